#!/usr/bin/env python
"""Key-switch throughput of RNS-CKKS at N = 2^16 on one MI355X, batched vs plain.

Workload (one step): 64 independent ciphertexts at N = 2^16 with a 24-prime
chain (one 60-bit base prime, 23 x 50-bit), hybrid key switching with 3 digits
of 8 primes and 8 special 60-bit primes; each ciphertext does mult_relin with a
second ciphertext, rescale, and 32 rotations (k = 1..32) hoisted over one
ModUp.  That is 64 x 33 = 2112 key switches per step.  Inputs are seeded
synthetic slot vectors, uniform in [-1, 1], encrypted under a uniform ternary
secret; all inputs are resident in HBM before the timed region.

* batched: one call per stage for all 64 ciphertexts (every NTT, base
  conversion and key inner product of the batch in one launch; each key word
  read once per launch);
* plain:   one call per ciphertext (mult_relin, rescale, hoisted rotations).

value = batched key switches per second.  The hoisted rotations' ModDowns
run on three lanes (side streams) unless --lanes 1.  Per-kernel HIP-event
timers run over a second pass of the same steps (not the timed one; kernels
do not overlap there); the kernel with the largest total time is reported
against the MI355X HBM roofline.  The CPU oracle is timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LOG_N = 16
Q_BITS = [60] + [50] * 23
P_BITS = [60] * 8
ALPHA = 8
SCALE = 2.0 ** 50
ROTS = list(range(1, 33))
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def log_free(torch, where):
    """Device memory left free after a part (torch's cache emptied first)."""
    import gc

    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    log("%s: %.1f of %.1f GiB free" % (where, free / 2.0 ** 30, total / 2.0 ** 30))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--count", type=int, default=64, help="ciphertexts per step")
    ap.add_argument("--rots", type=int, default=32, help="hoisted rotations per ciphertext")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ks", action="store_true", help="skip the key-switch part (the headline value is then null)")
    ap.add_argument("--no-boot", action="store_true", help="skip the bootstrap throughput part")
    ap.add_argument("--no-mlp", action="store_true", help="skip the MLP train_step part")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving part")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-ring-degree part")
    ap.add_argument("--no-paper-mlps", action="store_true", help="skip the paper's eMLP architectures")
    ap.add_argument("--train-small-b", type=int, default=8,
                    help="samples of the small-batch block-parallel timing of the train_step leg (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-lambda", type=float, default=0.0,
                    help="Poisson arrival rate, jobs/s (default: 0.8 x the capacity measured in the same run)")
    ap.add_argument("--serve-budget-gib", type=float, default=150.0)
    ap.add_argument("--no-serve-cross", action="store_true", help="no cross-tenant batching in the serving part")
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--serve-max-boot", type=int, default=16)
    ap.add_argument("--serve-mlp-b", type=int, default=8, help="samples per training step of serving jobs")
    ap.add_argument("--lanes", type=int, default=3,
                    help="side-stream lanes of hoisted-rotation ModDowns and bootstrap giant steps "
                         "(1: no overlapping kernels, as for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB device to device before the timed region (calibrates HBM byte counters)")
    return ap.parse_args()


def _tune_cache():
    """the autotuner's text cache (per user), or None when there is no cache directory"""
    d = os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(d, "rbk_tune.txt") if os.path.isdir(d) else None


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def setup(ctx, count, rots):
    import numpy as np

    import synth_inputs as S

    N, L = ctx.N, ctx.L
    g = S.rng(1, 16)
    s = S.ternary(g, N)
    ctx.set_secret(s)
    ctx.keygen_public(S.uniform_residues(g, ctx.moduli[: ctx.nQ], N), S.gaussian(g, N))
    a, e = S.key_randomness(g, ctx.beta, ctx.moduli, N)
    ctx.keygen_relin(a, e)
    for k in rots:
        a, e = S.key_randomness(g, ctx.beta, ctx.moduli, N)
        ctx.keygen_galois(ctx.galois_elt(k), a, e)
    A = ctx.empty_ct(L, count)
    B = ctx.empty_ct(L, count)
    z0 = []
    for i in range(count):
        for T in (A, B):
            z = S.uniform_slots(g, N // 2)
            if i == count - 1:
                z0.append(z)
            T[i].copy_(ctx.encrypt(ctx.encode(z, L, SCALE), L, *S.encryption_randomness(g, N)))
    ctx.sync()
    return s, A, B, z0


def batched_step(ctx, A, B, out_m, out_r, out_h, ks):
    L = ctx.L
    ctx.mult_relin_batch(A, B, L, out=out_m)
    ctx.rescale_batch(out_m, L, out=out_r)
    ctx.rotate_hoisted_batch(out_r, ks, L - 1, out=out_h)


def plain_ct(ctx, a, b, ks):
    L = ctx.L
    m = ctx.mult_relin(a, b, L)
    r = ctx.rescale(m, L)
    return ctx.rotate_hoisted(r, ks, L - 1)


BOOT_Q_BITS = [60] + [50] * 25
BOOT_P_BITS = [60] * 9
BOOT_ALPHA = 9


def bench_bootstrap(args, torch):
    """16 level-0 ciphertexts at scales 2^(35 + 10 i / 15), N = 2^16, full
    slots, HW-192 secret: batched (one call) vs plain (one call each)."""
    import numpy as np

    import synth_inputs as S
    from paper_2506_19693_amd import Context

    ctx = Context(LOG_N, BOOT_Q_BITS, BOOT_P_BITS, BOOT_ALPHA)
    ctx.set_lanes(args.lanes)
    ctx.boot_setup(K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2)
    N = ctx.N
    g = S.rng(3, 16)
    s = S.ternary_hw(g, N, 192)
    ctx.set_secret(s)
    ctx.keygen_public(S.uniform_residues(g, ctx.moduli[: ctx.nQ], N), S.gaussian(g, N))
    ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, N))
    for k in ctx.boot_rotations() + ["conj"]:
        gal = 2 * N - 1 if k == "conj" else ctx.galois_elt(k)
        ctx.keygen_galois(gal, *S.key_randomness(g, ctx.beta, ctx.moduli, N))
    count = 16
    tuned = ctx.autotune(ctx.L, count, _tune_cache())
    log("bootstrap: autotuned NTT split 2^%d, chunk %d, %d ciphertexts per inner-product thread" % (
        tuned["logC"], tuned["chunk"], tuned["cpc"]))
    scales = [2.0 ** (35 + 10 * i / 15) for i in range(count)]
    zs = [S.uniform_slots(g, N // 2) for _ in range(count)]
    cts = ctx.empty(count, 2, 1, N)
    for i in range(count):
        cts[i].copy_(ctx.encrypt(ctx.encode(zs[i], 0, scales[i]), 0, *S.encryption_randomness(g, N)))
    lo = ctx.boot_levels[3]
    out = ctx.empty_ct(lo, count)
    for _ in range(args.warmup):
        ctx.bootstrap_batch(cts, scales, out=out)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, so = ctx.bootstrap_batch(cts, scales, out=out)
    ctx.sync()
    t_b = (time.perf_counter() - t0) / args.steps
    err = max(float(np.max(np.abs(ctx.decode(ctx.decrypt(out[i], lo), lo, so[i]).real - zs[i]))) for i in range(count))
    # one more batched call with per-kernel timers and the key-switch count
    ctx.timer_enable(True)
    ctx.bootstrap_batch(cts, scales, out=out)
    ctx.sync()
    timers = ctx.timer_read()
    n_ks, ks_bytes = ctx.ks_stats()
    ctx.timer_enable(False)
    dom = max(timers, key=lambda k: timers[k][0])
    roof = ks_roofline(timers, dom, n_ks, ks_bytes, t_b, "bootstrap_c2")
    # the same batch captured once into a HIP graph and replayed
    out_g = ctx.empty_ct(lo, count)
    graph = ctx.capture(lambda: ctx.bootstrap_batch(cts, scales, out=out_g))
    graph.launch()
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    ctx.sync()
    t_g = (time.perf_counter() - t0) / args.steps
    graph_equal = bool(torch.equal(out_g, out))
    graph.close()
    lat = []
    t0 = time.perf_counter()
    for i in range(count):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.bootstrap(cts[i], scales[i])
        e1.record()
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1))
    t_p = time.perf_counter() - t0
    # the lower-failure-rate EvalMod: K = 25 with three double angles (one level more)
    ctx.boot_setup(K=25, degree=59, double_angle=3, cts_levels=3, stc_levels=3, log2_rho=2)
    lo25 = ctx.boot_levels[3]
    out25 = ctx.empty_ct(lo25, count)
    ctx.bootstrap_batch(cts, scales, out=out25)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, so25 = ctx.bootstrap_batch(cts, scales, out=out25)
    ctx.sync()
    t25 = (time.perf_counter() - t0) / args.steps
    err25 = max(float(np.max(np.abs(ctx.decode(ctx.decrypt(out25[i], lo25), lo25, so25[i]).real - zs[i])))
                for i in range(count))
    k25 = {"bootstraps_per_s_batched": count / t25, "output_level": lo25, "max_slot_error_log2": float(np.log2(err25)),
           "failure_rate_per_bootstrap": 1.3e-5}
    log("bootstrap K=25, r=3: %.2f/s batched, output level %d, max error 2^%.2f" % (
        count / t25, lo25, np.log2(err25)))
    res = {
        "workload": "bootstrap: 16 level-0 ciphertexts at scales 2^35..2^45, N=2^16, full 2^15 slots, HW-192 secret, "
                    "CtS/StC 3-level BSGS, EvalMod Chebyshev degree 59 + 2 double angles, 26 primes (60 + 25x50), "
                    "9 special primes",
        "bootstraps_per_s_batched": count / t_b,
        "bootstraps_per_s_plain": count / t_p,
        "bootstraps_per_s_graph": count / t_g,
        "graph_equals_eager": graph_equal,
        "batched_vs_plain": t_p / t_b,
        "ms_per_batch": t_b * 1e3,
        "plain_latency_ms_p50": percentile(lat, 50),
        "plain_latency_ms_p99": percentile(lat, 99),
        "output_level": lo,
        "max_slot_error_log2": float(np.log2(err)),
        "autotuned": tuned,
        "failure_rate_per_bootstrap": 3.0e-4,
        "evalmod_K25_r3": k25,
        "key_switches_per_bootstrap": n_ks / count,
        "roofline": roof,
        "kernels": {k: {"ms": round(v[0], 3), "launches": v[1], "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1)}
                    for k, v in timers.items()},
    }
    ctx.close()
    return res


MLP_Q_BITS = [60] + [50] * 27
MLP_P_BITS = [60] * 10
MLP_ALPHA = 10


def bench_train_step(args, torch):
    """The packed MLP training step at N = 2^16: 64 samples x 784 features
    uniform in [0, 1], one-hot labels over 10 classes; 784 -> 128 (RE block)
    -> 128 (CE block), each with a 10-way local classifier; degree-3
    activation z + z^2 + z^3/3; r = 256, c = 128, four input tiles; gamma =
    eta = 0.001, mu = 0.9; every W and V bootstrapped each step (14
    ciphertexts).  Batched (every operation on the 64 samples at once, each
    block's backward pass on a second stream beside the next block's
    forward pass) vs single-stream batched vs plain (one sample at a time)."""
    import numpy as np

    import synth_inputs as S
    from paper_2506_19693_amd import Context, Mlp

    k0, widths, o, r, c = 784, [128, 128], 10, 256, 128
    act = (1.0, 1.0, 1.0 / 3.0)
    b = 64
    ctx = Context(LOG_N, MLP_Q_BITS, MLP_P_BITS, MLP_ALPHA)
    ctx.set_lanes(args.lanes)
    ctx.boot_setup(K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2)
    mlp = Mlp(ctx, k0, widths, o, r, c, act=act, gamma=0.001, eta=0.001, mu=0.9, log2_scale=50.0)
    N = ctx.N
    g = S.rng(4, 16)
    ctx.set_secret(S.ternary_hw(g, N, 192))
    ctx.keygen_public(S.uniform_residues(g, ctx.moduli[: ctx.nQ], N), S.gaussian(g, N))
    ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, N))
    gals = sorted({ctx.galois_elt(k) for k in mlp.rotations() + ctx.boot_rotations()} | {2 * N - 1})
    for gal in gals:
        ctx.keygen_galois(gal, *S.key_randomness(g, ctx.beta, ctx.moduli, N))
    lo = ctx.boot_levels[3]
    T = 2.0 ** 50
    tiles = mlp.tiles
    tuned = ctx.autotune(lo, b, _tune_cache())
    log("train_step: autotuned NTT split 2^%d, chunk %d, %d ciphertexts per inner-product thread" % (
        tuned["logC"], tuned["chunk"], tuned["cpc"]))

    def enc(v):
        return ctx.encrypt(ctx.encode(v, lo, T), lo, *S.encryption_randomness(g, N))

    dims = [(k0, widths[0]), (widths[0], widths[1])]
    Ws = S.mlp_weights(g, dims)
    Wst = S.mlp_weights(g, [(k, o) for _, k in dims])
    # the state in the order W tiles, W*, V tiles, V* per block (V set by step 1)
    st = []
    for h, (W, Wsh) in enumerate(zip(Ws, Wst), start=1):
        M = np.zeros((r, c))
        if h == 1:
            for t in range(tiles):
                M[:] = 0.0
                blk = W[t * r: (t + 1) * r]
                M[: blk.shape[0], : blk.shape[1]] = blk
                st.append(M.ravel().copy())
            M[:] = 0.0
            M[:o, : Wsh.shape[0]] = Wsh.T
            st.append(M.ravel().copy())
            st += [None] * (tiles + 1)
        else:
            M[:] = 0.0
            M[: W.shape[1], : W.shape[0]] = W.T
            st.append(M.ravel().copy())
            M[:] = 0.0
            M[: Wsh.shape[0], : Wsh.shape[1]] = Wsh
            st.append(M.ravel().copy())
            st += [None, None]
    assert len(st) == mlp.n_state
    for i, v in enumerate(st):
        if v is not None:
            mlp.set_state(i, enc(v), lo, T)
    X, Y = S.mlp_batch(g, b, k0, o)
    x = ctx.empty(b, tiles, 2, lo + 1, N)
    ye = ctx.empty(b, 2, lo + 1, N)
    yr = ctx.empty(b, 2, lo + 1, N)
    for i in range(b):
        for t in range(tiles):
            M = np.zeros((r, c))
            seg = X[i, t * r: (t + 1) * r]
            M[: len(seg), :] = seg[:, None]
            x[i, t].copy_(enc(M.ravel()))
        M = np.zeros((r, c))
        M[:o, :] = Y[i][:, None]
        ye[i].copy_(enc(M.ravel()))
        M = np.zeros((r, c))
        M[:, :o] = Y[i]
        yr[i].copy_(enc(M.ravel()))
    ctx.sync()
    step = [1]

    def run(**kw):
        mlp.train_step(x, ye, yr, lo, T, step[0], **kw)
        step[0] += 1

    for _ in range(max(1, args.warmup)):
        run()
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    ctx.sync()
    t_b = (time.perf_counter() - t0) / args.steps
    # the same steps with every block's backward pass on the context stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(block_parallel=False)
    ctx.sync()
    t_s = (time.perf_counter() - t0) / args.steps
    # a small batch (8 samples), where one operation leaves the device part idle
    nb = min(args.train_small_b, b)
    xs, yes, yrs = x[:nb], ye[:nb], yr[:nb]

    def small(par):
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mlp.train_step(xs, yes, yrs, lo, T, step[0], block_parallel=par)
            step[0] += 1
        ctx.sync()
        return (time.perf_counter() - t0) / args.steps

    small_res = None
    if nb > 0:
        small(True)
        t_8p, t_8s = small(True), small(False)
        small_res = {"samples": nb, "ms_per_step_block_parallel": t_8p * 1e3,
                     "ms_per_step_single_stream": t_8s * 1e3, "block_parallel_gain": t_8s / t_8p}
    # one step captured into a HIP graph; each replay runs the next step
    graph = ctx.capture(lambda: mlp.train_step(x, ye, yr, lo, T, 2))
    graph.launch()
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    ctx.sync()
    t_g = (time.perf_counter() - t0) / args.steps
    graph.close()
    t0 = time.perf_counter()
    run(per_sample=True)
    ctx.sync()
    t_p = time.perf_counter() - t0
    ctx.timer_enable(True)               # one more step with per-kernel timers and the key-switch count
    run()
    ctx.sync()
    timers = ctx.timer_read()
    n_ks, ks_bytes = ctx.ks_stats()
    ctx.timer_enable(False)
    dom = max(timers, key=lambda k: timers[k][0])
    roof = ks_roofline(timers, dom, n_ks, ks_bytes, t_b, "train_step_c3")
    t0 = time.perf_counter()
    run(bootstrap=False)                  # the same step without its bootstrap (last: it leaves the state unrefreshed)
    ctx.sync()
    t_nb = time.perf_counter() - t0
    lr, lc = int(np.log2(r)), int(np.log2(c))
    rot_per_sample = (lr + 2 * lc + lr) + (2 * lc + lr + 2 * lc)
    res = {
        "workload": "packed MLP train_step: 64 samples x 784 features, 784->128 (RE)->128 (CE), 10-way local "
                    "classifiers, degree-3 activation, r=256 c=128 (4 input tiles), N=2^16, 28 primes (60 + 27x50), "
                    "10 special primes, HW-192 secret, bootstrap of all 14 W/V ciphertexts per step",
        "train_steps_per_s_batched": 1.0 / t_b,
        "train_steps_per_s_plain": 1.0 / t_p,
        "train_steps_per_s_graph": 1.0 / t_g,
        "train_steps_per_s_single_stream": 1.0 / t_s,
        "block_parallel_gain": t_s / t_b,
        "small_batch": small_res,
        "batched_vs_plain": t_p / t_b,
        "ms_per_step_batched": t_b * 1e3,
        "ms_per_step_plain": t_p * 1e3,
        "bootstrap_share_of_step": max(0.0, 1.0 - t_nb / t_b),
        "rotations_per_step": b * rot_per_sample,
        "bootstraps_per_step": mlp.n_state,
        "weight_level": lo,
        "depth": mlp.depth,
        "autotuned": tuned,
        "key_switches_per_step": n_ks,
        "roofline": roof,
        "kernels": {k: {"ms": round(v[0], 3), "launches": v[1], "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1)}
                    for k, v in timers.items()},
    }
    mlp.close()
    ctx.close()
    return res


SERVE_Q_BITS = [60] + [50] * 30
SERVE_P_BITS = [60] * 11
SERVE_ALPHA = 11
SERVE_LOG_NS = [14, 14, 14, 15, 15, 15, 16, 16]
# The Poisson arrival rate is this fraction of the capacity measured in the
# same run (all jobs submitted at once)
SERVE_LOAD = 0.8


def _dev_residues(ctx, gen, lead, level):
    """uniform residues [*lead][level+1][N] drawn on the device (inputs whose
    values do not matter to the cost of the operations)"""
    import torch

    t = torch.empty(*lead, level + 1, ctx.N, dtype=torch.int64, device="cuda")
    for i in range(level + 1):
        t[..., i, :] = torch.randint(0, ctx.moduli[i], (*lead, ctx.N), generator=gen, device="cuda",
                                     dtype=torch.int64)
    return t


class _Tenant:
    """A serving tenant: context with resident keys (relinearisation,
    bootstrap, MLP rotations at N = 2^16), input pools, MLPs."""

    def __init__(self, log_n, idx, rand_cache, mlp_b):
        import numpy as np

        import synth_inputs as S
        from paper_2506_19693_amd import Context, Mlp

        self.ctx = ctx = Context(log_n, SERVE_Q_BITS, SERVE_P_BITS, SERVE_ALPHA)
        ctx.boot_setup(K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2)
        N = ctx.N
        self.log_n = log_n
        g = S.rng(5, 100 + idx)
        ctx.set_secret(S.ternary_hw(g, N, 192))
        ctx.keygen_public(S.uniform_residues(g, ctx.moduli[: ctx.nQ], N), S.gaussian(g, N))
        self.mlps = {}
        if log_n == 16:
            for w in (64, 128, 256):
                widths = [w, w] if w <= 128 else [w]
                r, c = (256, 128) if w <= 128 else (128, 256)
                self.mlps[w] = Mlp(ctx, 784, widths, 10, r, c, act=(1.0, 1.0, 1.0 / 3.0), gamma=0.001, eta=0.001,
                                   mu=0.9, log2_scale=50.0)
        rots = set(ctx.boot_rotations())
        for m in self.mlps.values():
            rots |= set(m.rotations())
        gals = [0] + sorted({ctx.galois_elt(k) for k in rots} | {2 * N - 1})
        for i, gal in enumerate(gals):
            # the uniform part of a key is shared by the tenants of one ring degree (their secrets differ)
            key = (log_n, i)
            if key not in rand_cache:
                rand_cache[key] = S.key_randomness(S.rng(6, log_n, i), ctx.beta, ctx.moduli, N)
            a, e = rand_cache[key]
            if gal == 0:
                ctx.keygen_relin(a, e)
            else:
                ctx.keygen_galois(gal, a, e)
        L = ctx.L
        self.lo = ctx.boot_levels[3]
        T = 2.0 ** 50
        self.T = T
        # input pools: 64 ciphertext pairs at the top level (mult jobs read limbs 0..l),
        # 16 level-0 ciphertexts (bootstrap jobs)
        import torch

        gen = torch.Generator(device="cuda")
        gen.manual_seed(1000 + idx)
        self.A = _dev_residues(ctx, gen, (64, 2), L)
        self.B = _dev_residues(ctx, gen, (64, 2), L)
        self.C0 = _dev_residues(ctx, gen, (16, 2), 0)
        # result buffers shared by the tenant's jobs (the benchmark does not read results)
        self.out_mult = ctx.empty(64 * 2 * L * N)
        self.out_boot = ctx.empty(16 * 2 * (ctx.boot_levels[3] + 1) * N)
        self.mlp_in = {}
        lo = self.lo
        for w, m in self.mlps.items():
            r, c = (256, 128) if w <= 128 else (128, 256)
            X, Y = S.mlp_batch(g, mlp_b, 784, 10)
            enc = lambda v: ctx.encrypt(ctx.encode(v, lo, T), lo, *S.encryption_randomness(g, N))
            x = ctx.empty(mlp_b, m.tiles, 2, lo + 1, N)
            ye = ctx.empty(mlp_b, 2, lo + 1, N)
            yr = ctx.empty(mlp_b, 2, lo + 1, N)
            for i in range(mlp_b):
                for t in range(m.tiles):
                    M = np.zeros((r, c))
                    seg = X[i, t * r: (t + 1) * r]
                    M[: len(seg), :] = seg[:, None]
                    x[i, t].copy_(enc(M.ravel()))
                M = np.zeros((r, c))
                M[:10, :] = Y[i][:, None]
                ye[i].copy_(enc(M.ravel()))
                M = np.zeros((r, c))
                M[:, :10] = Y[i]
                yr[i].copy_(enc(M.ravel()))
            self.mlp_in[w] = (x, ye, yr)
            # random state at the weights' level and scale (the step's cost does not depend on the values)
            for i in range(m.n_state):
                m.set_state(i, _dev_residues(ctx, gen, (2,), lo), lo, T)
        ctx.sync()


def _serve_jobs(n_jobs, tenants, lam):
    """The job list: (arrival s, tenant, kind, params).  Types: mult+rescale
    batches (8..64 ciphertexts, levels 8..30), bootstraps (1..16), 1..3
    training steps (N = 2^16 tenants, widths 64 / 128 / 256)."""
    import numpy as np

    import synth_inputs as S

    g = S.rng(7, n_jobs)
    t = 0.0
    jobs = []
    mlp_tenants = [i for i, tn in enumerate(tenants) if tn.mlps]
    for _ in range(n_jobs):
        t += float(g.exponential(1.0 / lam)) if lam > 0 else 0.0
        u = g.uniform()
        if u < 0.55:
            ten = int(g.integers(0, len(tenants)))
            jobs.append((t, ten, "mult", dict(count=int(g.integers(8, 65)), level=int(g.integers(8, 31)))))
        elif u < 0.85:
            ten = int(g.integers(0, len(tenants)))
            n = int(g.integers(1, 17))
            jobs.append((t, ten, "boot", dict(count=n, scales=[2.0 ** float(g.uniform(35, 45)) for _ in range(n)])))
        else:
            ten = mlp_tenants[int(g.integers(0, len(mlp_tenants)))]
            jobs.append((t, ten, "train", dict(steps=int(g.integers(1, 4)), width=int((64, 128, 256)[g.integers(0, 3)]))))
    return jobs


_SERVE_CROSS = [True]   # cross-tenant batching of mult jobs (--no-serve-cross turns it off)


def _serve_run(tenants, jobs, budget, max_batch, max_boot, torch):
    """Submit at the arrival times; returns (makespan s, per-job latency ms, stats)."""
    import threading

    from paper_2506_19693_amd import Server

    srv = Server(budget, max_batch, max_boot)
    for tn in tenants:
        srv.add_tenant(tn.ctx)
    srv.set_cross_tenant(_SERVE_CROSS[0])
    srv.start()
    step = {id(tn): {w: 1 for w in tn.mlps} for tn in tenants}
    ids = []
    lock = threading.Lock()
    t0 = time.perf_counter()
    for (t_arr, ti, kind, p) in jobs:
        now = time.perf_counter() - t0
        if t_arr > now:
            time.sleep(t_arr - now)
        tn = tenants[ti]
        ctx = tn.ctx
        if kind == "mult":
            n, lv = p["count"], p["level"]
            out = tn.out_mult[: n * 2 * lv * ctx.N]
            ids.append(srv.submit_mult(ti, tn.A[:n], tn.B[:n], lv, out, in_level=ctx.L))
        elif kind == "boot":
            n = p["count"]
            out = tn.out_boot[: n * 2 * (tn.lo + 1) * ctx.N]
            ids.append(srv.submit_bootstrap(ti, tn.C0[:n], p["scales"], out)[0])
        else:
            w = p["width"]
            x, ye, yr = tn.mlp_in[w]
            with lock:
                t_first = step[id(tn)][w]
                step[id(tn)][w] += p["steps"]
            ids.append(srv.submit_train(ti, tn.mlps[w], x, ye, yr, tn.lo, tn.T, t_first, steps=p["steps"]))
    res = [srv.wait(j) for j in ids]
    srv.drain()
    makespan = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    return makespan, [r["latency_ms"] for r in res], stats


def _serial_run(tenants, jobs, torch):
    """Serial plain FIFO: one job at a time in arrival order, one ciphertext
    (or one sample) per call."""
    t0 = time.perf_counter()
    lat = []
    busy = 0.0
    step = {id(tn): {w: 10 ** 6 for w in tn.mlps} for tn in tenants}
    for (t_arr, ti, kind, p) in jobs:
        now = time.perf_counter() - t0
        if t_arr > now:
            time.sleep(t_arr - now)
        t_start = time.perf_counter()
        tn = tenants[ti]
        ctx = tn.ctx
        if kind == "mult":
            lv = p["level"]
            for i in range(p["count"]):
                a = tn.A[i][:, : lv + 1].contiguous()
                b = tn.B[i][:, : lv + 1].contiguous()
                ctx.rescale(ctx.mult_relin(a, b, lv), lv)
        elif kind == "boot":
            for i in range(p["count"]):
                ctx.bootstrap(tn.C0[i], p["scales"][i])
        else:
            w = p["width"]
            x, ye, yr = tn.mlp_in[w]
            for _ in range(p["steps"]):
                tn.mlps[w].train_step(x, ye, yr, tn.lo, tn.T, step[id(tn)][w], per_sample=True)
                step[id(tn)][w] += 1
        torch.cuda.synchronize()
        busy += time.perf_counter() - t_start
        lat.append((time.perf_counter() - t0 - t_arr) * 1e3)
    return time.perf_counter() - t0, lat, busy


def bench_serve(args, torch):
    """Serving workload: 8 tenants (N = 2^14 x 3, 2^15 x 3, 2^16 x 2; 31
    primes, 11 special; HW-192 secrets; resident relinearisation, bootstrap
    and MLP keys), Poisson arrivals of mixed jobs, served (continuous batching,
    HBM-ledger admission, per-tenant streams) vs serial plain FIFO."""
    _SERVE_CROSS[0] = not args.no_serve_cross
    rand_cache = {}
    tenants = [_Tenant(ln, i, rand_cache, args.serve_mlp_b) for i, ln in enumerate(SERVE_LOG_NS)]
    rand_cache.clear()
    free, total = torch.cuda.mem_get_info()
    log("serving: tenants set up, %.1f of %.1f GiB free" % (free / 2.0 ** 30, total / 2.0 ** 30))
    budget = int(args.serve_budget_gib * (1 << 30))
    # warm every tenant's workspaces and pools with one of each job kind
    _serve_run(tenants, [(0.0, i, "mult", dict(count=8, level=30)) for i in range(len(tenants))]
               + [(0.0, i, "boot", dict(count=2, scales=[2.0 ** 40] * 2)) for i in range(len(tenants))],
               budget, args.serve_max_batch, args.serve_max_boot, torch)
    log("serving: warm-up done, %.1f GiB free" % (torch.cuda.mem_get_info()[0] / 2.0 ** 30))
    # capacity: the job list submitted at once (the queue builds up, so batches merge)
    burst = [(0.0, i, k, p) for (_, i, k, p) in _serve_jobs(args.serve_jobs, tenants, 0.0)]
    mk_b, lat_b, st_b = _serve_run(tenants, burst, budget, args.serve_max_batch, args.serve_max_boot, torch)
    capacity = len(burst) / mk_b
    log("serving: burst of %d jobs done in %.1f s (%.2f jobs/s), %d batches, %d jobs merged" % (
        len(burst), mk_b, capacity, st_b["batches"], st_b["jobs_merged"]))
    lam = args.serve_lambda if args.serve_lambda > 0 else SERVE_LOAD * capacity
    jobs = _serve_jobs(args.serve_jobs, tenants, lam)
    mk, lat, stats = _serve_run(tenants, jobs, budget, args.serve_max_batch, args.serve_max_boot, torch)
    log("serving: Poisson run at %.2f jobs/s done in %.1f s, %d jobs merged (%d across tenants), %.1f GiB free" % (
        lam, mk, stats["jobs_merged"], stats["jobs_cross_tenant"], torch.cuda.mem_get_info()[0] / 2.0 ** 30))
    if stats["jobs_merged"] == 0:
        log("serving: WARNING: no job merged into another's batch at this arrival rate")
    out = {
        "workload": "serving: %d jobs, Poisson arrivals at %.2f jobs/s (%.2f x the capacity measured in this run), "
                    "8 tenants (N=2^14 x3, 2^15 x3, 2^16 x2), 31 primes (60 + 30x50) + 11 special, HW-192 secrets; "
                    "jobs: 55%% mult+rescale batches (8-64 ciphertexts, levels 8-30), 30%% bootstraps (1-16), 15%% "
                    "1-3 train_steps (784-w-w-10, w in 64/128; 784-256-10; %d samples) on the N=2^16 tenants; batch "
                    "caps %d ciphertexts (mult), %d (bootstrap)" % (
                        len(jobs), lam, lam / capacity, args.serve_mlp_b, args.serve_max_batch, args.serve_max_boot),
        "arrival_rate_jobs_per_s": lam,
        "jobs_per_s": len(jobs) / mk,
        "makespan_s": mk,
        "latency_ms_p50": percentile(lat, 50),
        "latency_ms_p99": percentile(lat, 99),
        "batches": stats["batches"],
        "jobs_merged": stats["jobs_merged"],
        "jobs_cross_tenant": stats["jobs_cross_tenant"],
        "cross_tenant_batching": _SERVE_CROSS[0],
        "ledger_peak_gib": stats["ledger_peak"] / 2.0 ** 30,
        "budget_gib": stats["budget"] / 2.0 ** 30,
        "burst": {
            "jobs_per_s": capacity,
            "makespan_s": mk_b,
            "latency_ms_p50": percentile(lat_b, 50),
            "latency_ms_p99": percentile(lat_b, 99),
            "batches": st_b["batches"],
            "jobs_merged": st_b["jobs_merged"],
            "jobs_cross_tenant": st_b["jobs_cross_tenant"],
        },
    }
    if not args.no_plain:
        mk_s, lat_s, busy_s = _serial_run(tenants, jobs, torch)
        log("serving: serial plain at the same arrivals done in %.1f s (%.1f s busy: %.2f jobs/s capacity)" % (
            mk_s, busy_s, len(jobs) / busy_s))
        out["serial_plain"] = {
            "capacity_jobs_per_s": len(jobs) / busy_s,
            "jobs_per_s": len(jobs) / mk_s,
            "makespan_s": mk_s,
            "latency_ms_p50": percentile(lat_s, 50),
            "latency_ms_p99": percentile(lat_s, 99),
        }
    for tn in tenants:
        for m in tn.mlps.values():
            m.close()
        tn.ctx.close()
    return out


def _oracle_worker(idx, barrier, out):
    """One ciphertext of the key-switch workload on the oracle: mult_relin +
    rescale + one hoisted rotation (2 key switches); the timed region starts
    when every worker is ready."""
    import oracle as O
    import synth_inputs as S

    orc = O.Oracle(LOG_N, Q_BITS, P_BITS, ALPHA)
    N, L = orc.N, orc.L
    g = S.rng(2, 16, idx)
    s = S.ternary(g, N)
    rlk = orc.keygen_relin(s, *S.key_randomness(g, orc.beta, orc.moduli, N))
    gal = orc.galois_rot(1)
    gk = orc.keygen_galois(s, gal, *S.key_randomness(g, orc.beta, orc.moduli, N))
    x = S.uniform_residues(g, orc.Q, N, lead=(2,))
    y = S.uniform_residues(g, orc.Q, N, lead=(2,))
    barrier.wait()
    t0 = time.perf_counter()
    m = orc.mult_relin(L, rlk, x, y)
    r = orc.rescale(L, m)
    orc.rotate_hoisted(L - 1, [gk], [gal], r)
    out.put(time.perf_counter() - t0)


# worker processes of the CPU oracle legs: every host core, at most the 16
# cores that one GPU's share of a GPU host is
CPU_WORKERS_CAP = 16


def cpu_workers():
    return max(1, min(CPU_WORKERS_CAP, os.cpu_count() or 1))


def cpu_baseline():
    """The oracle (plain C, one thread per process) on independent ciphertexts
    of the key-switch workload, one process per host core (at most 16): each
    does mult_relin + rescale + one hoisted rotation (2 key switches)."""
    import multiprocessing as mp

    workers = cpu_workers()
    nproc, model = _host_cpu()
    ctxm = mp.get_context("fork")
    barrier = ctxm.Barrier(workers)
    q = ctxm.Queue()
    procs = [ctxm.Process(target=_oracle_worker, args=(i, barrier, q)) for i in range(workers)]
    for p_ in procs:
        p_.start()
    dts = [q.get() for _ in procs]
    for p_ in procs:
        p_.join()
    wall = max(dts)
    return {
        "value": 2.0 * workers / wall,
        "unit": "key-switches/s",
        "cores": workers,
        "host_nproc": nproc,
        "host_cpu": model,
        "cores_cap": "one process per core up to %d (a GPU's share of the host)" % CPU_WORKERS_CAP,
        "kind": "oracle",
        "sample": "%d independent ciphertexts at N=2^16, 24 limbs, one oracle process per core: mult_relin + rescale "
                  "+ 1 hoisted rotation each (2 key switches), %.1f s wall (single-process time %.1f s)" % (
                      workers, wall, min(dts)),
    }


def bench_graph_small(args, torch):
    """Launch-bound work where a captured graph pays: the small-ring pipeline
    (N = 2^12, 50 + 3 x 40-bit chain, one 50-bit special prime, one prime per
    digit): mult_relin -> rescale -> rotations +1 and +7 (hoisted) -> add, on
    one ciphertext pair, eager (one launch sequence per call) vs one graph
    replay."""
    import numpy as np

    from paper_2506_19693_amd import Context

    ctx = Context(12, [50, 40, 40, 40], [50], 1)
    ctx.set_lanes(1)
    ctx.keygen(5, 0, [1, 7])
    N, L = ctx.N, ctx.L
    g = np.random.default_rng(5)
    x = ctx.empty_ct(L, 1)
    y = ctx.empty_ct(L, 1)
    zx, zy = g.uniform(-1, 1, N // 2), g.uniform(-1, 1, N // 2)
    x[0].copy_(ctx.encrypt_seeded(ctx.encode(zx, L, 2.0 ** 40), L, 5, 0))
    y[0].copy_(ctx.encrypt_seeded(ctx.encode(zy, L, 2.0 ** 40), L, 5, 1))
    m = ctx.empty_ct(L, 1)
    r = ctx.empty_ct(L - 1, 1)
    h = ctx.empty(1, 2, 2, L, N)
    out = ctx.empty_ct(L - 1)

    def pipeline():
        ctx.mult_relin_batch(x, y, L, out=m)
        ctx.rescale_batch(m, L, out=r)
        ctx.rotate_hoisted_batch(r, [1, 7], L - 1, out=h)
        _check_rc(ctx, ctx.lib.rbk_add(ctx.h, _dptr(h[0, 0]), _dptr(h[0, 1]), _dptr(out), L - 1, 2))

    pipeline()
    ctx.sync()
    want = out.clone()
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        pipeline()
    ctx.sync()
    t_e = (time.perf_counter() - t0) / reps
    graph = ctx.capture(pipeline)
    graph.launch()
    ctx.sync()
    same = bool(torch.equal(out, want))
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.launch()
    ctx.sync()
    t_g = (time.perf_counter() - t0) / reps
    graph.close()
    s_out = 2.0 ** 80 / ctx.moduli[L]
    got = ctx.decode(ctx.decrypt(out, L - 1), L - 1, s_out).real
    p = zx * zy
    err = float(np.max(np.abs(got - (np.roll(p, -1) + np.roll(p, -7)))))
    ctx.close()
    return {
        "workload": "N=2^12, 50 + 3x40-bit chain + one 50-bit special prime, one prime per digit: mult_relin, "
                    "rescale, hoisted rotations +1 and +7, add, on one ciphertext pair",
        "eager_us": t_e * 1e6,
        "graph_us": t_g * 1e6,
        "graph_speedup": t_e / t_g,
        "graph_equals_eager": same,
        "max_slot_error_log2": float(np.log2(err)),
    }


def _dptr(t):
    import ctypes

    return ctypes.c_void_p(t.data_ptr())


def _check_rc(ctx, rc):
    if rc < 0:
        raise RuntimeError("librbk error %d: %s" % (rc, ctx.lib.rbk_last_error().decode()))


# The paper's own architectures (Section 5.1, Table 3) on synthetic
# MNIST-shaped data (784 features in [0, 1), 10 one-hot classes; Table 8's
# MNIST settings: b = 48, gamma = 0.001, eta = 0.001 / 0.005):
#   eMLP-1: RE-Block(32), N = 2^16, depth 8;   eMLP-2: RE-Block(64) -> CE-Block(32), N = 2^17, depth 11.
# Chains: depth + the 14 levels this bootstrap consumes, 49-bit primes for
# eMLP-1 (Delta = 2^49); eMLP-2 uses 50-bit primes (Delta = 2^50: the
# bootstrap's q_0 / Delta >= 4 with a 60-bit q_0 excludes the paper's 2^59).
PAPER_MLPS = {
    "eMLP-1": dict(logN=16, widths=[32], r=1024, c=32, qbits=[60] + [49] * 22, pbits=[60] * 8, alpha=8,
                   log2_scale=49.0, eta=0.001),
    "eMLP-2": dict(logN=17, widths=[64, 32], r=1024, c=64, qbits=[60] + [50] * 25, pbits=[60] * 9, alpha=9,
                   log2_scale=50.0, eta=0.005),
}


def bench_paper_mlp(name, args, torch):
    """Seconds per encrypted training iteration of one of the paper's
    architectures: keys and encryptions drawn in the library from a seed,
    float64 weights set through the library, 48 samples per step, every
    weight and velocity bootstrapped each step."""
    import numpy as np

    import synth_inputs as S
    from paper_2506_19693_amd import Context, Mlp

    p = PAPER_MLPS[name]
    k0, o, b = 784, 10, 48
    ctx = Context(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    ctx.boot_setup(K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2)
    mlp = Mlp(ctx, k0, p["widths"], o, p["r"], p["c"], act=(1.0, 1.0, 0.0), gamma=0.001, eta=p["eta"], mu=0.9,
              log2_scale=p["log2_scale"])
    lo = ctx.boot_levels[3]
    if lo < mlp.depth:
        raise RuntimeError("%s: bootstrap output level %d below the step's depth %d" % (name, lo, mlp.depth))
    t0 = time.perf_counter()
    ctx.keygen(21, 192, sorted(set(mlp.rotations()) | set(ctx.boot_rotations())), conj=True)
    g = S.rng(22, p["logN"])
    dims = [(k0, p["widths"][0])] + [(p["widths"][h - 1], p["widths"][h]) for h in range(1, len(p["widths"]))]
    mlp.set_weights(S.mlp_weights(g, dims), S.mlp_weights(g, [(k, o) for _, k in dims]), level=lo, seed=23)
    X, Y = S.mlp_batch(g, b, k0, o)
    r, c, N = p["r"], p["c"], ctx.N
    T = 2.0 ** p["log2_scale"]
    tiles = mlp.tiles
    x = ctx.empty(b, tiles, 2, lo + 1, N)
    ye = ctx.empty(b, 2, lo + 1, N)
    yr = ctx.empty(b, 2, lo + 1, N)
    idx = 1000
    for i in range(b):
        for t in range(tiles):
            M = np.zeros((r, c))
            seg = X[i, t * r: (t + 1) * r]
            M[: len(seg), :] = seg[:, None]
            x[i, t].copy_(ctx.encrypt_seeded(ctx.encode(M.ravel(), lo, T), lo, 23, idx))
            idx += 1
        M = np.zeros((r, c))
        M[:o, :] = Y[i][:, None]
        ye[i].copy_(ctx.encrypt_seeded(ctx.encode(M.ravel(), lo, T), lo, 23, idx))
        M = np.zeros((r, c))
        M[:, :o] = Y[i]
        yr[i].copy_(ctx.encrypt_seeded(ctx.encode(M.ravel(), lo, T), lo, 23, idx + 1))
        idx += 2
    ctx.sync()
    t_setup = time.perf_counter() - t0
    step = 1
    for _ in range(max(1, args.warmup)):
        mlp.train_step(x, ye, yr, lo, T, step)
        step += 1
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mlp.train_step(x, ye, yr, lo, T, step)
        step += 1
    ctx.sync()
    t_it = (time.perf_counter() - t0) / args.steps
    Ws, Wst, Vs, Vst = mlp.get_weights(dims, o)
    finite = all(np.all(np.isfinite(w)) and np.max(np.abs(w)) < 4.0 for w in Ws + Wst + Vs + Vst)
    # encrypted inference of the same 48 samples through every local classifier (early exit at block 1 .. H)
    H = len(p["widths"])
    t_inf = {}
    for last in sorted({1, H}):
        mlp.infer(x, lo, T, last)
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mlp.infer(x, lo, T, last)
        ctx.sync()
        t_inf["exit_after_block_%d" % last] = (time.perf_counter() - t0) / args.steps
    res = {
        "workload": "%s (paper Table 3): %s, N=2^%d, %d primes (%s) + %d special, HW-192 secret, 784 -> %s -> 10 "
                    "classes, r=%d c=%d, %d samples per step, paper activation z + z^2, gamma 0.001, eta %g, mu 0.9; "
                    "every W and V bootstrapped each step" % (
                        name, " -> ".join(("RE" if h % 2 == 0 else "CE") + "(%d)" % w for h, w in enumerate(p["widths"])),
                        p["logN"], len(p["qbits"]), "60 + %dx%d" % (len(p["qbits"]) - 1, p["qbits"][1]),
                        len(p["pbits"]), "-".join(str(w) for w in p["widths"]), r, c, b, p["eta"]),
        "s_per_iteration": t_it,
        "depth": mlp.depth,
        "weight_level": lo,
        "setup_s": t_setup,
        "weights_decrypt_finite_and_bounded": bool(finite),
        "inference_s_per_batch": t_inf,
        "paper_cpu_s_per_iteration": {"eMLP-1": 190.32, "eMLP-2": 629.65}[name],
        "paper_hardware": "2x Intel Xeon Gold 5318S, OpenFHE (context only: other hardware, other software)",
    }
    mlp.close()
    ctx.close()
    return res


MIXED_RINGS = [14, 15, 16]
MIXED_COUNT = 16


def bench_mixed(args, torch):
    """Mixed ring degrees: 16 ciphertexts at each of N = 2^14, 2^15, 2^16 (the
    serving chain, 31 primes + 11 special, at levels 8..30), each multiplied,
    relinearised and rescaled: one multi-context call vs one batched call per
    context vs one call per ciphertext."""
    import synth_inputs as S
    from paper_2506_19693_amd import Context, rbk

    ctxs = [Context(ln, SERVE_Q_BITS, SERVE_P_BITS, SERVE_ALPHA) for ln in MIXED_RINGS]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    g = S.rng(12, 1)
    jobs, per_ctx = [], []
    for ctx in ctxs:
        N = ctx.N
        ctx.set_secret(S.ternary(g, N))
        ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, N))
        levels = [int(x) for x in g.integers(8, 31, size=MIXED_COUNT)]
        lm = max(levels)
        A = _dev_residues(ctx, gen, (MIXED_COUNT, 2), lm)
        B = _dev_residues(ctx, gen, (MIXED_COUNT, 2), lm)
        mine = []
        for i, lv in enumerate(levels):
            a = A[i][:, : lv + 1].contiguous()
            b = B[i][:, : lv + 1].contiguous()
            jobs.append((ctx, a, b, lv))
            mine.append((a, b, lv))
        per_ctx.append((ctx, A, B, levels))
    host = ctxs[0]
    outs = [c.empty_ct(lv - 1) for c, _, _, lv in jobs]

    def multi():
        rbk.mult_relin_rescale_multi(host, jobs, outs)

    def per_context():
        for ctx, A, B, levels in per_ctx:
            ctx.mult_relin_rescale_list(A, B, levels)

    def plain():
        for ctx, a, b, lv in jobs:
            ctx.rescale(ctx.mult_relin(a, b, lv), lv)

    res = {"workload": "mixed ring degrees: %d ciphertexts at each of N=2^14, 2^15, 2^16, levels 8-30 of a 31-prime "
                       "chain (60 + 30x50) + 11 special primes, mult_relin + rescale each" % MIXED_COUNT,
           "key_switches_per_call": len(jobs)}
    for name, fn in (("multi_context_call", multi), ("per_context_list_calls", per_context), ("plain", plain)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"ms": dt * 1e3, "key_switches_per_s": len(jobs) / dt}
    res["multi_vs_plain"] = res["plain"]["ms"] / res["multi_context_call"]["ms"]
    res["multi_vs_per_context"] = res["per_context_list_calls"]["ms"] / res["multi_context_call"]["ms"]
    del jobs, outs, per_ctx
    for c in ctxs:
        c.close()
    return res


# ---------------------------------------------------------------- oracle cost of the bootstrap and train_step legs

def _host_cpu():
    """(nproc, CPU model) of this host"""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


class _OpCounter:
    """Stands in for the oracle inside the oracle's own bootstrap and MLP
    code: records every ciphertext operation with its level and returns
    placeholder arrays of the right limb count (one coefficient each)."""

    def __init__(self, orc):
        self.N = orc.N
        self.nQ, self.nP = orc.nQ, orc.nP
        self.moduli = orc.moduli
        self.Q = orc.Q
        self.ops = []
        self.orc = orc

    def _ct(self, level, npoly=2):
        import numpy as np

        return np.zeros((npoly, level + 1, 1), dtype=np.uint64)

    def _rec(self, op, level, n=1):
        self.ops.append((op, level, n))

    def galois_rot(self, k):
        return self.orc.galois_rot(k)

    def galois_conj(self):
        return 2 * self.N - 1

    def drop(self, lf, lt, ct):
        return ct[..., : lt + 1, :]

    def mult_relin(self, level, rlk, a, b):
        self._rec("mult_relin", level)
        return self._ct(level)

    def rotate(self, level, key, g, ct):
        self._rec("rotate", level)
        return self._ct(level)

    def rotate_hoisted(self, level, keys, gs, ct):
        self._rec("hoisted", level, len(keys))
        return [self._ct(level) for _ in keys]

    def rescale(self, level, ct):
        self._rec("rescale", level)
        return self._ct(level - 1, ct.shape[0])

    def _ew(self, name, level, a):
        self._rec(name, level)
        return self._ct(level, a.shape[0] if a.ndim == 3 else 1)

    def add(self, level, a, b):
        return self._ew("add", level, a)

    def sub(self, level, a, b):
        return self._ew("add", level, a)

    def mul_plain(self, level, ct, pt):
        return self._ew("mul_plain", level, ct)

    def mul_scalar(self, level, a, sc):
        return self._ew("mul_scalar", level, a)

    def add_scalar(self, level, ct, sc):
        return self._ew("add", level, ct)

    def monomial(self, level, e, a):
        return self._ew("add", level, a)

    def modraise(self, level, ct0):
        self._rec("add", level)
        return self._ct(level)


def _op_sample_worker(idx, qbits, pbits, alpha, barrier, out):
    """Times, at the top level of the chain, of the oracle operations the
    bootstrap and the training step are made of: ModUp, key inner product,
    ModDown, tensor product, rescale and the element-wise products / sums."""
    import numpy as np

    import oracle as O
    import synth_inputs as S

    orc = O.Oracle(LOG_N, qbits, pbits, alpha)
    N, L = orc.N, orc.L
    g = S.rng(9, 16, idx)
    s = S.ternary(g, N)
    rlk = orc.keygen_relin(s, *S.key_randomness(g, orc.beta, orc.moduli, N))
    x = S.uniform_residues(g, orc.Q, N, lead=(2,))
    y = S.uniform_residues(g, orc.Q, N, lead=(2,))
    pt = S.uniform_residues(g, orc.Q, N)
    sc = np.array([3 % q for q in orc.Q], dtype=np.uint64)
    barrier.wait()
    t = {}
    t0 = time.perf_counter()
    ext = orc.modup(L, x[1])
    t["modup"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    u = orc.key_inner_product(L, ext, rlk)
    t["ip"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.moddown(L, u[0])
    t["moddown"] = 2 * (time.perf_counter() - t0)          # both polynomials
    for name, fn in (("tensor", lambda: orc.tensor(L, x, y)),
                     ("rescale", lambda: orc.rescale(L, x)),
                     ("mul_plain", lambda: orc.mul_plain(L, x, pt)),
                     ("mul_scalar", lambda: orc.mul_scalar(L, x, sc)),
                     ("add", lambda: orc.add(L, x, y))):
        t0 = time.perf_counter()
        fn()
        t[name] = time.perf_counter() - t0
    out.put(t)


def _op_times(qbits, pbits, alpha, workers):
    """Median over `workers` concurrent processes of the per-operation times."""
    import multiprocessing as mp

    ctxm = mp.get_context("fork")
    barrier = ctxm.Barrier(workers)
    q = ctxm.Queue()
    procs = [ctxm.Process(target=_op_sample_worker, args=(i, qbits, pbits, alpha, barrier, q)) for i in range(workers)]
    for p_ in procs:
        p_.start()
    res = [q.get() for _ in procs]
    for p_ in procs:
        p_.join()
    med = {}
    for k in res[0]:
        v = sorted(r[k] for r in res)
        med[k] = v[len(v) // 2]
    return med


def _oracle_seconds(ops, t, L0, k0, k):
    """Oracle time of an operation list, from the top-level op times t of a
    chain with top level L0 and k0 special primes: key-switching work scales
    with the extended basis (l+1+k), element-wise work with (l+1), rescale
    with l.  A rotation is a ModUp, an inner product and a ModDown (plus the
    automorphism, priced as an addition); a hoisted call of n rotations is
    one ModUp plus n inner products and ModDowns; mult_relin adds the tensor
    product."""
    up, md = t["modup"], t["ip"] + t["moddown"]
    tot = 0.0
    for op, l, n in ops:
        ks = (l + 1 + k) / (L0 + 1 + k0)
        ew = (l + 1) / (L0 + 1)
        if op == "rotate":
            tot += (up + md) * ks + t["add"] * ew
        elif op == "hoisted":
            tot += (up + n * md) * ks + n * t["add"] * ew
        elif op == "mult_relin":
            tot += (up + md) * ks + (t["tensor"] + t["add"]) * ew
        elif op == "rescale":
            tot += t["rescale"] * max(l, 1) / L0
        elif op in ("mul_plain", "mul_scalar", "add"):
            tot += t[op] * ew
    return tot


def cpu_baseline_boot_and_train(workers):
    """Oracle bootstraps/s and train_steps/s on the host cores, from a
    bounded sample: every worker process times each ciphertext operation
    once at the top level of the bootstrap chain (N = 2^16, 26 primes, 9
    special); the op lists of one bootstrap and of one training step come
    from running the oracle's own bootstrap and packed-step code with an
    operation counter in place of the arithmetic; each op is priced by its
    level; the workers run independent bootstraps (steps) in parallel."""
    import oracle as O
    from oracle import boot as B
    from oracle import mlp as M

    t_wall = time.perf_counter()
    t = _op_times(BOOT_Q_BITS, BOOT_P_BITS, BOOT_ALPHA, workers)
    L0, k0 = len(BOOT_Q_BITS) - 1, len(BOOT_P_BITS)
    # one bootstrap
    orc = O.Oracle(LOG_N, BOOT_Q_BITS, BOOT_P_BITS, BOOT_ALPHA)
    plan = B.Plan(orc.N, orc.Q, B.BootParams(log2_rho=2))
    cnt = _OpCounter(orc)
    from collections import defaultdict

    B.Evaluator(cnt, plan, None, defaultdict(lambda: None)).bootstrap(cnt._ct(0), 2.0 ** 40)
    boot_ops = list(cnt.ops)
    t_boot = _oracle_seconds(boot_ops, t, L0, k0, k0)
    n_ks = sum(n for op, _, n in boot_ops if op in ("rotate", "hoisted", "mult_relin"))
    # one training step (64 samples, 14 bootstraps), on the training chain
    orc_m = O.Oracle(LOG_N, MLP_Q_BITS, MLP_P_BITS, MLP_ALPHA)
    plan_m = B.Plan(orc_m.N, orc_m.Q, B.BootParams(log2_rho=2))
    cnt_m = _OpCounter(orc_m)
    cfg = M.MlpConfig(k0=784, widths=[128, 128], o=10, r=256, c=128, act=(1.0, 1.0, 1.0 / 3.0), gamma=0.001,
                      eta=0.001, mu=0.9, log2_scale=50.0)
    ev = B.Evaluator(cnt_m, plan_m, None, defaultdict(lambda: None))
    ev.plan = plan_m
    ops = M.EncOps(cnt_m, cfg, None, defaultdict(lambda: None), boot=ev)
    ops.masks = {lv: None for lv in range(orc_m.nQ)}
    lo, T = plan_m.level_out, 2.0 ** 50
    state = [M.Ct(cnt_m._ct(lo), lo, T) for _ in cfg.state_layout()]
    smp = [([M.Ct(cnt_m._ct(lo), lo, T) for _ in range(cfg.tiles)], M.Ct(cnt_m._ct(lo), lo, T),
            M.Ct(cnt_m._ct(lo), lo, T)) for _ in range(64)]
    M.packed_step(ops, cfg, state, smp, 2)
    t_step = _oracle_seconds(cnt_m.ops, t, L0, k0, len(MLP_P_BITS))
    n_ks_step = sum(n for op, _, n in cnt_m.ops if op in ("rotate", "hoisted", "mult_relin"))
    wall = time.perf_counter() - t_wall
    sample = ("each of %d processes times ModUp, key inner product, ModDown, tensor, rescale, mul_plain, mul_scalar "
              "and add once at N=2^16, level 25 (26 primes + 9 special); the oracle's own bootstrap / packed-step "
              "code run with an operation counter gives the op list, each op priced by its level "
              "(key switching x (l+1+k), element-wise x (l+1)); %.1f s wall" % (workers, wall))
    return t, {
        "value": workers / t_boot,
        "unit": "bootstraps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": sample,
        "extrapolated_oracle_s_per_bootstrap": t_boot,
        "key_switches_per_bootstrap": n_ks,
        "ops_per_bootstrap": len(boot_ops),
    }, {
        "value": workers / t_step,
        "unit": "train_steps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": sample,
        "extrapolated_oracle_s_per_step": t_step,
        "key_switches_per_step": n_ks_step,
    }


def _counters(profile, dom):
    """(HBM bytes per launch, VALUBusy %) of kernel class `dom` from the committed
    rocprofv3 counter runs, or None each when absent or taken on another source
    of the kernel."""
    import hashlib

    traffic = valu = None
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", profile + "_hbm_counters.json")))
        ent = prof["kernels"].get(dom)
        if ent and hashlib.sha256(open(os.path.join(ROOT, ent["source"]), "rb").read()).hexdigest() == ent["source_sha256"]:
            traffic = ent["hbm_bytes_per_launch"]
            valu = ent.get("valu_busy_pct")
    except (OSError, KeyError, ValueError):
        pass
    return traffic, valu


def ks_roofline(timers, dom, n_ks, ks_bytes, t_total_s, profile):
    """The roofline block: the dominant kernel's achieved rate on method bytes
    (the key switches it finishes per launch x the per-key-switch minimum:
    the switched polynomial read, one polynomial written, the level's key
    words once per call) next to its rate on its own I/O, and the rate of the
    whole measured region on method bytes."""
    ms, n, bts = timers[dom]
    traffic, valu = _counters(profile, dom)
    per_launch = ks_bytes / n if dom == "ntt_rows_fwd+moddown_ip" and n else None
    achieved = ks_bytes / (ms * 1e-3) / 1e9 if per_launch else bts / (ms * 1e-3) / 1e9
    io = bts / (ms * 1e-3) / 1e9
    return {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated by a 1 GiB copy)",
        "method_bytes_per_launch": per_launch,
        "key_switches_per_launch": n_ks / n if per_launch else None,
        "avg_launch_us": round(1e3 * ms / n, 2),
        "launches": n,
        "kernel_io": {"bytes_per_launch": bts / n, "GBps": round(io, 1), "frac": round(io / HBM_PEAK_GBS, 4)},
        "valu_busy_pct": valu,
        "whole_region": {
            "key_switches": n_ks,
            "method_bytes": ks_bytes,
            "GBps": round(ks_bytes / t_total_s / 1e9, 1),
            "frac": round(ks_bytes / t_total_s / 1e9 / HBM_PEAK_GBS, 4),
        },
    }


def bench_keyswitch(args, torch):
    """The key-switch workload (module docstring): batched and plain, kernel timers, roofline."""
    from paper_2506_19693_amd import Context

    count, ks = args.count, ROTS[: args.rots]
    log("setup: N=2^16, %d limbs, %d special, alpha %d, %d ciphertexts, %d rotations" % (
        len(Q_BITS), len(P_BITS), ALPHA, count, len(ks)))
    t0 = time.time()
    ctx = Context(LOG_N, Q_BITS, P_BITS, ALPHA)
    ctx.set_lanes(args.lanes)
    s, A, B, z_last = setup(ctx, count, ks)
    L = ctx.L
    ctx.reserve(L, count)
    tuned = ctx.autotune(L - 1, count, _tune_cache())
    log("autotuned: NTT split 2^%d columns, NTT chunk %d limbs, %d ciphertexts per inner-product thread" % (
        tuned["logC"], tuned["chunk"], tuned["cpc"]))
    out_m = ctx.empty_ct(L, count)
    out_r = ctx.empty_ct(L - 1, count)
    out_h = ctx.empty(count, len(ks), 2, L, ctx.N)
    log("setup done in %.1f s" % (time.time() - t0))
    ks_per_step = count * (1 + len(ks))

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------------------------------------------------------- batched
    for _ in range(args.warmup):
        batched_step(ctx, A, B, out_m, out_r, out_h, ks)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        batched_step(ctx, A, B, out_m, out_r, out_h, ks)
    ctx.sync()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    log("batched: %.2f ms/step, %.0f key-switches/s" % (t_batched * 1e3, ks_per_step / t_batched))
    # the same steps again with per-kernel HIP-event timers (kept out of the
    # headline: an event pair around every launch adds a little time)
    ctx.timer_enable(True)
    for i in range(args.steps):
        batched_step(ctx, A, B, out_m, out_r, out_h, ks)
    ctx.sync()
    torch.cuda.synchronize()
    timers = ctx.timer_read()
    n_ks, ks_bytes = ctx.ks_stats()
    ctx.timer_enable(False)

    # correctness spot check of the timed output: the last ciphertext's first,
    # middle and last rotation decrypt to the rotated slot-wise product
    import numpy as np

    prod = z_last[0] * z_last[1]
    s_out = SCALE * SCALE / ctx.moduli[L]
    check = 0.0
    for j in sorted({0, len(ks) // 2, len(ks) - 1}):
        got = ctx.decode(ctx.decrypt(out_h[count - 1, j], L - 1), L - 1, s_out).real
        check = max(check, float(np.max(np.abs(got - np.roll(prod, -ks[j])))))
    log("spot check: rotations of the last ciphertext decrypt within 2^%.1f of the rotated product" % np.log2(check))
    if not check < 2.0 ** -20:
        raise RuntimeError("the timed key-switch output does not decrypt to the expected slots (error %g)" % check)

    # ---------------------------------------------------------------- plain
    plain = None
    if not args.no_plain:
        for _ in range(args.warmup):
            for i in range(count):
                plain_ct(ctx, A[i], B[i], ks)
        ctx.sync()
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            evs = []
            for i in range(count):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                plain_ct(ctx, A[i], B[i], ks)
                e1.record()
                evs.append((e0, e1))
            torch.cuda.synchronize()
            lat += [a.elapsed_time(b) for a, b in evs]
        t_plain = (time.perf_counter() - t0) / args.steps
        plain = {
            "ms_per_step": t_plain * 1e3,
            "key_switches_per_s": ks_per_step / t_plain,
            "per_ct_latency_ms_p50": percentile(lat, 50),
            "per_ct_latency_ms_p99": percentile(lat, 99),
        }
        log("plain: %.2f ms/step, %.0f key-switches/s, p50 %.2f ms p99 %.2f ms per ciphertext" % (
            t_plain * 1e3, ks_per_step / t_plain, plain["per_ct_latency_ms_p50"], plain["per_ct_latency_ms_p99"]))

    # ---------------------------------------------------------------- roofline of the dominant kernel
    kern = {k: {"ms_total": v[0], "launches": v[1], "avg_us": 1e3 * v[0] / v[1], "GBps": v[2] / (v[0] * 1e-3) / 1e9}
            for k, v in timers.items()}
    dom = max(timers, key=lambda k: timers[k][0])
    roofline = ks_roofline(timers, dom, n_ks, ks_bytes, t_batched * args.steps, "keyswitch_c1")
    roofline["share_of_step"] = round(timers[dom][0] / (t_batched * 1e3 * args.steps), 3)

    # release the key-switch workload before the next parts
    del out_m, out_r, out_h, A, B
    ctx.close()
    torch.cuda.empty_cache()
    return {
        "value": ks_per_step / t_batched,
        "ms_per_step": t_batched * 1e3,
        "count": count,
        "rots": len(ks),
        "ks_per_step": ks_per_step,
        "tuned": tuned,
        "plain": plain,
        "roofline": roofline,
        "kernels": kern,
    }



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    log_free(torch, "start")
    ksw = None
    if not args.no_ks:
        ksw = bench_keyswitch(args, torch)
        log_free(torch, "after key switches")

    boot = None
    if not args.no_boot:
        log("bootstrap: 16 ciphertexts, N=2^16 ...")
        boot = bench_bootstrap(args, torch)
        log("bootstrap: %.2f/s batched, %.2f/s graph, %.2f/s plain, p99 %.1f ms, max error 2^%.2f" % (
            boot["bootstraps_per_s_batched"], boot["bootstraps_per_s_graph"], boot["bootstraps_per_s_plain"],
            boot["plain_latency_ms_p99"], boot["max_slot_error_log2"]))
        log_free(torch, "after bootstraps")

    mlp = None
    if not args.no_mlp:
        torch.cuda.empty_cache()
        log("train_step: 784-128-128, 64 samples, N=2^16 ...")
        mlp = bench_train_step(args, torch)
        log("train_step: %.3f steps/s batched (%.0f ms), %.3f graph, %.3f plain, bootstrap share %.2f" % (
            mlp["train_steps_per_s_batched"], mlp["ms_per_step_batched"], mlp["train_steps_per_s_graph"],
            mlp["train_steps_per_s_plain"], mlp["bootstrap_share_of_step"]))
        log_free(torch, "after training steps")

    paper = None
    if not args.no_paper_mlps:
        paper = {}
        for name in PAPER_MLPS:
            torch.cuda.empty_cache()
            log("%s: ..." % name)
            paper[name] = bench_paper_mlp(name, args, torch)
            log("%s: %.2f s per iteration (paper, on CPUs: %.2f s)" % (
                name, paper[name]["s_per_iteration"], paper[name]["paper_cpu_s_per_iteration"]))
            log_free(torch, "after " + name)

    small = None
    if not args.no_mixed:
        small = bench_graph_small(args, torch)
        log("small ring pipeline: eager %.1f us, graph %.1f us (%.2fx), graph == eager: %s, error 2^%.1f" % (
            small["eager_us"], small["graph_us"], small["graph_speedup"], small["graph_equals_eager"],
            small["max_slot_error_log2"]))
        log_free(torch, "after the small ring pipeline")

    mixed = None
    if not args.no_mixed:
        torch.cuda.empty_cache()
        log("mixed rings: 3 x %d ciphertexts at N=2^14, 2^15, 2^16 ..." % MIXED_COUNT)
        mixed = bench_mixed(args, torch)
        log("mixed rings: one call %.2f ms, per-context calls %.2f ms, plain %.2f ms" % (
            mixed["multi_context_call"]["ms"], mixed["per_context_list_calls"]["ms"], mixed["plain"]["ms"]))
        log_free(torch, "after mixed rings")

    serve = None
    if not args.no_serve:
        torch.cuda.empty_cache()
        log("serving: %d jobs, 8 tenants ..." % args.serve_jobs)
        serve = bench_serve(args, torch)
        log("serving: %.2f jobs/s, p50 %.0f ms, p99 %.0f ms%s" % (
            serve["jobs_per_s"], serve["latency_ms_p50"], serve["latency_ms_p99"],
            "" if "serial_plain" not in serve else "; serial plain %.2f jobs/s, p50 %.0f ms, p99 %.0f ms" % (
                serve["serial_plain"]["jobs_per_s"], serve["serial_plain"]["latency_ms_p50"],
                serve["serial_plain"]["latency_ms_p99"])))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample) ...")
        cpu = cpu_baseline()
        log("cpu baseline: %.3f key-switches/s" % cpu["value"])
        if boot is not None or mlp is not None:
            _, cb, cm = cpu_baseline_boot_and_train(cpu_workers())
            cb["host_nproc"] = cm["host_nproc"] = cpu["host_nproc"]
            cb["host_cpu"] = cm["host_cpu"] = cpu["host_cpu"]
            if boot is not None:
                boot["cpu_baseline"] = cb
            if mlp is not None:
                mlp["cpu_baseline"] = cm
            log("cpu baseline: %.5f bootstraps/s, %.2e train_steps/s (extrapolated from op timings)" % (
                cb["value"], cm["value"]))

    line = {
        "metric": "bootstraps/s + key-switches/s at N=2^16, batched vs plain; p99 latency",
        "value": round(ksw["value"], 1) if ksw else None,
        "unit": "key-switches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ksw["ms_per_step"], 3) if ksw else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": ("key-switch throughput: %d ciphertexts x (mult_relin + rescale + %d hoisted rotations), "
                         "N=2^16, 24 primes (60 + 23x50 bits), 8 special 60-bit primes, dnum=3" % (
                             ksw["count"], ksw["rots"])) if ksw else None,
            "key_switches_per_step": ksw["ks_per_step"] if ksw else None,
            "path": "batched",
            "lanes": args.lanes,
            "autotuned": ksw["tuned"] if ksw else None,
        },
        "plain": ksw["plain"] if ksw else None,
        "batched_vs_plain": round(ksw["plain"]["ms_per_step"] / ksw["ms_per_step"], 3) if ksw and ksw["plain"] else None,
        "roofline": ksw["roofline"] if ksw else None,
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in ksw["kernels"].items()} if ksw else None,
        "bootstrap": boot,
        "train_step": mlp,
        "paper_mlps": paper,
        "mixed_rings": mixed,
        "graph_small_ring": small,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
