"""The packed MLP training step on the GPU against the oracle.

* N = 2^10, two blocks, two input tiles, two samples, t = 2, no bootstrap:
  every state ciphertext is bit-exact with the oracle's step (same inputs,
  the oracle's SumCols masks imported), with the same levels, scales and
  integer constants, for the paper's activation, a degree-3 activation, the
  literal derivative and L2 decay; the batched form equals the per-sample form;
* N = 2^11 with the bootstrap (oracle constants imported): the bootstrapped
  state is bit-exact with the oracle's bootstrap of its updated state;
* block parallelism (a block's backward pass on a second stream) gives the
  single-stream residues: four blocks, and two blocks with the bootstrap;
  a step that fails part-way leaves the context usable;
* N = 2^16 at the full workload shape (784 -> 128 -> 128, ten classes,
  r = 256, c = 128, four input tiles, 64 samples, degree-3 activation): two
  steps decrypt to the float64 packed step within 2^-10.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from oracle import boot as B
from oracle import mlp as M

pytestmark = pytest.mark.gpu


class Pair:
    """GPU context + oracle with identical keys, and an MLP on each side."""

    def __init__(self, cfg, logN, qbits, pbits, alpha, hw=None, boot_rho=None, oracle=True, seed=21):
        from paper_2506_19693_amd import Context, Mlp

        d = Context(logN, qbits, pbits, alpha)
        self.d = d
        N = d.N
        self.N = N
        self.cfg = cfg
        g = S.rng(seed, logN)
        self.g = g
        self.s = S.ternary(g, N) if hw is None else S.ternary_hw(g, N, hw)
        d.set_secret(self.s)
        pa, pe = S.uniform_residues(g, d.moduli[: d.nQ], N), S.gaussian(g, N)
        d.keygen_public(pa, pe)
        ra, re_ = S.key_randomness(g, d.beta, d.moduli, N)
        d.keygen_relin(ra, re_)
        self.mlp = Mlp(d, cfg.k0, cfg.widths, cfg.o, cfg.r, cfg.c, act=cfg.act, gamma=cfg.gamma, eta=cfg.eta,
                       mu=cfg.mu, log2_scale=cfg.log2_scale, literal_deriv=cfg.literal_deriv, l2_decay=cfg.l2_decay)
        assert self.mlp.rotations() == M.rotations(cfg)
        assert self.mlp.depth == M.depth(cfg)
        gals = [d.galois_elt(k) for k in self.mlp.rotations()]
        if boot_rho is not None:
            d.boot_setup(log2_rho=boot_rho)
            gals += [d.galois_elt(k) for k in d.boot_rotations()] + [2 * N - 1]
        gal_rand = {}
        for gal in sorted(set(gals)):
            a, e = S.key_randomness(g, d.beta, d.moduli, N)
            d.keygen_galois(gal, a, e)
            gal_rand[gal] = (a, e)
        self.o = None
        if oracle:
            o = O.Oracle(logN, qbits, pbits, alpha)
            assert o.moduli == d.moduli
            self.o = o
            self.pk = o.keygen_public(self.s, pa, pe)
            self.rlk = o.keygen_relin(self.s, ra, re_)
            self.keys = {gal: o.keygen_galois(self.s, gal, a, e) for gal, (a, e) in gal_rand.items()}

    def oracle_enc(self, z, lv, scale):
        o = self.o
        pt = O.encode(z, self.N, scale, o.Q[: lv + 1])
        return M.Ct(o.encrypt(lv, self.pk, pt, *S.encryption_randomness(self.g, self.N)), lv, scale)

    def gpu_enc(self, z, lv, scale):
        d = self.d
        return d.encrypt(d.encode(z, lv, scale), lv, *S.encryption_randomness(self.g, self.N))

    def upload_inputs(self, samples, lv):
        """oracle-encrypted samples -> device x [b][tiles][2][lv+1][N], y_exp, y_rep"""
        d = self.d
        x = np.stack([np.stack([c.d for c in xt]) for xt, _, _ in samples])
        ye = np.stack([s[1].d for s in samples])
        yr = np.stack([s[2].d for s in samples])
        return d.to_ntt(x, lv), d.to_ntt(ye, lv), d.to_ntt(yr, lv)

    def set_state(self, cts):
        for i, c in enumerate(cts):
            if c is not None:
                self.mlp.set_state(i, self.d.to_ntt(c.d, c.lv), c.lv, c.s)

    def state(self):
        out = []
        for i in range(self.mlp.n_state):
            t, lv, s = self.mlp.get_state(i)
            out.append((self.d.to_coef(t, lv), lv, s))
        return out


def _model(cfg, g, with_v):
    dims = [cfg.layer_dims(h) for h in range(1, cfg.H + 1)]
    Ws = S.mlp_weights(g, dims)
    Wst = S.mlp_weights(g, [(k, cfg.o) for _, k in dims])
    if not with_v:
        return Ws, Wst, None, None
    Vs = [g.normal(size=w.shape) * 0.05 for w in Ws]
    Vst = [g.normal(size=w.shape) * 0.05 for w in Wst]
    return Ws, Wst, Vs, Vst


VARIANTS = {
    "paper": dict(),
    "deg3": dict(act=(1.0, 1.0, 1.0 / 3.0)),
    "literal": dict(literal_deriv=True),
    "l2": dict(l2_decay=True),
}


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_train_step_bit_exact_no_bootstrap(name):
    cfg = M.MlpConfig(k0=20, widths=[8, 8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0, **VARIANTS[name])
    L = 14
    p = Pair(cfg, 10, [60] + [40] * L, [60] * 3, 3)
    assert cfg.tiles == 2 and M.depth(cfg) <= L - 1
    g = S.rng(22, 1)
    Ws, Wst, Vs, Vst = _model(cfg, g, True)
    X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    wl = M.depth(cfg) + 1
    st = [p.oracle_enc(v, wl, T) for v in M.pack_state(cfg, Ws, Wst, Vs, Vst)]
    samples = [tuple([[p.oracle_enc(x, L, T) for x in xt], p.oracle_enc(ye, L, T), p.oracle_enc(yr, L, T)])
               for xt, ye, yr in (M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X)))]
    ops = M.EncOps(p.o, cfg, p.rlk, p.keys)
    want = M.packed_step(ops, cfg, st, samples, 2, bootstrap=False)
    for lv, pt in ops.masks.items():
        p.mlp.set_mask(lv, p.d.to_ntt(pt, lv))
    x, ye, yr = p.upload_inputs(samples, L)
    # per sample; batched on one stream; batched with the blocks' backward passes on the side stream
    for per_sample, par in ((True, False), (False, False), (False, True)):
        p.set_state(st)
        p.mlp.train_step(x, ye, yr, L, T, 2, bootstrap=False, per_sample=per_sample, block_parallel=par)
        got = p.state()
        for (res, lv, s), w in zip(got, want):
            assert lv == w.lv and s == w.s
            assert np.array_equal(res, w.d)
        if per_sample:
            assert p.mlp.scalars() == ops.scalars


def test_block_parallel_equals_sequential_four_blocks():
    """Section 4.2.3: no information flows between blocks in the backward
    pass, so block h's classifier and backward pass may run beside block
    h+1's forward pass.  Four blocks (RE, CE, RE, CE), three samples, steps
    t = 1 and t = 2 from the same state, repeated so that the side stream
    reuses its buffers: every state ciphertext, level, scale and integer
    constant equals the single-stream step's."""
    cfg = M.MlpConfig(k0=20, widths=[8, 8, 8, 8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0)
    L = 18
    p = Pair(cfg, 10, [60] + [40] * L, [60] * 3, 3, oracle=False)
    d = p.d
    assert cfg.H == 4 and M.depth(cfg) <= L - 1
    g = S.rng(23, 1)
    Ws, Wst, Vs, Vst = _model(cfg, g, True)
    X, Y = S.mlp_batch(g, 3, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    wl = M.depth(cfg) + 1
    st = [p.gpu_enc(v, wl, T) for v in M.pack_state(cfg, Ws, Wst, Vs, Vst)]
    packed = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
    x = d.empty(len(X), cfg.tiles, 2, L + 1, p.N)
    ye, yr = d.empty(len(X), 2, L + 1, p.N), d.empty(len(X), 2, L + 1, p.N)
    for i, (xt, e, r) in enumerate(packed):
        for t, v in enumerate(xt):
            x[i, t].copy_(p.gpu_enc(v, L, T))
        ye[i].copy_(p.gpu_enc(e, L, T))
        yr[i].copy_(p.gpu_enc(r, L, T))

    def step(t, par):
        for i, c in enumerate(st):
            p.mlp.set_state(i, c, wl, T)
        p.mlp.train_step(x, ye, yr, L, T, t, bootstrap=False, block_parallel=par)
        return p.state(), p.mlp.scalars()

    for t in (1, 2, 2):
        want = step(t, False)
        got = step(t, True)
        assert got[1] == want[1]
        for (a, la, sa), (b, lb, sb) in zip(got[0], want[0]):
            assert la == lb and sa == sb
            assert np.array_equal(a, b)


def test_block_parallel_with_bootstrap_equals_sequential():
    """Two blocks at N = 2^11 with the bootstrap of every W and V after the
    update (one batched call on the context stream, after it has waited for
    the side stream): steps t = 1 and t = 2 give the same residues, levels
    and scales with and without block parallelism."""
    cfg = M.MlpConfig(k0=24, widths=[16, 16], o=4, r=32, c=32, gamma=0.05, log2_scale=50.0)
    p = Pair(cfg, 11, [60] + [50] * 26, [60] * 6, 6, hw=64, boot_rho=4, oracle=False)
    d = p.d
    lo = d.boot_levels[3]
    assert lo >= M.depth(cfg)
    g = S.rng(28, 1)
    Ws, Wst, _, _ = _model(cfg, g, False)
    X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    st = {i: p.gpu_enc(v, lo, T) for i, v in enumerate(M.pack_state(cfg, Ws, Wst))
          if cfg.state_layout()[i][0] in ("W", "Wstar")}
    packed = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
    x = d.empty(2, cfg.tiles, 2, lo + 1, p.N)
    ye, yr = d.empty(2, 2, lo + 1, p.N), d.empty(2, 2, lo + 1, p.N)
    for i, (xt, e, r) in enumerate(packed):
        for t, v in enumerate(xt):
            x[i, t].copy_(p.gpu_enc(v, lo, T))
        ye[i].copy_(p.gpu_enc(e, lo, T))
        yr[i].copy_(p.gpu_enc(r, lo, T))
    got = []
    for par in (True, False):
        for i, c in st.items():
            p.mlp.set_state(i, c, lo, T)
        states = []
        for t in (1, 2):
            p.mlp.train_step(x, ye, yr, lo, T, t, block_parallel=par)
            states.append(p.state())
        got.append(states)
    for sa, sb in zip(*got):
        for (a, la, xa), (b, lb, xb) in zip(sa, sb):
            assert la == lb == lo and xa == xb
            assert np.array_equal(a, b)


def test_failed_step_leaves_context_and_mlp_usable():
    """Steps whose inputs sit too low fail part-way -- for the middle levels
    in block 1's classifier or backward pass, issued on the side stream --
    with RBK_ELEVEL.  Afterwards the context is back on its own stream and
    workspace: a full step gives the single-stream step's residues, and once
    the MLP (and with it the side stream's workspace) is gone, the context's
    own mult_relin still matches the oracle."""
    from paper_2506_19693_amd import RbkError

    cfg = M.MlpConfig(k0=20, widths=[8, 8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0)
    L = 14
    p = Pair(cfg, 10, [60] + [40] * L, [60] * 3, 3)
    d = p.d
    g = S.rng(27, 1)
    Ws, Wst, Vs, Vst = _model(cfg, g, True)
    X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    wl = M.depth(cfg) + 1
    st = [p.gpu_enc(v, wl, T) for v in M.pack_state(cfg, Ws, Wst, Vs, Vst)]
    packed = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]

    def inputs(lv):
        x = d.empty(2, cfg.tiles, 2, lv + 1, p.N)
        ye, yr = d.empty(2, 2, lv + 1, p.N), d.empty(2, 2, lv + 1, p.N)
        for i, (xt, e, r) in enumerate(packed):
            for t, v in enumerate(xt):
                x[i, t].copy_(p.gpu_enc(v, lv, T))
            ye[i].copy_(p.gpu_enc(e, lv, T))
            yr[i].copy_(p.gpu_enc(r, lv, T))
        return x, ye, yr

    def run(lv, ins, par=True):
        for i, c in enumerate(st):
            p.mlp.set_state(i, c, wl, T)
        p.mlp.train_step(*ins, lv, T, 2, bootstrap=False, block_parallel=par)

    failed = []
    for lv in range(1, L):
        try:
            run(lv, inputs(lv))
        except RbkError:
            failed.append(lv)
    print("steps that failed part-way: input levels %s" % failed)
    assert len(failed) >= 4
    ins = inputs(L)                      # encrypted once: both forms see the same ciphertexts
    got = []
    for par in (True, False):
        run(L, ins, par)
        got.append(p.state())
    for (a, la, sa), (b, lb, sb) in zip(*got):
        assert la == lb and sa == sb and np.array_equal(a, b)
    p.mlp.close()
    a = S.uniform_residues(p.g, p.o.Q, p.N, lead=(2,))
    b = S.uniform_residues(p.g, p.o.Q, p.N, lead=(2,))
    res = d.to_coef(d.mult_relin(d.to_ntt(a, L), d.to_ntt(b, L), L), L)
    assert np.array_equal(res, p.o.mult_relin(L, p.rlk, a, b))


def test_train_step_t1_ignores_velocities_and_rejects_missing_state():
    from paper_2506_19693_amd import RbkError

    cfg = M.MlpConfig(k0=12, widths=[8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0)
    L = 10
    p = Pair(cfg, 10, [60] + [40] * L, [60] * 3, 3)
    g = S.rng(23, 1)
    Ws, Wst, _, _ = _model(cfg, g, False)
    X, Y = S.mlp_batch(g, 3, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    wl = M.depth(cfg) + 1
    st = [p.oracle_enc(v, wl, T) for v in M.pack_state(cfg, Ws, Wst)]
    samples = [tuple([[p.oracle_enc(x, L, T) for x in xt], p.oracle_enc(ye, L, T), p.oracle_enc(yr, L, T)])
               for xt, ye, yr in (M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X)))]
    x, ye, yr = p.upload_inputs(samples, L)
    layout = cfg.state_layout()
    with pytest.raises(RbkError):          # no state yet
        p.mlp.train_step(x, ye, yr, L, T, 1, bootstrap=False)
    p.set_state([c if layout[i][0] in ("W", "Wstar") else None for i, c in enumerate(st)])
    with pytest.raises(RbkError):          # velocities are needed from t = 2 on
        p.mlp.train_step(x, ye, yr, L, T, 2, bootstrap=False)
    ops = M.EncOps(p.o, cfg, p.rlk, p.keys)
    want = M.packed_step(ops, cfg, st, samples, 1, bootstrap=False)
    for lv, pt in ops.masks.items():
        p.mlp.set_mask(lv, p.d.to_ntt(pt, lv))
    p.mlp.train_step(x, ye, yr, L, T, 1, bootstrap=False)
    for (res, lv, s), w in zip(p.state(), want):
        assert lv == w.lv and s == w.s and np.array_equal(res, w.d)
    # weights one level below what the step's depth needs
    low = [p.oracle_enc(v, wl - 2, T) for v in M.pack_state(cfg, Ws, Wst)]
    p.set_state(low)
    with pytest.raises(RbkError):
        p.mlp.train_step(x, ye, yr, L, T, 1, bootstrap=False)


def test_train_step_with_bootstrap_bit_exact():
    """N = 2^11, one RE block (depth 8), bootstrap output level 8."""
    cfg = M.MlpConfig(k0=24, widths=[16], o=4, r=32, c=32, gamma=0.05, log2_scale=50.0)
    qbits, pbits = [60] + [50] * 22, [60] * 6
    p = Pair(cfg, 11, qbits, pbits, 6, hw=64, boot_rho=4)
    d, o = p.d, p.o
    plan = B.Plan(p.N, o.Q, B.BootParams(log2_rho=4))
    assert d.boot_levels[3] == plan.level_out == M.depth(cfg)
    d.boot_import([pt for _, pt in plan.plains], [sc for _, sc in plan.scalars])
    g = S.rng(24, 1)
    Ws, Wst, _, _ = _model(cfg, g, False)
    X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    lo = plan.level_out
    st = [p.oracle_enc(v, lo, T) for v in M.pack_state(cfg, Ws, Wst)]
    samples = [tuple([[p.oracle_enc(x, lo, T) for x in xt], p.oracle_enc(ye, lo, T), p.oracle_enc(yr, lo, T)])
               for xt, ye, yr in (M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X)))]
    ops = M.EncOps(o, cfg, p.rlk, p.keys)
    upd = M.packed_step(ops, cfg, st, samples, 1, bootstrap=False)
    for lv, pt in ops.masks.items():
        p.mlp.set_mask(lv, d.to_ntt(pt, lv))
    x, ye, yr = p.upload_inputs(samples, lo)
    p.set_state(st)
    p.mlp.train_step(x, ye, yr, lo, T, 1)
    got = p.state()
    ev = B.Evaluator(o, plan, p.rlk, p.keys)
    for i in (0, 3):                       # W and V*: two oracle bootstraps keep the test short
        want, s_want = ev.bootstrap(o.drop(upd[i].lv, 0, upd[i].d), upd[i].s)
        res, lv, s = got[i]
        assert lv == lo and s == pytest.approx(s_want, rel=1e-12)
        assert np.array_equal(res, want)
    assert all(lv == lo for _, lv, _ in got)


def test_train_step_full_size_two_steps():
    """N = 2^16, chain 60 + 27 x 50 bits, 10 special primes, HW-192 secret;
    784 -> 128 (RE) -> 128 (CE), ten classes, degree-3 activation, 64
    samples: after two steps every W and V decrypts to the float64 packed
    step within 2^-10."""
    cfg = M.MlpConfig(k0=784, widths=[128, 128], o=10, r=256, c=128, act=(1.0, 1.0, 1.0 / 3.0),
                      gamma=0.001, eta=0.001, mu=0.9, log2_scale=50.0)
    p = Pair(cfg, 16, [60] + [50] * 27, [60] * 10, 10, hw=192, boot_rho=2, oracle=False)
    d = p.d
    lo = d.boot_levels[3]
    assert lo >= M.depth(cfg) == 13
    g = S.rng(25, 1)
    Ws, Wst, _, _ = _model(cfg, g, False)
    X, Y = S.mlp_batch(g, 64, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    plain = M.pack_state(cfg, Ws, Wst)
    for i, v in enumerate(plain):
        if cfg.state_layout()[i][0] in ("W", "Wstar"):
            p.mlp.set_state(i, p.gpu_enc(v, lo, T), lo, T)
    packed = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
    x = d.empty(len(X), cfg.tiles, 2, lo + 1, p.N)
    ye = d.empty(len(X), 2, lo + 1, p.N)
    yr = d.empty(len(X), 2, lo + 1, p.N)
    for i, (xt, e, r) in enumerate(packed):
        for t, v in enumerate(xt):
            x[i, t].copy_(p.gpu_enc(v, lo, T))
        ye[i].copy_(p.gpu_enc(e, lo, T))
        yr[i].copy_(p.gpu_enc(r, lo, T))
    ref = plain
    worst = -100.0
    for t in (1, 2):
        p.mlp.train_step(x, ye, yr, lo, T, t)
        ref = M.packed_step(M.PlainOps(cfg), cfg, ref, packed, t)
        for i in range(p.mlp.n_state):
            ct, lv, s = p.mlp.get_state(i)
            assert lv == lo
            back = d.decode(d.decrypt(ct, lv), lv, s).real
            worst = max(worst, math.log2(np.max(np.abs(back - ref[i])) + 1e-300))
    print("full-size train_step: max slot error after two steps 2^%.2f" % worst)
    assert worst < -10


@pytest.mark.parametrize("name", ["paper", "deg3"])
def test_inference_early_exit_bit_exact(name):
    """Encrypted inference through the local classifiers (forward pass of
    blocks 1..last, two input tiles, two samples in one call): every output
    ciphertext bit-exact with the oracle's packed inference, the same
    levels, scales and constants; and it decrypts to the float64 forward pass."""
    cfg = M.MlpConfig(k0=20, widths=[8, 8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0, **VARIANTS[name])
    L = 14
    p = Pair(cfg, 10, [60] + [40] * L, [60] * 3, 3)
    g = S.rng(26, 1)
    Ws, Wst, _, _ = _model(cfg, g, False)
    X, _ = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    T = 2.0 ** cfg.log2_scale
    wl = L
    st = [p.oracle_enc(v, wl, T) for v in M.pack_state(cfg, Ws, Wst)]
    layout = cfg.state_layout()
    p.set_state([c if layout[i][0] in ("W", "Wstar") else None for i, c in enumerate(st)])
    xs = [[p.oracle_enc(v, L, T) for v in M.pack_sample(cfg, X[i], np.zeros(cfg.o))[0]] for i in range(2)]
    ops = M.EncOps(p.o, cfg, p.rlk, p.keys)
    want = [M.packed_infer(ops, cfg, st, xs[i], cfg.H) for i in range(2)]
    for lv, pt in ops.masks.items():
        p.mlp.set_mask(lv, p.d.to_ntt(pt, lv))
    x = p.d.to_ntt(np.stack([np.stack([c.d for c in xt]) for xt in xs]), L)
    for last in (1, 2):
        got = p.mlp.infer(x, L, T, last)
        assert len(got) == last
        for h, (cts, lv, s) in enumerate(got):
            for i in range(2):
                w = want[i][h]
                assert lv == w.lv and s == w.s
                assert np.array_equal(p.d.to_coef(cts[i], lv), w.d), (last, h, i)
    # precision against the float64 forward pass (class j of block h's output)
    got = p.mlp.infer(x, L, T, cfg.H)
    for i in range(2):
        ref = M.reference_infer(cfg, Ws, Wst, X[i])
        for h, (cts, lv, s) in enumerate(got, start=1):
            back = p.d.decode(p.d.decrypt(cts[i], lv), lv, s).real.reshape(cfg.r, cfg.c)
            vals = back[: cfg.o, 0] if h % 2 == 1 else back[0, : cfg.o]
            assert np.max(np.abs(vals - ref[h - 1])) < 2.0 ** -20, (i, h)
