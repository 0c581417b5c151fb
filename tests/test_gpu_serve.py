"""The serving loop on the GPU: a mix of jobs from three tenants (two ring
degrees, mult+rescale batches at several levels, bootstraps, MLP training
steps) gives every job exactly the result it gets alone, whether jobs are
merged freely (large budget) or queued by a tight HBM budget with small chunk
caps (jobs split across launches); the ledger stays within the budget and
jobs do get merged."""
import pytest

import synth_inputs as S
from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _keys(ctx, g, gals, hw=None):
    N = ctx.N
    ctx.set_secret(S.ternary(g, N) if hw is None else S.ternary_hw(g, N, hw))
    ctx.keygen_public(S.uniform_residues(g, ctx.moduli[: ctx.nQ], N), S.gaussian(g, N))
    ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, N))
    for gal in sorted(set(gals)):
        ctx.keygen_galois(gal, *S.key_randomness(g, ctx.beta, ctx.moduli, N))


def _rand_cts(ctx, g, count, level):
    return ctx.to_ntt(S.uniform_residues(g, ctx.moduli[: level + 1], ctx.N, lead=(count, 2)), level)


class World:
    def __init__(self):
        import torch

        from paper_2506_19693_amd import Context, Mlp

        g = S.rng(31, 1)
        self.g = g
        # tenant A: N = 2^12, mult jobs only
        a = Context(12, [60] + [40] * 8, [60] * 3, 3)
        _keys(a, g, [])
        # tenant B: N = 2^11 with bootstrapping and an MLP (depth 8 = bootstrap output level)
        b = Context(11, [60] + [50] * 22, [60] * 6, 6)
        b.boot_setup(log2_rho=4)
        self.cfg = M.MlpConfig(k0=24, widths=[16], o=4, r=32, c=32, gamma=0.05, log2_scale=50.0)
        cfg = self.cfg
        mk = lambda: Mlp(b, cfg.k0, cfg.widths, cfg.o, cfg.r, cfg.c, act=cfg.act, gamma=cfg.gamma, eta=cfg.eta,
                         mu=cfg.mu, log2_scale=cfg.log2_scale)
        self.mlp = mk()
        gals = [b.galois_elt(k) for k in self.mlp.rotations() + b.boot_rotations()] + [2 * b.N - 1]
        _keys(b, g, gals, hw=64)
        # tenant C: N = 2^12, a second key set
        c = Context(12, [60] + [40] * 8, [60] * 3, 3)
        _keys(c, g, [])
        self.ctxs = [a, b, c]
        self.lo = b.boot_levels[3]
        T = 2.0 ** 50
        self.T = T
        lo = self.lo
        enc = lambda v: b.encrypt(b.encode(v, lo, T), lo, *S.encryption_randomness(g, b.N))
        Ws = S.mlp_weights(g, [cfg.layer_dims(1)])
        Wst = S.mlp_weights(g, [(cfg.widths[0], cfg.o)])
        self.state0 = [enc(v) if key[0] in ("W", "Wstar") else None
                       for v, key in zip(M.pack_state(cfg, Ws, Wst), cfg.state_layout())]
        X, Y = S.mlp_batch(g, 3, cfg.k0, cfg.o)
        packed = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
        self.x = torch.stack([torch.stack([enc(v) for v in xt]) for xt, _, _ in packed])
        self.ye = torch.stack([enc(e) for _, e, _ in packed])
        self.yr = torch.stack([enc(r) for _, _, r in packed])
        # the job list: (kind, tenant, args)
        self.jobs = []
        for i in range(14):
            t = (0, 1, 2)[i % 3]
            ctx = self.ctxs[t]
            lv = [3, 5, 8, 5, 2][i % 5]
            lv = min(lv, ctx.L)
            in_lv = min(ctx.L, lv + (i % 2) * 2)
            n = 1 + (i * 5) % 7
            self.jobs.append(("mult", t, dict(a=_rand_cts(ctx, g, n, in_lv), b=_rand_cts(ctx, g, n, in_lv), level=lv,
                                             in_level=in_lv)))
        for i in range(5):
            n = 1 + i % 3
            in_lv = i % 2
            self.jobs.append(("boot", 1, dict(cts=_rand_cts(b, g, n, in_lv), in_level=in_lv,
                                              scales=[2.0 ** (36 + i + 0.5 * k) for k in range(n)])))
        self.jobs.insert(4, ("train", 1, dict(t0=1)))
        self.jobs.insert(12, ("train", 1, dict(t0=2)))
        torch.cuda.synchronize()
        self.mk_mlp = mk

    def reset_mlp(self, mlp):
        for i, ct in enumerate(self.state0):
            if ct is not None:
                mlp.set_state(i, ct, self.lo, self.T)

    def alone(self):
        """every job by direct calls, one at a time"""
        want = []
        self.reset_mlp(self.mlp)
        for kind, t, a in self.jobs:
            ctx = self.ctxs[t]
            if kind == "mult":
                lv = a["level"]
                A = a["a"][:, :, : lv + 1].contiguous()
                B = a["b"][:, :, : lv + 1].contiguous()
                out = ctx.rescale_batch(ctx.mult_relin_batch(A, B, lv), lv)
                want.append(out.cpu())
            elif kind == "boot":
                res = []
                for i in range(a["cts"].shape[0]):
                    o, s = ctx.bootstrap(a["cts"][i][:, :1].contiguous(), a["scales"][i])
                    res.append((o.cpu(), s))
                want.append(res)
            else:
                self.mlp.train_step(self.x, self.ye, self.yr, self.lo, self.T, a["t0"])
                want.append([self.mlp.get_state(i)[0].cpu() for i in range(self.mlp.n_state)])
        ctx.sync()
        return want

    def served(self, budget, max_batch, max_boot_batch=16, cross=False):
        import torch

        from paper_2506_19693_amd import Server

        mlp = self.mk_mlp()
        self.reset_mlp(mlp)
        torch.cuda.synchronize()
        srv = Server(budget, max_batch, max_boot_batch)
        for c in self.ctxs:
            srv.add_tenant(c)
        if cross:
            srv.set_cross_tenant(True)
        srv.start()
        ids, outs = [], []
        for kind, t, a in self.jobs:
            ctx = self.ctxs[t]
            if kind == "mult":
                out = ctx.empty_ct(a["level"] - 1, a["a"].shape[0])
                ids.append(srv.submit_mult(t, a["a"], a["b"], a["level"], out, in_level=a["in_level"]))
                outs.append(out)
            elif kind == "boot":
                out = ctx.empty_ct(self.lo, a["cts"].shape[0])
                jid, so = srv.submit_bootstrap(t, a["cts"], a["scales"], out, in_level=a["in_level"])
                ids.append(jid)
                outs.append((out, so))
            else:
                ids.append(srv.submit_train(t, mlp, self.x, self.ye, self.yr, self.lo, self.T, a["t0"]))
                outs.append(None)
        res = [srv.wait(j) for j in ids]
        srv.drain()
        stats = srv.stats()
        srv.close()
        got = []
        for (kind, t, a), o in zip(self.jobs, outs):
            if kind == "mult":
                got.append(o.cpu())
            elif kind == "boot":
                got.append([(o[0][i].cpu(), o[1][i]) for i in range(o[0].shape[0])])
            else:
                got.append(None)
        final = [mlp.get_state(i)[0].cpu() for i in range(mlp.n_state)]
        mlp.close()
        return got, final, res, stats


_W = {}


def world():
    if "w" not in _W:
        _W["w"] = World()
    return _W["w"]


def _compare(w, want, got, final):
    import torch

    last_train = None
    for (kind, _, _), wv, gv in zip(w.jobs, want, got):
        if kind == "mult":
            assert torch.equal(wv, gv)
        elif kind == "boot":
            for (wo, ws), (go, gs) in zip(wv, gv):
                assert ws == gs and torch.equal(wo, go)
        else:
            last_train = wv
    for a, b in zip(last_train, final):
        assert torch.equal(a, b)


def test_mix_equals_alone_free_batching():
    w = world()
    want = w.alone()
    got, final, res, stats = w.served(budget=200 << 30, max_batch=64)
    _compare(w, want, got, final)
    assert stats["jobs_done"] == len(w.jobs)
    assert stats["jobs_merged"] > 0 and stats["batches"] < len(w.jobs)
    assert stats["ledger_peak"] <= stats["budget"]
    assert max(r["batch_cts"] for r in res) > 1
    _W["want"] = want


def test_mix_equals_alone_tight_budget():
    w = world()
    want = _W.get("want") or w.alone()
    # room for the resident keys plus roughly one large job at a time
    from paper_2506_19693_amd import Server

    probe = Server(1 << 60, 8, 2)
    for c in w.ctxs:
        probe.add_tenant(c)
    resident = probe.stats()["ledger_now"]
    probe.close()
    # bootstraps run in chunks of 2 ciphertexts (about 72 MiB of estimated
    # working set), mult batches in chunks of at most 8: one bootstrap at a time
    budget = resident + (100 << 20)
    got, final, res, stats = w.served(budget=budget, max_batch=8, max_boot_batch=2)
    _compare(w, want, got, final)
    assert resident < stats["ledger_peak"] <= budget
    assert stats["jobs_done"] == len(w.jobs)


def test_mix_equals_alone_cross_tenant_batching():
    """Mult jobs of different tenants (N = 2^11 and 2^12, different keys and
    chains) merged into one multi-context launch set: every result is still
    the one the job gets alone."""
    w = world()
    want = _W.get("want") or w.alone()
    got, final, res, stats = w.served(budget=200 << 30, max_batch=64, cross=True)
    _compare(w, want, got, final)
    assert stats["jobs_done"] == len(w.jobs)
    print("cross-tenant: %d jobs merged, %d ran in another tenant's batch, %d batches" % (
        stats["jobs_merged"], stats["jobs_cross_tenant"], stats["batches"]))
    assert stats["jobs_cross_tenant"] > 0
