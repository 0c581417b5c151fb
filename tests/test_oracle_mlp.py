"""Pins of the oracle's packed MLP training step (paper Section 4, Algorithms 1
and 2) against independent definitions.  CPU only.

* the matrix-form gradients equal torch autograd of the local RSS losses;
* the update equals torch's SGD with Nesterov momentum (the decay folded into
  the gradient as printed, or torch's own weight decay for the L2 reading);
* the packed step on float64 slot vectors (rotations as np.roll) equals the
  matrix-form step, for tiled inputs, both activation degrees, both decay
  readings and the literal derivative;
* the level count of the packed step reproduces Table 1's depths 8 / 11 / 13;
* the encrypted step on the oracle decrypts to the float64 packed step.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S
from oracle import mlp as M


def _cfg(**kw):
    base = dict(k0=20, widths=[8, 8], o=4, r=16, c=32)
    base.update(kw)
    return M.MlpConfig(**base)


def _model(cfg, seed):
    g = S.rng(seed, 1)
    dims = [cfg.layer_dims(h) for h in range(1, cfg.H + 1)]
    Ws = S.mlp_weights(g, dims)
    Wst = S.mlp_weights(g, [(k, cfg.o) for _, k in dims])
    return Ws, Wst


def test_gradients_equal_autograd_of_local_losses():
    cfg = _cfg(widths=[8, 8, 6], act=(0.5, 0.7, 0.2))
    Ws, Wst = _model(cfg, 1)
    X, Y = S.mlp_batch(S.rng(1, 2), 5, cfg.k0, cfg.o)
    G, Gs = M.reference_grads(cfg, Ws, Wst, X, Y)
    tW = [torch.tensor(w, requires_grad=True) for w in Ws]
    tS = [torch.tensor(w, requires_grad=True) for w in Wst]
    a1, a2, a3 = cfg.act
    loss = 0
    a = torch.tensor(X)
    for h in range(cfg.H):
        z = a @ tW[h]
        an = a1 * z + a2 * z ** 2 + a3 * z ** 3
        yhat = an @ tS[h]
        loss = loss + 0.5 * ((yhat - torch.tensor(Y)) ** 2).sum() / X.shape[0]
        a = an.detach()                  # local losses: no gradient crosses blocks
    loss.backward()
    for h in range(cfg.H):
        assert np.allclose(G[h], tW[h].grad.numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(Gs[h], tS[h].grad.numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("l2", [False, True])
def test_update_equals_torch_nesterov_sgd(l2):
    cfg = _cfg(gamma=0.03, eta=0.01, mu=0.9, l2_decay=l2)
    g = S.rng(2, 1)
    W0 = g.normal(size=(6, 5))
    grads = [g.normal(size=(6, 5)) for _ in range(5)]
    p = torch.tensor(W0, requires_grad=True)
    opt = torch.optim.SGD([p], lr=cfg.gamma, momentum=cfg.mu, nesterov=True,
                          weight_decay=cfg.eta if l2 else 0.0)
    W, V = W0.copy(), None
    for t, G in enumerate(grads, start=1):
        p.grad = torch.tensor(G if l2 else (1.0 + cfg.eta) * G)
        opt.step()
        W, V = M.reference_update(cfg, W, V, G, t)
        assert np.allclose(W, p.detach().numpy(), rtol=1e-13, atol=1e-15)


CASES = {
    "paper": dict(),
    "tiled3": dict(k0=40, widths=[8, 8, 5]),
    "deg3": dict(act=(1.0, 1.0, 1.0 / 3.0)),
    "literal": dict(literal_deriv=True),
    "l2": dict(l2_decay=True, widths=[8]),
    "coeffs": dict(act=(0.4, 0.3, 0.05), widths=[6, 7]),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("t", [1, 3])
def test_packed_step_equals_matrix_step(name, t):
    cfg = _cfg(gamma=0.05, **CASES[name])
    Ws, Wst = _model(cfg, 3)
    g = S.rng(3, 7)
    Vs = [g.normal(size=w.shape) * 0.1 for w in Ws] if t > 1 else None
    Vst = [g.normal(size=w.shape) * 0.1 for w in Wst] if t > 1 else None
    X, Y = S.mlp_batch(g, 3, cfg.k0, cfg.o)
    want = M.reference_step(cfg, Ws, Wst, Vs, Vst, X, Y, t)
    state = M.pack_state(cfg, Ws, Wst, Vs, Vst)
    samples = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
    got = M.unpack_state(cfg, M.packed_step(M.PlainOps(cfg), cfg, state, samples, t))
    for wl, gl in zip(want, got):
        for a, b in zip(wl, gl):
            assert a.shape == b.shape
            assert np.max(np.abs(a - b)) < 1e-12
    if cfg.literal_deriv:
        return           # 1 + 2 dA is 1 in the padding, so padded weights move
    # every slot outside the packed matrices stays zero
    new = M.packed_step(M.PlainOps(cfg), cfg, state, samples, t)
    again = M.pack_state(cfg, *got)
    for a, b in zip(new, again):
        assert np.max(np.abs(a - b)) < 1e-12


def test_packed_matmuls_equal_vector_matrix_products():
    cfg = _cfg()
    ops = M.PlainOps(cfg)
    g = S.rng(4, 1)
    a = g.normal(size=13)
    W = g.normal(size=(13, 29))
    re = M.sum_rows(ops, M.vec_exp(a, cfg.r, cfg.c) * M.mat_row(W, cfg.r, cfg.c), cfg)
    assert np.max(np.abs(re - M.vec_rep(a @ W, cfg.r, cfg.c))) < 1e-12
    W2 = g.normal(size=(29, 11))
    b = g.normal(size=29)
    ce = M.sum_cols(ops, M.vec_rep(b, cfg.r, cfg.c) * M.mat_col(W2, cfg.r, cfg.c), cfg)
    assert np.max(np.abs(ce - M.vec_exp(b @ W2, cfg.r, cfg.c))) < 1e-12


@pytest.mark.parametrize("H,want", [(1, 8), (2, 11), (3, 13)])
def test_depth_matches_table_1(H, want):
    """Table 1: forward floor(2.5H) + floor(1.5 + H mod 2), backward
    floor(4.5 + 1 - H mod 2): 8, 11, 13 for H = 1, 2, 3."""
    cfg = _cfg(widths=[8] * H)
    fw = math.floor(2.5 * H) + math.floor(1.5 + H % 2)
    bw = math.floor(4.5 + 1 - H % 2)
    assert fw + bw == want
    assert M.depth(cfg) == want


def test_depth_other_variants():
    assert M.depth(_cfg(widths=[8, 8], act=(1.0, 1.0, 1.0 / 3.0))) == 13
    assert M.depth(_cfg(widths=[8, 8], literal_deriv=True)) == 10


def test_rotation_set():
    cfg = _cfg()
    assert M.rotations(cfg) == sorted({32 * k for k in (1, 2, 4, 8)} | {k for k in (1, 2, 4, 8, 16)}
                                      | {-k for k in (1, 2, 4, 8, 16)})


class EncSetup:
    def __init__(self, cfg, logN, qbits, pbits, alpha, seed=5):
        o = O.Oracle(logN, qbits, pbits, alpha)
        self.o = o
        N = o.N
        assert cfg.n == N // 2
        g = S.rng(seed, logN)
        self.g = g
        self.s = S.ternary(g, N)
        self.pk = o.keygen_public(self.s, S.uniform_residues(g, o.Q, N), S.gaussian(g, N))
        self.rlk = o.keygen_relin(self.s, *S.key_randomness(g, o.beta, o.moduli, N))
        self.keys = {}
        for k in M.rotations(cfg):
            gal = o.galois_rot(k)
            self.keys[gal] = o.keygen_galois(self.s, gal, *S.key_randomness(g, o.beta, o.moduli, N))

    def enc(self, z, lv, scale):
        o = self.o
        pt = O.encode(z, o.N, scale, o.Q[: lv + 1])
        return M.Ct(o.encrypt(lv, self.pk, pt, *S.encryption_randomness(self.g, o.N)), lv, scale)

    def dec(self, ct):
        o = self.o
        return O.decode(o.decrypt(ct.lv, self.s, ct.d), o.N, ct.s, o.Q[: ct.lv + 1]).real


@pytest.mark.slow
def test_encrypted_step_decrypts_to_packed_step():
    """N = 2^10 (r = 16, c = 32), two blocks, two input tiles, two samples,
    t = 2 with velocities, no bootstrap: every state ciphertext decrypts to
    the float64 packed step within 2^-18."""
    cfg = _cfg(gamma=0.05, log2_scale=40.0)
    L = 12
    es = EncSetup(cfg, 10, [60] + [40] * L, [60] * 3, 3)
    assert M.depth(cfg) <= L - 1
    Ws, Wst = _model(cfg, 6)
    g = S.rng(6, 2)
    Vs = [g.normal(size=w.shape) * 0.1 for w in Ws]
    Vst = [g.normal(size=w.shape) * 0.1 for w in Wst]
    X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    state = M.pack_state(cfg, Ws, Wst, Vs, Vst)
    samples = [M.pack_sample(cfg, X[i], Y[i]) for i in range(len(X))]
    want = M.packed_step(M.PlainOps(cfg), cfg, state, samples, 2)
    wl = L - 1
    T = 2.0 ** cfg.log2_scale
    enc_state = [es.enc(v, wl, T) for v in state]
    enc_samples = [([es.enc(x, L, T) for x in xt], es.enc(ye, L, T), es.enc(yr, L, T)) for xt, ye, yr in samples]
    ops = M.EncOps(es.o, cfg, es.rlk, es.keys)
    got = M.packed_step(ops, cfg, enc_state, enc_samples, 2, bootstrap=False)
    worst = max(np.max(np.abs(es.dec(c) - w)) for c, w in zip(got, want))
    assert math.log2(worst) < -18, math.log2(worst)
    assert min(c.lv for c in got) == wl - M.depth(cfg)
    assert all(c.s == T for c in got)


@pytest.mark.parametrize("act", [(1.0, 1.0, 0.0), (0.5, 0.7, 0.2)])
def test_packed_inference_equals_matrix_forward(act):
    """Early-exit inference: the packed forward pass of blocks 1..3 (two input
    tiles) gives every local classifier's output, in the expanded format
    after a RE-block and the repeated format after a CE-block, equal to the
    unpacked float64 forward pass; the float64 pass itself equals torch's."""
    cfg = _cfg(widths=[8, 8, 6], act=act)
    Ws, Wst = _model(cfg, 5)
    g = S.rng(5, 9)
    X, _ = S.mlp_batch(g, 2, cfg.k0, cfg.o)
    state = M.pack_state(cfg, Ws, Wst)
    for x in X:
        want = M.reference_infer(cfg, Ws, Wst, x)
        a = torch.tensor(x)
        for h in range(cfg.H):
            z = a @ torch.tensor(Ws[h])
            a = act[0] * z + act[1] * z * z + act[2] * z ** 3
            assert np.max(np.abs((a @ torch.tensor(Wst[h])).numpy() - want[h])) < 1e-12
        xt, _, _ = M.pack_sample(cfg, x, np.zeros(cfg.o))
        for last in (1, 3):
            got = M.packed_infer(M.PlainOps(cfg), cfg, state, xt, last)
            assert len(got) == last
            for h, (gv, wv) in enumerate(zip(got, want), start=1):
                packed = M.vec_exp(wv, cfg.r, cfg.c) if h % 2 == 1 else M.vec_rep(wv, cfg.r, cfg.c)
                assert np.max(np.abs(gv - packed)) < 1e-12, (h, last)
