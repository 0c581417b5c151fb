"""Keys and encryption drawn inside the library from one seed, and the
ciphertext export / import calls, against the oracle (paper Section 3: the
secret and public key, one rotation key per index, encryption with added
noise).

The oracle draws the same randomness with its own ChaCha20 sampler and runs
its own key generation and encryption; every residue must agree.
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

CASES = {
    # uniform ternary secret, one prime per digit (N = 2^12, 50 + 3 x 40, one special prime)
    "c0": dict(logN=12, qbits=[50, 40, 40, 40], pbits=[50], alpha=1, hw=0),
    # fixed-weight secret, two digits, register NTT geometry
    "mid": dict(logN=13, qbits=[60] + [50] * 5, pbits=[60] * 3, alpha=3, hw=192),
}


@pytest.mark.parametrize("name", list(CASES))
def test_seeded_keys_and_encryption_match_oracle(name):
    from paper_2506_19693_amd import Context

    p = CASES[name]
    seed = 0x5EED0000 + (1 << 40) + len(name)
    d = Context(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    o = O.Oracle(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    try:
        assert d.moduli == o.moduli
        N, L = o.N, o.L
        steps = [1, -3, 5, 1, N // 2]          # a repeat and a multiple of N/2 (no key) included
        print("seeded keygen %s: N=2^%d, hw %d" % (name, p["logN"], p["hw"]), flush=True)
        d.keygen(seed, p["hw"], steps, conj=True)
        s = o.seeded_secret(seed, p["hw"])
        if p["hw"]:
            assert int(np.count_nonzero(s)) == p["hw"]
        rlk = o.keygen_relin(s, *o.seeded_key_randomness(seed, 0))
        assert np.array_equal(d.key_export(0), rlk)
        gals = sorted({o.galois_rot(k) for k in steps} - {1}) + [o.galois_conj()]
        for g in gals:
            want = o.keygen_galois(s, g, *o.seeded_key_randomness(seed, g))
            assert np.array_equal(d.key_export(g), want), g
        # public-key encryption with library-drawn (v, e0, e1)
        pk = o.keygen_public(s, *o.seeded_public_randomness(seed))
        g = S.rng(3, p["logN"])
        m = S.uniform_residues(g, o.Q, N)
        for index in (0, 7, (5 << 32) | 2):
            ct = d.encrypt_seeded(d.ct_import(m, L), L, seed, index)
            want = o.encrypt(L, pk, m, *o.seeded_encryption_randomness(seed, index))
            assert np.array_equal(d.ct_export(ct, L), want), index
        # the seeded keys work: mult_relin + rotation of seeded encryptions decrypt against the oracle
        x = d.encrypt_seeded(d.ct_import(m, L), L, seed, 11)
        y = d.encrypt_seeded(d.ct_import(m, L), L, seed, 12)
        r = d.rotate(d.mult_relin(x, y, L), 1, L)
        xo = o.encrypt(L, pk, m, *o.seeded_encryption_randomness(seed, 11))
        yo = o.encrypt(L, pk, m, *o.seeded_encryption_randomness(seed, 12))
        ro = o.rotate(L, o.keygen_galois(s, o.galois_rot(1), *o.seeded_key_randomness(seed, o.galois_rot(1))),
                      o.galois_rot(1), o.mult_relin(L, rlk, xo, yo))
        assert np.array_equal(d.ct_export(r, L), ro)
    finally:
        d.close()


def test_ct_export_import_roundtrip_and_errors():
    from paper_2506_19693_amd import Context
    from paper_2506_19693_amd.rbk import RbkError

    d = Context(12, [50, 40, 40, 40], [50], 1)
    try:
        g = S.rng(5, 12)
        for level in (3, 1, 0):
            ct = S.uniform_residues(g, d.moduli[: level + 1], d.N, lead=(2,))
            t = d.ct_import(ct, level)
            # the device form is the NTT domain: equal to the plain transform
            assert np.array_equal(d.to_coef(t, level), ct)
            assert np.array_equal(d.ct_export(t, level), ct)
        bad = S.uniform_residues(g, d.moduli[:4], d.N, lead=(2,))
        bad[1, 2, 17] = d.moduli[2]           # a residue equal to its prime
        with pytest.raises(RbkError):
            d.ct_import(bad, 3)
        with pytest.raises(RbkError):
            d.ct_export(d.empty_ct(3), 4)    # level above the chain
    finally:
        d.close()


def test_scaled_additions_check_scales():
    """Section 3's slot-wise add / sub: equal scales give the oracle's sums,
    scales that differ by more than 2^-30 (relative) give RBK_ESCALE."""
    from paper_2506_19693_amd import Context
    from paper_2506_19693_amd.rbk import RbkError

    d = Context(12, [50, 40, 40, 40], [50], 1)
    o = O.Oracle(12, [50, 40, 40, 40], [50], 1)
    try:
        g = S.rng(8, 12)
        L = 3
        a = S.uniform_residues(g, o.Q, o.N, lead=(2,))
        b = S.uniform_residues(g, o.Q, o.N, lead=(2,))
        pt = S.uniform_residues(g, o.Q, o.N)
        A, B, P = d.ct_import(a, L), d.ct_import(b, L), d.ct_import(pt, L)
        s = 2.0 ** 40
        out, so = d.add_scaled(A, s, B, s * (1 + 2.0 ** -32), L)
        assert so == s and np.array_equal(d.ct_export(out, L), o.add(L, a, b))
        out, so = d.sub_scaled(A, s, B, s, L)
        assert so == s and np.array_equal(d.ct_export(out, L), o.sub(L, a, b))
        out, so = d.add_plain_scaled(A, s, P, s, L)
        assert so == s and np.array_equal(d.ct_export(out, L), o.add_plain(L, a, pt))
        for fn, other in ((d.add_scaled, B), (d.sub_scaled, B), (d.add_plain_scaled, P)):
            with pytest.raises(RbkError, match="-8"):
                fn(A, s, other, s * (1 + 2.0 ** -20), L)
            with pytest.raises(RbkError, match="-1"):
                fn(A, s, other, -1.0, L)
    finally:
        d.close()


def test_mlp_weights_float64_roundtrip_and_step():
    """Algorithm 1's weights go in and come out as float64 matrices: the
    library packs them (Section 4.1 formats, two input tiles) into the same
    slot vectors as the oracle's packing, encrypts them with keys drawn from
    a seed, and after one training step (t = 2, no bootstrap) the decrypted
    weights and velocities follow the unpacked float64 reference step."""
    from paper_2506_19693_amd import Context, Mlp
    from oracle import mlp as M

    cfg = M.MlpConfig(k0=20, widths=[8, 8], o=4, r=16, c=32, gamma=0.05, log2_scale=40.0)
    L = 14
    d = Context(10, [60] + [40] * L, [60] * 3, 3)
    mlp = None
    try:
        mlp = Mlp(d, cfg.k0, cfg.widths, cfg.o, cfg.r, cfg.c, act=cfg.act, gamma=cfg.gamma, eta=cfg.eta, mu=cfg.mu,
                  log2_scale=cfg.log2_scale)
        d.keygen(77, 0, mlp.rotations())
        g = S.rng(31, 1)
        dims = [cfg.layer_dims(h) for h in range(1, cfg.H + 1)]
        Ws = S.mlp_weights(g, dims)
        Wst = S.mlp_weights(g, [(k, cfg.o) for _, k in dims])
        Vs = [g.normal(size=w.shape) * 0.05 for w in Ws]
        Vst = [g.normal(size=w.shape) * 0.05 for w in Wst]
        wl = M.depth(cfg) + 1
        mlp.set_weights(Ws, Wst, Vs, Vst, level=wl, seed=78)
        # the library's packing equals the oracle's: every state slot vector
        for i, v in enumerate(M.pack_state(cfg, Ws, Wst, Vs, Vst)):
            ct, lv, s = mlp.get_state(i)
            assert lv == wl and s == 2.0 ** cfg.log2_scale
            back = d.decode(d.decrypt(ct, lv), lv, s).real
            assert np.max(np.abs(back - v)) < 2.0 ** -20, i
        got = mlp.get_weights(dims, cfg.o)
        for want, have in zip((Ws, Wst, Vs, Vst), got):
            for a, b in zip(want, have):
                assert a.shape == b.shape and np.max(np.abs(a - b)) < 2.0 ** -20
        # one step on library-encrypted samples
        X, Y = S.mlp_batch(g, 2, cfg.k0, cfg.o)
        T = 2.0 ** cfg.log2_scale
        x = d.empty(2, cfg.tiles, 2, L + 1, d.N)
        ye, yr = d.empty(2, 2, L + 1, d.N), d.empty(2, 2, L + 1, d.N)
        idx = 1000
        for i in range(2):
            xt, e, r = M.pack_sample(cfg, X[i], Y[i])
            for t, v in enumerate(xt):
                x[i, t].copy_(d.encrypt_seeded(d.encode(v, L, T), L, 78, idx))
                idx += 1
            ye[i].copy_(d.encrypt_seeded(d.encode(e, L, T), L, 78, idx))
            yr[i].copy_(d.encrypt_seeded(d.encode(r, L, T), L, 78, idx + 1))
            idx += 2
        mlp.train_step(x, ye, yr, L, T, 2, bootstrap=False)
        ref = M.reference_step(cfg, Ws, Wst, Vs, Vst, X, Y, 2)
        got = mlp.get_weights(dims, cfg.o)
        worst = max(float(np.max(np.abs(a - b))) for want, have in zip(ref, got) for a, b in zip(want, have))
        print("float64 weights after one encrypted step: max error 2^%.2f" % np.log2(worst))
        assert worst < 2.0 ** -12
    finally:
        if mlp is not None:
            mlp.close()            # before its context
        d.close()
