"""Bootstrapping on the GPU against the oracle.

* plan: the same levels and constant layout on both sides, and the library's
  own float64 constants within rounding of the oracle's;
* with the oracle's constants imported, every output residue is bit-exact;
* with its own constants, decrypted slots are within 2^-12 of the input
  (here at N = 2^11 and at the full N = 2^16 size, 16 ciphertexts of uneven
  scales in one batch), and the batched call equals the single calls.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from oracle import boot as B

pytestmark = pytest.mark.gpu

SMALL = dict(logN=11, qbits=[60] + [50] * 17, pbits=[60] * 6, alpha=6, log2_rho=4)


class BootPair:
    def __init__(self, logN, qbits, pbits, alpha, log2_rho, oracle=True, seed=17, K=23, r=2):
        from paper_2506_19693_amd import Context

        self.gpu = Context(logN, qbits, pbits, alpha)
        self.gpu.boot_setup(K=K, double_angle=r, log2_rho=log2_rho)
        d = self.gpu
        N = d.N
        self.N = N
        self.g = S.rng(seed, logN)
        self.s = S.ternary_hw(self.g, N, 192)
        d.set_secret(self.s)
        pa, pe = S.uniform_residues(self.g, d.moduli[: d.nQ], N), S.gaussian(self.g, N)
        d.keygen_public(pa, pe)
        ra, re_ = S.key_randomness(self.g, d.beta, d.moduli, N)
        d.keygen_relin(ra, re_)
        self.rots = d.boot_rotations()
        gal_rand = {}
        for k in self.rots + ["conj"]:
            gal = 2 * N - 1 if k == "conj" else d.galois_elt(k)
            a, e = S.key_randomness(self.g, d.beta, d.moduli, N)
            d.keygen_galois(gal, a, e)
            gal_rand[gal] = (a, e)
        self.orc = None
        if oracle:
            o = O.Oracle(logN, qbits, pbits, alpha)
            assert o.moduli == d.moduli
            self.orc = o
            self.pk = o.keygen_public(self.s, pa, pe)
            self.rlk = o.keygen_relin(self.s, ra, re_)
            self.keys = {gal: o.keygen_galois(self.s, gal, a, e) for gal, (a, e) in gal_rand.items()}
            self.plan = B.Plan(N, o.Q, B.BootParams(K=K, double_angle=r, log2_rho=log2_rho))

    def level0_ct(self, z, scale):
        d = self.gpu
        pt = d.encode(z, 0, scale)
        return d.encrypt(pt, 0, *S.encryption_randomness(self.g, self.N))


_BP = {}


def small():
    if "small" not in _BP:
        _BP["small"] = BootPair(**SMALL)
    return _BP["small"]


def test_plan_layout_and_own_constants():
    p = small()
    d, plan = p.gpu, p.plan
    levels, n_plain, n_scalar = d.boot_info()
    assert levels == [plan.L, plan.level_evalmod, plan.level_stc, plan.level_out]
    assert n_plain == len(plan.plains) and n_scalar == len(plan.scalars)
    pl, sl = d.boot_constant_levels()
    assert pl == [lv for lv, _ in plan.plains]
    assert sl == [lv for lv, _ in plan.scalars]
    assert d.boot_rotations() == plan.rotations()
    plains, scalars = d.boot_export()
    worst, hist = 0, {}
    for (lv, want), got in zip(plan.plains, plains):
        a = O.crt_centered(want, p.orc.Q[: lv + 1])
        b = O.crt_centered(got, p.orc.Q[: lv + 1])
        for x, y in zip(a, b):
            dlt = abs(int(x) - int(y))
            hist[dlt] = hist.get(dlt, 0) + 1
            worst = max(worst, dlt)
    print("diagonal coefficients: |difference| histogram", sorted(hist.items()))
    # Two float64 encoders round values that differ by far less than one unit
    # here, so the rounded integers differ by at most one (measured: 257 of
    # 188416 coefficients differ, each by one)
    assert worst <= 1, worst
    rel, absd = 0.0, 0
    for (lv, want), got in zip(plan.scalars, scalars):
        a = int(O.crt_centered(np.asarray(want).reshape(-1, 1), p.orc.Q[: lv + 1])[0])
        b = int(O.crt_centered(np.asarray(got).reshape(-1, 1), p.orc.Q[: lv + 1])[0])
        absd = max(absd, abs(a - b))
        if a:
            rel = max(rel, abs(a - b) / abs(a))
        # both planners derive these from float64 scales and 60-term Chebyshev
        # sums evaluated in a different order; a sum's absolute rounding error
        # (about 60 ulp of its largest term) is a larger relative error for the
        # small high-degree coefficients (measured worst: 2^-36.8; bound with a
        # margin of 2^2.8)
        assert abs(a - b) <= max(1, abs(a) >> 34), (a, b)
    print("scalars: worst |difference| %d, worst relative 2^%.1f" % (absd, np.log2(rel) if rel else -999))


def test_bootstrap_bit_exact_with_oracle_constants():
    p = small()
    d, o, plan = p.gpu, p.orc, p.plan
    d.boot_import([pt for _, pt in plan.plains], [s for _, s in plan.scalars])
    try:
        z = S.uniform_slots(p.g, p.N // 2)
        scale = 2.0 ** 40
        # the input is made by the oracle and uploaded
        ct_host = o.encrypt(0, p.pk, O.encode(z, p.N, scale, o.Q[:1]), *S.encryption_randomness(p.g, p.N))
        out, so = d.bootstrap(d.to_ntt(ct_host, 0), scale)
        ev = B.Evaluator(o, plan, p.rlk, p.keys)
        want, so_o = ev.bootstrap(ct_host, scale)
        assert so == pytest.approx(so_o, rel=1e-12)
        got = d.to_coef(out, plan.level_out)
        assert np.array_equal(got, want)
    finally:
        d.boot_setup(log2_rho=SMALL["log2_rho"])   # back to the library's own constants


def _max_err(d, out, lv, scales, zs):
    worst = -100.0
    for i in range(len(zs)):
        back = d.decode(d.decrypt(out[i], lv), lv, scales[i]).real
        worst = max(worst, math.log2(np.max(np.abs(back - zs[i]))))
    return worst


def test_bootstrap_precision_and_batch_small():
    p = small()
    d = p.gpu
    lo = d.boot_levels[3]
    scales = [2.0 ** 30, 2.0 ** 33.5, 2.0 ** 37, 2.0 ** 40]
    zs = [S.uniform_slots(p.g, p.N // 2) for _ in scales]
    cts = d.empty(len(scales), 2, 1, p.N)
    for i, (z, sc) in enumerate(zip(zs, scales)):
        cts[i].copy_(p.level0_ct(z, sc))
    out, so = d.bootstrap_batch(cts, scales)
    assert _max_err(d, out, lo, so, zs) < -12
    for i in (0, 3):
        single, s1 = d.bootstrap(cts[i], scales[i])
        assert s1 == so[i]
        assert np.array_equal(d.to_coef(single, lo), d.to_coef(out[i], lo))


def test_bootstrap_full_size_batch():
    """N = 2^16, full 2^15 slots, HW-192 secret, chain 60 + 25 x 50 bits, 9
    special primes: 16 ciphertexts at scales 2^(35 + 10 i / 15) in one batch,
    output at level >= 10 and within 2^-12 of the input slots."""
    p = BootPair(16, [60] + [50] * 25, [60] * 9, 9, log2_rho=2, oracle=False)
    d = p.gpu
    lo = d.boot_levels[3]
    assert lo >= 10
    scales = [2.0 ** (35 + 10 * i / 15) for i in range(16)]
    zs = [S.uniform_slots(p.g, p.N // 2) for _ in scales]
    cts = d.empty(16, 2, 1, p.N)
    for i, (z, sc) in enumerate(zip(zs, scales)):
        cts[i].copy_(p.level0_ct(z, sc))
    out, so = d.bootstrap_batch(cts, scales)
    err = _max_err(d, out, lo, so, zs)
    print("full-size bootstrap: output level %d, max slot error 2^%.2f" % (lo, err))
    assert err < -12


def test_bootstrap_n17_precision():
    """N = 2^17 (the paper's eMLP-2/3 ring), full 2^16 slots, HW-192 secret,
    chain 60 + 25 x 50 bits, 9 special primes: four ciphertexts at uneven
    scales in one batch decrypt within 2^-12 of the input slots."""
    p = BootPair(17, [60] + [50] * 25, [60] * 9, 9, log2_rho=2, oracle=False)
    d = p.gpu
    lo = d.boot_levels[3]
    assert lo >= 10
    scales = [2.0 ** 35, 2.0 ** 38.5, 2.0 ** 42, 2.0 ** 45]
    zs = [S.uniform_slots(p.g, p.N // 2) for _ in scales]
    cts = d.empty(len(scales), 2, 1, p.N)
    for i, (z, sc) in enumerate(zip(zs, scales)):
        cts[i].copy_(p.level0_ct(z, sc))
    out, so = d.bootstrap_batch(cts, scales)
    err = _max_err(d, out, lo, so, zs)
    print("N=2^17 bootstrap: output level %d, max slot error 2^%.2f" % (lo, err))
    assert err < -12


def test_bootstrap_k25_r3_bit_exact_and_full_size_precision():
    """EvalMod with K = 25 and three double angles (failure rate 1.3e-5 per
    N = 2^16 bootstrap instead of 3e-4, one level more): residue-exact with
    the oracle's constants at N = 2^11, and at N = 2^16 (26 primes, 9
    special) eight ciphertexts of uneven scales within 2^-12, output level 10."""
    p = BootPair(**SMALL, K=25, r=3, seed=18)
    d, o, plan = p.gpu, p.orc, p.plan
    try:
        assert d.boot_levels[3] == plan.level_out == SMALL["qbits"].__len__() - 1 - 15
        d.boot_import([pt for _, pt in plan.plains], [s for _, s in plan.scalars])
        z = S.uniform_slots(p.g, p.N // 2)
        scale = 2.0 ** 39
        ct_host = o.encrypt(0, p.pk, O.encode(z, p.N, scale, o.Q[:1]), *S.encryption_randomness(p.g, p.N))
        out, so = d.bootstrap(d.to_ntt(ct_host, 0), scale)
        want, so_o = B.Evaluator(o, plan, p.rlk, p.keys).bootstrap(ct_host, scale)
        assert so == pytest.approx(so_o, rel=1e-12)
        assert np.array_equal(d.to_coef(out, plan.level_out), want)
    finally:
        d.close()
    q = BootPair(16, [60] + [50] * 25, [60] * 9, 9, log2_rho=2, oracle=False, K=25, r=3)
    try:
        d = q.gpu
        lo = d.boot_levels[3]
        assert lo == 10
        scales = [2.0 ** (35 + 10 * i / 7) for i in range(8)]
        zs = [S.uniform_slots(q.g, q.N // 2) for _ in scales]
        cts = d.empty(len(scales), 2, 1, q.N)
        for i, (z, sc) in enumerate(zip(zs, scales)):
            cts[i].copy_(q.level0_ct(z, sc))
        out, so = d.bootstrap_batch(cts, scales)
        err = _max_err(d, out, lo, so, zs)
        print("N=2^16 bootstrap, K=25, r=3: output level %d, max slot error 2^%.2f" % (lo, err))
        assert err < -12
    finally:
        q.gpu.close()
