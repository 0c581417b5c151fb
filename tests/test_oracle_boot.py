"""Pins of the oracle's bootstrapping pieces against plain mathematics:
the butterfly factorisation equals the decoding map (direct evaluation of the
canonical embedding), the Chebyshev split is an identity, the interpolant
error is within its expected bound, and a full encrypted bootstrap at
N = 2^11 decrypts within 2^-12 of the input slots.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from oracle import boot as B
from oracle import encoding as ENC


def _brv(j, bits):
    return int(format(j, "0%db" % bits)[::-1], 2)


@pytest.mark.parametrize("logN,levels", [(5, 2), (7, 3), (9, 3), (11, 3)])
def test_butterfly_factorisation_is_the_decoding_map(logN, levels):
    N = 1 << logN
    n, M = N // 2, 2 * N
    logn = logN - 1
    g = S.rng(40, logN)
    t = g.uniform(-1, 1, N)                       # a real polynomial
    w = t[:n] + 1j * t[n:]
    v = w[[_brv(j, logn) for j in range(n)]]      # bit-reversed w
    # SlotToCoeff direction: groups innermost first
    x = v.copy()
    for grp in B.stage_groups(logn, levels)[::-1]:
        x = B.apply_diag(B.group_matrix(n, M, grp, False), x)
    want = ENC.embed(t, N)                        # z_j = t(zeta^(5^j))
    assert np.max(np.abs(x - want)) < 1e-9 * n
    # CoeffToSlot direction recovers the bit-reversed coefficients
    y = want.copy()
    for grp in B.stage_groups(logn, levels):
        y = B.apply_diag(B.group_matrix(n, M, grp, True), y)
    assert np.max(np.abs(y - v)) < 1e-9
    # every diagonal offset lies in the planned set
    for grp in B.stage_groups(logn, levels):
        h0, kks = B.group_offsets(n, grp)
        offs = {(k * h0) % n for k in kks}
        assert set(B.group_matrix(n, M, grp, False)) <= offs


def test_decoding_map_direct_definition_small():
    N = 16
    n, M = 8, 32
    t = np.arange(N, dtype=float) - 7.5
    zeta = np.exp(2j * np.pi / M)
    direct = np.array([sum(t[k] * zeta ** (pow(5, j, M) * k) for k in range(N)) for j in range(n)])
    assert np.max(np.abs(ENC.embed(t, N) - direct)) < 1e-12


@pytest.mark.parametrize("K,r,fit_log2,sin_log2", [(23, 2, -24, -20), (25, 3, -44, -40)])
def test_chebyshev_split_identity_and_error(K, r, fit_log2, sin_log2):
    """Degree 59 at K = 23 with two double angles (the default), and the
    SURVEY's fallback K = 25 with three (one more level, failure rate per
    N = 2^16 bootstrap 1.3e-5 instead of 3e-4)."""
    deg = 59
    c = B.cheb_coeffs(B.evalmod_function(K, r), deg)
    u = np.linspace(-1, 1, 4001)
    T = np.polynomial.chebyshev
    for m, cc in ((32, c), (16, c[:31]), (8, c[:12])):
        q, rr = B.cheb_split(cc, m)
        lhs = T.chebval(u, cc)
        rhs = T.chebval(u, q) * T.chebval(u, np.eye(m + 1)[m]) + T.chebval(u, rr)
        assert np.max(np.abs(lhs - rhs)) < 1e-12
    err = np.max(np.abs(T.chebval(u, c) - B.evalmod_function(K, r)(u)))
    assert err < 2.0 ** fit_log2   # degree 59 on [-(K+1), K+1]
    # after r double angles the result approximates sin(2 pi x) near integers
    x = np.concatenate([I + np.linspace(-1e-3, 1e-3, 101) for I in range(-K, K + 1)])
    y = T.chebval(x / (K + 1), c)
    for _ in range(r):
        y = 2 * y * y - 1
    assert np.max(np.abs(y - np.sin(2 * np.pi * x))) < 2.0 ** sin_log2


@pytest.mark.parametrize("K,r", [(23, 2), (25, 3)])
def test_oracle_bootstrap_precision(K, r):
    logN = 11
    orc = O.Oracle(logN, [60] + [50] * 17, [60] * 6, 6)
    N = orc.N
    g = S.rng(41, logN)
    plan = B.Plan(N, orc.Q, B.BootParams(K=K, double_angle=r, log2_rho=4))
    # 17 - 3 (CoeffToSlot) - 6 + r (EvalMod: degree 59, r double angles) - 3 (SlotToCoeff)
    assert plan.level_out == 17 - 3 - (6 + r) - 3
    s = S.ternary_hw(g, N, 192)
    pk = orc.keygen_public(s, S.uniform_residues(g, orc.Q, N), S.gaussian(g, N))
    rlk = orc.keygen_relin(s, *S.key_randomness(g, orc.beta, orc.moduli, N))
    keys = {}
    for k in plan.rotations() + ["conj"]:
        gal = 2 * N - 1 if k == "conj" else orc.galois_rot(k)
        keys[gal] = orc.keygen_galois(s, gal, *S.key_randomness(g, orc.beta, orc.moduli, N))
    z = S.uniform_slots(g, N // 2)
    scale = 2.0 ** 38.3
    ct = orc.encrypt(0, pk, O.encode(z, N, scale, orc.Q[:1]), *S.encryption_randomness(g, N))
    out, so = B.Evaluator(orc, plan, rlk, keys).bootstrap(ct, scale)
    back = O.decode(orc.decrypt(plan.level_out, s, out), N, so, orc.Q[: plan.level_out + 1])
    assert math.log2(np.max(np.abs(back - z))) < -12


# ---------------------------------------------------------------- ModRaise and monomials, directly

def _crt_centred(res, mods):
    """the integer in (-Q/2, Q/2] with the given residues (Python big integers)"""
    Q = 1
    for m in mods:
        Q *= m
    x = 0
    for r, m in zip(res, mods):
        Qi = Q // m
        x += int(r) * Qi * pow(Qi % m, -1, m)
    x %= Q
    return x - Q if x > Q // 2 else x


def test_modraise_is_the_centred_lift():
    """ModRaise reads a level-0 residue as the integer of least absolute
    value and re-expresses it modulo every prime of the chain: the CRT of
    the outputs is that integer (every input, including 0, +-(q0-1)/2 and
    q0 - 1)."""
    orc = O.Oracle(5, [50, 40, 40, 40, 40], [50], 5)
    q0, N, L = orc.Q[0], orc.N, orc.L
    g = S.rng(41, 5)
    x = S.uniform_residues(g, orc.Q[:1], N, lead=(2,))
    x[0, 0, :4] = [0, (q0 - 1) // 2, (q0 + 1) // 2, q0 - 1]
    out = orc.modraise(L, x)
    assert out.shape == (2, L + 1, N)
    for p in range(2):
        for k in range(N):
            v = int(x[p, 0, k])
            want = v if v <= (q0 - 1) // 2 else v - q0
            assert _crt_centred(out[p, :, k], orc.Q) == want


def _negacyclic(a, b, q):
    """schoolbook product in Z_q[X] / (X^N + 1), Python integers"""
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            t = int(a[i]) * int(b[j])
            if i + j < N:
                out[i + j] += t
            else:
                out[i + j - N] -= t
    return [v % q for v in out]


def test_monomial_is_the_product_with_x_to_the_e():
    orc = O.Oracle(4, [50, 40, 40], [50], 3)
    N, L = orc.N, orc.L
    g = S.rng(42, 4)
    a = S.uniform_residues(g, orc.Q, N, lead=(2,))
    for e in (0, 1, 5, N - 1, N, N + 3, 3 * N // 2, 2 * N - 1):
        out = orc.monomial(L, e, a)
        xe = [0] * N
        xe[e % N] = 1 if e < N else -1          # X^e with X^N = -1
        for p in range(2):
            for t in range(L + 1):
                assert [int(v) for v in out[p, t]] == _negacyclic(a[p, t], xe, orc.Q[t]), (e, p, t)


def test_monomial_of_quarter_turn_multiplies_slots_by_i():
    """X^(N/2) evaluates to zeta^(5^j N/2) = i at every slot root (5^j = 1 mod 4),
    which is how the bootstrap splits real and imaginary parts."""
    N = 1 << 6
    orc = O.Oracle(6, [50, 40], [50], 2)
    g = S.rng(43, 6)
    z = g.uniform(-1, 1, N // 2) + 1j * g.uniform(-1, 1, N // 2)
    scale = 2.0 ** 30
    pt = O.encode(z, N, scale, orc.Q)
    back = O.decode(orc.monomial(orc.L, N // 2, pt[None])[0], N, scale, orc.Q)
    assert np.max(np.abs(back - 1j * z)) < 2.0 ** -20


# ---------------------------------------------------------------- ModRaise overflow and the bootstrap's failure rate

def test_modraise_overflow_matches_big_integers():
    """I from the wrapping-word computation equals (c0 + c1 s - m) / q_0 over
    the integers (Python big integers, schoolbook negacyclic product)."""
    orc = O.Oracle(6, [60, 50], [60], 2)
    N, q0 = orc.N, orc.Q[0]
    g = S.rng(44, 6)
    s = S.ternary_hw(g, N, 20)
    ct = S.uniform_residues(g, orc.Q[:1], N, lead=(2,))
    got = B.modraise_overflow(orc, s, ct)
    cen = lambda v: int(v) if int(v) <= (q0 - 1) // 2 else int(v) - q0
    c0 = [cen(v) for v in ct[0, 0]]
    c1 = [cen(v) for v in ct[1, 0]]
    t = list(c0)
    for i in range(N):
        for j in range(N):
            if s[j]:
                k = i + j
                if k < N:
                    t[k] += c1[i] * int(s[j])
                else:
                    t[k - N] -= c1[i] * int(s[j])
    for k in range(N):
        m = t[k] % q0
        m = m if m <= (q0 - 1) // 2 else m - q0
        assert (t[k] - m) % q0 == 0
        assert got[k] == (t[k] - m) // q0


def test_bootstrap_failure_rate_over_seeds():
    """Empirical law of I at the bootstrap workload's shape (N = 2^16,
    HW-192 secret, fresh level-0 encryptions): its spread matches
    sqrt((h + 1) / 12), the tail counts match the normal law where the
    sample reaches, and the failure rate P(some |I_j| > K) per bootstrap
    follows: about 3e-4 at K = 23 (EvalMod r = 2) and below 2e-5 at K = 25
    (r = 3)."""
    from math import erfc, sqrt

    logN, h, n_ct = 16, 192, 24
    orc = O.Oracle(logN, [60, 50], [60], 2)
    N = orc.N
    g = S.rng(45, logN)
    samples = []
    for i in range(n_ct):
        s = S.ternary_hw(g, N, h)
        pk = orc.keygen_public(s, S.uniform_residues(g, orc.Q, N), S.gaussian(g, N))
        m = S.uniform_residues(g, orc.Q, N) % np.uint64(1 << 40)      # any small message
        ct = orc.encrypt(0, pk, m[:1], *S.encryption_randomness(g, N))
        samples.append(B.modraise_overflow(orc, s, ct))
    I = np.concatenate(samples).astype(np.float64)
    sigma = sqrt((h + 1) / 12.0)
    assert abs(I.std() / sigma - 1) < 0.02 and abs(I.mean()) < 0.02
    tail = lambda t: erfc((t + 0.5) / (sigma * sqrt(2.0)))     # P(|I| > t), I integer
    for t in (8, 12, 15):
        want = tail(t) * I.size
        got = float(np.sum(np.abs(I) > t))
        assert abs(got - want) < 5 * sqrt(want) + 1, (t, got, want)
    per_bootstrap = {K: 1 - (1 - tail(K)) ** N for K in (23, 25)}
    print("failure rate per N=2^16 bootstrap: K=23 %.1e, K=25 %.1e (max |I| seen %d over %d coefficients)" % (
        per_bootstrap[23], per_bootstrap[25], int(np.abs(I).max()), I.size))
    assert 1e-4 < per_bootstrap[23] < 1e-3 and per_bootstrap[25] < 2e-5
