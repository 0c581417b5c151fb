"""Pins of the CPU oracle against mathematics that does not come from the
oracle itself: trial division, the DFT definition, schoolbook negacyclic
convolution, exact big-integer CRT arithmetic, and decryption of the scheme
against float64 plaintext arithmetic.  CPU only."""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from oracle import encoding as ENC


# ---------------------------------------------------------------- primes

def test_miller_rabin_matches_trial_division():
    for n in list(range(0, 3000)) + [561, 1105, 1729, 2465, 2821, 6601, 8911, 3215031751 % 100003]:
        assert O.is_prime(n) == O.is_prime_trial(n), n
    # strong pseudoprimes to several small bases, and known primes
    for n in [3215031751, 2152302898747, 3474749660383, 341550071728321]:
        assert not O.is_prime(n)
    for n in [(1 << 61) - 1, 1000000007, 998244353]:
        assert O.is_prime(n)


@pytest.mark.parametrize("logN,bits", [(4, [12, 12, 14]), (5, [14, 13]), (3, [10, 10, 10, 11])])
def test_prime_rule_by_brute_force(logN, bits):
    got = O.gen_primes(logN, bits)
    twoN = 2 << logN
    want = []
    for b in bits:
        j = 1
        while True:
            q = (1 << b) - j * twoN + 1
            if O.is_prime_trial(q) and q not in want:
                want.append(q)
                break
            j += 1
    assert got == want
    for q, b in zip(got, bits):
        assert q % twoN == 1 and q.bit_length() == b


@pytest.mark.parametrize("logN,b", [(3, 10), (4, 11), (5, 12)])
def test_min_psi_is_smallest_primitive_root(logN, b):
    q = O.gen_primes(logN, [b])[0]
    N = 1 << logN
    roots = [x for x in range(1, q) if pow(x, N, q) == q - 1]
    assert len(roots) == N          # exactly the N primitive 2N-th roots
    assert O.min_psi(q, logN) == min(roots)


# ---------------------------------------------------------------- NTT

def _direct_eval(a, q, psi, logN):
    """a(psi^(2k+1)) placed at bit-reversed k, in Python integers."""
    N = 1 << logN
    out = [0] * N
    for k in range(N):
        w = pow(psi, 2 * k + 1, q)
        v = sum(int(a[j]) * pow(w, j, q) for j in range(N)) % q
        r = int(format(k, "0%db" % logN)[::-1], 2)
        out[r] = v
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("logN", [3, 4, 5, 6, 7])
def test_ntt_matches_definition(logN):
    q = O.gen_primes(logN, [40])[0]
    psi = O.min_psi(q, logN)
    g = S.rng(7, logN)
    a = g.integers(0, q, 1 << logN, dtype=np.uint64)
    want = _direct_eval(a, q, psi, logN)
    assert np.array_equal(O.ntt(logN, q, psi, a), want)
    assert np.array_equal(O.ntt_direct(logN, q, psi, a), want)
    assert np.array_equal(O.intt(logN, q, psi, want), a)


@pytest.mark.parametrize("logN,b", [(3, 30), (6, 50), (8, 60), (10, 55)])
def test_ntt_convolution_theorem(logN, b):
    q = O.gen_primes(logN, [b])[0]
    psi = O.min_psi(q, logN)
    N = 1 << logN
    g = S.rng(11, logN)
    a = g.integers(0, q, N, dtype=np.uint64)
    c = g.integers(0, q, N, dtype=np.uint64)
    A, C = O.ntt(logN, q, psi, a), O.ntt(logN, q, psi, c)
    prod = np.array([(int(x) * int(y)) % q for x, y in zip(A, C)], dtype=np.uint64)
    got = O.intt(logN, q, psi, prod)
    # schoolbook in Python integers: X^N = -1
    want = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                want[k] += int(a[i]) * int(c[j])
            else:
                want[k - N] -= int(a[i]) * int(c[j])
    want = np.array([w % q for w in want], dtype=np.uint64)
    assert np.array_equal(got, want)
    assert np.array_equal(O.negacyclic_schoolbook(logN, q, a, c), want)


def test_psi_order():
    for logN in (10, 12, 16):
        for q in O.gen_primes(logN, [60, 50, 40]):
            psi = O.min_psi(q, logN)
            assert pow(psi, 1 << logN, q) == q - 1


# ---------------------------------------------------------------- base conversion, big integers

def _crt(res, mods):
    Q = 1
    for m in mods:
        Q *= m
    x = 0
    for r, m in zip(res, mods):
        Qi = Q // m
        x += int(r) * Qi * pow(Qi % m, -1, m)
    return x % Q, Q


def _small_ctx():
    return O.Oracle(5, [50, 40, 40, 40, 40], [50, 50], 2)


def test_bconv_is_crt_plus_small_multiple():
    orc = _small_ctx()
    g = S.rng(3)
    src = [0, 1, 2]
    dst = [3, 4, orc.nQ, orc.nQ + 1]
    x = S.uniform_residues(g, [orc.moduli[i] for i in src], orc.N)
    out = orc.bconv(src, x, dst)
    B = 1
    for i in src:
        B *= orc.moduli[i]
    for k in range(orc.N):
        X, _ = _crt([x[i][k] for i in range(len(src))], [orc.moduli[i] for i in src])
        for o, t in enumerate(dst):
            tm = orc.moduli[t]
            ok = [(X + u * B) % tm for u in range(len(src))]
            assert int(out[o][k]) in ok


def test_modup_digits():
    orc = _small_ctx()
    level = 4
    g = S.rng(4)
    d = S.uniform_residues(g, orc.Q[: level + 1], orc.N)
    ext = orc.modup(level, d)
    idx = orc.ext_indices(level)
    assert ext.shape == (orc.num_digits(level), len(idx), orc.N)
    for j in range(orc.num_digits(level)):
        lo, hi = j * orc.alpha, min(j * orc.alpha + orc.alpha, level + 1)
        mods = [orc.moduli[i] for i in range(lo, hi)]
        B = 1
        for m in mods:
            B *= m
        for k in range(0, orc.N, 3):
            X, _ = _crt([d[i][k] for i in range(lo, hi)], mods)
            for e, t in enumerate(idx):
                tm = orc.moduli[t]
                if lo <= e < hi:
                    assert ext[j][e][k] == d[e][k]
                else:
                    assert int(ext[j][e][k]) in [(X + u * B) % tm for u in range(hi - lo)]


def test_moddown_is_division_by_P():
    orc = _small_ctx()
    level = 3
    g = S.rng(5)
    idx = orc.ext_indices(level)
    u = S.uniform_residues(g, [orc.moduli[t] for t in idx], orc.N)
    out = orc.moddown(level, u)
    P = orc.P[0] * orc.P[1]
    Qs = orc.Q[: level + 1]
    for k in range(orc.N):
        U, QP = _crt([u[e][k] for e in range(len(idx))], [orc.moduli[t] for t in idx])
        Y, Q = _crt([out[i][k] for i in range(level + 1)], Qs)
        # out = (U - [U]_P - v P) / P  with 0 <= v < nP: floor division, off by at most nP
        base = (U - (U % P)) // P
        assert any((base - v - Y) % Q == 0 for v in range(orc.nP))


def test_rescale_is_exact_rounded_division():
    orc = _small_ctx()
    level = 4
    g = S.rng(6)
    ct = S.uniform_residues(g, orc.Q[: level + 1], orc.N, lead=(2,))
    out = orc.rescale(level, ct)
    ql = orc.Q[level]
    for p in range(2):
        for k in range(orc.N):
            C, Q = _crt([ct[p][i][k] for i in range(level + 1)], orc.Q[: level + 1])
            r = C % ql
            lift = r if r <= (ql - 1) // 2 else r - ql
            want = (C - lift) // ql
            Y, Qm = _crt([out[p][i][k] for i in range(level)], orc.Q[:level])
            assert (want - Y) % Qm == 0


def test_automorphism_is_substitution():
    orc = _small_ctx()
    N = orc.N
    g = S.rng(8)
    a = S.uniform_residues(g, orc.Q, N)
    for gal in (5, 25, 2 * N - 1, 3):
        out = orc.automorph(orc.L, gal, a)
        q = orc.Q[0]
        want = [0] * N
        for i in range(N):   # a(X^g) with X^N = -1
            e = (i * gal) % (2 * N)
            v = int(a[0][i])
            if e < N:
                want[e] = (want[e] + v) % q
            else:
                want[e - N] = (want[e - N] - v) % q
        assert np.array_equal(out[0], np.array(want, dtype=np.uint64))


# ---------------------------------------------------------------- encoding

@pytest.mark.parametrize("logN", [3, 4, 6])
def test_encoding_matches_direct_embedding(logN):
    N = 1 << logN
    n = N // 2
    g = S.rng(9, logN)
    z = g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)
    t = ENC.embed_inverse(z, N)
    zeta = np.exp(1j * np.pi / N)
    roots = [zeta ** pow(5, j, 2 * N) for j in range(n)]
    # the direct definition: evaluating t at the slot roots returns z
    back = np.array([sum(t[k] * r ** k for k in range(N)) for r in roots])
    assert np.max(np.abs(back - z)) < 1e-12
    assert np.max(np.abs(ENC.embed(t, N) - z)) < 1e-12
    # t is real: it must also vanish the conjugate condition t(conj root) = conj(z)
    back_c = np.array([sum(t[k] * np.conj(r) ** k for k in range(N)) for r in roots])
    assert np.max(np.abs(back_c - np.conj(z))) < 1e-12


def test_encode_decode_roundtrip_and_rotation_direction():
    orc = _small_ctx()
    N = orc.N
    g = S.rng(10)
    z = g.uniform(-1, 1, N // 2)
    scale = 2.0 ** 40
    m = O.encode(z, N, scale, orc.Q)
    back = O.decode(m, N, scale, orc.Q)
    assert np.max(np.abs(back - z)) < 2.0 ** -30
    for k in (1, 3, -2):
        rot = orc.automorph(orc.L, orc.galois_rot(k), m)
        zr = O.decode(rot, N, scale, orc.Q)
        assert np.max(np.abs(zr - np.roll(z, -k))) < 2.0 ** -30     # Rot(a,k)_j = a_{j+k}
    conj = orc.automorph(orc.L, orc.galois_conj(), O.encode(z * (1 + 1j), N, scale, orc.Q))
    assert np.max(np.abs(O.decode(conj, N, scale, orc.Q) - z * (1 - 1j))) < 2.0 ** -30


# ---------------------------------------------------------------- scheme-level semantics

class Scheme:
    def __init__(self, orc, seed=1, rots=(1, 7)):
        self.o = orc
        N = orc.N
        g = S.rng(seed, 100)
        self.s = S.ternary(g, N)
        self.pk = orc.keygen_public(self.s, S.uniform_residues(g, orc.Q, N), S.gaussian(g, N))
        a, e = S.key_randomness(g, orc.beta, orc.moduli, N)
        self.rlk = orc.keygen_relin(self.s, a, e)
        self.keys = {}
        for k in list(rots):
            gal = orc.galois_rot(k)
            a, e = S.key_randomness(g, orc.beta, orc.moduli, N)
            self.keys[k] = (gal, orc.keygen_galois(self.s, gal, a, e))
        self.g = g

    def enc(self, z, level, scale):
        m = O.encode(z, self.o.N, scale, self.o.Q[: level + 1])
        return self.o.encrypt(level, self.pk, m, *S.encryption_randomness(self.g, self.o.N))

    def dec(self, ct, level, scale):
        return O.decode(self.o.decrypt(level, self.s, ct), self.o.N, scale, self.o.Q[: level + 1])


def test_fresh_noise_bound():
    orc = _small_ctx()
    sch = Scheme(orc, rots=())
    N = orc.N
    m = np.zeros((orc.nQ, N), dtype=np.uint64)
    ct = orc.encrypt(orc.L, sch.pk, m, *S.encryption_randomness(sch.g, N))
    noise = O.crt_centered(orc.decrypt(orc.L, sch.s, ct), orc.Q)
    # v e + e0 + e1 s with |v|,|s| <= 1 and |e| <= 19: at most 19 (2N + 1)
    assert max(abs(int(x)) for x in noise) <= 19 * (2 * N + 1)


def test_c0_flow_precision():
    """N = 2^12, 50 + 3x40-bit chain, one 50-bit special prime: mult_relin,
    rescale, rotations by +1 and +7, add; decrypted within 2^-20 of float64."""
    orc = O.Oracle(12, [50, 40, 40, 40], [50], 1)
    sch = Scheme(orc, seed=2, rots=(1, 7, -1))
    N, L = orc.N, orc.L
    x = S.uniform_slots(sch.g, N // 2)
    y = S.uniform_slots(sch.g, N // 2)
    D = 2.0 ** 40
    cx, cy = sch.enc(x, L, D), sch.enc(y, L, D)
    cm = orc.mult_relin(L, sch.rlk, cx, cy)
    assert np.max(np.abs(sch.dec(cm, L, D * D) - x * y)) < 2.0 ** -20
    cr = orc.rescale(L, cm)
    sc = D * D / orc.Q[L]
    xy = x * y
    assert np.max(np.abs(sch.dec(cr, L - 1, sc) - xy)) < 2.0 ** -20
    r1 = orc.rotate(L - 1, sch.keys[1][1], sch.keys[1][0], cr)
    r7 = orc.rotate(L - 1, sch.keys[7][1], sch.keys[7][0], cr)
    tot = orc.add(L - 1, r1, r7)
    want = np.roll(xy, -1) + np.roll(xy, -7)
    assert np.max(np.abs(sch.dec(tot, L - 1, sc) - want)) < 2.0 ** -20
    # rotate(k) then rotate(-k) is the identity on the slots
    back = orc.rotate(L - 1, sch.keys[-1][1], sch.keys[-1][0], r1)
    assert np.max(np.abs(sch.dec(back, L - 1, sc) - xy)) < 2.0 ** -20
    # hoisted rotations decrypt like the plain ones
    h = orc.rotate_hoisted(L - 1, [sch.keys[1][1], sch.keys[7][1]], [sch.keys[1][0], sch.keys[7][0]], cr)
    assert np.max(np.abs(sch.dec(h[0], L - 1, sc) - np.roll(xy, -1))) < 2.0 ** -20
    assert np.max(np.abs(sch.dec(h[1], L - 1, sc) - np.roll(xy, -7))) < 2.0 ** -20


def test_multi_digit_keyswitch_and_plain_ops():
    orc = _small_ctx()     # alpha = 2: digits of 2, 2, 1 primes at the top level
    sch = Scheme(orc, seed=3, rots=(2,))
    N, L = orc.N, orc.L
    D = 2.0 ** 35
    x = S.uniform_slots(sch.g, N // 2)
    y = S.uniform_slots(sch.g, N // 2)
    for level in (L, L - 1, 2):
        cx, cy = sch.enc(x, level, D), sch.enc(y, level, D)
        assert np.max(np.abs(sch.dec(orc.add(level, cx, cy), level, D) - (x + y))) < 2.0 ** -25
        assert np.max(np.abs(sch.dec(orc.sub(level, cx, cy), level, D) - (x - y))) < 2.0 ** -25
        assert np.max(np.abs(sch.dec(orc.neg(level, cx), level, D) + x)) < 2.0 ** -25
        cm = orc.mult_relin(level, sch.rlk, cx, cy)
        assert np.max(np.abs(sch.dec(cm, level, D * D) - x * y)) < 2.0 ** -20
        py = O.encode(y, N, D, orc.Q[: level + 1])
        assert np.max(np.abs(sch.dec(orc.mul_plain(level, cx, py), level, D * D) - x * y)) < 2.0 ** -20
        assert np.max(np.abs(sch.dec(orc.add_plain(level, cx, py), level, D) - (x + y))) < 2.0 ** -25
        three = np.array([3 % q for q in orc.Q[: level + 1]], dtype=np.uint64)
        assert np.max(np.abs(sch.dec(orc.mul_scalar(level, cx, three), level, D) - 3 * x)) < 2.0 ** -25
        half = np.array([int(D * 0.5) % q for q in orc.Q[: level + 1]], dtype=np.uint64)
        assert np.max(np.abs(sch.dec(orc.add_scalar(level, cx, half), level, D) - (x + 0.5))) < 2.0 ** -25
        r = orc.rotate(level, sch.keys[2][1], sch.keys[2][0], cx)
        assert np.max(np.abs(sch.dec(r, level, D) - np.roll(x, -2))) < 2.0 ** -20
