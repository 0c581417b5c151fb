"""CPU oracle for the RNS-CKKS hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2506_19693_amd``); the two only see the same seeded inputs.

* ``ckks_oracle.c`` holds the integer arithmetic (primes, NTT, ring ops, key
  switching, rescale, automorphisms), written as plain definitions.
* ``encoding.py`` holds the canonical-embedding encoder/decoder (paper
  Section 3) in float64 numpy with Python big integers for the CRT.
* ``boot.py`` and ``mlp.py`` build the bootstrap and the packed MLP step out of
  these operations.

Every polynomial crossing this interface is in the coefficient domain.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
intp = ctypes.POINTER(ctypes.c_int)
u32p = ctypes.POINTER(ctypes.c_uint32)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        sigs = {
            "orc_mulmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
            "orc_powmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
            "orc_invmod": (ctypes.c_uint64, [ctypes.c_uint64] * 2),
            "orc_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
            "orc_is_prime_trial": (ctypes.c_int, [ctypes.c_uint64]),
            "orc_gen_primes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, intp, u64p]),
            "orc_min_psi": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int]),
            "orc_ntt_direct": (None, [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]),
            "orc_ntt": (None, [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]),
            "orc_intt": (None, [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]),
            "orc_negacyclic_schoolbook": (None, [ctypes.c_int, ctypes.c_uint64, u64p, u64p, u64p]),
            "orc_ctx_new": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, intp, ctypes.c_int, intp, ctypes.c_int]),
            "orc_ctx_free": (None, [ctypes.c_void_p]),
            "orc_ctx_moduli": (None, [ctypes.c_void_p, u64p]),
            "orc_ctx_psi": (None, [ctypes.c_void_p, u64p]),
            "orc_num_digits": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
            "orc_limb_mul": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_limb_ntt": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_limb_intt": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_bconv": (None, [ctypes.c_void_p, ctypes.c_int, intp, u64p, ctypes.c_int, intp, u64p]),
            "orc_keygen_switch": (None, [ctypes.c_void_p, i64p, u64p, u64p, i64p, u64p]),
            "orc_keygen_public": (None, [ctypes.c_void_p, i64p, u64p, i64p, u64p]),
            "orc_secret_square": (None, [ctypes.c_void_p, i64p, u64p]),
            "orc_secret_automorph": (None, [ctypes.c_void_p, i64p, ctypes.c_uint64, u64p]),
            "orc_encrypt": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, i64p, i64p, i64p, u64p]),
            "orc_decrypt": (None, [ctypes.c_void_p, ctypes.c_int, i64p, u64p, u64p]),
            "orc_add": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, u64p, u64p, u64p]),
            "orc_sub": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, u64p, u64p, u64p]),
            "orc_neg": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, u64p, u64p]),
            "orc_mul_plain": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_add_plain": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_mul_scalar": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, u64p, u64p, u64p]),
            "orc_add_scalar": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_tensor": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_modup": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_key_inner_product": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_moddown": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_keyswitch": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p]),
            "orc_mult_relin": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p, u64p, u64p]),
            "orc_rescale": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_automorph_limbs": (None, [ctypes.c_void_p, ctypes.c_int, intp, ctypes.c_uint64, u64p, u64p]),
            "orc_automorph": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, u64p]),
            "orc_galois_rot": (ctypes.c_uint64, [ctypes.c_void_p, ctypes.c_int64]),
            "orc_rotate": (None, [ctypes.c_void_p, ctypes.c_int, u64p, ctypes.c_uint64, u64p, u64p]),
            "orc_rotate_hoisted": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(u64p), u64p, u64p, u64p]),
            "orc_modraise": (None, [ctypes.c_void_p, ctypes.c_int, u64p, u64p]),
            "orc_monomial": (None, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, u64p]),
            "orc_chacha_quarter": (None, [u32p]),
            "orc_chacha_block": (None, [u32p, ctypes.c_uint32, u32p, u32p]),
            "orc_sample_uniform": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_int, u64p]),
            "orc_sample_ternary": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_int, i64p]),
            "orc_sample_gauss": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_int, i64p]),
            "orc_gauss_table": (None, [u64p]),
            "orc_sample_ternary_hw": (None, [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, i64p]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _u(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(i64p)


def _ints(v):
    arr = (ctypes.c_int * len(v))(*[int(x) for x in v])
    return arr


# ---------------------------------------------------------------- primitives

def is_prime(n):
    return bool(lib().orc_is_prime(int(n)))


def is_prime_trial(n):
    return bool(lib().orc_is_prime_trial(int(n)))


def gen_primes(logN, bits):
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = lib().orc_gen_primes(logN, len(bits), _ints(bits), out.ctypes.data_as(u64p))
    if rc != 0:
        raise ValueError("no prime for the requested bit sizes")
    return [int(x) for x in out]


def min_psi(q, logN):
    return int(lib().orc_min_psi(int(q), logN))


def mulmod(a, b, q):
    return int(lib().orc_mulmod(int(a), int(b), int(q)))


def ntt_direct(logN, q, psi, a):
    a, pa = _u(a)
    out = np.zeros_like(a)
    lib().orc_ntt_direct(logN, int(q), int(psi), pa, out.ctypes.data_as(u64p))
    return out


def ntt(logN, q, psi, a):
    a, pa = _u(a)
    out = np.zeros_like(a)
    lib().orc_ntt(logN, int(q), int(psi), pa, out.ctypes.data_as(u64p))
    return out


def intt(logN, q, psi, a):
    a, pa = _u(a)
    out = np.zeros_like(a)
    lib().orc_intt(logN, int(q), int(psi), pa, out.ctypes.data_as(u64p))
    return out


def negacyclic_schoolbook(logN, q, a, b):
    a, pa = _u(a)
    b, pb = _u(b)
    out = np.zeros_like(a)
    lib().orc_negacyclic_schoolbook(logN, int(q), pa, pb, out.ctypes.data_as(u64p))
    return out


# ---------------------------------------------------------------- seeded sampling (ChaCha20, RFC 8439)

P_SECRET, P_PK_A, P_PK_E, P_KEY_A, P_KEY_E, P_ENC_V, P_ENC_E0, P_ENC_E1 = range(1, 9)


def chacha_quarter(x4):
    a = (ctypes.c_uint32 * 4)(*[int(v) for v in x4])
    lib().orc_chacha_quarter(a)
    return [int(v) for v in a]


def chacha_block(key8, counter, nonce3):
    k = (ctypes.c_uint32 * 8)(*[int(v) for v in key8])
    n = (ctypes.c_uint32 * 3)(*[int(v) for v in nonce3])
    out = (ctypes.c_uint32 * 16)()
    lib().orc_chacha_block(k, int(counter), n, out)
    return [int(v) for v in out]


def sample_uniform(seed, purpose, ident, sub, q, logN):
    out = np.zeros(1 << logN, dtype=np.uint64)
    lib().orc_sample_uniform(int(seed), purpose, int(ident), int(sub), int(q), logN, out.ctypes.data_as(u64p))
    return out


def sample_ternary(seed, purpose, ident, sub, logN):
    out = np.zeros(1 << logN, dtype=np.int64)
    lib().orc_sample_ternary(int(seed), purpose, int(ident), int(sub), logN, out.ctypes.data_as(i64p))
    return out


def sample_gauss(seed, purpose, ident, sub, logN):
    out = np.zeros(1 << logN, dtype=np.int64)
    lib().orc_sample_gauss(int(seed), purpose, int(ident), int(sub), logN, out.ctypes.data_as(i64p))
    return out


def gauss_table():
    out = np.zeros(20, dtype=np.uint64)
    lib().orc_gauss_table(out.ctypes.data_as(u64p))
    return [int(x) for x in out]


def sample_ternary_hw(seed, logN, h):
    out = np.zeros(1 << logN, dtype=np.int64)
    lib().orc_sample_ternary_hw(int(seed), logN, int(h), out.ctypes.data_as(i64p))
    return out


# ---------------------------------------------------------------- context

class Oracle:
    """RNS-CKKS context of the oracle: ring degree 2^logN, the Q chain with
    the given prime sizes, nP special primes, alpha limbs per key-switch digit."""

    def __init__(self, logN, qbits, pbits, alpha):
        self.logN = int(logN)
        self.N = 1 << self.logN
        self.nQ = len(qbits)
        self.nP = len(pbits)
        self.alpha = int(alpha)
        self.L = self.nQ - 1
        h = lib().orc_ctx_new(self.logN, self.nQ, _ints(qbits), self.nP, _ints(pbits), self.alpha)
        if not h:
            raise ValueError("bad oracle parameters")
        self._h = ctypes.c_void_p(h)
        m = np.zeros(self.nQ + self.nP, dtype=np.uint64)
        lib().orc_ctx_moduli(self._h, m.ctypes.data_as(u64p))
        self.moduli = [int(x) for x in m]
        p = np.zeros(self.nQ + self.nP, dtype=np.uint64)
        lib().orc_ctx_psi(self._h, p.ctypes.data_as(u64p))
        self.psi = [int(x) for x in p]
        self.beta = self.num_digits(self.L)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.orc_ctx_free(h)
            self._h = None

    @property
    def Q(self):
        return self.moduli[: self.nQ]

    @property
    def P(self):
        return self.moduli[self.nQ:]

    def num_digits(self, level):
        return int(lib().orc_num_digits(self._h, level))

    def ext_indices(self, level):
        return list(range(level + 1)) + list(range(self.nQ, self.nQ + self.nP))

    # ------------------------------------------------------------ small helpers
    def _new(self, *shape):
        return np.zeros(shape, dtype=np.uint64)

    def limb_mul(self, t, a, b):
        a, pa = _u(a)
        b, pb = _u(b)
        out = self._new(self.N)
        lib().orc_limb_mul(self._h, t, pa, pb, out.ctypes.data_as(u64p))
        return out

    def limb_ntt(self, t, a):
        a, pa = _u(a)
        out = self._new(self.N)
        lib().orc_limb_ntt(self._h, t, pa, out.ctypes.data_as(u64p))
        return out

    def limb_intt(self, t, a):
        a, pa = _u(a)
        out = self._new(self.N)
        lib().orc_limb_intt(self._h, t, pa, out.ctypes.data_as(u64p))
        return out

    def bconv(self, in_idx, x, out_idx):
        x, px = _u(x)
        out = self._new(len(out_idx), self.N)
        lib().orc_bconv(self._h, len(in_idx), _ints(in_idx), px, len(out_idx), _ints(out_idx), out.ctypes.data_as(u64p))
        return out

    def signed_to_residues(self, v, idx):
        v = np.asarray(v, dtype=np.int64)
        return np.stack([(v % np.int64(self.moduli[t])).astype(np.uint64) for t in idx])

    # ------------------------------------------------------------ keys
    def secret_square(self, s):
        s, ps = _i(s)
        out = self._new(self.nQ + self.nP, self.N)
        lib().orc_secret_square(self._h, ps, out.ctypes.data_as(u64p))
        return out

    def secret_automorph(self, s, g):
        s, ps = _i(s)
        out = self._new(self.nQ + self.nP, self.N)
        lib().orc_secret_automorph(self._h, ps, int(g), out.ctypes.data_as(u64p))
        return out

    def keygen_switch(self, s, s_from, a, e):
        s, ps = _i(s)
        s_from, pf = _u(s_from)
        a, pa = _u(a)
        e, pe = _i(e)
        assert a.shape == (self.beta, self.nQ + self.nP, self.N)
        assert e.shape == (self.beta, self.N)
        out = self._new(self.beta, 2, self.nQ + self.nP, self.N)
        lib().orc_keygen_switch(self._h, ps, pf, pa, pe, out.ctypes.data_as(u64p))
        return out

    def keygen_relin(self, s, a, e):
        return self.keygen_switch(s, self.secret_square(s), a, e)

    def keygen_galois(self, s, g, a, e):
        return self.keygen_switch(s, self.secret_automorph(s, g), a, e)

    def keygen_public(self, s, a, e):
        s, ps = _i(s)
        a, pa = _u(a)
        e, pe = _i(e)
        out = self._new(2, self.nQ, self.N)
        lib().orc_keygen_public(self._h, ps, pa, pe, out.ctypes.data_as(u64p))
        return out

    # ------------------------------------------------------------ enc / dec
    def encrypt(self, level, pk, m, v, e0, e1):
        pk, ppk = _u(pk)
        m, pm = _u(m)
        v, pv = _i(v)
        e0, p0 = _i(e0)
        e1, p1 = _i(e1)
        out = self._new(2, level + 1, self.N)
        lib().orc_encrypt(self._h, level, ppk, pm, pv, p0, p1, out.ctypes.data_as(u64p))
        return out

    def decrypt(self, level, s, ct):
        s, ps = _i(s)
        ct, pc = _u(ct)
        out = self._new(level + 1, self.N)
        lib().orc_decrypt(self._h, level, ps, pc, out.ctypes.data_as(u64p))
        return out

    # ------------------------------------------------------------ ring ops
    def _binop(self, fn, level, a, b):
        a, pa = _u(a)
        b, pb = _u(b)
        npoly = a.size // ((level + 1) * self.N)
        out = np.zeros_like(a)
        fn(self._h, level, npoly, pa, pb, out.ctypes.data_as(u64p))
        return out

    def add(self, level, a, b):
        return self._binop(lib().orc_add, level, a, b)

    def sub(self, level, a, b):
        return self._binop(lib().orc_sub, level, a, b)

    def neg(self, level, a):
        a, pa = _u(a)
        out = np.zeros_like(a)
        lib().orc_neg(self._h, level, a.size // ((level + 1) * self.N), pa, out.ctypes.data_as(u64p))
        return out

    def mul_plain(self, level, ct, pt):
        ct, pc = _u(ct)
        pt, pp = _u(pt)
        out = np.zeros_like(ct)
        lib().orc_mul_plain(self._h, level, pc, pp, out.ctypes.data_as(u64p))
        return out

    def add_plain(self, level, ct, pt):
        ct, pc = _u(ct)
        pt, pp = _u(pt)
        out = np.zeros_like(ct)
        lib().orc_add_plain(self._h, level, pc, pp, out.ctypes.data_as(u64p))
        return out

    def mul_scalar(self, level, a, scal):
        a, pa = _u(a)
        scal, ps = _u(scal)
        out = np.zeros_like(a)
        lib().orc_mul_scalar(self._h, level, a.size // ((level + 1) * self.N), pa, ps, out.ctypes.data_as(u64p))
        return out

    def add_scalar(self, level, ct, scal):
        ct, pc = _u(ct)
        scal, ps = _u(scal)
        out = np.zeros_like(ct)
        lib().orc_add_scalar(self._h, level, pc, ps, out.ctypes.data_as(u64p))
        return out

    def tensor(self, level, a, b):
        a, pa = _u(a)
        b, pb = _u(b)
        out = self._new(3, level + 1, self.N)
        lib().orc_tensor(self._h, level, pa, pb, out.ctypes.data_as(u64p))
        return out

    # ------------------------------------------------------------ key switching
    def modup(self, level, d):
        d, pd = _u(d)
        out = self._new(self.num_digits(level), level + 1 + self.nP, self.N)
        lib().orc_modup(self._h, level, pd, out.ctypes.data_as(u64p))
        return out

    def key_inner_product(self, level, ext, key):
        ext, pe = _u(ext)
        key, pk = _u(key)
        out = self._new(2, level + 1 + self.nP, self.N)
        lib().orc_key_inner_product(self._h, level, pe, pk, out.ctypes.data_as(u64p))
        return out

    def moddown(self, level, u):
        u, pu = _u(u)
        out = self._new(level + 1, self.N)
        lib().orc_moddown(self._h, level, pu, out.ctypes.data_as(u64p))
        return out

    def keyswitch(self, level, key, d):
        key, pk = _u(key)
        d, pd = _u(d)
        out = self._new(2, level + 1, self.N)
        lib().orc_keyswitch(self._h, level, pk, pd, out.ctypes.data_as(u64p))
        return out

    def mult_relin(self, level, rlk, a, b):
        rlk, pr = _u(rlk)
        a, pa = _u(a)
        b, pb = _u(b)
        out = self._new(2, level + 1, self.N)
        lib().orc_mult_relin(self._h, level, pr, pa, pb, out.ctypes.data_as(u64p))
        return out

    def rescale(self, level, ct):
        ct, pc = _u(ct)
        out = self._new(2, level, self.N)
        lib().orc_rescale(self._h, level, pc, out.ctypes.data_as(u64p))
        return out

    def automorph(self, level, g, a):
        a, pa = _u(a)
        out = np.zeros_like(a)
        lib().orc_automorph(self._h, level, a.size // ((level + 1) * self.N), int(g), pa, out.ctypes.data_as(u64p))
        return out

    def galois_rot(self, k):
        return int(lib().orc_galois_rot(self._h, int(k)))

    def galois_conj(self):
        return 2 * self.N - 1

    def rotate(self, level, key, g, ct):
        key, pk = _u(key)
        ct, pc = _u(ct)
        out = self._new(2, level + 1, self.N)
        lib().orc_rotate(self._h, level, pk, int(g), pc, out.ctypes.data_as(u64p))
        return out

    def rotate_hoisted(self, level, keys, gs, ct):
        keys = [np.ascontiguousarray(k, dtype=np.uint64) for k in keys]
        kp = (u64p * len(keys))(*[k.ctypes.data_as(u64p) for k in keys])
        gs_a = np.ascontiguousarray(gs, dtype=np.uint64)
        ct, pc = _u(ct)
        out = self._new(len(keys), 2, level + 1, self.N)
        lib().orc_rotate_hoisted(self._h, level, len(keys), kp, gs_a.ctypes.data_as(u64p), pc, out.ctypes.data_as(u64p))
        return out

    def modraise(self, level, ct0):
        ct0, pc = _u(ct0)
        out = self._new(2, level + 1, self.N)
        lib().orc_modraise(self._h, level, pc, out.ctypes.data_as(u64p))
        return out

    def monomial(self, level, e, a):
        a, pa = _u(a)
        out = np.zeros_like(a)
        lib().orc_monomial(self._h, level, a.size // ((level + 1) * self.N), int(e), pa, out.ctypes.data_as(u64p))
        return out

    # ------------------------------------------------------------ keys and encryption from one seed
    def seeded_secret(self, seed, hw=0):
        """hw = 0: uniform ternary; hw > 0: exactly hw non-zero coefficients."""
        if hw:
            return sample_ternary_hw(seed, self.logN, hw)
        return sample_ternary(seed, P_SECRET, 0, 0, self.logN)

    def seeded_key_randomness(self, seed, g):
        """(a, e) of the switching key with Galois element g (0 = relinearisation):
        a limb t of digit j from nonce (KEY_A, g, j * 2^16 + t), e of digit j from
        (KEY_E, g, j)."""
        nT = self.nQ + self.nP
        a = np.stack([np.stack([sample_uniform(seed, P_KEY_A, g, (j << 16) | t, self.moduli[t], self.logN)
                                for t in range(nT)]) for j in range(self.beta)])
        e = np.stack([sample_gauss(seed, P_KEY_E, g, j, self.logN) for j in range(self.beta)])
        return a, e

    def seeded_public_randomness(self, seed):
        a = np.stack([sample_uniform(seed, P_PK_A, 0, t, self.moduli[t], self.logN) for t in range(self.nQ)])
        return a, sample_gauss(seed, P_PK_E, 0, 0, self.logN)

    def seeded_encryption_randomness(self, seed, index):
        """(v, e0, e1) of encryption number `index` (64-bit: low word = id, high word = sub)."""
        lo, hi = int(index) & 0xFFFFFFFF, int(index) >> 32
        return (sample_ternary(seed, P_ENC_V, lo, hi, self.logN), sample_gauss(seed, P_ENC_E0, lo, hi, self.logN),
                sample_gauss(seed, P_ENC_E1, lo, hi, self.logN))

    def drop(self, level_from, level_to, ct):
        """Keep limbs 0..level_to of every polynomial (the value is unchanged)."""
        ct = np.asarray(ct, dtype=np.uint64)
        return np.ascontiguousarray(ct[..., : level_to + 1, :])


from .encoding import encode, decode, crt_centered, slot_exponents  # noqa: E402,F401
