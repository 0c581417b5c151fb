"""Canonical-embedding encoder/decoder of the oracle -- TEST INFRASTRUCTURE ONLY.

Paper Section 3: a vector z of up to N/2 complex values is mapped into
R = Z[X]/(X^N + 1) by (a variant of) the inverse canonical embedding, and
decoding evaluates the polynomial back.  The variant used here:

* slot j corresponds to the root zeta^(5^j), zeta = exp(i pi / N), j < N/2;
  with this order X -> X^(5^k) rotates the slots left by k, as Rot(a, k) of
  Section 3 requires;
* encode:  t_k = (1/n) Re( sum_j z_j zeta^(-k 5^j) ),  k < N,  n = N/2, then
  m_k = round_half_even(scale * t_k) reduced modulo every prime;
* decode:  centred CRT of the residues, then z_j = m(zeta^(5^j)) / scale.

The sums are taken with numpy's FFT of length 2N (a library primitive): the
slot values are scattered to the positions 5^j mod 2N of a length-2N array.
"""
import numpy as np


def slot_exponents(N):
    """5^j mod 2N for j = 0 .. N/2-1."""
    n = N // 2
    e = np.empty(n, dtype=np.int64)
    x = 1
    for j in range(n):
        e[j] = x
        x = (x * 5) % (2 * N)
    return e


def embed_inverse(z, N):
    """Real coefficients t_k (k < N) whose canonical embedding is z."""
    n = N // 2
    zz = np.zeros(n, dtype=np.complex128)
    z = np.asarray(z, dtype=np.complex128).ravel()
    zz[: len(z)] = z
    A = np.zeros(2 * N, dtype=np.complex128)
    A[slot_exponents(N)] = zz
    F = np.fft.fft(A)                       # F[k] = sum_m A[m] zeta^(-m k)
    return F[:N].real / n


def embed(t, N):
    """Slot values z_j = t(zeta^(5^j)) of a real coefficient vector t."""
    B = np.zeros(2 * N, dtype=np.complex128)
    B[:N] = np.asarray(t, dtype=np.float64)
    G = np.fft.ifft(B) * (2 * N)            # G[p] = sum_k t_k zeta^(p k)
    return G[slot_exponents(N)]


def encode(z, N, scale, moduli):
    """Plaintext residues [len(moduli)][N] (uint64) of the vector z at 'scale'."""
    t = embed_inverse(z, N)
    m = np.rint(t * float(scale))
    if np.max(np.abs(m)) >= 2.0 ** 62:
        raise ValueError("encoded coefficient exceeds 2^62")
    mi = m.astype(np.int64)
    return np.stack([(mi % np.int64(q)).astype(np.uint64) for q in moduli])


def crt_centered(res, moduli):
    """Exact centred integers (numpy object array of Python ints) from residues
    [len(moduli)][N] by the Chinese remainder theorem."""
    res = np.asarray(res, dtype=np.uint64)
    Q = 1
    for q in moduli:
        Q *= int(q)
    acc = np.zeros(res.shape[1], dtype=object)
    for i, q in enumerate(moduli):
        q = int(q)
        Qi = Q // q
        ci = pow(Qi % q, -1, q)
        yi = np.array([(int(x) * ci) % q for x in res[i]], dtype=object)
        acc = acc + yi * Qi
    acc = acc % Q
    half = Q // 2
    return np.array([int(x) - Q if x > half else int(x) for x in acc], dtype=object)


def decode(res, N, scale, moduli):
    """Slot values (complex, length N/2) of plaintext residues at 'scale'."""
    m = crt_centered(res, moduli)
    t = np.array([float(x) for x in m], dtype=np.float64) / float(scale)
    return embed(t, N)
