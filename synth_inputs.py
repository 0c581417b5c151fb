"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws random numbers and nothing else: it holds none of the
CKKS arithmetic.  Every random quantity the scheme needs (secret key, key and
encryption noise, public uniform polynomials, slot values) is drawn here and
handed, identically, to the GPU library and to the CPU oracle.

Distributions:
* secret: uniform ternary {-1, 0, 1}, or ternary with exactly h non-zeros;
* errors: rounded Gaussian, sigma = 3.2, clipped to |x| <= 19 (6 sigma);
* public randomness: uniform residues in [0, q) for every prime q;
* slot values: uniform reals in [lo, hi).
"""
import numpy as np

SIGMA = 3.2
ERR_BOUND = 19


def rng(seed, *stream):
    """Independent generator for (seed, stream...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed)] + [int(s) for s in stream])))


def ternary(g, N):
    return g.integers(-1, 2, size=N, dtype=np.int64)


def ternary_hw(g, N, h):
    s = np.zeros(N, dtype=np.int64)
    pos = g.choice(N, size=h, replace=False)
    s[pos] = np.where(g.integers(0, 2, size=h) == 0, -1, 1)
    return s


def gaussian(g, *shape, sigma=SIGMA):
    e = np.rint(g.normal(0.0, sigma, size=shape))
    return np.clip(e, -ERR_BOUND, ERR_BOUND).astype(np.int64)


def uniform_residues(g, moduli, N, lead=()):
    """Array lead + [len(moduli)][N] of uniform residues, limb i below moduli[i]."""
    lead = tuple(lead)
    out = np.empty(lead + (len(moduli), N), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[(Ellipsis, i, slice(None))] = g.integers(0, int(q), size=lead + (N,), dtype=np.uint64)
    return out


def uniform_slots(g, n, lo=-1.0, hi=1.0):
    return g.uniform(lo, hi, size=n)


def key_randomness(g, beta, moduli, N):
    """(a, e) of a switching key with beta digits over the primes 'moduli'."""
    a = uniform_residues(g, moduli, N, lead=(beta,))
    e = gaussian(g, beta, N)
    return a, e


def encryption_randomness(g, N):
    """(v, e0, e1) of one public-key encryption."""
    return ternary(g, N), gaussian(g, N), gaussian(g, N)


def mlp_batch(g, b, k0, o):
    """A synthetic classification batch: features uniform in [0, 1), one-hot
    labels of classes drawn uniformly from o."""
    X = g.uniform(0.0, 1.0, size=(b, k0))
    Y = np.zeros((b, o))
    Y[np.arange(b), g.integers(0, o, size=b)] = 1.0
    return X, Y


def mlp_weights(g, dims):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) matrices of the given (fan_in, fan_out) shapes."""
    return [g.uniform(-1.0, 1.0, size=(d, k)) / np.sqrt(d) for d, k in dims]
