"""Pins of the oracle's seeded sampler (CPU only).

The keystream is the ChaCha20 block function of RFC 8439; the test vectors
below are the RFC's own (Section 2.1.1 quarter round, Section 2.3.2 block
function, Appendix A.1 test vector #1).  The samplers built on it are pinned
by what their distributions must be: residues below q and uniform (chi-square
against the flat law), ternary thirds, the Gaussian's probabilities
exp(-x^2 / 2 sigma^2) / Z (chi-square against them, computed here from the
definition), exactly h non-zeros for the fixed-weight secret, and streams
that differ when the nonce differs.  The library's own Gaussian table is
compared with the oracle's (both are host float64 computations).
"""
import math
import struct

import numpy as np
import pytest

import oracle as O


def words_le(hexstr):
    b = bytes.fromhex(hexstr)
    return [struct.unpack("<I", b[4 * i: 4 * i + 4])[0] for i in range(len(b) // 4)]


def test_rfc8439_quarter_round():
    # Section 2.1.1
    assert O.chacha_quarter([0x11111111, 0x01020304, 0x9B8D6F43, 0x01234567]) == [
        0xEA2A92F4, 0xCB1CF8CE, 0x4581472E, 0x5881C4BB]


def test_rfc8439_block_function():
    # Section 2.3.2: key 00:01:..:1f, nonce 00:00:00:09:00:00:00:4a:00:00:00:00, counter 1
    key = words_le(bytes(range(32)).hex())
    nonce = words_le("000000090000004a00000000")
    assert O.chacha_block(key, 1, nonce) == [
        0xE4E7F110, 0x15593BD1, 0x1FDD0F50, 0xC47120A3, 0xC7F4D1C7, 0x0368C033, 0x9AAA2204, 0x4E6CD4C3,
        0x466482D2, 0x09AA9F07, 0x05D7C214, 0xA2028BD9, 0xD19C12B5, 0xB94E16DE, 0xE883D0CB, 0x4E3C50A2]


def test_rfc8439_zero_key_keystream():
    # Appendix A.1, test vector #1: all-zero key and nonce, counter 0
    want = words_le("76b8e0ada0f13d90405d6ae55386bd28bdd219b8a08ded1aa836efcc8b770dc7"
                    "da41597c5157488d7724e03fb8d84a376a43b8f41518a11cc387b669b2ee6586")
    assert O.chacha_block([0] * 8, 0, [0] * 3) == want


def chi2_ok(counts, probs, n):
    """chi-square statistic within 5 standard deviations of its mean (df = bins - 1)."""
    exp = np.asarray(probs) * n
    stat = float(np.sum((np.asarray(counts) - exp) ** 2 / exp))
    df = len(counts) - 1
    return stat < df + 5 * math.sqrt(2 * df), stat


@pytest.mark.parametrize("q", [97, 257, 12289])
def test_uniform_is_below_q_and_flat(q):
    x = np.concatenate([O.sample_uniform(5, O.P_KEY_A, 1, s, q, 14) for s in range(4)]).astype(np.int64)
    assert x.max() < q and x.min() >= 0
    bins = 16
    counts = np.bincount(x * bins // q, minlength=bins)
    probs = [(math.ceil((b + 1) * q / bins) - math.ceil(b * q / bins)) / q for b in range(bins)]
    ok, stat = chi2_ok(counts, probs, x.size)
    assert ok, stat


def test_uniform_large_prime_moments():
    q = O.gen_primes(14, [50])[0]
    x = O.sample_uniform(9, O.P_PK_A, 0, 3, q, 14).astype(np.float64) / q
    assert x.max() < 1.0
    n = x.size
    assert abs(x.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(x.var() - 1 / 12) < 0.01


def test_ternary_thirds():
    x = O.sample_ternary(3, O.P_SECRET, 0, 0, 16)
    assert set(np.unique(x)) <= {-1, 0, 1}
    counts = [int(np.sum(x == v)) for v in (-1, 0, 1)]
    ok, stat = chi2_ok(counts, [1 / 3] * 3, x.size)
    assert ok, stat


def test_gaussian_follows_the_discrete_law():
    sigma = 3.2
    x = np.concatenate([O.sample_gauss(7, O.P_KEY_E, 0, j, 16) for j in range(4)])
    assert np.abs(x).max() <= 19
    vals = np.arange(-19, 20)
    rho = np.exp(-vals.astype(np.float64) ** 2 / (2 * sigma ** 2))
    probs = rho / rho.sum()
    # pool the tails (expected counts below 5) into the outermost kept bins
    keep = np.nonzero(probs * x.size >= 5)[0]
    lo, hi = keep[0], keep[-1]
    counts = np.array([np.sum(x == v) for v in vals])
    c = counts[lo: hi + 1].astype(np.float64)
    p = probs[lo: hi + 1].copy()
    c[0] += counts[:lo].sum()
    p[0] += probs[:lo].sum()
    c[-1] += counts[hi + 1:].sum()
    p[-1] += probs[hi + 1:].sum()
    ok, stat = chi2_ok(c, p, x.size)
    assert ok, stat
    assert abs(x.mean()) < 5 * sigma / math.sqrt(x.size)
    assert abs(x.var() / float(np.sum(probs * vals ** 2)) - 1) < 0.02


def test_gaussian_table_shape():
    T = O.gauss_table()
    assert all(a < b for a, b in zip(T, T[1:]))
    assert T[-1] == 1 << 63
    # P(x = 0) = 1 / Z
    sigma = 3.2
    Z = 1 + 2 * sum(math.exp(-m * m / (2 * sigma * sigma)) for m in range(1, 20))
    assert abs(T[0] / 2.0 ** 63 - 1 / Z) < 1e-15


@pytest.mark.parametrize("logN,h", [(10, 64), (16, 192), (4, 16)])
def test_fixed_weight_secret(logN, h):
    s = O.sample_ternary_hw(21, logN, h)
    assert int(np.count_nonzero(s)) == h
    assert set(np.unique(s[s != 0])) <= {-1, 1}
    if h >= 64:
        assert abs(int(np.sum(s == 1)) - h / 2) < 5 * math.sqrt(h / 4)
    assert np.array_equal(s, O.sample_ternary_hw(21, logN, h))
    assert not np.array_equal(s, O.sample_ternary_hw(22, logN, h))


def test_streams_are_separate():
    a = O.sample_uniform(1, O.P_KEY_A, 5, 0, 97, 10)
    assert np.array_equal(a, O.sample_uniform(1, O.P_KEY_A, 5, 0, 97, 10))
    for other in (O.sample_uniform(2, O.P_KEY_A, 5, 0, 97, 10), O.sample_uniform(1, O.P_PK_A, 5, 0, 97, 10),
                  O.sample_uniform(1, O.P_KEY_A, 6, 0, 97, 10), O.sample_uniform(1, O.P_KEY_A, 5, 1, 97, 10)):
        assert np.mean(a == other) < 0.05


def test_seed_reaches_the_high_key_word():
    lo = O.sample_gauss(1, O.P_ENC_E0, 0, 0, 10)
    hi = O.sample_gauss(1 | (1 << 32), O.P_ENC_E0, 0, 0, 10)
    assert not np.array_equal(lo, hi)


def test_library_gauss_table_equals_oracle():
    from paper_2506_19693_amd import rbk

    assert rbk.gauss_table() == O.gauss_table()
