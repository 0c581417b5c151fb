"""Full-size parity cases: parameters and the order of their seeded draws.

Both the script that writes the expected digests (``make_golden.py``, oracle
only) and the GPU tests draw their inputs through these functions, so the two
see the same keys' randomness and the same ciphertexts.  Nothing here
computes any of the scheme's arithmetic; it only fixes parameters and the
sequence of calls into ``synth_inputs``.
"""
import hashlib

import synth_inputs as S

# Key switching at the headline geometry: N = 2^16, 24 primes (one 60-bit
# base prime, 23 x 50-bit), 8 special 60-bit primes, digits of 8 primes.
KS = dict(logN=16, qbits=[60] + [50] * 23, pbits=[60] * 8, alpha=8, seed=11)
KS_ROTS = [1, -3, 32]          # hoisted rotations after mult_relin + rescale
KS_COUNT = 2                    # ciphertexts in the batch
KS_LIST_LEVELS = [23, 12, 5]    # uneven levels of one list call

# Bootstrapping at the headline geometry: N = 2^16, 26 primes (60 + 25 x 50),
# 9 special primes, HW-192 secret, q_0 / scale in [4, 8).
BOOT = dict(logN=16, qbits=[60] + [50] * 25, pbits=[60] * 9, alpha=9, seed=19, log2_rho=2)
BOOT_SCALE = 2.0 ** 40


def ks_draws(moduli, nQ, beta, N):
    """secret, relinearisation and Galois-key randomness, the batch's two
    operands and the list case's operands (uniform residues)."""
    g = S.rng(KS["seed"], KS["logN"])
    s = S.ternary(g, N)
    rlk = S.key_randomness(g, beta, moduli, N)
    gal = [S.key_randomness(g, beta, moduli, N) for _ in KS_ROTS]
    A = S.uniform_residues(g, moduli[:nQ], N, lead=(KS_COUNT, 2))
    B = S.uniform_residues(g, moduli[:nQ], N, lead=(KS_COUNT, 2))
    lst = [(S.uniform_residues(g, moduli[: l + 1], N, lead=(2,)),
            S.uniform_residues(g, moduli[: l + 1], N, lead=(2,))) for l in KS_LIST_LEVELS]
    return dict(s=s, rlk=rlk, gal=gal, A=A, B=B, lst=lst)


def boot_draws(moduli, nQ, beta, N, rotations):
    """HW-192 secret, public-key, relinearisation and Galois-key randomness
    (rotations in the given order, then the conjugation), slot values and the
    encryption randomness of the level-0 input."""
    g = S.rng(BOOT["seed"], BOOT["logN"])
    s = S.ternary_hw(g, N, 192)
    pk = (S.uniform_residues(g, moduli[:nQ], N), S.gaussian(g, N))
    rlk = S.key_randomness(g, beta, moduli, N)
    gal = [S.key_randomness(g, beta, moduli, N) for _ in list(rotations) + ["conj"]]
    z = S.uniform_slots(g, N // 2)
    enc = S.encryption_randomness(g, N)
    return dict(s=s, pk=pk, rlk=rlk, gal=gal, z=z, enc=enc)


def limb_digests(arr):
    """SHA-256 (hex) of every limb of a [..][limbs][N] uint64 array, in C order."""
    flat = arr.reshape(-1, arr.shape[-1])
    return [hashlib.sha256(x.astype("<u8").tobytes()).hexdigest() for x in flat]
