"""rbk_rescale_batch_noalloc (the allocation-free entry point) against
rbk_rescale_batch, through the C ABI: bit-exact on two calls in a row (the
second with a smaller input), no device memory allocated by the call, and a
clear error above the scratch limit."""
import numpy as np
import pytest

import synth_inputs as S

pytestmark = pytest.mark.gpu

# N = 2^16, 24 primes: the key-switch workload's ring
QB, PB, ALPHA = [60] + [50] * 23, [60] * 8, 8


def test_noalloc_rescale_matches_rescale_batch():
    import torch

    from paper_2506_19693_amd import Context, RbkError

    d = Context(16, QB, PB, ALPHA)
    try:
        N = d.N
        g = S.rng(31, 16)
        limit_words = (64 << 20) // 8
        # first call: 2 ciphertexts at level 20 (2 x 2 x 21 x 2^16 words = 42 MiB of scratch)
        # second call: 1 ciphertext at level 9 (smaller, so stale words of the first remain)
        for count, level in ((2, 20), (1, 9)):
            assert 2 * count * (1 + level) * N <= limit_words
            ct = d.to_ntt(S.uniform_residues(g, d.moduli[: level + 1], N, lead=(count, 2)), level)
            want = d.rescale_batch(ct, level)
            torch.cuda.synchronize()
            out = torch.full((count, 2, level, N), -1, dtype=torch.int64, device="cuda")
            free0 = torch.cuda.mem_get_info()[0]
            d.rescale_batch_noalloc(ct, level, out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            assert free1 >= free0 - (4 << 20), "the call allocated device memory"
            assert torch.equal(out, want), (count, level)
            print("noalloc rescale: %d ciphertexts at level %d equal to rbk_rescale_batch" % (count, level), flush=True)
        # above the scratch limit: 3 ciphertexts at level 23 need 72 MiB
        ct = d.empty(3, 2, 24, N)
        out = d.empty(3, 2, 23, N)
        with pytest.raises(RbkError):
            d.rescale_batch_noalloc(ct, 23, out)
        # overlapping input and output
        with pytest.raises(RbkError):
            d.rescale_batch_noalloc(ct[:1], 23, ct[:1])
    finally:
        d.close()


def test_noalloc_rescale_small_ring_and_oracle():
    """The unfused path (N = 2^10) against the oracle itself."""
    import oracle as O
    from paper_2506_19693_amd import Context

    qb, pb = [60, 50, 50, 50], [60]
    d = Context(10, qb, pb, 1)
    o = O.Oracle(10, qb, pb, 1)
    try:
        g = S.rng(32, 10)
        L = o.L
        a = S.uniform_residues(g, o.Q, d.N, lead=(3, 2))
        out = d.empty(3, 2, L, d.N)
        d.rescale_batch_noalloc(d.to_ntt(a, L), L, out)
        for i in range(3):
            assert np.array_equal(d.to_coef(out[i], L - 1), o.rescale(L, a[i]))
    finally:
        d.close()
