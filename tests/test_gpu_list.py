"""Descriptor-list entry points on the GPU: a list transform over limbs of
several ring degrees (2^11 .. 2^16) and primes in one launch matches the
oracle limb by limb, and the uneven-level mult_relin + rescale list at the
key-switch workload's ring (N = 2^16, 24 primes, 8 special, dnum 3) gives
the residues of the per-level batched calls."""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


def test_ntt_list_mixed_rings_matches_oracle():
    import random

    from paper_2506_19693_amd import Context, to_device, to_host

    qb, pb = [60, 50, 40], [60, 55]
    rings = []
    for logN in (11, 13, 14, 15, 16):
        ctx = Context(logN, qb, pb, 1)
        orc = O.Oracle(logN, qb, pb, 1)
        assert ctx.moduli == orc.moduli
        g = S.rng(41, logN)
        a = S.uniform_residues(g, orc.moduli, 1 << logN, lead=(3,))
        rings.append((ctx, orc, a, to_device(a)))
    items = []
    for ctx, _, _, t in rings:
        for c in range(3):
            for l in range(5):
                items.append((ctx, t, (c * 5 + l) * ctx.N, l))
    random.Random(3).shuffle(items)      # rings and primes interleaved in the list
    drv = rings[0][0]
    drv.ntt_list(items)
    for ctx, orc, a, t in rings:
        got = to_host(t)
        for c in range(3):
            for l in range(5):
                assert np.array_equal(got[c][l], orc.limb_ntt(l, a[c][l])), (ctx.N, c, l)
    drv.ntt_list(items, inverse=True)
    for ctx, orc, a, t in rings:
        assert np.array_equal(to_host(t), a), ctx.N


def test_uneven_levels_full_size_match_batched():
    import torch

    from paper_2506_19693_amd import Context, to_device

    ctx = Context(16, [60] + [50] * 23, [60] * 8, 8)
    g = S.rng(43, 16)
    N = ctx.N
    ctx.set_secret(S.ternary(g, N))
    ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, N))
    levels = [23, 9, 17, 4, 23, 12]
    Lm, cnt = max(levels), len(levels)
    A = torch.zeros(cnt, 2, Lm + 1, N, dtype=torch.int64, device="cuda")
    B = torch.zeros_like(A)
    for i, l in enumerate(levels):
        A[i, :, : l + 1] = to_device(S.uniform_residues(g, ctx.moduli[: l + 1], N, lead=(2,)))
        B[i, :, : l + 1] = to_device(S.uniform_residues(g, ctx.moduli[: l + 1], N, lead=(2,)))
    out = ctx.mult_relin_rescale_list(A, B, levels)
    for i, l in enumerate(levels):
        a = A[i : i + 1, :, : l + 1].contiguous()
        b = B[i : i + 1, :, : l + 1].contiguous()
        want = ctx.rescale_batch(ctx.mult_relin_batch(a, b, l), l)
        assert torch.equal(out[i, :, :l], want[0]), (i, l)


def test_list_errors():
    from paper_2506_19693_amd import Context, RbkError

    ctx = Context(12, [50, 40, 40, 40], [50], 1)
    g = S.rng(44, 12)
    ctx.set_secret(S.ternary(g, ctx.N))
    ctx.keygen_relin(*S.key_randomness(g, ctx.beta, ctx.moduli, ctx.N))
    A = ctx.empty_ct(3, 2).zero_()
    with pytest.raises(RbkError):
        ctx.mult_relin_rescale_list(A, A, [3, 0])       # level 0 cannot be rescaled
    A4 = ctx.empty_ct(4, 2).zero_()
    with pytest.raises(RbkError):
        ctx.mult_relin_rescale_list(A4, A4, [3, 4])     # above the chain
