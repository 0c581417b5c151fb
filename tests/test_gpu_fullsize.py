"""Bit-exact parity at the headline geometries, through the batched path the
benchmark times.

* N = 2^16, 24 primes (60 + 23 x 50 bits), 8 special 60-bit primes, digits
  of 8 primes, NTT split 2^8 x 2^8: mult_relin -> rescale -> hoisted
  rotations (+1, -3, +32) on a batch of two ciphertexts, with one and two
  ModDown lanes, plus the uneven-level list call; against per-limb SHA-256
  digests the CPU oracle wrote (tests/golden/make_golden.py);
* N = 2^16 bootstrap (26 primes, 9 special, HW-192 secret, q_0 / scale in
  [4, 8)), with the oracle planner's integer constants imported: the output
  of the single and the batched call against the oracle's digests;
* N = 2^14 and 2^15 with every NTT split the register kernels take, against
  the oracle run live.
Paper Section 3: multiplication, relinearisation, rescaling, Rot(a, k) and
the bootstrapping of the last paragraph.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from golden import cases as C
from oracle import boot as B

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def mismatches(got, want):
    """indices of limbs whose digest differs"""
    have = C.limb_digests(got)
    assert len(have) == len(want)
    return [i for i, (a, b) in enumerate(zip(have, want)) if a != b]


# ---------------------------------------------------------------- key switching, N = 2^16

class KsCase:
    def __init__(self):
        from paper_2506_19693_amd import Context

        p = C.KS
        self.gold = golden("keyswitch_n16.json")
        self.d = d = Context(p["logN"], p["qbits"], p["pbits"], p["alpha"])
        assert d.moduli == self.gold["moduli"]
        N = d.N
        self.dr = dr = C.ks_draws(d.moduli, d.nQ, d.beta, N)
        d.set_secret(dr["s"])
        d.keygen_relin(*dr["rlk"])
        for k, r in zip(C.KS_ROTS, dr["gal"]):
            d.keygen_galois(d.galois_elt(k), *r)
        L = d.L
        self.A = d.to_ntt(dr["A"], L)
        self.B = d.to_ntt(dr["B"], L)


_KS = []


def ks_case():
    if not _KS:
        _KS.append(KsCase())
    return _KS[0]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("lanes", [1, 2])
def test_keyswitch_n16_batched_matches_oracle(lanes):
    c = ks_case()
    d, gold = c.d, c.gold
    L = d.L
    d.set_lanes(lanes)
    d.tune_set(logC=8, cpc=d.tune_get()["cpc"])
    print("N=2^16 batched key switching, lanes %d, split %s" % (lanes, d.tune_get()), flush=True)
    m = d.mult_relin_batch(c.A, c.B, L)
    r = d.rescale_batch(m, L)
    h = d.rotate_hoisted_batch(r, C.KS_ROTS, L - 1)
    for i in range(C.KS_COUNT):
        assert mismatches(d.to_coef(m[i], L), gold["mult_relin"][i]) == [], ("mult_relin", i)
        assert mismatches(d.to_coef(r[i], L - 1), gold["rescale"][i]) == [], ("rescale", i)
        assert mismatches(d.to_coef(h[i], L - 1), gold["hoisted"][i]) == [], ("hoisted", i)
    d.set_lanes(2)


@pytest.mark.timeout(600)
def test_keyswitch_n16_plain_and_list_match_oracle():
    import torch

    c = ks_case()
    d, gold = c.d, c.gold
    L = d.L
    d.tune_set(logC=8, cpc=d.tune_get()["cpc"])
    # plain: one ciphertext per call
    i = 1
    m = d.mult_relin(c.A[i], c.B[i], L)
    r = d.rescale(m, L)
    h = d.rotate_hoisted(r, C.KS_ROTS, L - 1)
    assert mismatches(d.to_coef(m, L), gold["mult_relin"][i]) == []
    assert mismatches(d.to_coef(r, L - 1), gold["rescale"][i]) == []
    assert mismatches(d.to_coef(h, L - 1), gold["hoisted"][i]) == []
    # uneven levels in one list call
    lv = C.KS_LIST_LEVELS
    Lm = max(lv)
    A = torch.zeros(len(lv), 2, Lm + 1, d.N, dtype=torch.int64, device="cuda")
    Bt = torch.zeros_like(A)
    for j, (l, (a, b)) in enumerate(zip(lv, c.dr["lst"])):
        A[j, :, : l + 1] = d.to_ntt(a, l)
        Bt[j, :, : l + 1] = d.to_ntt(b, l)
    out = d.mult_relin_rescale_list(A, Bt, lv)
    for j, l in enumerate(lv):
        got = d.to_coef(out[j, :, :l].contiguous(), l - 1)
        assert mismatches(got, gold["list"][j]) == [], ("list", j, l)


# ---------------------------------------------------------------- N = 2^14, 2^15: every register split

MID = dict(qbits=[60] + [50] * 5, pbits=[60] * 3, alpha=2)
# N = 2^17 (the paper's larger ring) takes the general two-pass transforms
SPLITS = [(14, 6), (14, 7), (14, 8), (15, 7), (15, 8), (17, 8), (17, 9)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("logN,logC", SPLITS)
def test_keyswitch_splits_match_oracle(logN, logC):
    from paper_2506_19693_amd import Context

    d = Context(logN, MID["qbits"], MID["pbits"], MID["alpha"])
    o = O.Oracle(logN, MID["qbits"], MID["pbits"], MID["alpha"])
    try:
        assert d.moduli == o.moduli
        N, L = d.N, d.L
        g = S.rng(23, logN)
        s = S.ternary(g, N)
        d.set_secret(s)
        ra = S.key_randomness(g, o.beta, o.moduli, N)
        rlk = o.keygen_relin(s, *ra)
        d.keygen_relin(*ra)
        ks = [1, -3, 5]
        gals, gks = [], []
        for k in ks:
            gal = o.galois_rot(k)
            r = S.key_randomness(g, o.beta, o.moduli, N)
            gals.append(gal)
            gks.append(o.keygen_galois(s, gal, *r))
            d.keygen_galois(gal, *r)
        a = S.uniform_residues(g, o.Q, N, lead=(2, 2))
        b = S.uniform_residues(g, o.Q, N, lead=(2, 2))
        d.tune_set(logC=logC, cpc=d.tune_get()["cpc"])
        assert d.tune_get()["logC"] == logC
        print("N=2^%d split 2^%d: batched mult_relin, rescale, hoisted rotations" % (logN, logC), flush=True)
        want = []
        for i in range(2):
            wm = o.mult_relin(L, rlk, a[i], b[i])
            wr = o.rescale(L, wm)
            want.append((wm, wr, np.stack(o.rotate_hoisted(L - 1, gks, gals, wr))))
        for lanes in (1, 2):
            d.set_lanes(lanes)
            m = d.mult_relin_batch(d.to_ntt(a, L), d.to_ntt(b, L), L)
            r = d.rescale_batch(m, L)
            h = d.rotate_hoisted_batch(r, ks, L - 1)
            for i, (wm, wr, wh) in enumerate(want):
                assert np.array_equal(d.to_coef(m[i], L), wm), (lanes, i)
                assert np.array_equal(d.to_coef(r[i], L - 1), wr), (lanes, i)
                assert np.array_equal(d.to_coef(h[i], L - 1), wh), (lanes, i)
    finally:
        d.close()


# ---------------------------------------------------------------- bootstrapping, N = 2^16

@pytest.mark.timeout(900)
def test_bootstrap_n16_matches_oracle():
    """The bootstrap at the headline geometry (log2 rho = 2, the setting the
    benchmark runs), with the oracle planner's integer constants imported:
    every output limb of the single and the batched call against the digests
    of the oracle's own bootstrap of the same ciphertext."""
    from paper_2506_19693_amd import Context

    p = C.BOOT
    gold = golden("bootstrap_n16.json")
    d = Context(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    try:
        assert d.moduli == gold["moduli"]
        o = O.Oracle(p["logN"], p["qbits"], p["pbits"], p["alpha"])
        N = d.N
        plan = B.Plan(N, o.Q, B.BootParams(log2_rho=p["log2_rho"]))
        rots = plan.rotations()
        assert rots == gold["rotations"]
        dr = C.boot_draws(d.moduli, d.nQ, d.beta, N, rots)
        d.set_secret(dr["s"])
        d.keygen_public(*dr["pk"])
        d.keygen_relin(*dr["rlk"])
        for k, r in zip(list(rots) + ["conj"], dr["gal"]):
            d.keygen_galois(d.galois_conj() if k == "conj" else d.galois_elt(k), *r)
        d.boot_setup(log2_rho=p["log2_rho"])
        assert d.boot_rotations() == rots and d.boot_levels[3] == gold["level_out"]
        d.boot_import([pt for _, pt in plan.plains], [sc for _, sc in plan.scalars])
        # the input: the oracle's encryption of the seeded slots at level 0
        pk = o.keygen_public(dr["s"], *dr["pk"])
        ct = o.encrypt(0, pk, O.encode(dr["z"], N, C.BOOT_SCALE, o.Q[:1]), *dr["enc"])
        assert C.limb_digests(ct) == gold["input"]
        lo = gold["level_out"]
        print("N=2^16 bootstrap with the oracle's constants, output level %d" % lo, flush=True)
        out, so = d.bootstrap(d.to_ntt(ct, 0), C.BOOT_SCALE)
        assert so == pytest.approx(gold["scale_out"], rel=1e-12)
        assert mismatches(d.to_coef(out, lo), gold["output"]) == []
        # the batched call: the same ciphertext twice, next to one at another scale
        cts = d.empty(3, 2, 1, N)
        x = d.to_ntt(ct, 0)
        cts[0].copy_(x)
        cts[1].copy_(d.encrypt(d.encode(dr["z"], 0, 2.0 ** 37), 0, *S.encryption_randomness(S.rng(5, 16), N)))
        cts[2].copy_(x)
        outs, sos = d.bootstrap_batch(cts, [C.BOOT_SCALE, 2.0 ** 37, C.BOOT_SCALE])
        for i in (0, 2):
            assert sos[i] == so
            assert mismatches(d.to_coef(outs[i], lo), gold["output"]) == [], i
    finally:
        d.close()
