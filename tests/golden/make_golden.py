"""Write the expected per-limb digests of the full-size parity cases.

Runs the CPU oracle only (paper Section 3: multiplication with
relinearisation, rescaling, rotations Rot(a, k), and the bootstrapping of its
last paragraph), on the inputs drawn by ``cases.py``, and stores SHA-256
digests of every output limb (coefficient domain) as JSON next to this file:

    python tests/golden/make_golden.py keyswitch   # about 2 minutes
    python tests/golden/make_golden.py bootstrap   # about 20 minutes

No value here comes from the GPU library.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from oracle import boot as B  # noqa: E402
from golden import cases as C  # noqa: E402


def log(msg):
    print("[%7.1f s] %s" % (time.time() - T0, msg), flush=True)


def keyswitch():
    p = C.KS
    o = O.Oracle(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    N, L = o.N, o.L
    d = C.ks_draws(o.moduli, o.nQ, o.beta, N)
    rlk = o.keygen_relin(d["s"], *d["rlk"])
    gals = [o.galois_rot(k) for k in C.KS_ROTS]
    gks = [o.keygen_galois(d["s"], gal, *r) for gal, r in zip(gals, d["gal"])]
    log("keys")
    out = dict(case=p, rots=C.KS_ROTS, count=C.KS_COUNT, list_levels=C.KS_LIST_LEVELS, moduli=o.moduli,
               mult_relin=[], rescale=[], hoisted=[], list=[])
    for i in range(C.KS_COUNT):
        m = o.mult_relin(L, rlk, d["A"][i], d["B"][i])
        r = o.rescale(L, m)
        h = o.rotate_hoisted(L - 1, gks, gals, r)
        out["mult_relin"].append(C.limb_digests(m))
        out["rescale"].append(C.limb_digests(r))
        out["hoisted"].append(C.limb_digests(np.stack(h)))
        log("ciphertext %d" % i)
    for l, (a, b) in zip(C.KS_LIST_LEVELS, d["lst"]):
        out["list"].append(C.limb_digests(o.rescale(l, o.mult_relin(l, rlk, a, b))))
        log("list level %d" % l)
    return out


def bootstrap():
    p = C.BOOT
    o = O.Oracle(p["logN"], p["qbits"], p["pbits"], p["alpha"])
    N = o.N
    plan = B.Plan(N, o.Q, B.BootParams(log2_rho=p["log2_rho"]))
    rots = plan.rotations()
    d = C.boot_draws(o.moduli, o.nQ, o.beta, N, rots)
    pk = o.keygen_public(d["s"], *d["pk"])
    rlk = o.keygen_relin(d["s"], *d["rlk"])
    gals = [o.galois_rot(k) for k in rots] + [o.galois_conj()]
    keys = {}
    for gal, r in zip(gals, d["gal"]):
        keys[gal] = o.keygen_galois(d["s"], gal, *r)
    log("plan and %d keys" % (len(keys) + 1))
    ct = o.encrypt(0, pk, O.encode(d["z"], N, C.BOOT_SCALE, o.Q[:1]), *d["enc"])
    ev = B.Evaluator(o, plan, rlk, keys)
    out_ct, s_out = ev.bootstrap(ct, C.BOOT_SCALE)
    log("bootstrap")
    lv = plan.level_out
    dec = O.decode(o.decrypt(lv, d["s"], out_ct), N, s_out, o.Q[: lv + 1])
    err = float(np.max(np.abs(dec - d["z"])))
    log("decrypted max slot error 2^%.2f" % np.log2(err))
    return dict(case=p, scale_in=C.BOOT_SCALE, rotations=rots, moduli=o.moduli, level_out=lv, scale_out=s_out,
                input=C.limb_digests(ct), output=C.limb_digests(out_ct), oracle_slot_error_log2=float(np.log2(err)))


if __name__ == "__main__":
    T0 = time.time()
    which = sys.argv[1]
    res = {"keyswitch": keyswitch, "bootstrap": bootstrap}[which]()
    res["written_by"] = "tests/golden/make_golden.py %s (CPU oracle only)" % which
    path = os.path.join(HERE, "%s_n16.json" % which)
    with open(path, "w") as f:
        json.dump(res, f, indent=0)
    log("wrote " + path)
