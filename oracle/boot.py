"""Approximate CKKS bootstrapping, oracle side -- TEST INFRASTRUCTURE ONLY.

Paper Section 3 (last paragraph and its footnote): a ciphertext at level 0 is
refreshed to a higher level by homomorphically applying the encoding step,
approximating the modular reduction by a scaled sine, and applying the
decoding step (Cheon-Han-Kim-Kim-Song 2018; as in Bossuat et al. 2021).
Steps, in order:

1. integer pre-scale at level 0 by 2^e, so that the scale lies in
   (D_ref/2, D_ref] with D_ref = 2^(bits(q_0) - log2_rho);
2. ModRaise: dec = m + q_0 I(X), |I| <= K with overwhelming probability;
3. CoeffToSlot: the inverse of the decoding map, factored into log2(n)
   radix-2 butterfly stages grouped into `cts_levels` sparse linear
   transforms, each evaluated baby-step/giant-step with hoisted baby
   rotations; the conjugation splits real and imaginary parts;
4. EvalMod on each part: a Chebyshev interpolant of
   cos(2 pi ((K+1) u - 1/4) / 2^r) on [-1, 1], then r double-angle steps
   y <- 2 y^2 - 1, giving sin(2 pi x) ~ 2 pi (m / q_0);
5. SlotToCoeff: the decoding map in `stc_levels` transforms, the constant
   q_0 / (2 pi D_ref) folded into its first level.

Only integer constants (encoded diagonals and scalars) cross into the
ciphertext arithmetic; they are produced in a fixed order (the plan order)
so that the same constants can be handed to another implementation.
"""
import math

import numpy as np

from .encoding import encode


class BootParams:
    """K: bound on |I|; degree of the Chebyshev interpolant; double_angle: r;
    cts_levels / stc_levels: transforms of each linear map; log2_rho: the
    reference scale is 2^(bits(q_0) - log2_rho), so q_0 / scale is in
    [2^log2_rho, 2^(log2_rho+1))."""

    def __init__(self, K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2):
        self.log2_rho = log2_rho
        self.K = K
        self.degree = degree
        self.r = double_angle
        self.cts_levels = cts_levels
        self.stc_levels = stc_levels


# ---------------------------------------------------------------- linear algebra of the decoding map

def twiddles(n, M, depth):
    """T_depth[l] = zeta^(2^depth * 5^l mod M), l < n / 2^(depth+1), zeta = exp(2 pi i / M)."""
    h = n >> (depth + 1)
    e = np.empty(h, dtype=np.int64)
    x = 1
    for l in range(h):
        e[l] = (x << depth) % M
        x = (x * 5) % M
    return np.exp(2j * np.pi * e / M)


def stage(n, M, s, inverse):
    """Butterfly stage S_s (s = 1 .. log2 n; S_1 has blocks of size n) as
    {offset: diagonal}, the matrix being sum_o diag(d_o) Rot_o.  Forward,
    inside each block of size 2h: out_j = v_j + T_l v_(j+h), out_(j+h) = v_j - T_l v_(j+h)."""
    size = n >> (s - 1)
    h = size // 2
    T = twiddles(n, M, s - 1)
    idx = np.arange(n)
    loc = idx % size
    top = loc < h
    Tl = T[np.where(top, loc, loc - h)]
    d0 = np.empty(n, dtype=np.complex128)
    dp = np.zeros(n, dtype=np.complex128)
    dm = np.zeros(n, dtype=np.complex128)
    if not inverse:
        d0[top] = 1.0
        d0[~top] = -Tl[~top]
        dp[top] = Tl[top]
        dm[~top] = 1.0
    else:
        d0[top] = 0.5
        d0[~top] = -0.5 / Tl[~top]
        dp[top] = 0.5
        dm[~top] = 0.5 / Tl[~top]
    out = {0: d0}
    out[h % n] = out.get(h % n, 0) + dp
    out[(-h) % n] = out.get((-h) % n, 0) + dm
    return out


def matmul_diag(A, B, n):
    """(A B) in diagonal form: C_(a+b) += A_a * roll(B_b, -a)."""
    C = {}
    for a, da in A.items():
        for b, db in B.items():
            o = (a + b) % n
            C[o] = C.get(o, 0) + da * np.roll(db, -a)
    return C


def apply_diag(A, v):
    out = np.zeros_like(v)
    for o, d in A.items():
        out = out + d * np.roll(v, -o)
    return out


def stage_groups(logn, levels):
    """Split stages 1..logn into `levels` contiguous groups, the first
    (logn mod levels) groups one stage longer."""
    base, extra = divmod(logn, levels)
    groups, s = [], 1
    for g in range(levels):
        cnt = base + (1 if g < extra else 0)
        groups.append(list(range(s, s + cnt)))
        s += cnt
    return groups


def group_matrix(n, M, stages, inverse):
    """Product of the stages in the order they are applied to a vector.
    Forward (decoding): group [s1..sk] is S_s1 ... S_sk, S_sk applied first.
    Inverse: (S_s1 ... S_sk)^-1 = S_sk^-1 ... S_s1^-1, S_s1^-1 applied first."""
    mats = [stage(n, M, s, inverse) for s in stages]
    if inverse:
        mats = mats[::-1]
    P = mats[0]
    for A in mats[1:]:
        P = matmul_diag(P, A, n)
    return P


def group_offsets(n, stages):
    """Base step h0 (half-size of the group's innermost stage) and the
    normalised multipliers kk of every diagonal offset kk*h0 of the group."""
    h0 = n >> stages[-1]
    k = len(stages)
    W = n // h0
    if (2 << k) - 1 <= W:
        kks = list(range(-((1 << k) - 1), (1 << k)))
    else:
        kks = list(range(-(W // 2), W // 2))
    return h0, kks


def baby_steps(k):
    """Baby-step count of a group of k stages: 2^ceil((k+1)/2)."""
    return 1 << ((k + 2) // 2)


def bsgs(kks, n1):
    """(g, b, kk) with kk = g*n1 + b, 0 <= b < n1, sorted by g then b."""
    out = [(kk // n1, kk - (kk // n1) * n1, kk) for kk in kks]
    return sorted(out)


# ---------------------------------------------------------------- EvalMod

def cheb_coeffs(f, degree):
    """Chebyshev interpolant at the degree+1 Chebyshev nodes of [-1, 1]."""
    d1 = degree + 1
    j = np.arange(d1)
    nodes = np.cos(np.pi * (j + 0.5) / d1)
    fv = f(nodes)
    c = np.empty(d1)
    for k in range(d1):
        c[k] = (2.0 / d1) * np.sum(fv * np.cos(np.pi * k * (j + 0.5) / d1))
    c[0] /= 2
    return c


def evalmod_function(K, r):
    return lambda u: np.cos(2 * np.pi * ((K + 1) * u - 0.25) / (1 << r))


def cheb_split(c, m):
    """p = q T_m + r for Chebyshev coefficients c (deg >= m), using
    T_(m+j) = 2 T_m T_j - T_(m-j)."""
    d = len(c) - 1
    assert m <= d < 2 * m
    q = np.zeros(d - m + 1)
    r = np.array(c[:m], dtype=np.float64)
    q[0] = c[m]
    for j in range(1, d - m + 1):
        q[j] = 2 * c[m + j]
        r[m - j] -= c[m + j]
    return q, r


POWER_RECIPE = [  # (k, a, b, c): T_k = 2 T_a T_b - T_c ; c = 0 means the constant 1
    (2, 1, 1, 0), (3, 1, 2, 1), (4, 2, 2, 0), (5, 2, 3, 1), (6, 3, 3, 0), (7, 3, 4, 1),
]
BABY = 8


def giant_powers(degree):
    out, m = [], BABY
    while m <= degree:
        out.append(m)
        m *= 2
    return out


# ---------------------------------------------------------------- plan

def _residues(v, moduli):
    v = int(v)
    return np.array([v % int(q) for q in moduli], dtype=np.uint64)


def _round_int(x):
    """Nearest integer of a double (exact: a double above 2^53 is an integer)."""
    return int(round(x))


class Plan:
    """Levels, scales and integer constants of one bootstrap for the chain
    `moduli` (Q primes) at ring degree N, full slots (n = N/2)."""

    def __init__(self, N, moduli, params):
        self.N = N
        self.n = N // 2
        self.M = 2 * N
        self.logn = int(math.log2(self.n))
        self.q = [int(x) for x in moduli]
        self.P = params
        self.L = len(self.q) - 1
        K = params.K
        q0 = self.q[0]
        self.dref_log2 = q0.bit_length() - params.log2_rho
        self.s_A = 2.0 ** math.ceil(math.log2(2.0 * q0 * (K + 1)))
        self.c_cts = self.s_A / (2.0 * q0 * (K + 1))
        self.c_stc = q0 / (2 * math.pi * 2.0 ** self.dref_log2)
        self.plains = []     # (level, residues [level+1][N]) in plan order
        self.scalars = []    # (level, residues [level+1]) in plan order
        self.cheb = cheb_coeffs(evalmod_function(K, params.r), params.degree)
        self._build()

    # -- linear transforms
    def _lt(self, groups, inverse, level0, s_in, fold, drops):
        lts = []
        s = s_in
        for gi, stages in enumerate(groups):
            lvl = level0 - gi
            A = group_matrix(self.n, self.M, stages, inverse)
            if gi == 0:
                A = {o: d * fold for o, d in A.items()}
            h0, kks = group_offsets(self.n, stages)
            n1 = baby_steps(len(stages))
            ql = self.q[lvl]
            Sd = float(ql) * 2.0 ** (-drops[gi])
            entries = []
            for (g, b, kk) in bsgs(kks, n1):
                diag = A.get((kk * h0) % self.n)
                if diag is None:
                    diag = np.zeros(self.n, dtype=np.complex128)
                vals = np.roll(diag, g * n1 * h0)
                pt = encode(vals, self.N, Sd, self.q[: lvl + 1])
                self.plains.append((lvl, pt))
                entries.append((g, b, kk, len(self.plains) - 1))
            lts.append(dict(level=lvl, h0=h0, n1=n1, entries=entries, Sd=Sd, s_in=s))
            s = s * Sd / ql
        return lts, s

    # -- EvalMod program
    def _scalar(self, level, value):
        self.scalars.append((level, _residues(value, self.q[: level + 1])))
        return len(self.scalars) - 1

    def _evalmod_plan(self, level, s):
        prog = []
        T = {1: (level, s)}

        def prod(k, a, b, c):
            la, sa = T[a]
            lb, sb = T[b]
            lv = min(la, lb)
            sp = sa * sb
            if c == 0:
                idx = self._scalar(lv, -_round_int(sp))
            else:
                lc, sc = T[c]
                idx = self._scalar(lv, _round_int(sp / sc))
            prog.append(("prod", k, a, b, c, lv, idx))
            T[k] = (lv - 1, sp / self.q[lv])

        for (k, a, b, c) in POWER_RECIPE:
            if k <= self.P.degree:
                prod(k, a, b, c)
        for m in giant_powers(self.P.degree):
            prod(m, m // 2, m // 2, 0)

        def level_of(deg):
            if deg < BABY:
                return min(T[k][0] for k in range(1, deg + 1)) - 1
            m = max(g for g in giant_powers(self.P.degree) if g <= deg)
            lq = level_of(deg - m)
            lr = level_of(m - 1)
            return min(min(lq, T[m][0]) - 1, lr)

        def ev(c, s_t, reg):
            deg = len(c) - 1
            if deg < BABY:
                assert deg >= 1
                lv = min(T[k][0] for k in range(1, deg + 1))
                terms = []
                for k in range(1, deg + 1):
                    if c[k] != 0.0:
                        terms.append((k, self._scalar(lv, _round_int(c[k] * s_t * self.q[lv] / T[k][1]))))
                cidx = self._scalar(lv, _round_int(c[0] * s_t * self.q[lv]))
                prog.append(("leaf", reg, lv, terms, cidx))
                return lv - 1
            m = max(g for g in giant_powers(self.P.degree) if g <= deg)
            qc, rc = cheb_split(c, m)
            lq = level_of(len(qc) - 1)
            lp = min(lq, T[m][0])
            s_q = s_t * self.q[lp] / T[m][1]
            ev(qc, s_q, reg + "q")
            ev(rc, s_t, reg + "r")
            lr = level_of(len(rc) - 1)
            out = min(lp - 1, lr)
            prog.append(("giant", reg, m, lp, out))
            return out

        s_t = s
        lvl = ev(self.cheb, s_t, "p")
        sc = s_t
        for _ in range(self.P.r):
            idx = self._scalar(lvl, -_round_int(sc * sc))
            prog.append(("dbl", lvl, idx))
            sc = sc * sc / self.q[lvl]
            lvl -= 1
        return prog, lvl, sc

    def _build(self):
        P = self.P
        groups_cts = stage_groups(self.logn, P.cts_levels)
        groups_stc = stage_groups(self.logn, P.stc_levels)
        # CoeffToSlot: scale s_A -> about the size of the top prime
        s_b_log2 = round(math.log2(self.q[self.L]))
        total = int(round(math.log2(self.s_A))) - s_b_log2
        drops = [total // P.cts_levels] * P.cts_levels
        drops[-1] += total - sum(drops)
        self.cts, s = self._lt(groups_cts, True, self.L, self.s_A, self.c_cts, drops)
        self.level_evalmod = self.L - P.cts_levels
        self.s_B = s
        self.evalmod, lvl, s = self._evalmod_plan(self.level_evalmod, s)
        self.level_stc = lvl
        self.s_E = s
        # SlotToCoeff applies the groups innermost first
        self.stc, s = self._lt(groups_stc[::-1], False, lvl, s, self.c_stc, [0] * P.stc_levels)
        self.level_out = lvl - P.stc_levels
        self.s_out = s
        if self.level_out < 0:
            raise ValueError("modulus chain too short for bootstrapping")

    def rotations(self):
        """Every rotation index the plan uses (the conjugation is separate)."""
        ks = set()
        for lt in self.cts + self.stc:
            for (g, b, kk, _) in lt["entries"]:
                if b:
                    ks.add(b * lt["h0"])
                if g:
                    ks.add(g * lt["n1"] * lt["h0"])
        n = self.n
        return sorted({k % n for k in ks} - {0})


# ---------------------------------------------------------------- execution on the oracle

class Evaluator:
    """Runs a plan with the oracle's ciphertext operations.  keys: dict
    Galois element -> switching key; rlk: relinearisation key."""

    def __init__(self, orc, plan, rlk, keys):
        self.o = orc
        self.p = plan
        self.rlk = rlk
        self.keys = keys

    def rot(self, level, ct, k):
        g = self.o.galois_rot(k)
        if g == 1:
            return ct
        return self.o.rotate(level, self.keys[g], g, ct)

    def lt(self, ct, lt):
        o, lvl = self.o, lt["level"]
        h0, n1 = lt["h0"], lt["n1"]
        babies = sorted({b for (g, b, kk, i) in lt["entries"] if b})
        rots = {0: ct}
        if babies:
            ks = [b * h0 for b in babies]
            gs = [o.galois_rot(k) for k in ks]
            outs = o.rotate_hoisted(lvl, [self.keys[g] for g in gs], gs, ct)
            for b, r in zip(babies, outs):
                rots[b] = r
        total = None
        for g in sorted({e[0] for e in lt["entries"]}):
            inner = None
            for (gg, b, kk, i) in lt["entries"]:
                if gg != g:
                    continue
                t = o.mul_plain(lvl, rots[b], self.p.plains[i][1])
                inner = t if inner is None else o.add(lvl, inner, t)
            if g:
                inner = self.rot(lvl, inner, g * n1 * h0)
            total = inner if total is None else o.add(lvl, total, inner)
        return o.rescale(lvl, total)

    def scalar(self, idx):
        return self.p.scalars[idx][1]

    def evalmod(self, ct):
        o, p = self.o, self.p
        T = {1: ct}
        lvT = {1: p.level_evalmod}

        def at(k, lv):
            return o.drop(lvT[k], lv, T[k])

        regs = {}
        for step in p.evalmod:
            kind = step[0]
            if kind == "prod":
                _, k, a, b, c, lv, idx = step
                x = o.mult_relin(lv, self.rlk, at(a, lv), at(b, lv))
                x = o.add(lv, x, x)
                if c == 0:
                    x = o.add_scalar(lv, x, self.scalar(idx))
                else:
                    x = o.sub(lv, x, o.mul_scalar(lv, at(c, lv), self.scalar(idx)))
                T[k] = o.rescale(lv, x)
                lvT[k] = lv - 1
            elif kind == "leaf":
                _, reg, lv, terms, cidx = step
                acc = None
                for (k, idx) in terms:
                    t = o.mul_scalar(lv, at(k, lv), self.scalar(idx))
                    acc = t if acc is None else o.add(lv, acc, t)
                acc = o.add_scalar(lv, acc, self.scalar(cidx))
                regs[reg] = (o.rescale(lv, acc), lv - 1)
            elif kind == "giant":
                _, reg, m, lp, out = step
                qct, lq = regs.pop(reg + "q")
                rct, lr = regs.pop(reg + "r")
                x = o.mult_relin(lp, self.rlk, o.drop(lq, lp, qct), at(m, lp))
                x = o.rescale(lp, x)
                x = o.drop(lp - 1, out, x)
                regs[reg] = (o.add(out, x, o.drop(lr, out, rct)), out)
            elif kind == "dbl":
                _, lv, idx = step
                y, ly = regs["p"]
                y = o.drop(ly, lv, y)
                x = o.mult_relin(lv, self.rlk, y, y)
                x = o.add(lv, x, x)
                x = o.add_scalar(lv, x, self.scalar(idx))
                regs["p"] = (o.rescale(lv, x), lv - 1)
        return regs["p"][0]

    def bootstrap(self, ct0, scale_in):
        """ct0: level-0 ciphertext [2][1][N] at scale scale_in.  Returns
        (ciphertext at plan.level_out, its scale)."""
        o, p = self.o, self.p
        frac, ex = math.frexp(scale_in)
        e = p.dref_log2 - (ex - 1 if frac == 0.5 else ex)
        if e < 0:
            raise ValueError("input scale above the bootstrapping reference scale")
        d_prime = scale_in * 2.0 ** e
        ct = o.mul_scalar(0, ct0, np.array([pow(2, e, p.q[0])], dtype=np.uint64))
        ct = o.modraise(p.L, ct)
        for lt in p.cts:
            ct = self.lt(ct, lt)
        lv = p.level_evalmod
        conj = o.rotate(lv, self.keys[2 * o.N - 1], 2 * o.N - 1, ct)
        re = o.add(lv, ct, conj)
        im = o.monomial(lv, 3 * o.N // 2, o.sub(lv, ct, conj))
        re = self.evalmod(re)
        im = self.evalmod(im)
        lv = p.level_stc
        ct = o.add(lv, re, o.monomial(lv, o.N // 2, im))
        for lt in p.stc:
            ct = self.lt(ct, lt)
        # the slots hold z * d' / D_ref at the arithmetic scale s_out
        return ct, p.s_out * d_prime / 2.0 ** p.dref_log2


# ---------------------------------------------------------------- the overflow polynomial I of ModRaise

def modraise_overflow(orc, s, ct0):
    """I(X) with c0 + c1 s = m + q_0 I over the integers, for a level-0
    ciphertext ct0 ([2][1][N], residues mod q_0) read as centred integers and
    the secret s (small integers).  The bootstrap's EvalMod is valid only
    while every |I_j| <= K.

    t = c0 + c1 s is known modulo 2^64 (wrapping uint64 arithmetic of the
    negacyclic product) and modulo q_0 (m, the decryption); |t| < 2^63 and
    q_0 is odd, so I = (t - m) q_0^-1 mod 2^64, read as a signed word."""
    N = orc.N
    q0 = int(orc.Q[0])
    c = np.asarray(ct0, dtype=np.uint64).reshape(2, N)
    half = np.uint64((q0 - 1) // 2)
    # centred lifts, as uint64 words (two's complement for negative values)
    lift = [np.where(c[p] <= half, c[p], c[p] - np.uint64(q0)) for p in range(2)]
    t = lift[0].copy()
    with np.errstate(over="ignore"):
        for j in np.nonzero(s)[0]:
            sh = np.roll(lift[1], int(j))          # X^j c1: coefficient k comes from k - j
            sh[: int(j)] = np.uint64(0) - sh[: int(j)]   # wrapped past X^N: negated
            t = t + sh if s[j] > 0 else t - sh
        m = orc.decrypt(0, s, ct0).reshape(N)
        mc = np.where(m <= half, m, m - np.uint64(q0))
        inv = pow(q0, -1, 1 << 64)
        I = (t - mc) * np.uint64(inv)
    return I.view(np.int64)
