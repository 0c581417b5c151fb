"""Packed local-loss MLP training step of ReBoot, oracle side -- TEST INFRASTRUCTURE ONLY.

What the step computes (paper Section 4):

* packing (Section 4.1): an r x c slot matrix (r c = N/2, slot (i, j) at index
  i c + j).  A vector is *repeated* (every row a copy) or *expanded* (every
  column a copy); a weight matrix is *row-wise* (W itself) or *column-wise*
  (W transposed), zero padded;
* RE-Matmul = SumRows(A_exp (.) W_row) -> repeated, CE-Matmul =
  SumCols(A_rep (.) W_col) -> expanded (Section 4.2.1); SumRows and SumCols
  are the rotate-and-add recursions of Section 3, SumCols with the first-slot
  mask between its two halves;
* blocks alternate RE (odd layers) and CE (even layers); block h trains layer
  h and its local classifier h* (opposite type) on the RSS gradient
  Yhat - Y (Section 4.3.2, Algorithm 1) and updates both with the NAG-style
  rule of Algorithm 2; every weight and velocity ciphertext is bootstrapped
  after the update.

Readings taken where the paper is silent, ambiguous or in conflict with itself:

* r c = N/2 with r >= every CE width, the input width (per tile) and the
  output count; c >= every RE width and the output count.  A first RE layer
  wider than r is tiled into ceil(k0 / r) row tiles: Z = SumRows(sum_t X_t (.) W_t)
  (SumRows is linear), and each tile gets its own gradient and velocity;
* activation f(z) = a1 z + a2 z^2 + a3 z^3 (the paper's z + z^2 is (1, 1, 0));
  the backward pass uses the chain rule dZ = dA (.) f'(Z); the flag
  ``literal_deriv`` takes the printed form dZ = 1 + 2 dA instead;
* the batch gradient is the mean of the per-sample gradients (it keeps the
  velocity inside the bootstrap's input range); decay as printed,
  dW <- (1 + eta) dW, or standard L2 (dW <- dW + eta W) with ``l2_decay``;
  the classifier uses its gradient of the same iteration;
* the three plaintext products of the update and the decay are folded into one
  scalar per operand, so W' = W - c_w dW - c_wv V and V' = c_v dW + c_vv V each
  cost one level;
* scale management: every ciphertext carries its exact float64 scale.  A
  product of ciphertexts has scale s_a s_b / q_l.  A product with a constant c
  encodes the integer round(c q_l T / s) (T the scale wanted after the
  rescale); the mask plaintext is encoded at scale q_l and keeps the scale; an
  affine map a x + b with a > 0 and one ciphertext is free: the scale becomes
  s / a and the integer round(b s / a) is added.  Additions therefore always
  meet equal scales.  The updated W and V get the scale 2^log2_scale.
"""
import math

import numpy as np

from .encoding import encode


# ---------------------------------------------------------------- configuration and packing

class MlpConfig:
    def __init__(self, k0, widths, o, r, c, act=(1.0, 1.0, 0.0), gamma=0.001, eta=0.001, mu=0.9,
                 log2_scale=50.0, literal_deriv=False, l2_decay=False):
        self.k0 = int(k0)
        self.widths = [int(w) for w in widths]
        self.o = int(o)
        self.r = int(r)
        self.c = int(c)
        self.act = tuple(float(a) for a in act)
        self.gamma, self.eta, self.mu = float(gamma), float(eta), float(mu)
        self.log2_scale = float(log2_scale)
        self.literal_deriv = bool(literal_deriv)
        self.l2_decay = bool(l2_decay)
        self.H = len(self.widths)
        assert self.H >= 1
        assert self.r & (self.r - 1) == 0 and self.c & (self.c - 1) == 0, "r and c are powers of two"
        a1, a2, a3 = self.act
        self.degree = 3 if a3 != 0.0 else 2
        lead = a3 if self.degree == 3 else a2
        assert lead > 0.0, "the leading activation coefficient must be positive"
        self.tiles = max(1, -(-self.k0 // self.r))
        for h in range(1, self.H + 1):
            d, k = self.layer_dims(h)
            if h % 2 == 1:
                assert (h == 1 or d <= self.r) and k <= self.c and self.o <= self.r
            else:
                assert d <= self.c and k <= self.r and self.o <= self.c

    @property
    def n(self):
        return self.r * self.c

    def layer_dims(self, h):
        ks = [self.k0] + self.widths
        return ks[h - 1], ks[h]

    def n_tiles(self, h):
        return self.tiles if h == 1 else 1

    def state_layout(self):
        """State ciphertexts in order: per block, W tiles, W*, V tiles, V*."""
        out = []
        for h in range(1, self.H + 1):
            nt = self.n_tiles(h)
            out += [("W", h, t) for t in range(nt)] + [("Wstar", h, 0)]
            out += [("V", h, t) for t in range(nt)] + [("Vstar", h, 0)]
        return out


def vec_rep(a, r, c):
    M = np.zeros((r, c))
    M[:, : len(a)] = a
    return M.ravel()


def vec_exp(a, r, c):
    M = np.zeros((r, c))
    M[: len(a), :] = np.asarray(a, dtype=np.float64)[:, None]
    return M.ravel()


def mat_row(W, r, c):
    M = np.zeros((r, c))
    M[: W.shape[0], : W.shape[1]] = W
    return M.ravel()


def mat_col(W, r, c):
    M = np.zeros((r, c))
    M[: W.shape[1], : W.shape[0]] = W.T
    return M.ravel()


def first_slot_mask(r, c):
    M = np.zeros((r, c))
    M[:, 0] = 1.0
    return M.ravel()


def pack_state(cfg, Ws, Wstars, Vs=None, Vstars=None):
    """Slot vectors of the state in state_layout() order (V entries zero if absent)."""
    r, c = cfg.r, cfg.c
    out = []
    for h in range(1, cfg.H + 1):
        for mats, stars in ((Ws, Wstars), (Vs, Vstars)):
            if mats is None:
                out += [np.zeros(cfg.n)] * (cfg.n_tiles(h) + 1)
                continue
            W, Wst = mats[h - 1], stars[h - 1]
            if h % 2 == 1:
                if cfg.n_tiles(h) > 1:
                    out += [mat_row(W[t * r: (t + 1) * r], r, c) for t in range(cfg.n_tiles(h))]
                else:
                    out.append(mat_row(W, r, c))
                out.append(mat_col(Wst, r, c))
            else:
                out.append(mat_col(W, r, c))
                out.append(mat_row(Wst, r, c))
    return out


def unpack_state(cfg, vecs):
    """(Ws, Wstars, Vs, Vstars) from state_layout()-ordered slot vectors."""
    r, c = cfg.r, cfg.c
    res = ([], [], [], [])
    i = 0
    for h in range(1, cfg.H + 1):
        d, k = cfg.layer_dims(h)
        nt = cfg.n_tiles(h)
        for which in (0, 1):
            if h % 2 == 1:
                if nt > 1:
                    rows = [vecs[i + t].reshape(r, c)[:, :k] for t in range(nt)]
                    W = np.vstack(rows)[:d].copy()
                else:
                    W = vecs[i].reshape(r, c)[:d, :k].copy()
                Wst = vecs[i + nt].reshape(r, c)[: cfg.o, :k].T.copy()
            else:
                W = vecs[i].reshape(r, c)[:k, :d].T.copy()
                Wst = vecs[i + nt].reshape(r, c)[:k, : cfg.o].copy()
            res[2 * which].append(W)
            res[2 * which + 1].append(Wst)
            i += nt + 1
    return res


def pack_sample(cfg, x, y):
    """(input tiles in the expanded format, label expanded, label repeated)"""
    r, c = cfg.r, cfg.c
    xs = [vec_exp(x[t * r: (t + 1) * r], r, c) for t in range(cfg.tiles)]
    return xs, vec_exp(y, r, c), vec_rep(y, r, c)


# ---------------------------------------------------------------- unpacked reference (float64)

def act(cfg, z):
    a1, a2, a3 = cfg.act
    return a1 * z + a2 * z * z + a3 * z ** 3


def act_deriv(cfg, z):
    a1, a2, a3 = cfg.act
    return a1 + 2.0 * a2 * z + 3.0 * a3 * z * z


def reference_grads(cfg, Ws, Wstars, X, Y):
    """Mean local-loss gradients in matrix form.  For every block h and sample:
    z = a W, a' = f(z), yhat = a' W*, g = yhat - y, dW* = a'^T g,
    da = g W*^T, dz = da * f'(z) (or 1 + 2 da, literal), dW = a^T dz; a' feeds
    block h+1 as a constant (local losses)."""
    b = X.shape[0]
    G = [np.zeros_like(W) for W in Ws]
    Gs = [np.zeros_like(W) for W in Wstars]
    for m in range(b):
        a = X[m]
        for h in range(cfg.H):
            z = a @ Ws[h]
            an = act(cfg, z)
            g = an @ Wstars[h] - Y[m]
            Gs[h] += np.outer(an, g)
            da = Wstars[h] @ g
            dz = 1.0 + 2.0 * da if cfg.literal_deriv else da * act_deriv(cfg, z)
            G[h] += np.outer(a, dz)
            a = an
    return [x / b for x in G], [x / b for x in Gs]


def reference_update(cfg, W, V, G, t):
    """Algorithm 2 on one matrix (V is None at t = 1); returns (W', V')."""
    g, e, m = cfg.gamma, cfg.eta, cfg.mu
    D = G + e * W if cfg.l2_decay else G + e * G
    if t == 1:
        return W - (g * D + g * m * D), D
    Vn = m * V + D
    return W - (g * D + g * m * D + g * m * m * V), Vn


def reference_step(cfg, Ws, Wstars, Vs, Vstars, X, Y, t):
    G, Gs = reference_grads(cfg, Ws, Wstars, X, Y)
    out = ([], [], [], [])
    for h in range(cfg.H):
        w, v = reference_update(cfg, Ws[h], None if t == 1 else Vs[h], G[h], t)
        ws, vs = reference_update(cfg, Wstars[h], None if t == 1 else Vstars[h], Gs[h], t)
        out[0].append(w)
        out[1].append(ws)
        out[2].append(v)
        out[3].append(vs)
    return out


# ---------------------------------------------------------------- the packed step, for any number system

def sum_rows(ops, s, cfg):
    k = cfg.r >> 1
    while k >= 1:
        s = ops.add(s, ops.rot(s, cfg.c * k))
        k >>= 1
    return s


def sum_cols(ops, u, cfg):
    k = cfg.c >> 1
    while k >= 1:
        u = ops.add(u, ops.rot(u, k))
        k >>= 1
    u = ops.mask(u)
    k = 1
    while k < cfg.c:
        u = ops.add(u, ops.rot(u, -k))
        k <<= 1
    return u


def activation(ops, cfg, z, need_deriv=True):
    """(f(z), f'(z)); f'(z) is None with the literal derivative or when
    need_deriv is False (a forward pass only)."""
    a1, a2, a3 = cfg.act
    z2 = ops.mul(z, z)
    if cfg.degree == 2:
        t2 = ops.affine(z2, a2, 0.0)
        a = ops.add(t2, ops.lincomb([(z, a1)], like=t2)) if a1 != 0.0 else t2
        d = None if (cfg.literal_deriv or not need_deriv) else ops.affine(z, 2.0 * a2, a1)
        return a, d
    z3 = ops.mul(z2, z)
    t3 = ops.affine(z3, a3, 0.0)
    terms = [(x, cf) for x, cf in ((z2, a2), (z, a1)) if cf != 0.0]
    a = ops.add(t3, ops.lincomb(terms, like=t3)) if terms else t3
    d = None
    if not cfg.literal_deriv and need_deriv:
        d2 = ops.affine(z2, 3.0 * a3, 0.0)
        d = ops.add(d2, ops.lincomb([(z, 2.0 * a2)], like=d2)) if a2 != 0.0 else d2
        d = ops.affine(d, 1.0, a1)
    return a, d


def reference_infer(cfg, Ws, Wstars, x):
    """Float64 forward pass of one sample: the output of every block's local
    classifier, yhat_h = f(a_(h-1) W_h) W*_h with a_0 = x."""
    outs, a = [], np.asarray(x, dtype=np.float64)
    for h in range(cfg.H):
        a = act(cfg, a @ Ws[h])
        outs.append(a @ Wstars[h])
    return outs


def packed_infer(ops, cfg, state, x_tiles, last):
    """Encrypted inference with early exit (Section 4.2.3: after training the
    local classifiers can serve as exits): the forward pass of blocks
    1..last on one sample, returning the local classifiers' outputs
    [yhat_1 .. yhat_last].  A RE-block's output is in the expanded format
    (class i in row i), a CE-block's in the repeated format (class j in
    column j), as in the training step."""
    layout = cfg.state_layout()
    pos = {key: i for i, key in enumerate(layout)}
    out, a_in = [], list(x_tiles)
    for h in range(1, last + 1):
        nt = cfg.n_tiles(h)
        W = [state[pos[("W", h, i)]] for i in range(nt)]
        Ws = state[pos[("Wstar", h, 0)]]
        if h % 2 == 1:
            p = None
            for i in range(nt):
                t = ops.mul(a_in[i], W[i])
                p = t if p is None else ops.add(p, t)
            a, _ = activation(ops, cfg, sum_rows(ops, p, cfg), need_deriv=False)
            out.append(sum_cols(ops, ops.mul(a, Ws), cfg))
        else:
            a, _ = activation(ops, cfg, sum_cols(ops, ops.mul(a_in[0], W[0]), cfg), need_deriv=False)
            out.append(sum_rows(ops, ops.mul(a, Ws), cfg))
        a_in = [a]
    return out


def packed_step(ops, cfg, state, samples, t, bootstrap=True):
    """One training step.  state: ciphertexts/vectors in cfg.state_layout()
    order (V entries ignored at t = 1); samples: [(x_tiles, y_exp, y_rep)].
    Returns the new state (bootstrapped unless bootstrap=False)."""
    layout = cfg.state_layout()
    pos = {key: i for i, key in enumerate(layout)}
    H = cfg.H
    b = len(samples)
    grads = {h: [None] * cfg.n_tiles(h) for h in range(1, H + 1)}
    gstar = {h: None for h in range(1, H + 1)}

    def acc(old, new):
        return new if old is None else ops.add(old, new)

    for (xt, ye, yr) in samples:
        a_in = list(xt)
        for h in range(1, H + 1):
            nt = cfg.n_tiles(h)
            W = [state[pos[("W", h, i)]] for i in range(nt)]
            Ws = state[pos[("Wstar", h, 0)]]
            if h % 2 == 1:                     # RE-block
                p = None
                for i in range(nt):
                    p = acc(p, ops.mul(a_in[i], W[i]))
                z = sum_rows(ops, p, cfg)
                a, d = activation(ops, cfg, z)
                yhat = sum_cols(ops, ops.mul(a, Ws), cfg)
                g = ops.sub(yhat, ops.lincomb([(ye, 1.0)], like=yhat))
                gstar[h] = acc(gstar[h], ops.mul(a, g))
                da = sum_rows(ops, ops.mul(g, Ws), cfg)
            else:                              # CE-block
                z = sum_cols(ops, ops.mul(a_in[0], W[0]), cfg)
                a, d = activation(ops, cfg, z)
                yhat = sum_rows(ops, ops.mul(a, Ws), cfg)
                g = ops.sub(yhat, ops.lincomb([(yr, 1.0)], like=yhat))
                gstar[h] = acc(gstar[h], ops.mul(a, g))
                da = sum_cols(ops, ops.mul(g, Ws), cfg)
            dz = ops.affine(da, 2.0, 1.0) if d is None else ops.mul(da, d)
            for i in range(nt):
                grads[h][i] = acc(grads[h][i], ops.mul(a_in[i], dz))
            a_in = [a]

    gm, e, m = cfg.gamma, cfg.eta, cfg.mu
    T = 2.0 ** cfg.log2_scale
    new = [None] * len(layout)
    for h in range(1, H + 1):
        pairs = [(("W", h, i), ("V", h, i), grads[h][i]) for i in range(cfg.n_tiles(h))]
        pairs.append((("Wstar", h, 0), ("Vstar", h, 0), gstar[h]))
        for kw, kv, G in pairs:
            W, V = state[pos[kw]], state[pos[kv]]
            if cfg.l2_decay:
                wt = [(W, 1.0 - gm * (1.0 + m) * e), (G, -gm * (1.0 + m) / b)]
                vt = [(G, 1.0 / b), (W, e)]
            else:
                wt = [(W, 1.0), (G, -gm * (1.0 + m) * (1.0 + e) / b)]
                vt = [(G, (1.0 + e) / b)]
            if t > 1:
                wt.append((V, -gm * m * m))
                vt.append((V, m))
            new[pos[kw]] = ops.lincomb(wt, scale=T)
            new[pos[kv]] = ops.lincomb(vt, scale=T)
    if bootstrap:
        new = ops.bootstrap(new)
    return new


class PlainOps:
    """float64 slot vectors; the same calls as the encrypted step."""

    def __init__(self, cfg):
        self.mask_v = first_slot_mask(cfg.r, cfg.c)

    def mul(self, a, b):
        return a * b

    def add(self, a, b):
        return a + b

    def sub(self, a, b):
        return a - b

    def rot(self, a, k):
        return np.roll(a, -k)

    def mask(self, a):
        return a * self.mask_v

    def affine(self, a, alpha, beta):
        return alpha * a + beta

    def lincomb(self, terms, like=None, scale=None):
        return sum(c * x for x, c in terms)

    def bootstrap(self, cts):
        return cts


class LevelOps:
    """Levels only: runs the step to count its multiplicative depth."""

    def mul(self, a, b):
        return min(a, b) - 1

    def add(self, a, b):
        return min(a, b)

    sub = add

    def rot(self, a, k):
        return a

    def mask(self, a):
        return a - 1

    def affine(self, a, alpha, beta):
        return a

    def lincomb(self, terms, like=None, scale=None):
        lv = min(x for x, _ in terms)
        if like is not None:
            lv = min(lv, like + 1)
        return lv - 1

    def bootstrap(self, cts):
        return cts


def depth(cfg):
    """Levels one step consumes below the level of the weights."""
    w = 1000
    state = [w] * len(cfg.state_layout())
    x = ([10 ** 6] * cfg.tiles, 10 ** 6, 10 ** 6)
    out = packed_step(LevelOps(), cfg, state, [x], t=2, bootstrap=False)
    return w - min(out)


def rotations(cfg):
    """Rotation indices the step uses."""
    ks = set()
    k = cfg.r >> 1
    while k >= 1:
        ks.add(cfg.c * k)
        k >>= 1
    k = cfg.c >> 1
    while k >= 1:
        ks.update((k, -k))
        k >>= 1
    return sorted(ks)


# ---------------------------------------------------------------- encrypted operations on the oracle

class Ct:
    __slots__ = ("d", "lv", "s")

    def __init__(self, d, lv, s):
        self.d, self.lv, self.s = d, lv, s


class EncOps:
    """Ciphertexts with exact scales on the oracle's primitives.

    ``scalars`` records every integer constant in evaluation order (the
    library exports its own list for comparison); ``masks`` maps a level to
    the mask plaintext encoded at scale q_level (the library may import these
    instead of encoding its own)."""

    def __init__(self, orc, cfg, rlk, gal_keys, boot=None):
        self.o = orc
        self.cfg = cfg
        self.rlk = rlk
        self.keys = gal_keys
        self.boot = boot
        self.q = [int(x) for x in orc.Q]
        self.masks = {}
        self.scalars = []

    # -- helpers
    def _drop(self, x, lv):
        if x.lv == lv:
            return x.d
        assert x.lv > lv
        return self.o.drop(x.lv, lv, x.d)

    def _res(self, k, lv):
        return np.array([k % q for q in self.q[: lv + 1]], dtype=np.uint64)

    def _int(self, v):
        if not abs(v) < 2.0 ** 62:
            raise ValueError("constant out of range (|k| >= 2^62): the scales do not fit the primes")
        k = int(np.rint(v))
        self.scalars.append(k)
        return k

    def mask_plain(self, lv):
        if lv not in self.masks:
            self.masks[lv] = encode(first_slot_mask(self.cfg.r, self.cfg.c), self.o.N, float(self.q[lv]),
                                    self.q[: lv + 1])
        return self.masks[lv]

    # -- operations
    def mul(self, a, b):
        lv = min(a.lv, b.lv)
        prod = self.o.mult_relin(lv, self.rlk, self._drop(a, lv), self._drop(b, lv))
        return Ct(self.o.rescale(lv, prod), lv - 1, a.s * b.s / float(self.q[lv]))

    def _same_scale(self, a, b):
        if a.s != b.s:
            raise ValueError("scale mismatch %r vs %r" % (a.s, b.s))

    def add(self, a, b):
        self._same_scale(a, b)
        lv = min(a.lv, b.lv)
        return Ct(self.o.add(lv, self._drop(a, lv), self._drop(b, lv)), lv, a.s)

    def sub(self, a, b):
        self._same_scale(a, b)
        lv = min(a.lv, b.lv)
        return Ct(self.o.sub(lv, self._drop(a, lv), self._drop(b, lv)), lv, a.s)

    def rot(self, a, k):
        g = self.o.galois_rot(k)
        return Ct(self.o.rotate(a.lv, self.keys[g], g, a.d), a.lv, a.s)

    def mask(self, a):
        lv = a.lv
        return Ct(self.o.rescale(lv, self.o.mul_plain(lv, a.d, self.mask_plain(lv))), lv - 1, a.s)

    def affine(self, a, alpha, beta):
        s = a.s / alpha
        if beta == 0.0:
            return Ct(a.d, a.lv, s)
        k = self._int(beta * s)
        return Ct(self.o.add_scalar(a.lv, a.d, self._res(k, a.lv)), a.lv, s)

    def lincomb(self, terms, like=None, scale=None):
        """sum c_i x_i, rescaled once, at scale `scale` or at like's level and scale."""
        lv = min(x.lv for x, _ in terms)
        if like is not None:
            lv = min(lv, like.lv + 1)
            T = like.s
        else:
            T = scale
        ql = float(self.q[lv])
        acc = None
        for x, cf in terms:
            k = self._int(cf * ql * T / x.s)
            y = self.o.mul_scalar(lv, self._drop(x, lv), self._res(k, lv))
            acc = y if acc is None else self.o.add(lv, acc, y)
        return Ct(self.o.rescale(lv, acc), lv - 1, T)

    def bootstrap(self, cts):
        out = []
        for x in cts:
            d, s = self.boot.bootstrap(self._drop(x, 0), x.s)
            out.append(Ct(d, self.boot.plan.level_out, s))
        return out
