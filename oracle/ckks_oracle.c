/*
 * ckks_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU reference for the RNS-CKKS
 * ciphertext arithmetic that ReBoot runs all of its encrypted training on
 * (paper Section 3: the parameter set {N, q, Delta}, the slot-wise add / sub /
 * mult of eqs. (add)-(mult), plaintext-ciphertext ops, and Rot(a, k)).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code, header, table or helper
 * with the GPU library; both sides only receive the same seeded random inputs.
 *
 * Conventions (each is a definition, written out as plainly as possible):
 *  - every residue is canonical, in [0, q);
 *  - every polynomial handed in or out is in the COEFFICIENT domain, a limb
 *    being N consecutive uint64 values;
 *  - a ciphertext at level l is [2][l+1][N];
 *  - the prime table is Q = (q_0 .. q_{nQ-1}) followed by P = (p_0 .. p_{nP-1});
 *  - the extended basis at level l is (q_0 .. q_l, p_0 .. p_{nP-1}).
 *
 * Modular products use the 128-bit product and the C '%' operator: the
 * definition of a*b mod q, nothing cleverer.
 *
 * Cited methods (the paper names them but does not spell them out):
 *  - negacyclic NTT: evaluation of a(X) at the odd powers of a primitive
 *    2N-th root psi (Longa-Naehrig 2016 ordering: output index brv(k) holds
 *    a(psi^(2k+1)));
 *  - hybrid key switching with digits of alpha limbs, ModUp by fast base
 *    conversion, ModDown by P (Han-Ki 2020; fast base conversion of
 *    Bajard-Eynard-Hasan-Zucca 2016, without the correction term);
 *  - rescale by the last prime with a centred lift (Cheon-Kim-Kim-Song 2017,
 *    RNS form of Cheon-Han-Kim-Kim-Song 2018);
 *  - Galois automorphisms X -> X^g, g = 5^k for a left rotation by k and
 *    g = 2N-1 for conjugation;
 *  - hoisted rotations: one ModUp shared by several automorphisms
 *    (Halevi-Shoup 2018).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

#define ORC_MAX_PRIMES 80

/* ------------------------------------------------------------------ */
/* modular arithmetic: the definitions                                */
/* ------------------------------------------------------------------ */

static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addm(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 subm(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - (b % q)) % q); }
static u64 negm(u64 a, u64 q) { return a == 0 ? 0 : q - a; }

static u64 powm(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulm(r, b, q);
        b = mulm(b, b, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime: Fermat's little theorem */
static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); }

/* a signed integer reduced into [0, q) */
static u64 from_signed(i64 v, u64 q)
{
    if (v >= 0) return (u64)v % q;
    u64 m = (u64)(-(v + 1)) % q;     /* careful with INT64_MIN */
    return (q - 1 - m) % q;
}

u64 orc_mulmod(u64 a, u64 b, u64 q) { return mulm(a, b, q); }
u64 orc_powmod(u64 b, u64 e, u64 q) { return powm(b, e, q); }
u64 orc_invmod(u64 a, u64 q) { return invm(a, q); }

/* ------------------------------------------------------------------ */
/* primes                                                             */
/* ------------------------------------------------------------------ */

/* Deterministic Miller-Rabin: the first twelve prime bases decide every
 * n < 3.3e24 (Sorenson-Webster 2015), which covers all 64-bit n. */
int orc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powm(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int r = 1; r < s; r++) {
            x = mulm(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* Trial division, used only to pin orc_is_prime on small inputs. */
int orc_is_prime_trial(u64 n)
{
    if (n < 2) return 0;
    for (u64 d = 2; d * d <= n; d++)
        if (n % d == 0) return 0;
    return 1;
}

/* NTT-friendly primes.  For each requested bit size b, in request order,
 * scan q = 2^b - j*2N + 1 for j = 1, 2, ... and take the first prime that is
 * not already in the list.  Every such q is = 1 (mod 2N), so Z_q holds a
 * primitive 2N-th root of unity.  Returns 0, or -1 if a bit size is invalid. */
int orc_gen_primes(int logN, int count, const int *bits, u64 *out)
{
    u64 twoN = (u64)2 << logN;
    for (int i = 0; i < count; i++) {
        int b = bits[i];
        if (b < logN + 2 || b > 62) return -1;
        u64 top = (u64)1 << b;
        u64 found = 0;
        for (u64 j = 1; j * twoN < top; j++) {
            u64 q = top - j * twoN + 1;
            if (!orc_is_prime(q)) continue;
            int dup = 0;
            for (int k = 0; k < i; k++)
                if (out[k] == q) dup = 1;
            if (dup) continue;
            found = q;
            break;
        }
        if (!found) return -1;
        out[i] = found;
    }
    return 0;
}

/* The smallest primitive 2N-th root of unity modulo q.  psi0 = x^((q-1)/2N)
 * is primitive exactly when psi0^N = -1; all primitive 2N-th roots are the
 * odd powers of psi0, and the smallest of them is returned. */
u64 orc_min_psi(u64 q, int logN)
{
    u64 N = (u64)1 << logN;
    u64 psi0 = 0;
    for (u64 x = 2; x < q; x++) {
        u64 c = powm(x, (q - 1) / (2 * N), q);
        if (powm(c, N, q) == q - 1) { psi0 = c; break; }
    }
    u64 best = psi0, psi2 = mulm(psi0, psi0, q), cur = psi0;
    for (u64 k = 0; k < N; k++) {
        if (cur < best) best = cur;
        cur = mulm(cur, psi2, q);
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT                                                     */
/* ------------------------------------------------------------------ */

static u64 bitrev(u64 x, int bits)
{
    u64 r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* The definition: out[brv(k)] = sum_j a_j psi^((2k+1) j) mod q.  O(N^2). */
void orc_ntt_direct(int logN, u64 q, u64 psi, const u64 *a, u64 *out)
{
    u64 N = (u64)1 << logN;
    for (u64 k = 0; k < N; k++) {
        u64 w = powm(psi, 2 * k + 1, q), wp = 1, acc = 0;
        for (u64 j = 0; j < N; j++) {
            acc = addm(acc, mulm(a[j], wp, q), q);
            wp = mulm(wp, w, q);
        }
        out[bitrev(k, logN)] = acc;
    }
}

/* Evaluate a (length n, coefficients with stride 'st' in src) at the points
 * w^(2k+1), k = 0..n-1, where w is a primitive 2n-th root, writing the n
 * values in natural k order to dst.  Even/odd split:
 *   a(x) = e(x^2) + x o(x^2),  (w^(2k+1))^2 = (w^2)^(2k+1),
 *   value_k       = e_k + w^(2k+1) o_k
 *   value_{k+n/2} = e_k - w^(2k+1) o_k     (w^n = -1).            */
static void eval_odd_powers(const u64 *src, size_t st, size_t n, u64 q, u64 w, u64 *dst, u64 *tmp)
{
    if (n == 1) { dst[0] = src[0] % q; return; }
    size_t h = n / 2;
    u64 w2 = mulm(w, w, q);
    u64 *E = tmp, *O = tmp + h;
    eval_odd_powers(src, 2 * st, h, q, w2, E, dst);
    eval_odd_powers(src + st, 2 * st, h, q, w2, O, dst);
    u64 wk = w;                         /* w^(2k+1) */
    for (size_t k = 0; k < h; k++) {
        u64 t = mulm(wk, O[k], q);
        dst[k] = addm(E[k], t, q);
        dst[k + h] = subm(E[k], t, q);
        wk = mulm(wk, w2, q);
    }
}

/* Inverse of eval_odd_powers: from the n values at w^(2k+1) (natural k order)
 * recover the coefficients, written with stride 1.  winv = w^-1, inv2 = 2^-1.
 *   e_k = (v_k + v_{k+n/2}) / 2,  o_k = (v_k - v_{k+n/2}) / (2 w^(2k+1)). */
static void interp_odd_powers(const u64 *v, size_t n, u64 q, u64 w, u64 winv, u64 inv2, u64 *coef, u64 *tmp)
{
    if (n == 1) { coef[0] = v[0]; return; }
    size_t h = n / 2;
    u64 w2 = mulm(w, w, q), winv2 = mulm(winv, winv, q);
    u64 *E = tmp, *O = tmp + h;
    u64 wk_inv = winv;                  /* w^-(2k+1) */
    for (size_t k = 0; k < h; k++) {
        E[k] = mulm(addm(v[k], v[k + h], q), inv2, q);
        O[k] = mulm(mulm(subm(v[k], v[k + h], q), inv2, q), wk_inv, q);
        wk_inv = mulm(wk_inv, winv2, q);
    }
    u64 *ce = (u64 *)malloc(h * sizeof(u64)), *co = (u64 *)malloc(h * sizeof(u64));
    interp_odd_powers(E, h, q, w2, winv2, inv2, ce, coef);
    interp_odd_powers(O, h, q, w2, winv2, inv2, co, coef);
    for (size_t i = 0; i < h; i++) { coef[2 * i] = ce[i]; coef[2 * i + 1] = co[i]; }
    free(ce);
    free(co);
}

/* Forward NTT with the same output convention as orc_ntt_direct. */
void orc_ntt(int logN, u64 q, u64 psi, const u64 *a, u64 *out)
{
    size_t N = (size_t)1 << logN;
    u64 *vals = (u64 *)malloc(N * sizeof(u64)), *tmp = (u64 *)malloc(N * sizeof(u64));
    eval_odd_powers(a, 1, N, q, psi, vals, tmp);
    for (size_t k = 0; k < N; k++) out[bitrev(k, logN)] = vals[k];
    free(vals);
    free(tmp);
}

/* Inverse NTT: input in the orc_ntt order, output coefficients. */
void orc_intt(int logN, u64 q, u64 psi, const u64 *in, u64 *out)
{
    size_t N = (size_t)1 << logN;
    u64 *vals = (u64 *)malloc(N * sizeof(u64)), *tmp = (u64 *)malloc(N * sizeof(u64));
    for (size_t k = 0; k < N; k++) vals[k] = in[bitrev(k, logN)];
    interp_odd_powers(vals, N, q, psi, invm(psi, q), invm(2, q), out, tmp);
    free(vals);
    free(tmp);
}

/* Schoolbook product in Z_q[X]/(X^N + 1): X^N = -1 wraps with a sign. */
void orc_negacyclic_schoolbook(int logN, u64 q, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = (size_t)1 << logN;
    for (size_t k = 0; k < N; k++) out[k] = 0;
    for (size_t i = 0; i < N; i++)
        for (size_t j = 0; j < N; j++) {
            u64 p = mulm(a[i], b[j], q);
            size_t k = i + j;
            if (k < N) out[k] = addm(out[k], p, q);
            else out[k - N] = subm(out[k - N], p, q);
        }
}

/* ------------------------------------------------------------------ */
/* context: ring degree, prime table, digit size                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int logN;
    size_t N;
    int nQ, nP, alpha;
    u64 mod[ORC_MAX_PRIMES];
    u64 psi[ORC_MAX_PRIMES];
} orc_ctx;

orc_ctx *orc_ctx_new(int logN, int nQ, const int *qbits, int nP, const int *pbits, int alpha)
{
    if (logN < 2 || logN > 17 || nQ < 1 || nP < 0 || nQ + nP > ORC_MAX_PRIMES || alpha < 1) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    int bits[ORC_MAX_PRIMES];
    for (int i = 0; i < nQ; i++) bits[i] = qbits[i];
    for (int i = 0; i < nP; i++) bits[nQ + i] = pbits[i];
    if (orc_gen_primes(logN, nQ + nP, bits, c->mod) != 0) { free(c); return NULL; }
    c->logN = logN;
    c->N = (size_t)1 << logN;
    c->nQ = nQ;
    c->nP = nP;
    c->alpha = alpha;
    for (int i = 0; i < nQ + nP; i++) c->psi[i] = orc_min_psi(c->mod[i], logN);
    return c;
}

void orc_ctx_free(orc_ctx *c) { free(c); }

void orc_ctx_moduli(const orc_ctx *c, u64 *out)
{
    for (int i = 0; i < c->nQ + c->nP; i++) out[i] = c->mod[i];
}

void orc_ctx_psi(const orc_ctx *c, u64 *out)
{
    for (int i = 0; i < c->nQ + c->nP; i++) out[i] = c->psi[i];
}

/* number of digits at level l: ceil((l+1)/alpha) */
int orc_num_digits(const orc_ctx *c, int level) { return (level + 1 + c->alpha - 1) / c->alpha; }

/* prime-table index of position i of the extended basis at level l */
static int ext_index(const orc_ctx *c, int level, int i) { return i <= level ? i : c->nQ + (i - level - 1); }

/* ring product of one limb (prime-table index t), through the NTT */
static void limb_mul(const orc_ctx *c, int t, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = c->N;
    u64 *A = (u64 *)malloc(N * sizeof(u64)), *B = (u64 *)malloc(N * sizeof(u64));
    orc_ntt(c->logN, c->mod[t], c->psi[t], a, A);
    orc_ntt(c->logN, c->mod[t], c->psi[t], b, B);
    for (size_t i = 0; i < N; i++) A[i] = mulm(A[i], B[i], c->mod[t]);
    orc_intt(c->logN, c->mod[t], c->psi[t], A, out);
    free(A);
    free(B);
}

void orc_limb_mul(const orc_ctx *c, int t, const u64 *a, const u64 *b, u64 *out) { limb_mul(c, t, a, b, out); }

void orc_limb_ntt(const orc_ctx *c, int t, const u64 *a, u64 *out) { orc_ntt(c->logN, c->mod[t], c->psi[t], a, out); }
void orc_limb_intt(const orc_ctx *c, int t, const u64 *a, u64 *out) { orc_intt(c->logN, c->mod[t], c->psi[t], a, out); }

/* ------------------------------------------------------------------ */
/* fast base conversion                                               */
/* ------------------------------------------------------------------ */

/* Fast base conversion of Bajard et al. without the correction term.
 * For x given by residues x_i modulo the primes B = {b_0..b_{m-1}} (table
 * indices in_idx), with Bh_i = prod_{k != i} b_k:
 *    y_i   = x_i * Bh_i^{-1} mod b_i
 *    out_t = sum_i y_i * (Bh_i mod t) mod t     for each target prime t.
 * The result equals x + u*B modulo t for some integer 0 <= u < m. */
void orc_bconv(const orc_ctx *c, int n_in, const int *in_idx, const u64 *in, int n_out, const int *out_idx, u64 *out)
{
    size_t N = c->N;
    u64 *bhinv = (u64 *)malloc(n_in * sizeof(u64));
    u64 *bh_mod_t = (u64 *)malloc((size_t)n_in * n_out * sizeof(u64));
    for (int i = 0; i < n_in; i++) {
        u64 bi = c->mod[in_idx[i]], prod = 1;
        for (int k = 0; k < n_in; k++)
            if (k != i) prod = mulm(prod, c->mod[in_idx[k]] % bi, bi);
        bhinv[i] = invm(prod, bi);
        for (int o = 0; o < n_out; o++) {
            u64 t = c->mod[out_idx[o]], pt = 1;
            for (int k = 0; k < n_in; k++)
                if (k != i) pt = mulm(pt, c->mod[in_idx[k]] % t, t);
            bh_mod_t[(size_t)i * n_out + o] = pt;
        }
    }
    for (size_t k = 0; k < N; k++) {
        u64 y[ORC_MAX_PRIMES];
        for (int i = 0; i < n_in; i++) y[i] = mulm(in[(size_t)i * N + k], bhinv[i], c->mod[in_idx[i]]);
        for (int o = 0; o < n_out; o++) {
            u64 t = c->mod[out_idx[o]], acc = 0;
            for (int i = 0; i < n_in; i++) acc = addm(acc, mulm(y[i] % t, bh_mod_t[(size_t)i * n_out + o], t), t);
            out[(size_t)o * N + k] = acc;
        }
    }
    free(bhinv);
    free(bh_mod_t);
}

/* ------------------------------------------------------------------ */
/* key generation, encryption, decryption (randomness is an input)    */
/* ------------------------------------------------------------------ */

/* Switching key from s_from to s (hybrid key switching, Han-Ki 2020).
 *   s      : [N] small signed coefficients of the secret
 *   s_from : [nQ+nP][N] residues of the source secret s' on every prime
 *   a      : [beta][nQ+nP][N] uniform residues, beta = ceil(nQ/alpha)
 *   e      : [beta][N] small signed error coefficients
 *   out    : [beta][2][nQ+nP][N], digit j holds (b_j, a_j) with
 *            b_j = -a_j s + e_j + [P]_{q_i} s'  (mod q_i, i in digit j)
 *            b_j = -a_j s + e_j                 (every other prime). */
void orc_keygen_switch(const orc_ctx *c, const i64 *s, const u64 *s_from, const u64 *a, const i64 *e, u64 *out)
{
    size_t N = c->N;
    int nT = c->nQ + c->nP, beta = orc_num_digits(c, c->nQ - 1);
    u64 *sl = (u64 *)malloc(N * sizeof(u64)), *as = (u64 *)malloc(N * sizeof(u64));
    for (int j = 0; j < beta; j++) {
        for (int t = 0; t < nT; t++) {
            u64 q = c->mod[t];
            const u64 *aj = a + ((size_t)j * nT + t) * N;
            u64 *bo = out + (((size_t)j * 2 + 0) * nT + t) * N;
            u64 *ao = out + (((size_t)j * 2 + 1) * nT + t) * N;
            for (size_t k = 0; k < N; k++) sl[k] = from_signed(s[k], q);
            limb_mul(c, t, aj, sl, as);
            int in_digit = (t < c->nQ) && (t / c->alpha == j);
            u64 Pmod = 1;
            for (int p = 0; p < c->nP; p++) Pmod = mulm(Pmod, c->mod[c->nQ + p] % q, q);
            for (size_t k = 0; k < N; k++) {
                u64 b = addm(negm(as[k], q), from_signed(e[(size_t)j * N + k], q), q);
                if (in_digit) b = addm(b, mulm(Pmod, s_from[(size_t)t * N + k], q), q);
                bo[k] = b;
                ao[k] = aj[k];
            }
        }
    }
    free(sl);
    free(as);
}

/* Public key over Q: pk = (-a s + e, a).  a: [nQ][N] uniform, e: [N]. out: [2][nQ][N]. */
void orc_keygen_public(const orc_ctx *c, const i64 *s, const u64 *a, const i64 *e, u64 *out)
{
    size_t N = c->N;
    u64 *sl = (u64 *)malloc(N * sizeof(u64)), *as = (u64 *)malloc(N * sizeof(u64));
    for (int t = 0; t < c->nQ; t++) {
        u64 q = c->mod[t];
        for (size_t k = 0; k < N; k++) sl[k] = from_signed(s[k], q);
        limb_mul(c, t, a + (size_t)t * N, sl, as);
        for (size_t k = 0; k < N; k++) {
            out[(size_t)t * N + k] = addm(negm(as[k], q), from_signed(e[k], q), q);
            out[((size_t)c->nQ + t) * N + k] = a[(size_t)t * N + k];
        }
    }
    free(sl);
    free(as);
}

/* Residues of s^2 (ring product) or sigma_g(s) on every prime, for key generation. */
void orc_secret_square(const orc_ctx *c, const i64 *s, u64 *out)
{
    size_t N = c->N;
    u64 *sl = (u64 *)malloc(N * sizeof(u64));
    for (int t = 0; t < c->nQ + c->nP; t++) {
        for (size_t k = 0; k < N; k++) sl[k] = from_signed(s[k], c->mod[t]);
        limb_mul(c, t, sl, sl, out + (size_t)t * N);
    }
    free(sl);
}

/* Public-key encryption of a plaintext at level l:
 *   ct = (v*pk0 + e0 + m, v*pk1 + e1)  modulo q_0..q_l.
 * m: [l+1][N] residues, v/e0/e1: [N] small signed coefficients. out: [2][l+1][N]. */
void orc_encrypt(const orc_ctx *c, int level, const u64 *pk, const u64 *m, const i64 *v, const i64 *e0, const i64 *e1, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1;
    u64 *vl = (u64 *)malloc(N * sizeof(u64)), *pr = (u64 *)malloc(N * sizeof(u64));
    for (int t = 0; t < L1; t++) {
        u64 q = c->mod[t];
        for (size_t k = 0; k < N; k++) vl[k] = from_signed(v[k], q);
        limb_mul(c, t, vl, pk + (size_t)t * N, pr);
        for (size_t k = 0; k < N; k++)
            out[(size_t)t * N + k] = addm(addm(pr[k], from_signed(e0[k], q), q), m[(size_t)t * N + k], q);
        limb_mul(c, t, vl, pk + ((size_t)c->nQ + t) * N, pr);
        for (size_t k = 0; k < N; k++) out[((size_t)L1 + t) * N + k] = addm(pr[k], from_signed(e1[k], q), q);
    }
    free(vl);
    free(pr);
}

/* Decryption: m' = c0 + c1 s modulo q_0..q_l.  out: [l+1][N]. */
void orc_decrypt(const orc_ctx *c, int level, const i64 *s, const u64 *ct, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1;
    u64 *sl = (u64 *)malloc(N * sizeof(u64)), *pr = (u64 *)malloc(N * sizeof(u64));
    for (int t = 0; t < L1; t++) {
        u64 q = c->mod[t];
        for (size_t k = 0; k < N; k++) sl[k] = from_signed(s[k], q);
        limb_mul(c, t, ct + ((size_t)L1 + t) * N, sl, pr);
        for (size_t k = 0; k < N; k++) out[(size_t)t * N + k] = addm(ct[(size_t)t * N + k], pr[k], q);
    }
    free(sl);
    free(pr);
}

/* ------------------------------------------------------------------ */
/* slot-wise ring operations (Section 3: add, sub, mult, pt ops)       */
/* ------------------------------------------------------------------ */

/* out = a + b, elementwise on npoly polynomials of l+1 limbs */
void orc_add(const orc_ctx *c, int level, int npoly, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < npoly; p++)
        for (int t = 0; t <= level; t++)
            for (size_t k = 0; k < N; k++) {
                size_t o = ((size_t)p * (level + 1) + t) * N + k;
                out[o] = addm(a[o], b[o], c->mod[t]);
            }
}

void orc_sub(const orc_ctx *c, int level, int npoly, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < npoly; p++)
        for (int t = 0; t <= level; t++)
            for (size_t k = 0; k < N; k++) {
                size_t o = ((size_t)p * (level + 1) + t) * N + k;
                out[o] = subm(a[o], b[o], c->mod[t]);
            }
}

void orc_neg(const orc_ctx *c, int level, int npoly, const u64 *a, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < npoly; p++)
        for (int t = 0; t <= level; t++)
            for (size_t k = 0; k < N; k++) {
                size_t o = ((size_t)p * (level + 1) + t) * N + k;
                out[o] = negm(a[o], c->mod[t]);
            }
}

/* ciphertext times plaintext: both polynomials of ct multiplied by pt ([l+1][N]) */
void orc_mul_plain(const orc_ctx *c, int level, const u64 *ct, const u64 *pt, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < 2; p++)
        for (int t = 0; t <= level; t++) {
            size_t o = ((size_t)p * (level + 1) + t) * N;
            limb_mul(c, t, ct + o, pt + (size_t)t * N, out + o);
        }
}

/* ct + pt: only the first polynomial changes */
void orc_add_plain(const orc_ctx *c, int level, const u64 *ct, const u64 *pt, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    for (size_t t = 0; t < L1; t++)
        for (size_t k = 0; k < N; k++) {
            out[t * N + k] = addm(ct[t * N + k], pt[t * N + k], c->mod[t]);
            out[(L1 + t) * N + k] = ct[(L1 + t) * N + k];
        }
}

/* every limb t of npoly polynomials multiplied by the integer scal[t] (< q_t) */
void orc_mul_scalar(const orc_ctx *c, int level, int npoly, const u64 *a, const u64 *scal, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < npoly; p++)
        for (int t = 0; t <= level; t++)
            for (size_t k = 0; k < N; k++) {
                size_t o = ((size_t)p * (level + 1) + t) * N + k;
                out[o] = mulm(a[o], scal[t], c->mod[t]);
            }
}

/* ct + constant: the constant (residues scal[t]) is the polynomial scal,
 * i.e. it adds to coefficient 0 of the first polynomial only. */
void orc_add_scalar(const orc_ctx *c, int level, const u64 *ct, const u64 *scal, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    memcpy(out, ct, 2 * L1 * N * sizeof(u64));
    for (size_t t = 0; t < L1; t++) out[t * N] = addm(out[t * N], scal[t], c->mod[t]);
}

/* Tensor product of two degree-1 ciphertexts:
 * d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1.  out: [3][l+1][N]. */
void orc_tensor(const orc_ctx *c, int level, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    u64 *t1 = (u64 *)malloc(N * sizeof(u64)), *t2 = (u64 *)malloc(N * sizeof(u64));
    for (size_t t = 0; t < L1; t++) {
        u64 q = c->mod[t];
        const u64 *a0 = a + t * N, *a1 = a + (L1 + t) * N, *b0 = b + t * N, *b1 = b + (L1 + t) * N;
        limb_mul(c, (int)t, a0, b0, out + t * N);
        limb_mul(c, (int)t, a0, b1, t1);
        limb_mul(c, (int)t, a1, b0, t2);
        for (size_t k = 0; k < N; k++) out[(L1 + t) * N + k] = addm(t1[k], t2[k], q);
        limb_mul(c, (int)t, a1, b1, out + (2 * L1 + t) * N);
    }
    free(t1);
    free(t2);
}

/* ------------------------------------------------------------------ */
/* hybrid key switching                                               */
/* ------------------------------------------------------------------ */

/* ModUp: split d ([l+1][N]) into digits of alpha consecutive limbs; digit j
 * is extended from its own primes to every other prime of the extended basis
 * by fast base conversion.  out: [beta_l][l+1+nP][N]. */
void orc_modup(const orc_ctx *c, int level, const u64 *d, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1, E = L1 + c->nP, beta = orc_num_digits(c, level);
    for (int j = 0; j < beta; j++) {
        int lo = j * c->alpha, hi = lo + c->alpha;
        if (hi > L1) hi = L1;
        int in_idx[ORC_MAX_PRIMES], out_idx[ORC_MAX_PRIMES], out_pos[ORC_MAX_PRIMES], n_in = 0, n_out = 0;
        for (int i = lo; i < hi; i++) in_idx[n_in++] = i;
        for (int e = 0; e < E; e++) {
            int t = ext_index(c, level, e);
            if (e >= lo && e < hi) continue;
            out_idx[n_out] = t;
            out_pos[n_out++] = e;
        }
        u64 *conv = (u64 *)malloc((size_t)n_out * N * sizeof(u64));
        orc_bconv(c, n_in, in_idx, d + (size_t)lo * N, n_out, out_idx, conv);
        u64 *dj = out + (size_t)j * E * N;
        for (int i = lo; i < hi; i++) memcpy(dj + (size_t)i * N, d + (size_t)i * N, N * sizeof(u64));
        for (int o = 0; o < n_out; o++) memcpy(dj + (size_t)out_pos[o] * N, conv + (size_t)o * N, N * sizeof(u64));
        free(conv);
    }
}

/* Inner product with a switching key at level l:
 *   (u0, u1) = sum_j ext_j * (b_j, a_j)   over the extended basis.
 * ext: [beta_l][l+1+nP][N]; key: [beta][2][nQ+nP][N]; out: [2][l+1+nP][N]. */
void orc_key_inner_product(const orc_ctx *c, int level, const u64 *ext, const u64 *key, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1, E = L1 + c->nP, nT = c->nQ + c->nP, beta = orc_num_digits(c, level);
    u64 *pr = (u64 *)malloc(N * sizeof(u64));
    memset(out, 0, 2 * (size_t)E * N * sizeof(u64));
    for (int j = 0; j < beta; j++)
        for (int e = 0; e < E; e++) {
            int t = ext_index(c, level, e);
            for (int h = 0; h < 2; h++) {
                limb_mul(c, t, ext + ((size_t)j * E + e) * N, key + (((size_t)j * 2 + h) * nT + t) * N, pr);
                u64 *o = out + ((size_t)h * E + e) * N;
                for (size_t k = 0; k < N; k++) o[k] = addm(o[k], pr[k], c->mod[t]);
            }
        }
    free(pr);
}

/* ModDown of one polynomial over the extended basis ([l+1+nP][N]):
 *   out_i = (u_i - BConv_{P -> q_i}(u_P)) * P^{-1}  mod q_i,  i = 0..l. */
void orc_moddown(const orc_ctx *c, int level, const u64 *u, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1;
    int in_idx[ORC_MAX_PRIMES] = {0}, out_idx[ORC_MAX_PRIMES] = {0};
    for (int p = 0; p < c->nP; p++) in_idx[p] = c->nQ + p;
    for (int i = 0; i < L1; i++) out_idx[i] = i;
    u64 *conv = (u64 *)malloc((size_t)L1 * N * sizeof(u64));
    orc_bconv(c, c->nP, in_idx, u + (size_t)L1 * N, L1, out_idx, conv);
    for (int i = 0; i < L1; i++) {
        u64 q = c->mod[i], P = 1;
        for (int p = 0; p < c->nP; p++) P = mulm(P, c->mod[c->nQ + p] % q, q);
        u64 Pinv = invm(P, q);
        for (size_t k = 0; k < N; k++)
            out[(size_t)i * N + k] = mulm(subm(u[(size_t)i * N + k], conv[(size_t)i * N + k], q), Pinv, q);
    }
    free(conv);
}

/* KS(d) = ModDown(<ModUp(d), key>).  out: [2][l+1][N]. */
void orc_keyswitch(const orc_ctx *c, int level, const u64 *key, const u64 *d, u64 *out)
{
    size_t N = c->N;
    int L1 = level + 1, E = L1 + c->nP, beta = orc_num_digits(c, level);
    u64 *ext = (u64 *)malloc((size_t)beta * E * N * sizeof(u64));
    u64 *u = (u64 *)malloc(2 * (size_t)E * N * sizeof(u64));
    orc_modup(c, level, d, ext);
    orc_key_inner_product(c, level, ext, key, u);
    orc_moddown(c, level, u, out);
    orc_moddown(c, level, u + (size_t)E * N, out + (size_t)L1 * N);
    free(ext);
    free(u);
}

/* ct x ct with relinearisation: (d0, d1) + KS_{s^2 -> s}(d2).  out: [2][l+1][N]. */
void orc_mult_relin(const orc_ctx *c, int level, const u64 *rlk, const u64 *a, const u64 *b, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    u64 *d = (u64 *)malloc(3 * L1 * N * sizeof(u64)), *ks = (u64 *)malloc(2 * L1 * N * sizeof(u64));
    orc_tensor(c, level, a, b, d);
    orc_keyswitch(c, level, rlk, d + 2 * L1 * N, ks);
    orc_add(c, level, 2, d, ks, out);
    free(d);
    free(ks);
}

/* ------------------------------------------------------------------ */
/* rescale                                                            */
/* ------------------------------------------------------------------ */

/* Divide by the last prime q_l with rounding: for every polynomial and every
 * i < l,  out_i = (c_i - lift(c_l)) * q_l^{-1} mod q_i,  where lift(c_l) is the
 * centred representative of c_l in (-q_l/2, q_l/2].  in: [2][l+1][N], out: [2][l][N]. */
void orc_rescale(const orc_ctx *c, int level, const u64 *in, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    u64 ql = c->mod[level];
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < level; i++) {
            u64 q = c->mod[i], qlinv = invm(ql % q, q);
            for (size_t k = 0; k < N; k++) {
                u64 x = in[((size_t)p * L1 + level) * N + k];
                u64 lifted;                       /* centred lift reduced mod q */
                if (x <= (ql - 1) / 2) lifted = x % q;
                else lifted = subm(x % q, ql % q, q);
                u64 ci = in[((size_t)p * L1 + i) * N + k];
                out[((size_t)p * level + i) * N + k] = mulm(subm(ci, lifted, q), qlinv, q);
            }
        }
}

/* ------------------------------------------------------------------ */
/* automorphisms and rotations                                        */
/* ------------------------------------------------------------------ */

/* sigma_g on nlimb limbs (table indices idx): coefficient i moves to i*g mod N
 * with sign (-1)^floor(i*g / N), because X^N = -1. */
void orc_automorph_limbs(const orc_ctx *c, int nlimb, const int *idx, u64 g, const u64 *in, u64 *out)
{
    size_t N = c->N;
    for (int l = 0; l < nlimb; l++) {
        u64 q = c->mod[idx[l]];
        for (size_t i = 0; i < N; i++) {
            u64 e = ((u64)i * g) % (2 * N);
            u64 v = in[(size_t)l * N + i];
            if (e < N) out[(size_t)l * N + e] = v;
            else out[(size_t)l * N + (e - N)] = negm(v, q);
        }
    }
}

/* sigma_g on npoly polynomials of the Q basis at level l */
void orc_automorph(const orc_ctx *c, int level, int npoly, u64 g, const u64 *in, u64 *out)
{
    int idx[ORC_MAX_PRIMES];
    for (int i = 0; i <= level; i++) idx[i] = i;
    for (int p = 0; p < npoly; p++)
        orc_automorph_limbs(c, level + 1, idx, g, in + (size_t)p * (level + 1) * c->N, out + (size_t)p * (level + 1) * c->N);
}

/* Galois element of a left rotation by k slots: 5^(k mod N/2) mod 2N. */
u64 orc_galois_rot(const orc_ctx *c, i64 k)
{
    i64 n = (i64)(c->N / 2);
    i64 r = ((k % n) + n) % n;
    return powm(5, (u64)r, 2 * c->N);
}

/* Rot(ct, k) via sigma_g and a key for sigma_g(s):
 *   out = (sigma_g(c0), 0) + KS(sigma_g(c1)). */
void orc_rotate(const orc_ctx *c, int level, const u64 *key, u64 g, const u64 *ct, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    u64 *rot = (u64 *)malloc(2 * L1 * N * sizeof(u64)), *ks = (u64 *)malloc(2 * L1 * N * sizeof(u64));
    orc_automorph(c, level, 2, g, ct, rot);
    orc_keyswitch(c, level, key, rot + L1 * N, ks);
    for (size_t t = 0; t < L1; t++)
        for (size_t k = 0; k < N; k++) {
            out[t * N + k] = addm(rot[t * N + k], ks[t * N + k], c->mod[t]);
            out[(L1 + t) * N + k] = ks[(L1 + t) * N + k];
        }
    free(rot);
    free(ks);
}

/* Hoisted rotations: ModUp(c1) once; for each Galois element g_r,
 * sigma_g is applied to every digit on the extended basis, the result goes
 * through the inner product with key_r and ModDown, and sigma_g(c0) is added.
 * keys: array of nrot key pointers; outs: [nrot][2][l+1][N]. */
void orc_rotate_hoisted(const orc_ctx *c, int level, int nrot, const u64 *const *keys, const u64 *gs, const u64 *ct, u64 *outs)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    int E = (int)L1 + c->nP, beta = orc_num_digits(c, level);
    int idx[ORC_MAX_PRIMES];
    for (int e = 0; e < E; e++) idx[e] = ext_index(c, level, e);
    u64 *ext = (u64 *)malloc((size_t)beta * E * N * sizeof(u64));
    u64 *extg = (u64 *)malloc((size_t)beta * E * N * sizeof(u64));
    u64 *u = (u64 *)malloc(2 * (size_t)E * N * sizeof(u64));
    u64 *c0g = (u64 *)malloc(L1 * N * sizeof(u64));
    u64 *ks = (u64 *)malloc(2 * L1 * N * sizeof(u64));
    orc_modup(c, level, ct + L1 * N, ext);
    for (int r = 0; r < nrot; r++) {
        for (int j = 0; j < beta; j++)
            orc_automorph_limbs(c, E, idx, gs[r], ext + (size_t)j * E * N, extg + (size_t)j * E * N);
        orc_key_inner_product(c, level, extg, keys[r], u);
        orc_moddown(c, level, u, ks);
        orc_moddown(c, level, u + (size_t)E * N, ks + L1 * N);
        orc_automorph(c, level, 1, gs[r], ct, c0g);
        u64 *o = outs + (size_t)r * 2 * L1 * N;
        for (size_t t = 0; t < L1; t++)
            for (size_t k = 0; k < N; k++) {
                o[t * N + k] = addm(c0g[t * N + k], ks[t * N + k], c->mod[t]);
                o[(L1 + t) * N + k] = ks[(L1 + t) * N + k];
            }
    }
    free(ext);
    free(extg);
    free(u);
    free(c0g);
    free(ks);
}

/* Residues of sigma_g(s) on every prime (source secret of a rotation key). */
void orc_secret_automorph(const orc_ctx *c, const i64 *s, u64 g, u64 *out)
{
    size_t N = c->N;
    int nT = c->nQ + c->nP;
    u64 *sl = (u64 *)malloc(N * sizeof(u64));
    for (int t = 0; t < nT; t++) {
        for (size_t k = 0; k < N; k++) sl[k] = from_signed(s[k], c->mod[t]);
        orc_automorph_limbs(c, 1, &t, g, sl, out + (size_t)t * N);
    }
    free(sl);
}

/* ------------------------------------------------------------------ */
/* bootstrapping primitives                                           */
/* ------------------------------------------------------------------ */

/* ModRaise: a ciphertext modulo q_0 ([2][1][N]) is read as centred integers
 * in (-q_0/2, q_0/2] and reduced modulo every prime of level l:
 * out [2][l+1][N].  The decryption then becomes m + q_0 I(X) for a small
 * integer polynomial I (Cheon-Han-Kim-Kim-Song 2018). */
void orc_modraise(const orc_ctx *c, int level, const u64 *in, u64 *out)
{
    size_t N = c->N, L1 = (size_t)level + 1;
    u64 q0 = c->mod[0];
    for (int p = 0; p < 2; p++)
        for (size_t k = 0; k < N; k++) {
            u64 x = in[(size_t)p * N + k];
            for (size_t i = 0; i < L1; i++) {
                u64 q = c->mod[i], v;
                if (x <= (q0 - 1) / 2) v = x % q;
                else v = subm(x % q, q0 % q, q);
                out[((size_t)p * L1 + i) * N + k] = v;
            }
        }
}

/* Multiplication by the monomial X^e (0 <= e < 2N) of npoly polynomials:
 * coefficient k moves to k+e, negated each time it wraps past X^N. */
void orc_monomial(const orc_ctx *c, int level, int npoly, u64 e, const u64 *in, u64 *out)
{
    size_t N = c->N;
    for (int p = 0; p < npoly; p++)
        for (int t = 0; t <= level; t++) {
            u64 q = c->mod[t];
            const u64 *a = in + ((size_t)p * (level + 1) + t) * N;
            u64 *o = out + ((size_t)p * (level + 1) + t) * N;
            for (size_t k = 0; k < N; k++) {
                u64 d = (k + e) % (2 * N);
                if (d < N) o[d] = a[k];
                else o[d - N] = negm(a[k], q);
            }
        }
}

/* ------------------------------------------------------------------ */
/* seeded sampling                                                    */
/* ------------------------------------------------------------------ */

/* Every random quantity of key generation and encryption (Section 3: the
 * secret, the uniform public polynomials, the added noise) can be drawn
 * from one 64-bit seed.  The paper does not say how; the reading used here:
 *
 *  - keystream: the ChaCha20 block function of RFC 8439 (20 rounds), key =
 *    (seed low 32 bits, seed high 32 bits, 0, 0, 0, 0, 0, 0), 32-bit block
 *    counter, nonce = (purpose, id, sub) naming the quantity;
 *  - per coefficient j of an N-coefficient polynomial: the block with
 *    counter j (then j + N, j + 2N, ... if that block yields no value);
 *  - uniform mod q: the block's eight little-endian 64-bit words, each masked
 *    to bitlen(q) bits; the first below q;
 *  - uniform ternary: the block's 256 2-bit fields (word 0 bits 1:0 first);
 *    the first that is not 3, with 0, 1, 2 meaning 0, +1, -1;
 *  - discrete Gaussian, sigma = 3.2, support |x| <= 19: word w = the block's
 *    first 64-bit word; u = w >> 1 is compared with the cumulative table
 *    T[m] = floor(2^63 P(|x| <= m)) (T[19] = 2^63), magnitude = the least m
 *    with u < T[m], negative when m > 0 and bit 0 of w is set;
 *  - secret with exactly h non-zero coefficients: 32-bit words of the
 *    stream (counters 0, 1, ... in order) taken two at a time, position =
 *    first & (N - 1), sign = bit 0 of the second (set = -1); a position
 *    already taken is skipped, until h are set. */

#define ORC_P_SECRET 1u
#define ORC_P_PK_A 2u
#define ORC_P_PK_E 3u
#define ORC_P_KEY_A 4u
#define ORC_P_KEY_E 5u
#define ORC_P_ENC_V 6u
#define ORC_P_ENC_E0 7u
#define ORC_P_ENC_E1 8u

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

static void quarter(uint32_t *x, int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

void orc_chacha_quarter(uint32_t *x4)
{
    quarter(x4, 0, 1, 2, 3);
}

/* RFC 8439 Section 2.3: the state is the four constants, the eight key
 * words, the counter and the three nonce words; ten double rounds (column
 * rounds then diagonal rounds); the output adds the input state. */
void orc_chacha_block(const uint32_t *key8, uint32_t counter, const uint32_t *nonce3, uint32_t *out16)
{
    uint32_t in[16], x[16];
    in[0] = 0x61707865u; in[1] = 0x3320646eu; in[2] = 0x79622d32u; in[3] = 0x6b206574u;
    for (int i = 0; i < 8; i++) in[4 + i] = key8[i];
    in[12] = counter;
    for (int i = 0; i < 3; i++) in[13 + i] = nonce3[i];
    for (int i = 0; i < 16; i++) x[i] = in[i];
    for (int r = 0; r < 10; r++) {
        quarter(x, 0, 4, 8, 12); quarter(x, 1, 5, 9, 13); quarter(x, 2, 6, 10, 14); quarter(x, 3, 7, 11, 15);
        quarter(x, 0, 5, 10, 15); quarter(x, 1, 6, 11, 12); quarter(x, 2, 7, 8, 13); quarter(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; i++) out16[i] = x[i] + in[i];
}

static void seed_block(u64 seed, uint32_t purpose, uint32_t id, uint32_t sub, uint32_t counter, uint32_t *out16)
{
    uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    uint32_t nonce[3] = {purpose, id, sub};
    orc_chacha_block(key, counter, nonce, out16);
}

static int bitlen(u64 q)
{
    int b = 0;
    while (b < 64 && (q >> b)) b++;
    return b;
}

void orc_sample_uniform(u64 seed, uint32_t purpose, uint32_t id, uint32_t sub, u64 q, int logN, u64 *out)
{
    size_t N = (size_t)1 << logN;
    int b = bitlen(q);
    u64 mask = b >= 64 ? ~(u64)0 : (((u64)1 << b) - 1);
    uint32_t blk[16];
    for (size_t j = 0; j < N; j++) {
        for (uint32_t ctr = (uint32_t)j;; ctr += (uint32_t)N) {
            seed_block(seed, purpose, id, sub, ctr, blk);
            int found = 0;
            for (int t = 0; t < 8 && !found; t++) {
                u64 w = ((u64)blk[2 * t] | ((u64)blk[2 * t + 1] << 32)) & mask;
                if (w < q) { out[j] = w; found = 1; }
            }
            if (found) break;
        }
    }
}

void orc_sample_ternary(u64 seed, uint32_t purpose, uint32_t id, uint32_t sub, int logN, i64 *out)
{
    size_t N = (size_t)1 << logN;
    uint32_t blk[16];
    for (size_t j = 0; j < N; j++) {
        for (uint32_t ctr = (uint32_t)j;; ctr += (uint32_t)N) {
            seed_block(seed, purpose, id, sub, ctr, blk);
            int found = 0;
            for (int f = 0; f < 256 && !found; f++) {
                uint32_t v = (blk[f / 16] >> (2 * (f % 16))) & 3u;
                if (v != 3) { out[j] = v == 0 ? 0 : (v == 1 ? 1 : -1); found = 1; }
            }
            if (found) break;
        }
    }
}

/* The cumulative table of the magnitude of the discrete Gaussian:
 * rho(x) = exp(-x^2 / (2 sigma^2)), P(|x| = 0) = rho(0) / Z,
 * P(|x| = m) = 2 rho(m) / Z, Z = rho(0) + 2 sum_{m=1}^{19} rho(m). */
void orc_gauss_table(u64 *T20)
{
    const double sigma = 3.2;
    double rho[20], Z = 0.0, acc = 0.0;
    for (int m = 0; m < 20; m++) rho[m] = exp(-(double)(m * m) / (2.0 * sigma * sigma));
    for (int m = 0; m < 20; m++) Z += m == 0 ? rho[m] : 2.0 * rho[m];
    for (int m = 0; m < 19; m++) {
        acc += m == 0 ? rho[m] : 2.0 * rho[m];
        T20[m] = (u64)floor(ldexp(acc / Z, 63));
    }
    T20[19] = (u64)1 << 63;
}

void orc_sample_gauss(u64 seed, uint32_t purpose, uint32_t id, uint32_t sub, int logN, i64 *out)
{
    size_t N = (size_t)1 << logN;
    u64 T[20];
    uint32_t blk[16];
    orc_gauss_table(T);
    for (size_t j = 0; j < N; j++) {
        seed_block(seed, purpose, id, sub, (uint32_t)j, blk);
        u64 w = (u64)blk[0] | ((u64)blk[1] << 32);
        u64 u = w >> 1;
        int m = 0;
        while (!(u < T[m])) m++;
        out[j] = (m > 0 && (w & 1)) ? -(i64)m : (i64)m;
    }
}

void orc_sample_ternary_hw(u64 seed, int logN, int h, i64 *out)
{
    size_t N = (size_t)1 << logN;
    uint32_t blk[16], ctr = 0;
    int pos = 16, set = 0;
    uint32_t pair[2];
    memset(out, 0, N * sizeof(i64));
    if (h > (int)N) h = (int)N;
    while (set < h) {
        for (int k = 0; k < 2; k++) {
            if (pos == 16) {
                seed_block(seed, ORC_P_SECRET, 1, 0, ctr++, blk);
                pos = 0;
            }
            pair[k] = blk[pos++];
        }
        size_t p = pair[0] & (uint32_t)(N - 1);
        if (out[p] != 0) continue;
        out[p] = (pair[1] & 1) ? -1 : 1;
        set++;
    }
}
