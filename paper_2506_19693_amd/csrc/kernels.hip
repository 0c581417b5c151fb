// Ring and key-switching kernels of librbk (gfx950).
//
// Every polynomial on the device is in the NTT (evaluation) domain unless a
// kernel says otherwise; a limb is N consecutive uint64 residues in [0, q).
// Layouts: ciphertext [2][l+1][N]; batch of ciphertexts outermost;
// ModUp output [beta_l][E][N] with E = l+1+nP positions (q_0..q_l, p_0..);
// inner-product output [2][E][N].
#include <algorithm>

#include "rbk_ctx.hpp"
#include "wide_arith.hpp"

#define EW_THREADS 256


// ---------------------------------------------------------------- elementwise

template <int OP>
__global__ void k_ew(const u64 *a, const u64 *b, u64 *out, size_t total, int logN, int nlimbs, LimbMap map,
                     const PrimeC *pc)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= total) return;
    if (OP == EW_ZERO) {
        out[i] = 0;
        return;
    }
    int limb = (int)((i >> logN) % nlimbs);
    u64 q = pc[map.prime(limb)].q;
    u64 x = a[i];
    if (OP == EW_ADD) out[i] = add_mod(x, b[i], q);
    else if (OP == EW_SUB) out[i] = sub_mod(x, b[i], q);
    else if (OP == EW_NEG) out[i] = x == 0 ? 0 : q - x;
    else if (OP == EW_MUL) out[i] = mul_mod(x, b[i], pc[map.prime(limb)]);
    else out[i] = x;
}

void ew_launch(const rbk_ctx_impl *c, EwOp op, const u64 *a, const u64 *b, u64 *out, int npoly, int nlimbs, LimbMap map,
               hipStream_t st)
{
    size_t total = (size_t)npoly * nlimbs * c->N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    switch (op) {
    case EW_ADD: hipLaunchKernelGGL(k_ew<EW_ADD>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    case EW_SUB: hipLaunchKernelGGL(k_ew<EW_SUB>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    case EW_NEG: hipLaunchKernelGGL(k_ew<EW_NEG>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    case EW_MUL: hipLaunchKernelGGL(k_ew<EW_MUL>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    case EW_ZERO: hipLaunchKernelGGL(k_ew<EW_ZERO>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    default: hipLaunchKernelGGL(k_ew<EW_COPY>, grid, dim3(EW_THREADS), 0, st, a, b, out, total, c->logN, nlimbs, map, c->d_pc); break;
    }
    kt_end(c, KC_ELEMENTWISE, (op == EW_NEG || op == EW_COPY ? 2.0 : 3.0) * total * sizeof(u64), st);
}

__global__ void k_mul_scalar(const u64 *a, u64 *out, size_t total, int logN, int nlimbs, LimbMap map, const PrimeC *pc,
                             ScalArg s)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= total) return;
    int limb = (int)((i >> logN) % nlimbs);
    u64 q = pc[map.prime(limb)].q;
    out[i] = shoup(a[i], s.w[limb], s.wsh[limb], q);
}

void mul_scalar_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int npoly, int nlimbs, LimbMap map, const ScalArg &s,
                       hipStream_t st)
{
    size_t total = (size_t)npoly * nlimbs * c->N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_mul_scalar, grid, dim3(EW_THREADS), 0, st, a, out, total, c->logN, nlimbs, map, c->d_pc, s);
    kt_end(c, KC_ELEMENTWISE, 2.0 * total * sizeof(u64), st);
}

// ct + constant: a constant polynomial evaluates to itself at every root, so
// in the NTT domain it is added to every entry of every limb of c0.
__global__ void k_add_scalar(const u64 *a, u64 *out, size_t per_poly, int logN, const PrimeC *pc, ScalArg s)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= 2 * per_poly) return;
    if (i >= per_poly) { out[i] = a[i]; return; }
    int limb = (int)(i >> logN);
    out[i] = add_mod(a[i], s.w[limb], pc[limb].q);
}

void add_scalar_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int nlimbs, const ScalArg &s, hipStream_t st)
{
    size_t per = (size_t)nlimbs * c->N;
    dim3 grid((unsigned)((2 * per + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_add_scalar, grid, dim3(EW_THREADS), 0, st, a, out, per, c->logN, c->d_pc, s);
    kt_end(c, KC_ELEMENTWISE, 4.0 * per * sizeof(u64), st);
}

// small signed integers (coefficient domain) reduced into each limb's prime
__global__ void k_signed_to_limbs(const i64 *v, u64 *out, size_t total, int logN, int nlimbs, LimbMap map, const PrimeC *pc)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= total) return;
    size_t k = i & (((size_t)1 << logN) - 1);
    size_t poly = (i >> logN) / nlimbs;
    int limb = (int)((i >> logN) % nlimbs);
    u64 q = pc[map.prime(limb)].q;
    i64 x = v[(poly << logN) + k];
    u64 m = x >= 0 ? (u64)x : (u64)(-x);
    m = m % q;
    out[i] = (x >= 0 || m == 0) ? m : q - m;
}

void signed_to_limbs_launch(const rbk_ctx_impl *c, const i64 *v, u64 *out, int npoly, int nlimbs, LimbMap map,
                            hipStream_t st)
{
    size_t total = (size_t)npoly * nlimbs * c->N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_signed_to_limbs, grid, dim3(EW_THREADS), 0, st, v, out, total, c->logN, nlimbs, map, c->d_pc);
}

// Tensor product (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1).
// a, b: [count][2][l+1][N]; out: [count][3][l+1][N].
__global__ void k_tensor(const u64 *a, const u64 *b, u64 *out, int logN, int L1, int count, const PrimeC *pc)
{
    size_t per = (size_t)L1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= per * count) return;
    size_t ct = i / per, r = i % per;
    int limb = (int)(r >> logN);
    const PrimeC p = pc[limb];
    const u64 *A = a + ct * 2 * per, *B = b + ct * 2 * per;
    u64 a0 = A[r], a1 = A[per + r], b0 = B[r], b1 = B[per + r];
    u64 *O = out + ct * 3 * per;
    O[r] = mul_mod(a0, b0, p);
    u128w s = mul_wide(a0, b1);
    acc_wide(s, mul_wide(a1, b0));
    u64 t = redc(s, p.q, p.qneg);                       // (a0 b1 + a1 b0) 2^-64
    O[per + r] = redc(mul_wide(t, p.r2), p.q, p.qneg);  // undo the 2^-64
    O[2 * per + r] = mul_mod(a1, b1, p);
}

void tensor_launch(const rbk_ctx_impl *c, const u64 *a, const u64 *b, u64 *out, int level, int count, hipStream_t st)
{
    size_t total = (size_t)count * (level + 1) * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_TENSOR, st);
    hipLaunchKernelGGL(k_tensor, grid, dim3(EW_THREADS), 0, st, a, b, out, c->logN, level + 1, count, c->d_pc);
    kt_end(c, KC_TENSOR, 7.0 * total * sizeof(u64), st);
}

// NTT-domain automorphism of npoly x nlimbs limbs (a pure permutation).
// PAIR: two adjacent outputs per thread, read as one aligned source pair
// (pairs map to pairs under any automorphism; in and out 16-byte aligned)
template <bool PAIR>
__global__ void k_automorph(const u64 *in, u64 *out, size_t total, int logN, u64 g)
{
    size_t i = (PAIR ? 2 : 1) * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    if (i >= total) return;
    size_t base = i & ~(((size_t)1 << logN) - 1);
    u32 o = (u32)(i & (((size_t)1 << logN) - 1));
    if (PAIR) {
        const u64x2 v = ld2_perm(in + base, auto_src(o, g, logN));
        st2(out + i, v.x, v.y);
    } else {
        out[i] = in[base + auto_src(o, g, logN)];
    }
}

void automorph_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int npoly, int nlimbs, u64 g, hipStream_t st)
{
    size_t total = (size_t)npoly * nlimbs * c->N;
    if (total == 0) return;
    const bool pair = (((uintptr_t)in | (uintptr_t)out) & 15) == 0 && c->N >= 2;
    const size_t threads = pair ? total / 2 : total;
    dim3 grid((unsigned)((threads + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    if (pair) hipLaunchKernelGGL(k_automorph<true>, grid, dim3(EW_THREADS), 0, st, in, out, total, c->logN, g);
    else hipLaunchKernelGGL(k_automorph<false>, grid, dim3(EW_THREADS), 0, st, in, out, total, c->logN, g);
    kt_end(c, KC_ELEMENTWISE, 2.0 * total * sizeof(u64), st);
}

// The same permutation of npoly polynomials of nlimbs limbs each, polynomial
// p read at in + p in_stride and written at out + p out_stride (grid.y runs
// over the polynomials)
template <bool PAIR>
__global__ void k_automorph_polys(const u64 *in, long in_stride, u64 *out, long out_stride, size_t per, int logN, u64 g)
{
    size_t i = (PAIR ? 2 : 1) * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    if (i >= per) return;
    const u64 *src = in + (size_t)blockIdx.y * in_stride;
    u64 *dst = out + (size_t)blockIdx.y * out_stride;
    size_t base = i & ~(((size_t)1 << logN) - 1);
    u32 o = (u32)(i & (((size_t)1 << logN) - 1));
    if (PAIR) {
        const u64x2 v = ld2_perm(src + base, auto_src(o, g, logN));
        st2(dst + i, v.x, v.y);
    } else {
        dst[i] = src[base + auto_src(o, g, logN)];
    }
}

void automorph_polys_launch(const rbk_ctx_impl *c, const u64 *in, long in_stride, u64 *out, long out_stride, int npoly,
                            int nlimbs, u64 g, hipStream_t st)
{
    const size_t per = (size_t)nlimbs * c->N;
    if (per == 0 || npoly <= 0) return;
    const bool pair = (((uintptr_t)in | (uintptr_t)out) & 15) == 0 && ((in_stride | out_stride) & 1) == 0 && c->N >= 2;
    const size_t threads = pair ? per / 2 : per;
    kt_begin(c, KC_ELEMENTWISE, st);
    for (int p0 = 0; p0 < npoly; p0 += 65535) {
        const int np = std::min(npoly - p0, 65535);
        dim3 grid((unsigned)((threads + EW_THREADS - 1) / EW_THREADS), (unsigned)np);
        const u64 *src = in + (size_t)p0 * in_stride;
        u64 *dst = out + (size_t)p0 * out_stride;
        if (pair) hipLaunchKernelGGL(k_automorph_polys<true>, grid, dim3(EW_THREADS), 0, st, src, in_stride, dst, out_stride, per, c->logN, g);
        else hipLaunchKernelGGL(k_automorph_polys<false>, grid, dim3(EW_THREADS), 0, st, src, in_stride, dst, out_stride, per, c->logN, g);
    }
    kt_end(c, KC_ELEMENTWISE, 2.0 * npoly * per * sizeof(u64), st);
}

// ---------------------------------------------------------------- base conversion

#define BCONV_MAX_IN 16
// the table is staged in LDS output-major, entry (i, o) at o * TS + i with the
// row stride TS = MAXIN rounded up to even (16-byte aligned rows), so the
// inputs of one output sit at one address plus immediate offsets; n_out is
// below the prime count
#define BCONV_TS(MAXIN) (((MAXIN) + 1) & ~1)
#define BCONV_TAB(MAXIN) (RBK_MAX_PRIMES * BCONV_TS(MAXIN))

// Base-conversion sums use the carry-free 30-bit split accumulation of
// wide_arith.hpp (at most 16 terms of residues and table entries below 2^60).
using wa::Acc4;
using wa::Half30;
using wa::split30;
__device__ __forceinline__ u128w acc4_sum(const Acc4 &a)
{
    const wa::Wide w = wa::acc4_value(a);
    u128w t;
    t.lo = w.lo;
    t.hi = w.hi;
    return t;
}

// ModUp also copies the digit's own limbs, in the NTT domain (own: the
// polynomial the coefficient-domain input was made from), into their positions.
template <bool MODUP, int MAXIN>
__global__ __launch_bounds__(EW_THREADS) void k_bconv(const u64 *in, long in_stride, u64 *out, long out_stride, int logN,
                                                      int L1, int E, int alpha, int nP, int nQ, const u64 *A,
                                                      const u64 *Ash, const u64 *M, long m_stride, const PrimeC *pc,
                                                      const u64 *own, long own_stride)
{
    __shared__ Half30 tab[BCONV_TAB(MAXIN)];
    const size_t N = (size_t)1 << logN;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int poly = blockIdx.z;
    int lo, n_in, n_out;
    const u64 *Aj, *Ashj, *Mj;
    u64 *dst;
    const u64 *x;
    if (MODUP) {
        const int j = blockIdx.y;
        lo = j * alpha;
        n_in = min(alpha, L1 - lo);
        n_out = E - n_in;
        Aj = A + j * alpha;
        Ashj = Ash + j * alpha;
        Mj = M + (size_t)j * alpha * m_stride;
        x = in + poly * in_stride + (size_t)lo * N;
        dst = out + poly * out_stride + (size_t)j * E * N;
    } else {
        lo = 0;
        n_in = nP;
        n_out = L1;
        Aj = A;
        Ashj = Ash;
        Mj = M;
        x = in + poly * in_stride;
        dst = out + poly * out_stride;
    }
    // zero columns past n_in: every output sums all MAXIN terms without branches
    constexpr int TS = BCONV_TS(MAXIN);
    for (int w = threadIdx.x; w < TS * n_out; w += EW_THREADS) {
        const int o = w / TS, i = w % TS;
        tab[w] = i < n_in ? split30(Mj[(size_t)i * m_stride + o]) : Half30{0, 0};
    }
    __syncthreads();
    if (k >= N) return;
    Half30 yh[MAXIN];
    const u64 *ownj = MODUP ? own + poly * own_stride + (size_t)lo * N : nullptr;
#pragma unroll
    for (int i = 0; i < MAXIN; i++) {
        yh[i] = Half30{0, 0};
        if (i < n_in) {
            const int pi = MODUP ? lo + i : nQ + i;
            yh[i] = split30(shoup(x[(size_t)i * N + k], Aj[i], Ashj[i], pc[pi].q));
            if (MODUP) dst[(size_t)(lo + i) * N + k] = ownj[(size_t)i * N + k];
        }
    }
    for (int o = 0; o < n_out; o++) {
        int pos, pr;
        if (MODUP) {
            pos = o < lo ? o : o + n_in;
            pr = pos < L1 ? pos : nQ + pos - L1;
        } else {
            pos = o;
            pr = o;
        }
        const PrimeC p = pc[pr];
        Acc4 acc;
#pragma unroll
        for (int i = 0; i < MAXIN; i++)
            wa::acc4(acc, yh[i], tab[o * TS + i]);
        // n_in <= 16 terms, each y (< 2^60) times a table entry (< p): the sum
        // stays below p 2^64, so a plain REDC reduces it
        dst[(size_t)pos * N + k] = redc(acc4_sum(acc), p.q, p.qneg);
    }
}

// terms per output of the base-conversion kernel for n inputs
static int bconv_terms(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n == 9 ? 9 : n == 10 ? 10 : n <= 12 ? 12 : 16; }

void bconv_modup_launch(const rbk_ctx_impl *c, const u64 *coef, long coef_stride, const u64 *own, long own_stride,
                        u64 *ext, long ext_stride, int level, int count, hipStream_t st)
{
    const ModUpTables &T = modup_tables(const_cast<rbk_ctx_impl *>(c), level);
    int L1 = level + 1, E = L1 + c->nP;
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), T.beta, count);
    kt_begin(c, KC_BCONV_UP, st);
#define BCU(M)                                                                                                         \
    hipLaunchKernelGGL((k_bconv<true, M>), grid, dim3(EW_THREADS), 0, st, coef, coef_stride, ext, ext_stride, c->logN, L1, \
                       E, c->alpha, c->nP, c->nQ, T.d_A, T.d_Ash, T.d_M, (long)E, c->d_pc, own, own_stride)
    // the digit size itself where it is common (no zero terms), else the next multiple of 4
    switch (bconv_terms(c->alpha)) {
    case 4: BCU(4); break;
    case 8: BCU(8); break;
    case 9: BCU(9); break;
    case 10: BCU(10); break;
    case 12: BCU(12); break;
    default: BCU(16); break;
    }
#undef BCU
    kt_end(c, KC_BCONV_UP, (double)count * T.beta * E * c->N * sizeof(u64), st);
}

void bconv_moddown_launch(const rbk_ctx_impl *c, const u64 *pcoef, long p_stride, u64 *conv, long conv_stride, int level,
                          int count, hipStream_t st)
{
    int L1 = level + 1;
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), 1, count);
    kt_begin(c, KC_BCONV_DOWN, st);
#define BCD(M)                                                                                                           \
    hipLaunchKernelGGL((k_bconv<false, M>), grid, dim3(EW_THREADS), 0, st, pcoef, p_stride, conv, conv_stride, c->logN, L1, \
                       L1 + c->nP, c->alpha, c->nP, c->nQ, c->d_md_A, c->d_md_Ash, c->d_md_M, (long)c->nQ, c->d_pc, nullptr, 0)
    switch (bconv_terms(c->nP)) {
    case 4: BCD(4); break;
    case 8: BCD(8); break;
    case 9: BCD(9); break;
    case 10: BCD(10); break;
    case 12: BCD(12); break;
    default: BCD(16); break;
    }
#undef BCD
    kt_end(c, KC_BCONV_DOWN, (double)count * (c->nP + L1) * c->N * sizeof(u64), st);
}

// ---------------------------------------------------------------- key inner product

// (u0, u1)[e] = sum_j ext_j[e] * (b_j, a_j)[t_e], one REDC per output (the key
// is stored times 2^64).  With g != 0 every digit is read through the
// automorphism sigma_g (hoisted rotation).  One thread serves one (e, k) for
// all 'count' ciphertexts, so each key word is fetched once per launch.
#define IP_MAX_BETA 8
__global__ __launch_bounds__(EW_THREADS) void k_ip(const u64 *ext, long ext_stride, const u64 *key, u64 *u, long u_stride,
                                                   int logN, int E, int beta, int nT, int count, LimbMap emap, u64 g,
                                                   const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int e = blockIdx.y;
    if (k >= N) return;
    const int t = emap.prime(e);
    const PrimeC p = pc[t];
    u64 kb[IP_MAX_BETA], ka[IP_MAX_BETA];
#pragma unroll
    for (int j = 0; j < IP_MAX_BETA; j++)
        if (j < beta) {
            kb[j] = key[(((size_t)j * 2 + 0) * nT + t) * N + k];
            ka[j] = key[(((size_t)j * 2 + 1) * nT + t) * N + k];
        }
    const size_t src = g ? auto_src((u32)k, g, logN) : k;
    for (int ct = 0; ct < count; ct++) {
        const u64 *x = ext + ct * ext_stride + (size_t)e * N + src;
        u128w s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int j = 0; j < IP_MAX_BETA; j++)
            if (j < beta) {
                u64 d = x[(size_t)j * E * N];
                acc_wide(s0, mul_wide(d, kb[j]));
                acc_wide(s1, mul_wide(d, ka[j]));
            }
        u64 *o = u + ct * u_stride + (size_t)e * N + k;
        o[0] = redc(s0, p.q, p.qneg);  // beta <= 8 products below p^2: the sum is below p 2^64
        o[(size_t)E * N] = redc(s1, p.q, p.qneg);
    }
}

void ip_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *u, long u_stride, int level,
               int count, u64 g, hipStream_t st)
{
    int L1 = level + 1, E = L1 + c->nP;
    int beta_l = (L1 + c->alpha - 1) / c->alpha;
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), E, 1);
    LimbMap emap{0, L1, c->nQ};
    kt_begin(c, KC_IP, st);
    hipLaunchKernelGGL(k_ip, grid, dim3(EW_THREADS), 0, st, ext, ext_stride, key, u, u_stride, c->logN, E, beta_l, c->nT,
                       count, emap, g, c->d_pc);
    kt_end(c, KC_IP, ((double)count * beta_l * E + 2.0 * beta_l * E + 2.0 * count * E) * c->N * sizeof(u64), st);
}

// out[p][i] = (u[p][i] - conv[p][i]) * P^-1 mod q_i  (+ add_p[i], read through
// sigma_{add_g} when add_g != 0).  u: [2][E][N] per ct (Q positions first);
// conv/out/add: [2][l+1][N] per ct.  add may be null; add is applied to
// poly 0 always and to poly 1 only when add_both != 0.
__global__ void k_moddown_finish(const u64 *u, long u_stride, const u64 *conv, long conv_stride, const u64 *add,
                                 long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int logN, int L1, int E,
                                 int count, const u64 *Pinv, const u64 *Pinv_sh, const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t per = (size_t)L1 * N;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= 2 * per * count) return;
    size_t ct = i / (2 * per), r = i % (2 * per);
    int poly = (int)(r / per);
    size_t rr = r % per;
    int limb = (int)(rr >> logN);
    size_t k = rr & (N - 1);
    u64 q = pc[limb].q;
    u64 uv = u[ct * u_stride + (size_t)poly * E * N + rr];
    u64 cv = conv[ct * conv_stride + r];
    u64 v = shoup(sub_mod(uv, cv, q), Pinv[limb], Pinv_sh[limb], q);
    if (add && (poly == 0 || add_both)) {
        size_t src = add_g ? auto_src((u32)k, add_g, logN) : k;
        v = add_mod(v, add[ct * add_stride + (size_t)poly * per + ((size_t)limb << logN) + src], q);
    }
    out[ct * out_stride + r] = v;
}

void moddown_finish_launch(const rbk_ctx_impl *c, const u64 *u, long u_stride, const u64 *conv, long conv_stride,
                           const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level,
                           int count, hipStream_t st)
{
    int L1 = level + 1, E = L1 + c->nP;
    size_t total = (size_t)2 * L1 * c->N * count;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_MODDOWN_FIN, st);
    hipLaunchKernelGGL(k_moddown_finish, grid, dim3(EW_THREADS), 0, st, u, u_stride, conv, conv_stride, add, add_stride,
                       add_g, add_both, out, out_stride, c->logN, L1, E, count, c->d_Pinv, c->d_Pinv_sh, c->d_pc);
    kt_end(c, KC_MODDOWN_FIN, ((double)count * L1 * (add ? (add_both ? 8 : 7) : 6)) * c->N * sizeof(u64), st);
}

// ---------------------------------------------------------------- key switching with a fused ModDown epilogue

// ciphertexts handled by one thread of the fused inner-product kernels: the
// key words are loaded once per thread, the grid's z dimension covers the rest

// Inner product restricted to the special-prime positions, written to
// tp[count][2][nP][N] (the input of the ModDown inverse NTT).
template <int BETA>
__global__ __launch_bounds__(EW_THREADS) void k_ip_p(const u64 *__restrict__ ext, long ext_stride,
                                                     const u64 *__restrict__ key, u64 *__restrict__ tp, int logN,
                                                     int L1, int E, int nT, int nQ, int nP, int count, int cpc, u64 g,
                                                     const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t k = 2 * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    const int t = blockIdx.y;
    const int ct0 = blockIdx.z * cpc, ct1 = min(count, ct0 + cpc);
    if (k >= N) return;
    const int pos = L1 + t, pr = nQ + t;
    const PrimeC p = pc[pr];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
            kb[j] = ld2(key + (((size_t)j * 2 + 0) * nT + pr) * N + k);
            ka[j] = ld2(key + (((size_t)j * 2 + 1) * nT + pr) * N + k);
        }
    const size_t src = g ? auto_src((u32)k, g, logN) : k;
#pragma unroll 2
    for (int ct = ct0; ct < ct1; ct++) {
        const u64 *x = ext + ct * ext_stride + (size_t)pos * N;
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++) {
                u64x2 d = ld2_perm(x + (size_t)j * E * N, src);
                acc_wide(s0, mul_wide(d.x, kb[j].x));
                acc_wide(t0, mul_wide(d.y, kb[j].y));
                acc_wide(s1, mul_wide(d.x, ka[j].x));
                acc_wide(t1, mul_wide(d.y, ka[j].y));
            }
        u64 *o = tp + ((size_t)ct * 2 * nP + t) * N + k;
        // beta <= 8 products below p^2: every sum is below p 2^64, a plain REDC suffices
        st2(o, redc(s0, p.q, p.qneg), redc(t0, p.q, p.qneg));
        st2(o + (size_t)nP * N, redc(s1, p.q, p.qneg), redc(t1, p.q, p.qneg));
    }
}

// Q positions: the inner product is recomputed here instead of being stored,
//   out[h][i] = (sum_j ext_j[i] key_j[h][i] - conv[h][i]) * P^-1 mod q_i (+ add_h[i]).
// add (through sigma_{add_g} when add_g != 0) goes to poly 0, and to poly 1
// when add_both != 0.
template <int BETA, int ADD>
__global__ __launch_bounds__(EW_THREADS) void k_moddown_ip(const u64 *__restrict__ ext, long ext_stride,
                                                           const u64 *__restrict__ key, const u64 *__restrict__ conv,
                                                           long conv_stride, const u64 *__restrict__ add, long add_stride,
                                                           u64 add_g, u64 *__restrict__ out, long out_stride, int logN,
                                                           int L1, int E, int nT, int count, int cpc, u64 g,
                                                           const u64 *Pinv, const u64 *Pinv_sh, const PrimeC *pc)
{
    // ADD: 0 none, 1 add to the first output polynomial, 2 to both
    const size_t N = (size_t)1 << logN;
    const size_t k = 2 * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    const int i = blockIdx.y;
    const int ct0 = blockIdx.z * cpc, ct1 = min(count, ct0 + cpc);
    if (k >= N) return;
    const PrimeC p = pc[i];
    const u64 pinv = Pinv[i], pinv_sh = Pinv_sh[i];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
            kb[j] = ld2(key + (((size_t)j * 2 + 0) * nT + i) * N + k);
            ka[j] = ld2(key + (((size_t)j * 2 + 1) * nT + i) * N + k);
        }
    const size_t src = g ? auto_src((u32)k, g, logN) : k;
    const size_t asrc = add_g ? auto_src((u32)k, add_g, logN) : k;
    const size_t per = (size_t)L1 * N, li = (size_t)i * N;
#pragma unroll 2
    for (int ct = ct0; ct < ct1; ct++) {
        // every load of the ciphertext first, then the arithmetic
        const u64 *x = ext + ct * ext_stride + li;
        u64x2 d[BETA];
#pragma unroll
        for (int j = 0; j < BETA; j++) d[j] = ld2_perm(x + (size_t)j * E * N, src);
        const u64 *cv = conv + ct * conv_stride + li + k;
        const u64x2 c0 = ld2(cv), c1 = ld2(cv + per);
        u64x2 a0 = {0, 0}, a1 = {0, 0};
        if (ADD >= 1) a0 = ld2_perm(add + ct * add_stride + li, asrc);
        if (ADD == 2) a1 = ld2_perm(add + ct * add_stride + li + per, asrc);
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++) {
                acc_wide(s0, mul_wide(d[j].x, kb[j].x));
                acc_wide(t0, mul_wide(d[j].y, kb[j].y));
                acc_wide(s1, mul_wide(d[j].x, ka[j].x));
                acc_wide(t1, mul_wide(d[j].y, ka[j].y));
            }
        // beta <= 8 products below q^2: every sum is below q 2^64, a plain REDC suffices
        u64 v0 = shoup(sub_mod(redc(s0, p.q, p.qneg), c0.x, p.q), pinv, pinv_sh, p.q);
        u64 w0 = shoup(sub_mod(redc(t0, p.q, p.qneg), c0.y, p.q), pinv, pinv_sh, p.q);
        u64 v1 = shoup(sub_mod(redc(s1, p.q, p.qneg), c1.x, p.q), pinv, pinv_sh, p.q);
        u64 w1 = shoup(sub_mod(redc(t1, p.q, p.qneg), c1.y, p.q), pinv, pinv_sh, p.q);
        if (ADD >= 1) {
            v0 = add_mod(v0, a0.x, p.q);
            w0 = add_mod(w0, a0.y, p.q);
        }
        if (ADD == 2) {
            v1 = add_mod(v1, a1.x, p.q);
            w1 = add_mod(w1, a1.y, p.q);
        }
        u64 *o = out + ct * out_stride + li + k;
        st2_nt(o, v0, w0);
        st2_nt(o + per, v1, w1);
    }
}

void ip_p_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *tp, int level, int count,
                 u64 g, hipStream_t st)
{
    int L1 = level + 1, E = L1 + c->nP;
    int beta_l = (L1 + c->alpha - 1) / c->alpha;
    if (c->nP == 0) return;
    const int cpc = c->ip_cpc;
    dim3 grid((unsigned)((c->N / 2 + EW_THREADS - 1) / EW_THREADS), c->nP, (count + cpc - 1) / cpc);
    kt_begin(c, KC_IP_P, st);
#define IPP_CASE(B)                                                                                          \
    case B:                                                                                                   \
        hipLaunchKernelGGL(k_ip_p<B>, grid, dim3(EW_THREADS), 0, st, ext, ext_stride, key, tp, c->logN, L1, E, c->nT, \
                           c->nQ, c->nP, count, cpc, g, c->d_pc);                                             \
        break;
    switch (beta_l) { IPP_CASE(1) IPP_CASE(2) IPP_CASE(3) IPP_CASE(4) IPP_CASE(5) IPP_CASE(6) IPP_CASE(7) default: IPP_CASE(8) }
#undef IPP_CASE
    kt_end(c, KC_IP_P, ((double)count * beta_l * c->nP + 2.0 * beta_l * c->nP + 2.0 * count * c->nP) * c->N * sizeof(u64),
           st);
}

void moddown_ip_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, const u64 *conv,
                       long conv_stride, const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out,
                       long out_stride, int level, int count, u64 g, hipStream_t st)
{
    int L1 = level + 1, E = L1 + c->nP;
    int beta_l = (L1 + c->alpha - 1) / c->alpha;
    const int cpc = c->ip_cpc;
    dim3 grid((unsigned)((c->N / 2 + EW_THREADS - 1) / EW_THREADS), L1, (count + cpc - 1) / cpc);
    kt_begin(c, KC_MODDOWN_IP, st);
    const int addm = add ? (add_both ? 2 : 1) : 0;
#define MDI_LAUNCH(B, A)                                                                                        \
    hipLaunchKernelGGL((k_moddown_ip<B, A>), grid, dim3(EW_THREADS), 0, st, ext, ext_stride, key, conv, conv_stride, add, \
                       add_stride, add_g, out, out_stride, c->logN, L1, E, c->nT, count, cpc, g, c->d_Pinv, c->d_Pinv_sh, \
                       c->d_pc)
#define MDI_CASE(B)                                                                                           \
    case B:                                                                                                    \
        if (addm == 0) MDI_LAUNCH(B, 0);                                                                       \
        else if (addm == 1) MDI_LAUNCH(B, 1);                                                                  \
        else MDI_LAUNCH(B, 2);                                                                                 \
        break;
    switch (beta_l) { MDI_CASE(1) MDI_CASE(2) MDI_CASE(3) MDI_CASE(4) MDI_CASE(5) MDI_CASE(6) MDI_CASE(7) default: MDI_CASE(8) }
#undef MDI_CASE
#undef MDI_LAUNCH
    double words = (double)count * L1 * (beta_l + 2 + 2 + (add ? (add_both ? 2 : 1) : 0)) + 2.0 * beta_l * L1;
    kt_end(c, KC_MODDOWN_IP, words * c->N * sizeof(u64), st);
}

// ---------------------------------------------------------------- rescale

// lifted[p][i] = centred(last[p]) mod q_i  for i < l   (coefficient domain)
__global__ void k_rescale_lift(const u64 *last, u64 *lifted, int logN, int level, int npoly, const PrimeC *pc,
                               const u64 *qmod)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)level * N;
    if (i >= per * npoly) return;
    size_t poly = i / per, r = i % per;
    int limb = (int)(r >> logN);
    size_t k = r & (N - 1);
    const PrimeC p = pc[limb];
    u64 ql = pc[level].q;
    u64 x = last[poly * N + k];
    u64 xm = shoup(x, 1, p.one_sh, p.q);
    lifted[i] = (x <= (ql - 1) / 2) ? xm : sub_mod(xm, qmod[limb], p.q);
}

void rescale_lift_launch(const rbk_ctx_impl *c, const u64 *last, u64 *lifted, int level, int npoly, hipStream_t st)
{
    size_t total = (size_t)npoly * level * c->N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_RESCALE, st);
    hipLaunchKernelGGL(k_rescale_lift, grid, dim3(EW_THREADS), 0, st, last, lifted, c->logN, level, npoly, c->d_pc,
                       c->d_rs_qmod + (size_t)level * c->nQ);
    kt_end(c, KC_RESCALE, (double)npoly * (1 + level) * c->N * sizeof(u64), st);
}

// out[p][i] = (in[p][i] - lifted[p][i]) * q_l^-1 mod q_i;  in: [npoly][l+1][N], out/lifted: [npoly][l][N]
__global__ void k_rescale_finish(const u64 *in, const u64 *lifted, u64 *out, int logN, int level, int npoly,
                                 const PrimeC *pc, const u64 *inv, const u64 *inv_sh)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)level * N;
    if (i >= per * npoly) return;
    size_t poly = i / per, r = i % per;
    int limb = (int)(r >> logN);
    u64 q = pc[limb].q;
    u64 x = in[poly * (per + N) + r];
    out[i] = shoup(sub_mod(x, lifted[i], q), inv[limb], inv_sh[limb], q);
}

void rescale_finish_launch(const rbk_ctx_impl *c, const u64 *in, const u64 *lifted, u64 *out, int level, int npoly,
                           hipStream_t st)
{
    size_t total = (size_t)npoly * level * c->N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_RESCALE, st);
    hipLaunchKernelGGL(k_rescale_finish, grid, dim3(EW_THREADS), 0, st, in, lifted, out, c->logN, level, npoly, c->d_pc,
                       c->d_rs_inv + (size_t)level * c->nQ, c->d_rs_inv_sh + (size_t)level * c->nQ);
    kt_end(c, KC_RESCALE, 3.0 * total * sizeof(u64), st);
}

// ---------------------------------------------------------------- bootstrapping helpers

// ModRaise, lifting step: x (coefficient domain, residues mod q_0, one limb
// per polynomial, npoly polynomials) is read as a centred integer and reduced
// into limbs 0..l: out [npoly][l+1][N].
__global__ void k_modraise_lift(const u64 *in, u64 *out, int logN, int L1, int npoly, const PrimeC *pc, const u64 *q0mod)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)L1 * N;
    if (i >= per * npoly) return;
    size_t poly = i / per, r = i % per;
    int limb = (int)(r >> logN);
    size_t k = r & (N - 1);
    const PrimeC p = pc[limb];
    const u64 q0 = pc[0].q;
    u64 x = in[poly * N + k];
    u64 xm = shoup(x, 1, p.one_sh, p.q);
    out[i] = (x <= (q0 - 1) / 2) ? xm : sub_mod(xm, q0mod[limb], p.q);
}

void modraise_lift_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int level, int npoly, hipStream_t st)
{
    size_t total = (size_t)npoly * (level + 1) * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_modraise_lift, grid, dim3(EW_THREADS), 0, st, in, out, c->logN, level + 1, npoly, c->d_pc,
                       c->d_q0mod);
    kt_end(c, KC_ELEMENTWISE, (double)npoly * (level + 2) * c->N * sizeof(u64), st);
}

// Multiplication by sign * X^(N/2) in the NTT domain: at psi^(2k+1) the
// monomial is i_q^(2k+1) = i_q (-1)^k with i_q = psi^(N/2) (a square root of -1),
// and k = bit_reverse(o) is odd exactly when the top index bit of o is set.
__global__ void k_monomial_half(const u64 *in, u64 *out, size_t total, int logN, int nlimbs, int neg, const PrimeC *pc,
                                const u64 *iq, const u64 *iq_sh)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= total) return;
    int limb = (int)((i >> logN) % nlimbs);
    u64 q = pc[limb].q;
    u64 v = shoup(in[i], iq[limb], iq_sh[limb], q);
    int odd = (int)((i >> (logN - 1)) & 1);
    if ((odd ^ neg) && v) v = q - v;
    out[i] = v;
}

void monomial_half_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int npoly, int level, int neg, hipStream_t st)
{
    size_t total = (size_t)npoly * (level + 1) * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_monomial_half, grid, dim3(EW_THREADS), 0, st, in, out, total, c->logN, level + 1, neg, c->d_pc,
                       c->d_iq, c->d_iq_sh);
    kt_end(c, KC_ELEMENTWISE, 2.0 * total * sizeof(u64), st);
}

// The lazy 128-bit sum of at most 16 products below q^2 stays below q 2^64:
// one REDC, and one more to undo its 2^-64, end it.
__device__ __forceinline__ u64 mac_finish(u128w acc, const PrimeC &p)
{
    return redc(mul_wide(redc(acc, p.q, p.qneg), p.r2), p.q, p.qneg);
}

// Several giant steps of a baby-step / giant-step product in one pass: each
// baby-step ciphertext is read once per launch and multiplied into the inner
// sums of up to GT_MAX_G giant steps (one position per thread, every
// plaintext weight of the thread's position held in registers across the
// batch), where a launch per giant step reads every baby step again.
__global__ __launch_bounds__(EW_THREADS) void k_mac_giants(GiantTerms T, int logN, int L1, int count, const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t n = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (n >= N) return;
    const int limb = blockIdx.y, poly = blockIdx.z;
    const PrimeC p = pc[limb];
    const size_t per = (size_t)L1 * N, lo = ((size_t)limb << logN) + n, off = (size_t)poly * per + lo;
    u64 w[GT_MAX_G][GT_MAX_B];
#pragma unroll
    for (int j = 0; j < GT_MAX_G; j++)
#pragma unroll
        for (int b = 0; b < GT_MAX_B; b++) w[j][b] = (j < T.ng && b < T.nb && T.pt[j][b]) ? T.pt[j][b][lo] : 0;
    for (int c = 0; c < count; c++) {
        u128w acc[GT_MAX_G];
#pragma unroll
        for (int j = 0; j < GT_MAX_G; j++) acc[j] = {0, 0};
#pragma unroll
        for (int b = 0; b < GT_MAX_B; b++) {
            if (b < T.nb) {
                const u64 v = T.src[b][(size_t)c * T.stride[b] + off];
#pragma unroll
                for (int j = 0; j < GT_MAX_G; j++)
                    if (j < T.ng && T.pt[j][b]) acc_wide(acc[j], mul_wide(v, w[j][b]));
            }
        }
#pragma unroll
        for (int j = 0; j < GT_MAX_G; j++)
            if (j < T.ng) {
                u64 *o = T.out[j] + (size_t)c * 2 * per + off;
                u64 r = mac_finish(acc[j], p);
                if (T.add[j]) r = add_mod(*o, r, p.q);
                *o = r;
            }
    }
}

void mac_giants_launch(const rbk_ctx_impl *c, const GiantTerms &T, int level, int count, hipStream_t st)
{
    if (T.ng <= 0 || T.nb <= 0 || count <= 0) return;
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), level + 1, 2);
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_mac_giants, grid, dim3(EW_THREADS), 0, st, T, c->logN, level + 1, count, c->d_pc);
    int n_pt = 0, n_rd = 0;
    for (int j = 0; j < T.ng; j++) {
        n_rd += T.add[j] ? 2 : 1;
        for (int b = 0; b < T.nb; b++) n_pt += T.pt[j][b] ? 1 : 0;
    }
    const double ct = 2.0 * (level + 1) * c->N * sizeof(u64);
    kt_end(c, KC_ELEMENTWISE, ct * count * (T.nb + n_rd) + ct * n_pt, st);
}

// ct + constant for count ciphertexts (the constant goes to every NTT point of c0)
__global__ void k_add_scalar_batch(const u64 *a, u64 *out, size_t per, int logN, int count, const PrimeC *pc, ScalArg s)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= 2 * per * count) return;
    size_t r = i % (2 * per);
    if (r >= per) { out[i] = a[i]; return; }
    int limb = (int)(r >> logN);
    out[i] = add_mod(a[i], s.w[limb], pc[limb].q);
}

void add_scalar_batch_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int level, int count, const ScalArg &s,
                             hipStream_t st)
{
    size_t per = (size_t)(level + 1) * c->N;
    dim3 grid((unsigned)((2 * per * count + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_ELEMENTWISE, st);
    hipLaunchKernelGGL(k_add_scalar_batch, grid, dim3(EW_THREADS), 0, st, a, out, per, c->logN, count, c->d_pc, s);
    kt_end(c, KC_ELEMENTWISE, 4.0 * per * count * sizeof(u64), st);
}

// ---------------------------------------------------------------- keys, encryption

// Switching key, NTT domain, every prime of the table:
//   b_j = -a_j s + e_j (+ [P]_{q_t} s' on the primes of digit j),  stored with a_j
// in Montgomery form.  a, e: [beta][nT][N]; s, s_from: [nT][N]; key: [beta][2][nT][N].
__global__ void k_keygen(const u64 *a, const u64 *e, const u64 *s, const u64 *s_from, u64 *key, int logN, int nT, int nQ,
                         int alpha, int beta, const PrimeC *pc, const u64 *Pmod, const u64 *Pmod_sh)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)nT * N;
    if (i >= per * beta) return;
    int j = (int)(i / per);
    size_t r = i % per;
    int t = (int)(r >> logN);
    const PrimeC p = pc[t];
    u64 av = a[i], ev = e[i], sv = s[r];
    u64 b = sub_mod(ev, mul_mod(av, sv, p), p.q);
    if (t < nQ && t / alpha == j) b = add_mod(b, shoup(s_from[r], Pmod[t], Pmod_sh[t], p.q), p.q);
    u64 *kj = key + (size_t)j * 2 * per;
    kj[r] = redc(mul_wide(b, p.r2), p.q, p.qneg);
    kj[per + r] = redc(mul_wide(av, p.r2), p.q, p.qneg);
}

void keygen_launch(const rbk_ctx_impl *c, const u64 *a_ntt, const u64 *e_ntt, const u64 *s_from, u64 *key_out,
                   hipStream_t st)
{
    size_t total = (size_t)c->beta * c->nT * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_keygen, grid, dim3(EW_THREADS), 0, st, a_ntt, e_ntt, c->d_s, s_from, key_out, c->logN, c->nT,
                       c->nQ, c->alpha, c->beta, c->d_pc, c->d_Pmod, c->d_Pmod_sh);
}

// x -> x 2^64 mod q (forward) or x 2^-64 mod q (inverse)
__global__ void k_to_mont(u64 *d, size_t total, int logN, int nlimbs, LimbMap map, const PrimeC *pc, int inverse)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= total) return;
    int limb = (int)((i >> logN) % nlimbs);
    const PrimeC p = pc[map.prime(limb)];
    u128w x = {d[i], 0};
    d[i] = inverse ? redc(x, p.q, p.qneg) : redc(mul_wide(d[i], p.r2), p.q, p.qneg);
}

void to_mont_launch(const rbk_ctx_impl *c, u64 *data, int npoly, int nlimbs, LimbMap map, bool inverse, hipStream_t st)
{
    size_t total = (size_t)npoly * nlimbs * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_to_mont, grid, dim3(EW_THREADS), 0, st, data, total, c->logN, nlimbs, map, c->d_pc, inverse ? 1 : 0);
}

// ct = (v pk0 + e0 + m, v pk1 + e1) at level l; all operands NTT domain.
__global__ void k_encrypt(const u64 *pt, const u64 *v, const u64 *e0, const u64 *e1, const u64 *pk, u64 *ct, int logN,
                          int L1, int nQ, const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)L1 * N;
    if (i >= per) return;
    int limb = (int)(i >> logN);
    const PrimeC p = pc[limb];
    u64 vv = v[i];
    ct[i] = add_mod(add_mod(mul_mod(vv, pk[i], p), e0[i], p.q), pt[i], p.q);
    ct[per + i] = add_mod(mul_mod(vv, pk[(size_t)nQ * N + i], p), e1[i], p.q);
}

void encrypt_launch(const rbk_ctx_impl *c, const u64 *pt, const u64 *v, const u64 *e0, const u64 *e1, u64 *ct, int level,
                    hipStream_t st)
{
    size_t total = (size_t)(level + 1) * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_encrypt, grid, dim3(EW_THREADS), 0, st, pt, v, e0, e1, c->d_pk, ct, c->logN, level + 1, c->nQ,
                       c->d_pc);
}

// m = c0 + c1 s at level l (NTT domain)
__global__ void k_decrypt(const u64 *ct, const u64 *s, u64 *pt, int logN, int L1, const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    size_t per = (size_t)L1 * N;
    if (i >= per) return;
    int limb = (int)(i >> logN);
    const PrimeC p = pc[limb];
    pt[i] = add_mod(ct[i], mul_mod(ct[per + i], s[i], p), p.q);
}

void decrypt_launch(const rbk_ctx_impl *c, const u64 *ct, u64 *pt, int level, hipStream_t st)
{
    size_t total = (size_t)(level + 1) * c->N;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_decrypt, grid, dim3(EW_THREADS), 0, st, ct, c->d_s, pt, c->logN, level + 1, c->d_pc);
}

// ---------------------------------------------------------------- batches of uneven level
//
// A batch of `count` ciphertexts whose levels differ.  Every buffer is laid
// out at the strides of the largest level Lm (L1m = Lm + 1 limbs per
// polynomial, Em = L1m + nP extended positions per ModUp digit, betam digits
// per ciphertext); ciphertext i uses the first level_i + 1 limbs (and E_i =
// level_i + 1 + nP positions, beta_i digits) of its slot.  Grids cover the
// largest shape and work outside a ciphertext's own shape returns at once.
// The arithmetic of every element is that of the uniform kernels above.

__global__ void k_tensor_list(const u64 *a, const u64 *b, u64 *out, int logN, int L1m, int count, const ListCt *cts,
                              const PrimeC *pc)
{
    const size_t per = (size_t)L1m << logN;
    const size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= per * count) return;
    const size_t ct = i / per, r = i % per;
    const int limb = (int)(r >> logN);
    if (limb > cts[ct].level) return;
    const PrimeC p = pc[limb];
    const u64 *A = a + ct * 2 * per, *B = b + ct * 2 * per;
    const u64 a0 = A[r], a1 = A[per + r], b0 = B[r], b1 = B[per + r];
    u64 *O = out + ct * 3 * per;
    O[r] = mul_mod(a0, b0, p);
    u128w s = mul_wide(a0, b1);
    acc_wide(s, mul_wide(a1, b0));
    const u64 t = redc(s, p.q, p.qneg);
    O[per + r] = redc(mul_wide(t, p.r2), p.q, p.qneg);
    O[2 * per + r] = mul_mod(a1, b1, p);
}

// ModUp base conversion of digit blockIdx.y of ciphertext blockIdx.z, with the
// digit's own limbs (NTT domain, from d) copied into their positions.
template <int MAXIN>
__global__ __launch_bounds__(EW_THREADS) void k_bconv_up_list(const u64 *coef, long coef_stride, const u64 *d, long d_stride,
                                                              u64 *ext, long ext_stride, long dig_stride, int logN,
                                                              int alpha, int nP, int nQ, const ListCt *cts,
                                                              const PrimeC *pc)
{
    __shared__ Half30 tab[BCONV_TAB(MAXIN)];
    const size_t N = (size_t)1 << logN;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int ct = blockIdx.z, j = blockIdx.y;
    const ListCt C = cts[ct];
    const int L1 = C.level + 1, E = L1 + nP, beta = (L1 + alpha - 1) / alpha;
    if (j >= beta) return;
    const int lo = j * alpha, n_in = min(alpha, L1 - lo), n_out = E - n_in;
    const u64 *Aj = C.A + j * alpha, *Ashj = C.Ash + j * alpha, *Mj = C.M + (size_t)j * alpha * E;
    // zero columns past n_in: every output sums all MAXIN terms without branches
    for (int w = threadIdx.x; w < MAXIN * n_out; w += EW_THREADS) {
        const int o = w / MAXIN, i = w % MAXIN;
        tab[w] = i < n_in ? split30(Mj[(size_t)i * E + o]) : Half30{0, 0};
    }
    __syncthreads();
    if (k >= N) return;
    const u64 *x = coef + ct * coef_stride + (size_t)lo * N;
    const u64 *own = d + ct * d_stride + (size_t)lo * N;
    u64 *dst = ext + ct * ext_stride + (size_t)j * dig_stride;
    Half30 yh[MAXIN];
#pragma unroll
    for (int i = 0; i < MAXIN; i++) {
        yh[i] = Half30{0, 0};
        if (i < n_in) {
            yh[i] = split30(shoup(x[(size_t)i * N + k], Aj[i], Ashj[i], pc[lo + i].q));
            dst[(size_t)(lo + i) * N + k] = own[(size_t)i * N + k];
        }
    }
    for (int o = 0; o < n_out; o++) {
        const int pos = o < lo ? o : o + n_in;
        const int pr = pos < L1 ? pos : nQ + pos - L1;
        const PrimeC p = pc[pr];
        Acc4 acc;
#pragma unroll
        for (int i = 0; i < MAXIN; i++)
            wa::acc4(acc, yh[i], tab[o * MAXIN + i]);
        dst[(size_t)pos * N + k] = redc(acc4_sum(acc), p.q, p.qneg);
    }
}

// ModDown base conversion P -> Q_l of polynomial blockIdx.z (ciphertext z / 2);
// tp: [2 count][nP][N], conv: polynomial stride conv_stride.
template <int MAXIN>
__global__ __launch_bounds__(EW_THREADS) void k_bconv_down_list(const u64 *tp, u64 *conv, long conv_stride, int logN,
                                                                int nP, int nQ, const ListCt *cts, const u64 *A,
                                                                const u64 *Ash, const u64 *M, const PrimeC *pc)
{
    __shared__ Half30 tab[BCONV_TAB(MAXIN)];
    const size_t N = (size_t)1 << logN;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int poly = blockIdx.z;
    const int n_out = cts[poly / 2].level + 1;
    // zero columns past nP: every output sums all MAXIN terms without branches
    for (int w = threadIdx.x; w < MAXIN * n_out; w += EW_THREADS) {
        const int o = w / MAXIN, i = w % MAXIN;
        tab[w] = i < nP ? split30(M[(size_t)i * nQ + o]) : Half30{0, 0};
    }
    __syncthreads();
    if (k >= N) return;
    const u64 *x = tp + (size_t)poly * nP * N;
    u64 *dst = conv + poly * conv_stride;
    Half30 yh[MAXIN];
#pragma unroll
    for (int i = 0; i < MAXIN; i++) {
        yh[i] = Half30{0, 0};
        if (i < nP) yh[i] = split30(shoup(x[(size_t)i * N + k], A[i], Ash[i], pc[nQ + i].q));
    }
    for (int o = 0; o < n_out; o++) {
        const PrimeC p = pc[o];
        Acc4 acc;
#pragma unroll
        for (int i = 0; i < MAXIN; i++)
            wa::acc4(acc, yh[i], tab[o * MAXIN + i]);
        dst[(size_t)o * N + k] = redc(acc4_sum(acc), p.q, p.qneg);
    }
}

// Special-prime part of the relinearisation inner product (no automorphism).
template <int BETA>
__global__ __launch_bounds__(EW_THREADS) void k_ip_p_list(const u64 *__restrict__ ext, long ext_stride, long dig_stride,
                                                          const u64 *__restrict__ key, u64 *__restrict__ tp, int logN,
                                                          int alpha, int nT, int nQ, int nP, int count, int cpc,
                                                          const ListCt *cts, const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t k = 2 * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    const int t = blockIdx.y;
    const int ct0 = blockIdx.z * cpc, ct1 = min(count, ct0 + cpc);
    if (k >= N) return;
    const int pr = nQ + t;
    const PrimeC p = pc[pr];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
        kb[j] = ld2(key + (((size_t)j * 2 + 0) * nT + pr) * N + k);
        ka[j] = ld2(key + (((size_t)j * 2 + 1) * nT + pr) * N + k);
    }
    for (int ct = ct0; ct < ct1; ct++) {
        const int L1 = cts[ct].level + 1, beta = (L1 + alpha - 1) / alpha;
        const u64 *x = ext + ct * ext_stride + (size_t)(L1 + t) * N + k;
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++)
            if (j < beta) {
                const u64x2 dd = ld2(x + (size_t)j * dig_stride);
                acc_wide(s0, mul_wide(dd.x, kb[j].x));
                acc_wide(t0, mul_wide(dd.y, kb[j].y));
                acc_wide(s1, mul_wide(dd.x, ka[j].x));
                acc_wide(t1, mul_wide(dd.y, ka[j].y));
            }
        u64 *o = tp + ((size_t)ct * 2 * nP + t) * N + k;
        st2(o, redc(s0, p.q, p.qneg), redc(t0, p.q, p.qneg));
        st2(o + (size_t)nP * N, redc(s1, p.q, p.qneg), redc(t1, p.q, p.qneg));
    }
}

// Q positions of the relinearisation: out = (IP - conv) * P^-1 + (d0, d1);
// conv, add and out have polynomial stride `per` inside a ciphertext.
template <int BETA>
__global__ __launch_bounds__(EW_THREADS) void k_moddown_ip_list(const u64 *__restrict__ ext, long ext_stride,
                                                                long dig_stride, const u64 *__restrict__ key,
                                                                const u64 *__restrict__ conv, long conv_stride, long per,
                                                                const u64 *__restrict__ add, long add_stride,
                                                                u64 *__restrict__ out, long out_stride, int logN,
                                                                int alpha, int nT, int count, int cpc,
                                                                const ListCt *cts, const u64 *Pinv, const u64 *Pinv_sh,
                                                                const PrimeC *pc)
{
    const size_t N = (size_t)1 << logN;
    const size_t k = 2 * ((size_t)blockIdx.x * EW_THREADS + threadIdx.x);
    const int i = blockIdx.y;
    const int ct0 = blockIdx.z * cpc, ct1 = min(count, ct0 + cpc);
    if (k >= N) return;
    const PrimeC p = pc[i];
    const u64 pinv = Pinv[i], pinv_sh = Pinv_sh[i];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
        kb[j] = ld2(key + (((size_t)j * 2 + 0) * nT + i) * N + k);
        ka[j] = ld2(key + (((size_t)j * 2 + 1) * nT + i) * N + k);
    }
    const size_t li = (size_t)i * N + k;
    for (int ct = ct0; ct < ct1; ct++) {
        const int L1 = cts[ct].level + 1;
        if (i >= L1) continue;
        const int beta = (L1 + alpha - 1) / alpha;
        const u64 *x = ext + ct * ext_stride + li;
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++)
            if (j < beta) {
                const u64x2 dd = ld2(x + (size_t)j * dig_stride);
                acc_wide(s0, mul_wide(dd.x, kb[j].x));
                acc_wide(t0, mul_wide(dd.y, kb[j].y));
                acc_wide(s1, mul_wide(dd.x, ka[j].x));
                acc_wide(t1, mul_wide(dd.y, ka[j].y));
            }
        const u64 *cv = conv + ct * conv_stride + li;
        const u64x2 c0 = ld2(cv), c1 = ld2(cv + per);
        const u64 *ad = add + ct * add_stride + li;
        const u64x2 a0 = ld2(ad), a1 = ld2(ad + per);
        const u64 v0 = add_mod(shoup(sub_mod(redc(s0, p.q, p.qneg), c0.x, p.q), pinv, pinv_sh, p.q), a0.x, p.q);
        const u64 w0 = add_mod(shoup(sub_mod(redc(t0, p.q, p.qneg), c0.y, p.q), pinv, pinv_sh, p.q), a0.y, p.q);
        const u64 v1 = add_mod(shoup(sub_mod(redc(s1, p.q, p.qneg), c1.x, p.q), pinv, pinv_sh, p.q), a1.x, p.q);
        const u64 w1 = add_mod(shoup(sub_mod(redc(t1, p.q, p.qneg), c1.y, p.q), pinv, pinv_sh, p.q), a1.y, p.q);
        u64 *o = out + ct * out_stride + li;
        st2(o, v0, w0);
        st2(o + per, v1, w1);
    }
}

// rescale: last[poly] = limb level_i of polynomial poly (coefficient pass follows)
__global__ void k_rescale_last_list(const u64 *in, long in_poly_stride, u64 *last, int logN, int count,
                                    const ListCt *cts)
{
    const size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= ((size_t)2 * count << logN)) return;
    const size_t poly = i >> logN, k = i & (((size_t)1 << logN) - 1);
    last[i] = in[poly * in_poly_stride + ((size_t)cts[poly / 2].level << logN) + k];
}

// lifted[poly][limb] for limb < level_i (layout [2 count][Lm][N])
__global__ void k_rescale_lift_list(const u64 *last, u64 *lifted, int logN, int Lm, int count, const ListCt *cts,
                                    const PrimeC *pc, const u64 *rs_qmod, int nQ)
{
    const size_t N = (size_t)1 << logN;
    const size_t per = (size_t)Lm * N;
    const size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= per * 2 * count) return;
    const size_t poly = i / per, r = i % per;
    const int limb = (int)(r >> logN), l = cts[poly / 2].level;
    if (limb >= l) return;
    const size_t k = r & (N - 1);
    const PrimeC p = pc[limb];
    const u64 ql = pc[l].q;
    const u64 x = last[poly * N + k];
    const u64 xm = shoup(x, 1, p.one_sh, p.q);
    lifted[i] = (x <= (ql - 1) / 2) ? xm : sub_mod(xm, rs_qmod[(size_t)l * nQ + limb], p.q);
}

// out[poly][limb] = (in - lifted) * q_l^-1 for limb < level_i
__global__ void k_rescale_finish_list(const u64 *in, long in_poly_stride, const u64 *lifted, u64 *out,
                                      long out_poly_stride, int logN, int Lm, int count, const ListCt *cts,
                                      const PrimeC *pc, const u64 *rs_inv, const u64 *rs_inv_sh, int nQ)
{
    const size_t N = (size_t)1 << logN;
    const size_t per = (size_t)Lm * N;
    const size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= per * 2 * count) return;
    const size_t poly = i / per, r = i % per;
    const int limb = (int)(r >> logN), l = cts[poly / 2].level;
    if (limb >= l) return;
    const u64 q = pc[limb].q;
    const u64 x = in[poly * in_poly_stride + r];
    const size_t ti = (size_t)l * nQ + limb;
    out[poly * out_poly_stride + r] = shoup(sub_mod(x, lifted[i], q), rs_inv[ti], rs_inv_sh[ti], q);
}

void tensor_list_launch(const rbk_ctx_impl *c, const u64 *a, const u64 *b, u64 *out, int Lm, int count,
                        const ListCt *cts, hipStream_t st)
{
    const size_t total = (size_t)count * (Lm + 1) * c->N;
    kt_begin(c, KC_TENSOR, st);
    hipLaunchKernelGGL(k_tensor_list, dim3((unsigned)((total + EW_THREADS - 1) / EW_THREADS)), dim3(EW_THREADS), 0, st, a,
                       b, out, c->logN, Lm + 1, count, cts, c->d_pc);
    kt_end(c, KC_TENSOR, 7.0 * total * sizeof(u64), st);
}

void bconv_up_list_launch(const rbk_ctx_impl *c, const u64 *coef, long coef_stride, const u64 *d, long d_stride, u64 *ext,
                          long ext_stride, long dig_stride, int Lm, int count, const ListCt *cts, hipStream_t st)
{
    const int betam = (Lm + 1 + c->alpha - 1) / c->alpha;
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), betam, count);
    kt_begin(c, KC_BCONV_UP, st);
    if (c->alpha <= 4)
        hipLaunchKernelGGL((k_bconv_up_list<4>), grid, dim3(EW_THREADS), 0, st, coef, coef_stride, d, d_stride, ext,
                           ext_stride, dig_stride, c->logN, c->alpha, c->nP, c->nQ, cts, c->d_pc);
    else if (c->alpha <= 8)
        hipLaunchKernelGGL((k_bconv_up_list<8>), grid, dim3(EW_THREADS), 0, st, coef, coef_stride, d, d_stride, ext,
                           ext_stride, dig_stride, c->logN, c->alpha, c->nP, c->nQ, cts, c->d_pc);
    else if (c->alpha <= 12)
        hipLaunchKernelGGL((k_bconv_up_list<12>), grid, dim3(EW_THREADS), 0, st, coef, coef_stride, d, d_stride, ext,
                           ext_stride, dig_stride, c->logN, c->alpha, c->nP, c->nQ, cts, c->d_pc);
    else
        hipLaunchKernelGGL((k_bconv_up_list<16>), grid, dim3(EW_THREADS), 0, st, coef, coef_stride, d, d_stride, ext,
                           ext_stride, dig_stride, c->logN, c->alpha, c->nP, c->nQ, cts, c->d_pc);
    kt_end(c, KC_BCONV_UP, (double)count * betam * (Lm + 1 + c->nP) * c->N * sizeof(u64), st);
}

void bconv_down_list_launch(const rbk_ctx_impl *c, const u64 *tp, u64 *conv, long conv_stride, int Lm, int count,
                            const ListCt *cts, hipStream_t st)
{
    dim3 grid((unsigned)((c->N + EW_THREADS - 1) / EW_THREADS), 1, 2 * count);
    kt_begin(c, KC_BCONV_DOWN, st);
    if (c->nP <= 4)
        hipLaunchKernelGGL((k_bconv_down_list<4>), grid, dim3(EW_THREADS), 0, st, tp, conv, conv_stride, c->logN, c->nP,
                           c->nQ, cts, c->d_md_A, c->d_md_Ash, c->d_md_M, c->d_pc);
    else if (c->nP <= 8)
        hipLaunchKernelGGL((k_bconv_down_list<8>), grid, dim3(EW_THREADS), 0, st, tp, conv, conv_stride, c->logN, c->nP,
                           c->nQ, cts, c->d_md_A, c->d_md_Ash, c->d_md_M, c->d_pc);
    else if (c->nP <= 12)
        hipLaunchKernelGGL((k_bconv_down_list<12>), grid, dim3(EW_THREADS), 0, st, tp, conv, conv_stride, c->logN, c->nP,
                           c->nQ, cts, c->d_md_A, c->d_md_Ash, c->d_md_M, c->d_pc);
    else
        hipLaunchKernelGGL((k_bconv_down_list<16>), grid, dim3(EW_THREADS), 0, st, tp, conv, conv_stride, c->logN, c->nP,
                           c->nQ, cts, c->d_md_A, c->d_md_Ash, c->d_md_M, c->d_pc);
    kt_end(c, KC_BCONV_DOWN, 2.0 * count * (c->nP + Lm + 1) * c->N * sizeof(u64), st);
}

void ip_p_list_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, long dig_stride, const u64 *key, u64 *tp,
                      int Lm, int count, const ListCt *cts, hipStream_t st)
{
    const int betam = (Lm + 1 + c->alpha - 1) / c->alpha;
    const int cpc = c->ip_cpc;
    dim3 grid((unsigned)((c->N / 2 + EW_THREADS - 1) / EW_THREADS), c->nP, (count + cpc - 1) / cpc);
    kt_begin(c, KC_IP_P, st);
#define IPL_CASE(B)                                                                                                \
    case B:                                                                                                         \
        hipLaunchKernelGGL(k_ip_p_list<B>, grid, dim3(EW_THREADS), 0, st, ext, ext_stride, dig_stride, key, tp, c->logN, \
                           c->alpha, c->nT, c->nQ, c->nP, count, cpc, cts, c->d_pc);                               \
        break;
    switch (betam) { IPL_CASE(1) IPL_CASE(2) IPL_CASE(3) IPL_CASE(4) IPL_CASE(5) IPL_CASE(6) IPL_CASE(7) default: IPL_CASE(8) }
#undef IPL_CASE
    kt_end(c, KC_IP_P, ((double)count * betam * c->nP + 2.0 * betam * c->nP + 2.0 * count * c->nP) * c->N * sizeof(u64), st);
}

void moddown_ip_list_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, long dig_stride, const u64 *key,
                            const u64 *conv, long conv_stride, long per, const u64 *add, long add_stride, u64 *out,
                            long out_stride, int Lm, int count, const ListCt *cts, hipStream_t st)
{
    const int betam = (Lm + 1 + c->alpha - 1) / c->alpha;
    const int cpc = c->ip_cpc;
    dim3 grid((unsigned)((c->N / 2 + EW_THREADS - 1) / EW_THREADS), Lm + 1, (count + cpc - 1) / cpc);
    kt_begin(c, KC_MODDOWN_IP, st);
#define MDL_CASE(B)                                                                                                   \
    case B:                                                                                                            \
        hipLaunchKernelGGL(k_moddown_ip_list<B>, grid, dim3(EW_THREADS), 0, st, ext, ext_stride, dig_stride, key, conv,   \
                           conv_stride, per, add, add_stride, out, out_stride, c->logN, c->alpha, c->nT, count, cpc, cts, \
                           c->d_Pinv, c->d_Pinv_sh, c->d_pc);                                                          \
        break;
    switch (betam) { MDL_CASE(1) MDL_CASE(2) MDL_CASE(3) MDL_CASE(4) MDL_CASE(5) MDL_CASE(6) MDL_CASE(7) default: MDL_CASE(8) }
#undef MDL_CASE
    kt_end(c, KC_MODDOWN_IP, ((double)count * (Lm + 1) * (betam + 6) + 2.0 * betam * (Lm + 1)) * c->N * sizeof(u64), st);
}

void rescale_list_launch(const rbk_ctx_impl *c, int step, const u64 *in, long in_poly_stride, u64 *last, u64 *lifted,
                         u64 *out, long out_poly_stride, int Lm, int count, const ListCt *cts, hipStream_t st)
{
    const size_t N = c->N;
    if (step == 0) {
        const size_t total = (size_t)2 * count * N;
        hipLaunchKernelGGL(k_rescale_last_list, dim3((unsigned)((total + EW_THREADS - 1) / EW_THREADS)), dim3(EW_THREADS),
                           0, st, in, in_poly_stride, last, c->logN, count, cts);
        return;
    }
    const size_t total = (size_t)2 * count * Lm * N;
    if (total == 0) return;
    dim3 grid((unsigned)((total + EW_THREADS - 1) / EW_THREADS));
    kt_begin(c, KC_RESCALE, st);
    if (step == 1)
        hipLaunchKernelGGL(k_rescale_lift_list, grid, dim3(EW_THREADS), 0, st, last, lifted, c->logN, Lm, count, cts,
                           c->d_pc, c->d_rs_qmod, c->nQ);
    else
        hipLaunchKernelGGL(k_rescale_finish_list, grid, dim3(EW_THREADS), 0, st, in, in_poly_stride, lifted, out,
                           out_poly_stride, c->logN, Lm, count, cts, c->d_pc, c->d_rs_inv, c->d_rs_inv_sh, c->nQ);
    kt_end(c, KC_RESCALE, 3.0 * total * sizeof(u64), st);
}
