// Multiplication with relinearisation and rescale (paper Section 3: mult
// followed by "switching to the next prime") of ciphertexts that belong to
// DIFFERENT contexts -- ring degree, modulus chain, special primes,
// relinearisation key -- in one set of launches.
//
// Every ciphertext brings its own descriptor (its context's prime constants,
// base-conversion tables, rescale tables and key, its buffers); a kernel's
// grid is the concatenation of the ciphertexts' block ranges, and a block
// finds its ciphertext by binary search in a prefix table.  The transforms
// are descriptor-list NTTs over exactly the limbs each ciphertext owns (the
// list transform already mixes ring degrees and primes).  The steps and
// their arithmetic are those of the single-context pipeline: tensor product,
// ModUp of d2 (fast base conversion of each digit), the key inner product on
// the special primes, ModDown (base conversion P -> Q, then
// (IP - conv) P^-1 + (d0, d1)), and the rescale by each ciphertext's own
// last prime with a centred lift.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"
#include "wide_arith.hpp"

namespace {

constexpr int MT = 256;
using wa::Acc4;
using wa::Half30;
using wa::split30;

__device__ __forceinline__ u128w sum4(const Acc4 &a)
{
    const wa::Wide w = wa::acc4_value(a);
    u128w t;
    t.lo = w.lo;
    t.hi = w.hi;
    return t;
}

// One ciphertext of a mixed batch: its context's tables and key, its inputs,
// output and workspace (all device pointers).
struct MultiCt {
    int logN, level, nQ, nP, nT, alpha;
    const PrimeC *pc;
    const u64 *upA, *upAsh, *upM;   // ModUp tables of this level: [beta][alpha], [beta][alpha][E]
    const u64 *mdA, *mdAsh, *mdM;   // ModDown P -> Q: [nP], [nP][nQ]
    const u64 *Pinv, *Pinv_sh;      // P^-1 mod q_i
    const u64 *rs_inv, *rs_inv_sh, *rs_qmod;  // [nQ][nQ] rescale tables
    const u64 *key;                 // relinearisation key [beta][2][nT][N]
    const u64 *a, *b;               // inputs [2][l+1][N]
    u64 *out;                       // output [2][l][N]
    u64 *d, *coef, *ext, *tp, *conv, *mr, *last, *lifted;  // workspace
};

// index of the ciphertext that owns block b: prefix[i] is its first block
__device__ __forceinline__ int owner(const int *prefix, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Up to MG ciphertexts of one context whose key inner products share their
// key-word loads: one thread serves one position of one limb for all of them
constexpr int MG = 8;
struct MultiGroup {
    int n, beta_max, l1_max;
    int ct[MG];
};

// (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1); d2 also into coef (its
// coefficient form is computed in place there)
__global__ __launch_bounds__(MT) void k_tensor_multi(const MultiCt *cts, const int *prefix, int n)
{
    const int ct = owner(prefix, n, blockIdx.x);
    const MultiCt &C = cts[ct];
    const size_t N = (size_t)1 << C.logN, per = (size_t)(C.level + 1) * N;
    const size_t r = (size_t)(blockIdx.x - prefix[ct]) * MT + threadIdx.x;
    if (r >= per) return;
    const PrimeC p = C.pc[r >> C.logN];
    const u64 a0 = C.a[r], a1 = C.a[per + r], b0 = C.b[r], b1 = C.b[per + r];
    C.d[r] = mul_mod(a0, b0, p);
    u128w s = mul_wide(a0, b1);
    acc_wide(s, mul_wide(a1, b0));
    const u64 t = redc(s, p.q, p.qneg);
    C.d[per + r] = redc(mul_wide(t, p.r2), p.q, p.qneg);
    const u64 d2 = mul_mod(a1, b1, p);
    C.d[2 * per + r] = d2;
    C.coef[r] = d2;
}

// ModUp base conversion of one digit (blocks per digit = ceil(N / MT)); the
// digit's own limbs are copied from d2 (NTT domain)
template <int MAXIN>
__global__ __launch_bounds__(MT) void k_bconv_up_multi(const MultiCt *cts, const int *prefix, int n)
{
    __shared__ Half30 tab[RBK_MAX_PRIMES * MAXIN];
    const int ct = owner(prefix, n, blockIdx.x);
    const MultiCt &C = cts[ct];
    const size_t N = (size_t)1 << C.logN;
    const int L1 = C.level + 1, E = L1 + C.nP, alpha = C.alpha;
    const int bpd = (int)((N + MT - 1) / MT);
    const int lb = blockIdx.x - prefix[ct];
    const int j = lb / bpd;
    const size_t k = (size_t)(lb % bpd) * MT + threadIdx.x;
    const int lo = j * alpha, n_in = min(alpha, L1 - lo), n_out = E - n_in;
    const u64 *Aj = C.upA + (size_t)j * alpha, *Ashj = C.upAsh + (size_t)j * alpha;
    const u64 *Mj = C.upM + (size_t)j * alpha * E;
    for (int w = threadIdx.x; w < MAXIN * n_out; w += MT) {
        const int o = w / MAXIN, i = w % MAXIN;
        tab[w] = i < n_in ? split30(Mj[(size_t)i * E + o]) : Half30{0, 0};
    }
    __syncthreads();
    if (k >= N) return;
    const u64 *x = C.coef + (size_t)lo * N;
    const u64 *own = C.d + (size_t)2 * L1 * N + (size_t)lo * N;
    u64 *dst = C.ext + (size_t)j * E * N;
    Half30 yh[MAXIN];
#pragma unroll
    for (int i = 0; i < MAXIN; i++) {
        yh[i] = Half30{0, 0};
        if (i < n_in) {
            yh[i] = split30(shoup(x[(size_t)i * N + k], Aj[i], Ashj[i], C.pc[lo + i].q));
            dst[(size_t)(lo + i) * N + k] = own[(size_t)i * N + k];
        }
    }
    for (int o = 0; o < n_out; o++) {
        const int pos = o < lo ? o : o + n_in;
        const int pr = pos < L1 ? pos : C.nQ + pos - L1;
        const PrimeC p = C.pc[pr];
        Acc4 acc;
#pragma unroll
        for (int i = 0; i < MAXIN; i++)
            wa::acc4(acc, yh[i], tab[o * MAXIN + i]);
        dst[(size_t)pos * N + k] = redc(sum4(acc), p.q, p.qneg);
    }
}

// special-prime part of the key inner product, tp [2][nP][N]; per group of
// ciphertexts one block range of ceil(N / 2 / MT) blocks per special prime,
// two coefficients a thread, the key words loaded once for the group
template <int BETA>
__global__ __launch_bounds__(MT) void k_ip_p_multi(const MultiCt *cts, const MultiGroup *grp, const int *prefix, int n)
{
    const int gi = owner(prefix, n, blockIdx.x);
    const MultiGroup &G = grp[gi];
    const MultiCt &C0 = cts[G.ct[0]];
    const size_t N = (size_t)1 << C0.logN;
    const int bpl = (int)((N / 2 + MT - 1) / MT);
    const int lb = blockIdx.x - prefix[gi];
    const int t = lb / bpl;
    const size_t k = 2 * ((size_t)(lb % bpl) * MT + threadIdx.x);
    if (k >= N) return;
    const int pr = C0.nQ + t;
    const PrimeC p = C0.pc[pr];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++)
        if (j < G.beta_max) {
            kb[j] = ld2(C0.key + (((size_t)j * 2 + 0) * C0.nT + pr) * N + k);
            ka[j] = ld2(C0.key + (((size_t)j * 2 + 1) * C0.nT + pr) * N + k);
        }
    for (int r = 0; r < G.n; r++) {
        const MultiCt &C = cts[G.ct[r]];
        const int L1 = C.level + 1, E = L1 + C.nP, beta = (L1 + C.alpha - 1) / C.alpha;
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++)
            if (j < beta) {
                const u64x2 dd = ld2(C.ext + ((size_t)j * E + L1 + t) * N + k);
                acc_wide(s0, mul_wide(dd.x, kb[j].x));
                acc_wide(t0, mul_wide(dd.y, kb[j].y));
                acc_wide(s1, mul_wide(dd.x, ka[j].x));
                acc_wide(t1, mul_wide(dd.y, ka[j].y));
            }
        u64 *o = C.tp + (size_t)t * N + k;
        st2(o, redc(s0, p.q, p.qneg), redc(t0, p.q, p.qneg));
        st2(o + (size_t)C.nP * N, redc(s1, p.q, p.qneg), redc(t1, p.q, p.qneg));
    }
}

// ModDown base conversion P -> Q_l of one polynomial (blocks per polynomial = ceil(N / MT))
template <int MAXIN>
__global__ __launch_bounds__(MT) void k_bconv_down_multi(const MultiCt *cts, const int *prefix, int n)
{
    __shared__ Half30 tab[RBK_MAX_PRIMES * MAXIN];
    const int ct = owner(prefix, n, blockIdx.x);
    const MultiCt &C = cts[ct];
    const size_t N = (size_t)1 << C.logN;
    const int L1 = C.level + 1, nP = C.nP;
    const int bpp = (int)((N + MT - 1) / MT);
    const int lb = blockIdx.x - prefix[ct];
    const int poly = lb / bpp;
    const size_t k = (size_t)(lb % bpp) * MT + threadIdx.x;
    for (int w = threadIdx.x; w < MAXIN * L1; w += MT) {
        const int o = w / MAXIN, i = w % MAXIN;
        tab[w] = i < nP ? split30(C.mdM[(size_t)i * C.nQ + o]) : Half30{0, 0};
    }
    __syncthreads();
    if (k >= N) return;
    const u64 *x = C.tp + (size_t)poly * nP * N;
    u64 *dst = C.conv + (size_t)poly * L1 * N;
    Half30 yh[MAXIN];
#pragma unroll
    for (int i = 0; i < MAXIN; i++) {
        yh[i] = Half30{0, 0};
        if (i < nP) yh[i] = split30(shoup(x[(size_t)i * N + k], C.mdA[i], C.mdAsh[i], C.pc[C.nQ + i].q));
    }
    for (int o = 0; o < L1; o++) {
        const PrimeC p = C.pc[o];
        Acc4 acc;
#pragma unroll
        for (int i = 0; i < MAXIN; i++)
            wa::acc4(acc, yh[i], tab[o * MAXIN + i]);
        dst[(size_t)o * N + k] = redc(sum4(acc), p.q, p.qneg);
    }
}

// Q positions: mr = (IP - conv) P^-1 + (d0, d1); per group of ciphertexts one
// block range per limb (up to the group's highest level), the key words
// loaded once for the ciphertexts of the group that have the limb
template <int BETA>
__global__ __launch_bounds__(MT) void k_moddown_ip_multi(const MultiCt *cts, const MultiGroup *grp, const int *prefix,
                                                         int n)
{
    const int gi = owner(prefix, n, blockIdx.x);
    const MultiGroup &G = grp[gi];
    const MultiCt &C0 = cts[G.ct[0]];
    const size_t N = (size_t)1 << C0.logN;
    const int bpl = (int)((N / 2 + MT - 1) / MT);
    const int lb = blockIdx.x - prefix[gi];
    const int i = lb / bpl;
    const size_t k = 2 * ((size_t)(lb % bpl) * MT + threadIdx.x);
    if (k >= N) return;
    const PrimeC p = C0.pc[i];
    const u64 pinv = C0.Pinv[i], pinv_sh = C0.Pinv_sh[i];
    u64x2 kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++)
        if (j < G.beta_max) {
            kb[j] = ld2(C0.key + (((size_t)j * 2 + 0) * C0.nT + i) * N + k);
            ka[j] = ld2(C0.key + (((size_t)j * 2 + 1) * C0.nT + i) * N + k);
        }
    for (int r = 0; r < G.n; r++) {
        const MultiCt &C = cts[G.ct[r]];
        const int L1 = C.level + 1, E = L1 + C.nP, beta = (L1 + C.alpha - 1) / C.alpha;
        if (i >= L1) continue;
        u128w s0 = {0, 0}, s1 = {0, 0}, t0 = {0, 0}, t1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++)
            if (j < beta) {
                const u64x2 dd = ld2(C.ext + ((size_t)j * E + i) * N + k);
                acc_wide(s0, mul_wide(dd.x, kb[j].x));
                acc_wide(t0, mul_wide(dd.y, kb[j].y));
                acc_wide(s1, mul_wide(dd.x, ka[j].x));
                acc_wide(t1, mul_wide(dd.y, ka[j].y));
            }
        const size_t li = (size_t)i * N + k, per = (size_t)L1 * N;
        const u64x2 c0 = ld2(C.conv + li), c1 = ld2(C.conv + per + li);
        const u64x2 a0 = ld2(C.d + li), a1 = ld2(C.d + per + li);
        const u64 v0 = add_mod(shoup(sub_mod(redc(s0, p.q, p.qneg), c0.x, p.q), pinv, pinv_sh, p.q), a0.x, p.q);
        const u64 w0 = add_mod(shoup(sub_mod(redc(t0, p.q, p.qneg), c0.y, p.q), pinv, pinv_sh, p.q), a0.y, p.q);
        const u64 v1 = add_mod(shoup(sub_mod(redc(s1, p.q, p.qneg), c1.x, p.q), pinv, pinv_sh, p.q), a1.x, p.q);
        const u64 w1 = add_mod(shoup(sub_mod(redc(t1, p.q, p.qneg), c1.y, p.q), pinv, pinv_sh, p.q), a1.y, p.q);
        st2(C.mr + li, v0, w0);
        st2(C.mr + per + li, v1, w1);
    }
}

// rescale step 0: last[poly] = limb l of mr (blocks per polynomial = ceil(N / MT))
__global__ __launch_bounds__(MT) void k_last_multi(const MultiCt *cts, const int *prefix, int n)
{
    const int ct = owner(prefix, n, blockIdx.x);
    const MultiCt &C = cts[ct];
    const size_t N = (size_t)1 << C.logN;
    const int bpp = (int)((N + MT - 1) / MT);
    const int lb = blockIdx.x - prefix[ct];
    const int poly = lb / bpp;
    const size_t k = (size_t)(lb % bpp) * MT + threadIdx.x;
    if (k >= N) return;
    C.last[(size_t)poly * N + k] = C.mr[((size_t)poly * (C.level + 1) + C.level) * N + k];
}

// rescale step 1 (STEP = 1): lifted [2][l][N] = centred lift of last to every
// lower prime; step 2 (STEP = 2): out = (mr - lifted) q_l^-1
template <int STEP>
__global__ __launch_bounds__(MT) void k_rescale_multi(const MultiCt *cts, const int *prefix, int n)
{
    const int ct = owner(prefix, n, blockIdx.x);
    const MultiCt &C = cts[ct];
    const int l = C.level;
    const size_t N = (size_t)1 << C.logN, per = (size_t)l * N;
    const size_t r = (size_t)(blockIdx.x - prefix[ct]) * MT + threadIdx.x;
    if (r >= 2 * per) return;
    const size_t poly = r / per, rr = r % per;
    const int limb = (int)(rr >> C.logN);
    const size_t k = rr & (N - 1);
    const PrimeC p = C.pc[limb];
    const size_t ti = (size_t)l * C.nQ + limb;
    if (STEP == 1) {
        const u64 ql = C.pc[l].q;
        const u64 x = C.last[poly * N + k];
        const u64 xm = shoup(x, 1, p.one_sh, p.q);
        C.lifted[r] = (x <= (ql - 1) / 2) ? xm : sub_mod(xm, C.rs_qmod[ti], p.q);
    } else {
        const u64 x = C.mr[(poly * (l + 1) + limb) * N + k];
        C.out[r] = shoup(sub_mod(x, C.lifted[r], p.q), C.rs_inv[ti], C.rs_inv_sh[ti], p.q);
    }
}

int round4(int x) { return x <= 4 ? 4 : x <= 8 ? 8 : x <= 12 ? 12 : 16; }

}  // namespace

extern "C" int rbk_mult_relin_rescale_multi(rbk_ctx *c, const rbk_mr_item *items, int n)
{
    if (!c || n < 0 || (n > 0 && !items)) return rbk_set_error(RBK_EINVAL, "bad argument");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "list calls cannot be captured");
    if (n == 0) return RBK_OK;
    int max_alpha = 1, max_np = 1, max_beta = 1;
    size_t words = 0;
    for (int i = 0; i < n; i++) {
        const rbk_ctx *ic = items[i].ctx;
        if (!ic || !items[i].d_a || !items[i].d_b || !items[i].d_out)
            return rbk_set_error(RBK_EINVAL, "null context or buffer in an item");
        if (ic->device != c->device) return rbk_set_error(RBK_EINVAL, "item context on another device");
        if (ic->nP < 1) return rbk_set_error(RBK_EUNSUPPORTED, "needs special primes (hybrid key switching)");
        if (!ic->relin.data) return rbk_set_error(RBK_ENOKEY, "relinearisation key not generated");
        const int l = items[i].level;
        if (l < 1 || l >= ic->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range (1..L)");
        const int r = ic->logN - ic->ntt_logC;
        const bool ntt_ok = ic->logN <= 12 || (ic->logN <= 16 && r >= 6 && r <= 8 && ic->ntt_logC >= 6 &&
                                              ic->ntt_logC <= 8);
        if (ic->logN < 4 || !ntt_ok)
            return rbk_set_error(RBK_EUNSUPPORTED, "ring degree not supported by the list transform (2^4..2^16)");
        const size_t N = ic->N, L1 = l + 1, E = L1 + ic->nP, beta = (L1 + ic->alpha - 1) / ic->alpha;
        if (ic->alpha > 16 || ic->nP > 16 || beta > 8)
            return rbk_set_error(RBK_EUNSUPPORTED, "at most 16 primes per digit, 16 special primes and 8 digits");
        if (ranges_overlap(items[i].d_a, 2 * L1 * N, items[i].d_out, 2 * (L1 - 1) * N) ||
            ranges_overlap(items[i].d_b, 2 * L1 * N, items[i].d_out, 2 * (L1 - 1) * N))
            return rbk_set_error(RBK_EINVAL, "inputs and output of an item overlap");
        max_alpha = std::max(max_alpha, ic->alpha);
        max_np = std::max(max_np, ic->nP);
        max_beta = std::max(max_beta, (int)beta);
        // d 3 L1, coef L1, ext beta E, tp 2 nP, conv 2 L1, mr 2 L1, last 2, lifted 2 l  (limbs of N)
        words += (3 * L1 + L1 + beta * E + 2 * ic->nP + 2 * L1 + 2 * L1 + 2 + 2 * (L1 - 1)) * N;
    }
    u64 *ws = ws_reserve(c, words);
    if (!ws) return rbk_set_error(RBK_ENOMEM, "device workspace allocation failed");

    std::vector<MultiCt> cts((size_t)n);
    std::vector<NttItem> l_coef, l_ext, l_tp, l_conv, l_last, l_lift;
    std::vector<int> p_ew(n + 1, 0), p_up(n + 1, 0), p_poly(n + 1, 0), p_rs(n + 1, 0);
    // groups of up to MG ciphertexts of one context (their key inner products
    // share the key-word loads), in the order the contexts first appear
    std::vector<MultiGroup> groups;
    {
        std::vector<std::pair<const rbk_ctx *, int>> open;   // context -> its group being filled
        for (int i = 0; i < n; i++) {
            const rbk_ctx *ic = items[i].ctx;
            int gi = -1;
            for (auto &o : open)
                if (o.first == ic && groups[o.second].n < MG) gi = o.second;
            if (gi < 0) {
                groups.push_back(MultiGroup{});
                gi = (int)groups.size() - 1;
                bool found = false;
                for (auto &o : open)
                    if (o.first == ic) {
                        o.second = gi;
                        found = true;
                    }
                if (!found) open.emplace_back(ic, gi);
            }
            MultiGroup &g = groups[gi];
            const int L1 = items[i].level + 1;
            g.ct[g.n++] = i;
            g.beta_max = std::max(g.beta_max, (L1 + ic->alpha - 1) / ic->alpha);
            g.l1_max = std::max(g.l1_max, L1);
        }
    }
    const int ng = (int)groups.size();
    std::vector<int> p_ipp(ng + 1, 0), p_mdip(ng + 1, 0);
    for (int gi = 0; gi < ng; gi++) {
        const rbk_ctx *ic = items[groups[gi].ct[0]].ctx;
        const int bH = (int)((ic->N / 2 + MT - 1) / MT);
        p_ipp[gi + 1] = p_ipp[gi] + ic->nP * bH;
        p_mdip[gi + 1] = p_mdip[gi] + groups[gi].l1_max * bH;
    }
    u64 *w = ws;
    for (int i = 0; i < n; i++) {
        rbk_ctx *ic = items[i].ctx;
        const int l = items[i].level, L1 = l + 1, E = L1 + ic->nP, beta = (L1 + ic->alpha - 1) / ic->alpha;
        const size_t N = ic->N;
        const ModUpTables &T = modup_tables(ic, l);
        if (!T.d_M) return rbk_set_error(RBK_ENOMEM, "ModUp tables");
        MultiCt &C = cts[i];
        C.logN = ic->logN;
        C.level = l;
        C.nQ = ic->nQ;
        C.nP = ic->nP;
        C.nT = ic->nT;
        C.alpha = ic->alpha;
        C.pc = ic->d_pc;
        C.upA = T.d_A;
        C.upAsh = T.d_Ash;
        C.upM = T.d_M;
        C.mdA = ic->d_md_A;
        C.mdAsh = ic->d_md_Ash;
        C.mdM = ic->d_md_M;
        C.Pinv = ic->d_Pinv;
        C.Pinv_sh = ic->d_Pinv_sh;
        C.rs_inv = ic->d_rs_inv;
        C.rs_inv_sh = ic->d_rs_inv_sh;
        C.rs_qmod = ic->d_rs_qmod;
        C.key = ic->relin.data;
        C.a = items[i].d_a;
        C.b = items[i].d_b;
        C.out = items[i].d_out;
        C.d = w;
        C.coef = C.d + 3 * (size_t)L1 * N;
        C.ext = C.coef + (size_t)L1 * N;
        C.tp = C.ext + (size_t)beta * E * N;
        C.conv = C.tp + 2 * (size_t)ic->nP * N;
        C.mr = C.conv + 2 * (size_t)L1 * N;
        C.last = C.mr + 2 * (size_t)L1 * N;
        C.lifted = C.last + 2 * N;
        w = C.lifted + 2 * (size_t)l * N;
        // block ranges of every kernel
        const int bN = (int)((N + MT - 1) / MT);
        p_ew[i + 1] = p_ew[i] + (int)(((size_t)L1 * N + MT - 1) / MT);
        p_up[i + 1] = p_up[i] + beta * bN;
        p_poly[i + 1] = p_poly[i] + 2 * bN;
        p_rs[i + 1] = p_rs[i] + (int)((2 * (size_t)l * N + MT - 1) / MT);
        // transforms: limbs each ciphertext owns
        auto item = [&](u64 *p, int prime) { return NttItem{p, ic->d_tabs, prime, ic->logN, ic->ntt_logC, 0}; };
        for (int limb = 0; limb < L1; limb++) l_coef.push_back(item(C.coef + (size_t)limb * N, limb));
        for (int j = 0; j < beta; j++) {
            const int lo = j * ic->alpha, hi = std::min(L1, lo + ic->alpha);
            for (int pos = 0; pos < E; pos++)
                if (pos < lo || pos >= hi)
                    l_ext.push_back(item(C.ext + ((size_t)j * E + pos) * N, pos < L1 ? pos : ic->nQ + pos - L1));
        }
        for (int p = 0; p < 2; p++) {
            for (int t = 0; t < ic->nP; t++) l_tp.push_back(item(C.tp + ((size_t)p * ic->nP + t) * N, ic->nQ + t));
            for (int limb = 0; limb < L1; limb++) l_conv.push_back(item(C.conv + ((size_t)p * L1 + limb) * N, limb));
            l_last.push_back(item(C.last + (size_t)p * N, l));
            for (int limb = 0; limb < l; limb++) l_lift.push_back(item(C.lifted + ((size_t)p * l + limb) * N, limb));
        }
        // method bytes of the key switch (the switched polynomial read, one written, the key words once)
        c->ks_bytes += 2.0 * L1 * N * 8.0 + (double)beta * 2.0 * E * N * 8.0;
        c->ks_units += 1;
    }
    DescBlob b;
    const size_t o_cts = b.put(cts.data(), cts.size());
    const size_t o_grp = b.put(groups.data(), groups.size());
    const size_t o_ew = b.put(p_ew.data(), p_ew.size()), o_up = b.put(p_up.data(), p_up.size());
    const size_t o_ipp = b.put(p_ipp.data(), p_ipp.size()), o_poly = b.put(p_poly.data(), p_poly.size());
    const size_t o_mdip = b.put(p_mdip.data(), p_mdip.size()), o_rs = b.put(p_rs.data(), p_rs.size());
    struct Packed {
        size_t items, p1, p2;
        int n, t1, t2;
    };
    auto pack = [&](const std::vector<NttItem> &v) {
        Packed P{0, 0, 0, (int)v.size(), 0, 0};
        std::vector<int> p1(v.size() + 1, 0), p2(v.size() + 1, 0);
        for (size_t i = 0; i < v.size(); i++) {
            p1[i + 1] = p1[i] + ntt_item_units(v[i].logN, true);
            p2[i + 1] = p2[i] + ntt_item_units(v[i].logN, false);
        }
        P.t1 = p1.back();
        P.t2 = p2.back();
        P.items = b.put(v.data(), v.size());
        P.p1 = b.put(p1.data(), p1.size());
        P.p2 = b.put(p2.data(), p2.size());
        return P;
    };
    const Packed P_coef = pack(l_coef), P_ext = pack(l_ext), P_tp = pack(l_tp), P_conv = pack(l_conv);
    const Packed P_last = pack(l_last), P_lift = pack(l_lift);
    int rc = RBK_OK;
    const char *dev = desc_upload(c, b, &rc);
    if (!dev) return rc;
    const MultiCt *dc = reinterpret_cast<const MultiCt *>(dev + o_cts);
    const MultiGroup *dg = reinterpret_cast<const MultiGroup *>(dev + o_grp);
    auto pre = [&](size_t o) { return reinterpret_cast<const int *>(dev + o); };
    hipStream_t st = c->stream;
    auto ntt = [&](const Packed &P, bool inverse) {
        if (P.n)
            ntt_list_launch(reinterpret_cast<const NttItem *>(dev + P.items), pre(P.p1), pre(P.p2), P.n, P.t1, P.t2,
                            inverse, st);
    };
    auto grid = [](const std::vector<int> &p) { return dim3((unsigned)p.back()); };

    kt_begin(c, KC_TENSOR, st);
    hipLaunchKernelGGL(k_tensor_multi, grid(p_ew), dim3(MT), 0, st, dc, pre(o_ew), n);
    kt_end(c, KC_TENSOR, 0.0, st);
    ntt(P_coef, true);
    kt_begin(c, KC_BCONV_UP, st);
    switch (round4(max_alpha)) {
    case 4: hipLaunchKernelGGL(k_bconv_up_multi<4>, grid(p_up), dim3(MT), 0, st, dc, pre(o_up), n); break;
    case 8: hipLaunchKernelGGL(k_bconv_up_multi<8>, grid(p_up), dim3(MT), 0, st, dc, pre(o_up), n); break;
    case 12: hipLaunchKernelGGL(k_bconv_up_multi<12>, grid(p_up), dim3(MT), 0, st, dc, pre(o_up), n); break;
    default: hipLaunchKernelGGL(k_bconv_up_multi<16>, grid(p_up), dim3(MT), 0, st, dc, pre(o_up), n); break;
    }
    kt_end(c, KC_BCONV_UP, 0.0, st);
    ntt(P_ext, false);
    kt_begin(c, KC_IP_P, st);
#define IPM(B) \
    case B: hipLaunchKernelGGL(k_ip_p_multi<B>, grid(p_ipp), dim3(MT), 0, st, dc, dg, pre(o_ipp), ng); break;
    switch (max_beta) { IPM(1) IPM(2) IPM(3) IPM(4) IPM(5) IPM(6) IPM(7) default: IPM(8) }
#undef IPM
    kt_end(c, KC_IP_P, 0.0, st);
    ntt(P_tp, true);
    kt_begin(c, KC_BCONV_DOWN, st);
    switch (round4(max_np)) {
    case 4: hipLaunchKernelGGL(k_bconv_down_multi<4>, grid(p_poly), dim3(MT), 0, st, dc, pre(o_poly), n); break;
    case 8: hipLaunchKernelGGL(k_bconv_down_multi<8>, grid(p_poly), dim3(MT), 0, st, dc, pre(o_poly), n); break;
    case 12: hipLaunchKernelGGL(k_bconv_down_multi<12>, grid(p_poly), dim3(MT), 0, st, dc, pre(o_poly), n); break;
    default: hipLaunchKernelGGL(k_bconv_down_multi<16>, grid(p_poly), dim3(MT), 0, st, dc, pre(o_poly), n); break;
    }
    kt_end(c, KC_BCONV_DOWN, 0.0, st);
    ntt(P_conv, false);
    kt_begin(c, KC_MODDOWN_IP, st);
#define MDM(B) \
    case B: hipLaunchKernelGGL(k_moddown_ip_multi<B>, grid(p_mdip), dim3(MT), 0, st, dc, dg, pre(o_mdip), ng); break;
    switch (max_beta) { MDM(1) MDM(2) MDM(3) MDM(4) MDM(5) MDM(6) MDM(7) default: MDM(8) }
#undef MDM
    kt_end(c, KC_MODDOWN_IP, 0.0, st);
    kt_begin(c, KC_RESCALE, st);
    hipLaunchKernelGGL(k_last_multi, grid(p_poly), dim3(MT), 0, st, dc, pre(o_poly), n);
    kt_end(c, KC_RESCALE, 0.0, st);
    ntt(P_last, true);
    kt_begin(c, KC_RESCALE, st);
    hipLaunchKernelGGL(k_rescale_multi<1>, grid(p_rs), dim3(MT), 0, st, dc, pre(o_rs), n);
    kt_end(c, KC_RESCALE, 0.0, st);
    ntt(P_lift, false);
    kt_begin(c, KC_RESCALE, st);
    hipLaunchKernelGGL(k_rescale_multi<2>, grid(p_rs), dim3(MT), 0, st, dc, pre(o_rs), n);
    kt_end(c, KC_RESCALE, 0.0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rbk_set_error(RBK_EDEVICE, hipGetErrorString(e));
    return RBK_OK;
}
