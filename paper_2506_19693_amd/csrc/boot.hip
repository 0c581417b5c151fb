// Approximate bootstrapping of full-slot ciphertexts (paper Section 3, last
// paragraph: encoding step, scaled-sine modular reduction, decoding step;
// Cheon-Han-Kim-Kim-Song 2018, Bossuat et al. 2021).
//
//   level-0 ct --(x 2^e)--> ModRaise --> CoeffToSlot (cts_levels BSGS
//   transforms) --> conjugation split --> EvalMod on re and im together
//   (Chebyshev interpolant of cos(2 pi ((K+1)u - 1/4)/2^r), r double angles)
//   --> recombine --> SlotToCoeff (stc_levels transforms)
//
// The plan (levels, scales, encoded diagonals, scalar constants) is built on
// the host from the parameters alone; its constants are listed in a fixed
// "plan order" so that another implementation's constants can be imported
// (rbk_boot_import) and the ciphertext arithmetic compared residue by residue.
// Every step runs on the device: the diagonals are encoded with the device
// encoder, and a batch of ciphertexts goes through each step in one launch
// (EvalMod runs the real and imaginary halves of the whole batch together).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

typedef std::complex<double> cd;
typedef std::map<long, std::vector<cd>> DiagMat;  // offset -> diagonal (length n)
typedef unsigned __int128 u128b;

struct BootLT {
    int level = 0, h0 = 1, n1 = 1;
    double Sd = 1, s_in = 1;
    struct E {
        int g, b, kk, plain;
    };
    std::vector<E> ents;
};

enum StepKind { ST_PROD = 0, ST_LEAF = 1, ST_GIANT = 2, ST_DBL = 3 };

struct BootStep {
    int kind = 0;
    int k = 0, a = 0, b = 0, cc = 0, lv = 0, sidx = -1;  // prod
    std::string reg;                                    // leaf / giant
    std::vector<std::pair<int, int>> terms;             // leaf: (power, scalar)
    int cidx = -1;                                      // leaf constant
    int m = 0, lp = 0, out = 0;                         // giant
};

struct BootPlan {
    rbk_boot_params prm{};
    int L = 0, level_evalmod = 0, level_stc = 0, level_out = 0, dref_log2 = 0;
    double s_A = 0, s_B = 0, s_E = 0, s_out = 0;
    std::vector<BootLT> cts, stc;
    std::vector<BootStep> prog;
    std::vector<int> plain_level;
    std::vector<u64 *> d_plain;  // NTT domain, [level+1][N]
    std::vector<int> scalar_level;
    std::vector<std::vector<u64>> scalars;  // residues [level+1]
    std::vector<int64_t> rots;
    // registers of earlier runs, with their capacities in words (kept for
    // later runs; a run takes any register at least as large as it needs)
    std::vector<std::pair<u64 *, size_t>> pool;
    u64 *rot_area = nullptr;  // hoisted baby rotations of a transform
    size_t rot_words = 0;
    // key-switching workspaces of the giant-step lanes (side streams)
    u64 *lane_ws[RBK_LANES] = {};
    size_t lane_ws_words[RBK_LANES] = {};
    // the scalars with Shoup quotients, [n_scalars][nQ][2], uploaded when they change
    u64 *d_scal = nullptr;
    bool scal_dirty = true;
};

// ---------------------------------------------------------------- host arithmetic

static u64 b_mul(u64 a, u64 b, u64 q) { return (u64)((u128b)a * b % q); }
static u64 b_pow(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = b_mul(r, b, q);
        b = b_mul(b, b, q);
    }
    return r;
}
static u64 b_shoup(u64 w, u64 q) { return (u64)(((u128b)w << 64) / q); }

// residue of the integer nearest to x (ties to even) modulo q; a double above
// 2^53 is an integer m 2^s with a 53-bit m.
static u64 round_mod(double x, u64 q)
{
    double r = std::nearbyint(x);
    if (r == 0) return 0;
    bool neg = r < 0;
    r = std::fabs(r);
    u64 v;
    if (r < 9007199254740992.0) {
        v = (u64)r % q;
    } else {
        int e;
        double f = std::frexp(r, &e);
        u64 m = (u64)std::ldexp(f, 53);
        v = b_mul(m % q, b_pow(2, (u64)(e - 53), q), q);
    }
    return (neg && v) ? q - v : v;
}

// ---------------------------------------------------------------- the decoding map

// Stage S_s (s = 1..log2 n): blocks of size n >> (s-1); inside a block of size
// 2h, out_j = v_j + T_l v_(j+h) and out_(j+h) = v_j - T_l v_(j+h), with
// T_l = zeta^(2^(s-1) 5^l mod M), zeta = exp(2 pi i / M), M = 4n.  The inverse
// stage is out_j = (v_j + v_(j+h))/2, out_(j+h) = (v_j - v_(j+h)) / (2 T_l).
static DiagMat stage_mat(long n, long M, int s, bool inv)
{
    const long size = n >> (s - 1), h = size / 2;
    std::vector<cd> T(h);
    u64 x = 1;
    for (long l = 0; l < h; l++) {
        u64 e = (x << (s - 1)) % (u64)M;
        T[l] = std::polar(1.0, 2.0 * M_PI * (double)e / (double)M);
        x = (x * 5) % (u64)M;
    }
    std::vector<cd> d0(n), dp(n, 0.0), dm(n, 0.0);
    for (long j = 0; j < n; j++) {
        long loc = j % size;
        bool top = loc < h;
        cd t = T[top ? loc : loc - h];
        if (!inv) {
            d0[j] = top ? cd(1.0) : -t;
            if (top) dp[j] = t;
            else dm[j] = 1.0;
        } else {
            d0[j] = top ? cd(0.5) : -0.5 / t;
            if (top) dp[j] = 0.5;
            else dm[j] = 0.5 / t;
        }
    }
    DiagMat A;
    A[0] = d0;
    auto addto = [&](long o, const std::vector<cd> &d) {
        auto it = A.find(o);
        if (it == A.end()) A[o] = d;
        else
            for (long j = 0; j < n; j++) it->second[j] += d[j];
    };
    addto(h % n, dp);
    addto(((-h) % n + n) % n, dm);
    return A;
}

// (A B)_(a+b)[j] += A_a[j] B_b[j+a]
static DiagMat mat_mul(const DiagMat &A, const DiagMat &B, long n)
{
    DiagMat C;
    for (auto &pa : A)
        for (auto &pb : B) {
            long o = (pa.first + pb.first) % n;
            auto &dst = C[o];
            if (dst.empty()) dst.assign(n, 0.0);
            const long a = pa.first;
            for (long j = 0; j < n; j++) dst[j] += pa.second[j] * pb.second[(j + a) % n];
        }
    return C;
}

static std::vector<std::vector<int>> stage_groups(int logn, int levels)
{
    std::vector<std::vector<int>> g;
    int base = logn / levels, extra = logn % levels, s = 1;
    for (int i = 0; i < levels; i++) {
        int cnt = base + (i < extra ? 1 : 0);
        std::vector<int> st;
        for (int k = 0; k < cnt; k++) st.push_back(s + k);
        s += cnt;
        g.push_back(st);
    }
    return g;
}

// ---------------------------------------------------------------- plan construction

static int plan_lt(rbk_ctx *c, BootPlan &P, const std::vector<std::vector<int>> &groups, bool inv, int level0, double s,
                   double fold, const std::vector<int> &drops, std::vector<BootLT> &out, double &s_end)
{
    const long n = (long)c->N / 2, M = 2 * (long)c->N;
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const std::vector<int> &st = groups[gi];
        std::vector<DiagMat> mats;
        for (int sidx : st) mats.push_back(stage_mat(n, M, sidx, inv));
        if (inv) std::reverse(mats.begin(), mats.end());
        DiagMat A = mats[0];
        for (size_t i = 1; i < mats.size(); i++) A = mat_mul(A, mats[i], n);
        if (gi == 0)
            for (auto &d : A)
                for (auto &v : d.second) v *= fold;
        BootLT lt;
        lt.level = level0 - (int)gi;
        lt.h0 = (int)(n >> st.back());
        const int k = (int)st.size();
        const long W = n / lt.h0;
        int kmin, kmax;
        if ((2L << k) - 1 <= W) {
            kmin = -((1 << k) - 1);
            kmax = (1 << k) - 1;
        } else {
            kmin = (int)(-W / 2);
            kmax = (int)(W / 2 - 1);
        }
        lt.n1 = 1 << ((k + 2) / 2);
        const u64 ql = c->mod[lt.level];
        lt.Sd = (double)ql * std::ldexp(1.0, -drops[gi]);
        lt.s_in = s;
        struct T3 {
            int g, b, kk;
        };
        std::vector<T3> order;
        for (int kk = kmin; kk <= kmax; kk++) {
            int g = (int)std::floor((double)kk / lt.n1);
            order.push_back({g, kk - g * lt.n1, kk});
        }
        std::sort(order.begin(), order.end(), [](const T3 &x, const T3 &y) { return x.g != y.g ? x.g < y.g : x.b < y.b; });
        std::vector<double> re(n), im(n);
        for (auto &t : order) {
            long o = (((long)t.kk * lt.h0) % n + n) % n;
            auto it = A.find(o);
            long shift = (long)t.g * lt.n1 * lt.h0;
            for (long j = 0; j < n; j++) {
                // vals = roll(diag, shift): vals[j] = diag[j - shift]
                cd v = it == A.end() ? cd(0.0) : it->second[(((j - shift) % n) + n) % n];
                re[j] = v.real();
                im[j] = v.imag();
            }
            u64 *d = nullptr;
            if (hipMalloc((void **)&d, (size_t)(lt.level + 1) * c->N * sizeof(u64)) != hipSuccess) return RBK_ENOMEM;
            P.d_plain.push_back(d);
            P.plain_level.push_back(lt.level);
            int rc = rbk_encode(c, re.data(), im.data(), (size_t)n, lt.level, lt.Sd, d);
            if (rc) return rc;
            lt.ents.push_back({t.g, t.b, t.kk, (int)P.d_plain.size() - 1});
        }
        out.push_back(lt);
        s = s * lt.Sd / (double)ql;
    }
    s_end = s;
    return RBK_OK;
}

static std::vector<double> cheb_coeffs(int K, int r, int degree)
{
    const int d1 = degree + 1;
    std::vector<double> f(d1), c(d1);
    for (int j = 0; j < d1; j++) {
        double u = std::cos(M_PI * (j + 0.5) / d1);
        f[j] = std::cos(2 * M_PI * ((K + 1) * u - 0.25) / (double)(1 << r));
    }
    for (int k = 0; k < d1; k++) {
        double acc = 0;
        for (int j = 0; j < d1; j++) acc += f[j] * std::cos(M_PI * k * (j + 0.5) / d1);
        c[k] = 2.0 / d1 * acc;
    }
    c[0] /= 2;
    return c;
}

static void cheb_split(const std::vector<double> &c, int m, std::vector<double> &q, std::vector<double> &r)
{
    const int d = (int)c.size() - 1;
    q.assign(d - m + 1, 0.0);
    r.assign(c.begin(), c.begin() + m);
    q[0] = c[m];
    for (int j = 1; j <= d - m; j++) {
        q[j] = 2 * c[m + j];
        r[m - j] -= c[m + j];
    }
}

static const int BABY = 8;

struct EvalPlanner {
    rbk_ctx *c;
    BootPlan &P;
    std::map<int, std::pair<int, double>> T;  // power -> (level, scale)
    std::vector<int> giants;

    int scalar(int level, double x)
    {
        std::vector<u64> r(level + 1);
        for (int i = 0; i <= level; i++) r[i] = round_mod(x, c->mod[i]);
        P.scalars.push_back(r);
        P.scalar_level.push_back(level);
        return (int)P.scalars.size() - 1;
    }

    void prod(int k, int a, int b, int cc)
    {
        auto ta = T[a], tb = T[b];
        int lv = std::min(ta.first, tb.first);
        double sp = ta.second * tb.second;
        BootStep st;
        st.kind = ST_PROD;
        st.k = k;
        st.a = a;
        st.b = b;
        st.cc = cc;
        st.lv = lv;
        st.sidx = cc == 0 ? scalar(lv, -std::nearbyint(sp)) : scalar(lv, sp / T[cc].second);
        P.prog.push_back(st);
        T[k] = {lv - 1, sp / (double)c->mod[lv]};
    }

    int level_of(int deg)
    {
        if (deg < BABY) {
            int lv = 1 << 30;
            for (int k = 1; k <= deg; k++) lv = std::min(lv, T[k].first);
            return lv - 1;
        }
        int m = 0;
        for (int g : giants)
            if (g <= deg) m = g;
        int lq = level_of(deg - m), lr = level_of(m - 1);
        return std::min(std::min(lq, T[m].first) - 1, lr);
    }

    int ev(const std::vector<double> &cf, double s_t, const std::string &reg)
    {
        const int deg = (int)cf.size() - 1;
        if (deg < BABY) {
            int lv = 1 << 30;
            for (int k = 1; k <= deg; k++) lv = std::min(lv, T[k].first);
            BootStep st;
            st.kind = ST_LEAF;
            st.reg = reg;
            st.lv = lv;
            const double ql = (double)c->mod[lv];
            for (int k = 1; k <= deg; k++)
                if (cf[k] != 0.0) st.terms.push_back({k, scalar(lv, cf[k] * s_t * ql / T[k].second)});
            st.cidx = scalar(lv, cf[0] * s_t * ql);
            P.prog.push_back(st);
            return lv - 1;
        }
        int m = 0;
        for (int g : giants)
            if (g <= deg) m = g;
        std::vector<double> qc, rc;
        cheb_split(cf, m, qc, rc);
        int lq = level_of((int)qc.size() - 1);
        int lp = std::min(lq, T[m].first);
        double s_q = s_t * (double)c->mod[lp] / T[m].second;
        ev(qc, s_q, reg + "q");
        ev(rc, s_t, reg + "r");
        int lr = level_of((int)rc.size() - 1);
        BootStep st;
        st.kind = ST_GIANT;
        st.reg = reg;
        st.m = m;
        st.lp = lp;
        st.out = std::min(lp - 1, lr);
        P.prog.push_back(st);
        return st.out;
    }
};

void boot_free(rbk_ctx_impl *ci)
{
    BootPlan *P = ci->boot;
    if (!P) return;
    for (u64 *d : P->d_plain) release_buffer(ci, d);
    for (auto &r : P->pool) release_buffer(ci, r.first);
    release_buffer(ci, P->rot_area);
    for (int k = 0; k < RBK_LANES; k++) release_buffer(ci, P->lane_ws[k]);
    release_buffer(ci, P->d_scal);
    delete P;
    ci->boot = nullptr;
}

static int build_plan(rbk_ctx *c, const rbk_boot_params &prm, BootPlan &P)
{
    P.prm = prm;
    P.L = c->nQ - 1;
    const u64 q0 = c->mod[0];
    int bits0 = 64 - __builtin_clzll(q0);
    P.dref_log2 = bits0 - (int)prm.log2_rho;
    const double K = prm.K;
    P.s_A = std::ldexp(1.0, (int)std::ceil(std::log2(2.0 * (double)q0 * (K + 1))));
    const double c_cts = P.s_A / (2.0 * (double)q0 * (K + 1));
    const double c_stc = (double)q0 / (2 * M_PI * std::ldexp(1.0, P.dref_log2));
    const int logn = c->logN - 1;
    auto gc = stage_groups(logn, prm.cts_levels), gs = stage_groups(logn, prm.stc_levels);
    int sb_log2 = (int)std::lround(std::log2((double)c->mod[P.L]));
    int total = (int)std::lround(std::log2(P.s_A)) - sb_log2;
    std::vector<int> drops(prm.cts_levels, total / (int)prm.cts_levels);
    drops.back() += total - (total / (int)prm.cts_levels) * (int)prm.cts_levels;
    if (P.L < (int)(prm.cts_levels + prm.stc_levels + prm.double_angle + 8)) return RBK_ELEVEL;
    int rc = plan_lt(c, P, gc, true, P.L, P.s_A, c_cts, drops, P.cts, P.s_B);
    if (rc) return rc;
    P.level_evalmod = P.L - (int)prm.cts_levels;

    EvalPlanner E{c, P, {}, {}};
    E.T[1] = {P.level_evalmod, P.s_B};
    for (int m = BABY; m <= (int)prm.degree; m *= 2) E.giants.push_back(m);
    const int recipe[6][4] = {{2, 1, 1, 0}, {3, 1, 2, 1}, {4, 2, 2, 0}, {5, 2, 3, 1}, {6, 3, 3, 0}, {7, 3, 4, 1}};
    for (auto &r : recipe)
        if (r[0] <= (int)prm.degree) E.prod(r[0], r[1], r[2], r[3]);
    for (int m : E.giants) E.prod(m, m / 2, m / 2, 0);
    std::vector<double> cf = cheb_coeffs((int)prm.K, (int)prm.double_angle, (int)prm.degree);
    int lvl = E.ev(cf, P.s_B, "p");
    double sc = P.s_B;
    for (unsigned i = 0; i < prm.double_angle; i++) {
        BootStep st;
        st.kind = ST_DBL;
        st.lv = lvl;
        st.sidx = E.scalar(lvl, -std::nearbyint(sc * sc));
        P.prog.push_back(st);
        sc = sc * sc / (double)c->mod[lvl];
        lvl--;
    }
    if (lvl - (int)prm.stc_levels < 0) return RBK_ELEVEL;
    P.level_stc = lvl;
    P.s_E = sc;
    std::vector<std::vector<int>> gsr(gs.rbegin(), gs.rend());
    rc = plan_lt(c, P, gsr, false, lvl, sc, c_stc, std::vector<int>(prm.stc_levels, 0), P.stc, P.s_out);
    if (rc) return rc;
    P.level_out = lvl - (int)prm.stc_levels;

    std::set<int64_t> ks;
    const int64_t n = (int64_t)c->N / 2;
    for (auto *v : {&P.cts, &P.stc})
        for (auto &lt : *v)
            for (auto &e : lt.ents) {
                if (e.b) ks.insert(((int64_t)e.b * lt.h0) % n);
                if (e.g) ks.insert((((int64_t)e.g * lt.n1 * lt.h0) % n + n) % n);
            }
    ks.erase(0);
    P.rots.assign(ks.begin(), ks.end());
    return RBK_OK;
}

// ---------------------------------------------------------------- execution

struct Reg {
    u64 *d = nullptr;
    int level = 0;
};

// out = (2 x if x) + sum_t (+-) s_t v_t + (constant on c0): the elementwise part
// of an EvalMod step in one pass.  Terms are views (ciphertext c, polynomial
// p of term t at v[t] + c vcs[t] + p vps[t]), read at the output level, so a
// power kept at a higher level needs no dropped copy.  A scalar index of -1
// is the coefficient 1.
constexpr int COMB_MAX = 8;
struct CombArgs {
    const u64 *x;
    const u64 *v[COMB_MAX];
    long vcs[COMB_MAX], vps[COMB_MAX];
    int vs[COMB_MAX], vneg[COMB_MAX];
    int n;
    int cidx;
};

__device__ __forceinline__ u64 comb_term(const CombArgs &A, int t, u64 v, const u64 *scal, int nQ, int limb, u64 q)
{
    if (A.vs[t] >= 0) {
        const u64 *w = scal + ((size_t)A.vs[t] * nQ + limb) * 2;
        v = shoup(v, w[0], w[1], q);
    }
    return v;
}

// PAIR: two adjacent coefficients per thread (every view and out 16-byte
// aligned, even strides), else one
template <bool PAIR>
__global__ __launch_bounds__(256) void k_boot_comb(CombArgs A, u64 *out, const u64 *scal, int nQ, int logN, int L1,
                                                    const PrimeC *pc)
{
    const size_t n = (PAIR ? 2 : 1) * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (n >= ((size_t)1 << logN)) return;
    const int limb = blockIdx.y;
    const unsigned ct = blockIdx.z >> 1, poly = blockIdx.z & 1;
    const u64 q = pc[limb].q;
    const size_t per = (size_t)L1 << logN;
    const size_t o = (size_t)ct * 2 * per + poly * per + ((size_t)limb << logN) + n;
    const u64 cadd = (poly == 0 && A.cidx >= 0) ? scal[((size_t)A.cidx * nQ + limb) * 2] : 0;
    if (PAIR) {
        u64 r0 = 0, r1 = 0;
        if (A.x) {
            const u64x2 x = ld2(A.x + o);
            r0 = add_mod(x.x, x.x, q);
            r1 = add_mod(x.y, x.y, q);
        }
#pragma unroll
        for (int t = 0; t < COMB_MAX; t++) {
            if (t >= A.n) break;
            const u64x2 v = ld2(A.v[t] + (size_t)ct * A.vcs[t] + poly * A.vps[t] + ((size_t)limb << logN) + n);
            const u64 v0 = comb_term(A, t, v.x, scal, nQ, limb, q), v1 = comb_term(A, t, v.y, scal, nQ, limb, q);
            r0 = A.vneg[t] ? sub_mod(r0, v0, q) : add_mod(r0, v0, q);
            r1 = A.vneg[t] ? sub_mod(r1, v1, q) : add_mod(r1, v1, q);
        }
        st2(out + o, add_mod(r0, cadd, q), add_mod(r1, cadd, q));
        return;
    }
    u64 r = 0;
    if (A.x) r = add_mod(A.x[o], A.x[o], q);
#pragma unroll
    for (int t = 0; t < COMB_MAX; t++) {
        if (t >= A.n) break;
        const u64 v = comb_term(A, t, A.v[t][(size_t)ct * A.vcs[t] + poly * A.vps[t] + ((size_t)limb << logN) + n], scal,
                                nQ, limb, q);
        r = A.vneg[t] ? sub_mod(r, v, q) : add_mod(r, v, q);
    }
    out[o] = add_mod(r, cadd, q);
}

static int upload_scalars(rbk_ctx *c, BootPlan &P)
{
    if (!P.scal_dirty && P.d_scal) return RBK_OK;
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "bootstrap scalars changed during graph capture");
    const size_t nQ = c->nQ, n = std::max<size_t>(P.scalars.size(), 1);
    std::vector<u64> h(n * nQ * 2, 0);
    for (size_t i = 0; i < P.scalars.size(); i++)
        for (size_t k = 0; k < P.scalars[i].size() && k < nQ; k++) {
            h[(i * nQ + k) * 2] = P.scalars[i][k];
            h[(i * nQ + k) * 2 + 1] = b_shoup(P.scalars[i][k], c->mod[k]);
        }
    if (!P.d_scal && hipMalloc((void **)&P.d_scal, h.size() * sizeof(u64)) != hipSuccess) {
        P.d_scal = nullptr;
        return rbk_set_error(RBK_ENOMEM, "bootstrap scalar table");
    }
    if (hipMemcpy(P.d_scal, h.data(), h.size() * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess)
        return rbk_set_error(RBK_EDEVICE, "bootstrap scalar upload");
    P.scal_dirty = false;
    return RBK_OK;
}

struct Runner {
    rbk_ctx *c;
    BootPlan &P;
    int cnt;                 // ciphertexts per register
    size_t reg_words;        // the words one register of this run needs
    std::vector<u64 *> free_;  // pooled registers not in use (each holds at least reg_words)

    u64 *take()
    {
        if (!free_.empty()) {
            u64 *d = free_.back();
            free_.pop_back();
            return d;
        }
        // a new register of exactly this run's size
        u64 *d = nullptr;
        if (hipMalloc((void **)&d, reg_words * sizeof(u64)) != hipSuccess) return nullptr;
        P.pool.emplace_back(d, reg_words);
        return d;
    }
    // while steps run on several lanes, registers they release are held back
    // until the lanes join (another lane could otherwise take one still in use)
    std::vector<u64 *> *held = nullptr;
    void give(u64 *d)
    {
        if (d) (held ? *held : free_).push_back(d);
    }
    size_t per(int level) const { return (size_t)(level + 1) * c->N; }

    // copy of limbs 0..to of every polynomial of src (at level from)
    int drop(const u64 *src, int from, int to, u64 *dst, int n_ct)
    {
        const size_t N = c->N;
        if (from == to && src == dst) return RBK_OK;
        if (hipMemcpy2DAsync(dst, (to + 1) * N * sizeof(u64), src, (from + 1) * N * sizeof(u64), (to + 1) * N * sizeof(u64),
                             (size_t)2 * n_ct, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return RBK_EDEVICE;
        return RBK_OK;
    }

    ScalArg scal(int idx, int level)
    {
        ScalArg s;
        const std::vector<u64> &r = P.scalars[idx];
        for (int i = 0; i <= level; i++) {
            s.w[i] = r[i];
            s.wsh[i] = b_shoup(r[i], c->mod[i]);
        }
        return s;
    }

    int rotate(const u64 *in, u64 *out, int level, int n_ct, int64_t k);
    // out = add + Rot_k(in) (add may be out)
    int rotate_add(const u64 *in, const u64 *add, u64 *out, int level, int n_ct, int64_t k);
    // one elementwise pass at level lv over n_ct ciphertexts (see k_boot_comb)
    void comb(CombArgs &A, u64 *out, int lv, int n_ct)
    {
        bool pair = ((uintptr_t)out & 15) == 0 && (!A.x || ((uintptr_t)A.x & 15) == 0) && c->N >= 2;
        for (int t = 0; t < A.n; t++) pair = pair && ((uintptr_t)A.v[t] & 15) == 0 && (A.vcs[t] | A.vps[t]) % 2 == 0;
        const size_t work = pair ? c->N / 2 : c->N;
        const unsigned thr = (unsigned)std::min<size_t>(256, work);
        dim3 grid((unsigned)(work / thr), lv + 1, 2 * n_ct);
        kt_begin(c, KC_ELEMENTWISE, c->stream);
        if (pair)
            hipLaunchKernelGGL(k_boot_comb<true>, grid, dim3(thr), 0, c->stream, A, out, P.d_scal, c->nQ, c->logN, lv + 1,
                               c->d_pc);
        else
            hipLaunchKernelGGL(k_boot_comb<false>, grid, dim3(thr), 0, c->stream, A, out, P.d_scal, c->nQ, c->logN, lv + 1,
                               c->d_pc);
        kt_end(c, KC_ELEMENTWISE, (double)n_ct * 2 * (lv + 1) * c->N * sizeof(u64) * (A.n + (A.x ? 2 : 1)), c->stream);
    }
    // a register seen as a view: ciphertexts 2 (level+1) N apart
    static void term(CombArgs &A, const Reg &r, size_t N, int sidx, int neg)
    {
        const int t = A.n++;
        A.v[t] = r.d;
        A.vps[t] = (long)((size_t)(r.level + 1) * N);
        A.vcs[t] = 2 * A.vps[t];
        A.vs[t] = sidx;
        A.vneg[t] = neg;
    }
    int lt(Reg &x, const BootLT &lt, int n_ct);
    int evalmod(Reg &x, int n_ct);
};

int Runner::rotate(const u64 *in, u64 *out, int level, int n_ct, int64_t k)
{
    return rotate_batch_g(c, in, out, level, n_ct, rbk_galois_elt(c, k));
}

int Runner::rotate_add(const u64 *in, const u64 *add, u64 *out, int level, int n_ct, int64_t k)
{
    return rotate_add_batch_g(c, in, add, out, level, n_ct, rbk_galois_elt(c, k));
}

int Runner::lt(Reg &x, const BootLT &L, int n_ct)
{
    const int lvl = L.level;
    const size_t ctw = 2 * per(lvl);
    std::vector<int> babies;
    for (auto &e : L.ents)
        if (e.b && std::find(babies.begin(), babies.end(), e.b) == babies.end()) babies.push_back(e.b);
    std::sort(babies.begin(), babies.end());
    const int nb = (int)babies.size();
    int rc = RBK_OK;
    u64 *rots = nullptr;
    if (nb) {
        const size_t need = (size_t)n_ct * nb * ctw;
        if (need > P.rot_words) {
            if (c->capturing) return rbk_set_error(RBK_ESTATE, "rotation area too small during graph capture");
            release_buffer(c, P.rot_area);
            P.rot_area = nullptr;
            P.rot_words = 0;
            if (hipMalloc((void **)&P.rot_area, need * sizeof(u64)) != hipSuccess)
                return rbk_set_error(RBK_ENOMEM, "rotation area");
            P.rot_words = need;
        }
        std::vector<int64_t> ks;
        for (int b : babies) ks.push_back((int64_t)b * L.h0);
        rc = rbk_rotate_hoisted_batch(c, x.d, ks.data(), nb, P.rot_area, lvl, n_ct);
        if (rc) return rc;
        rots = P.rot_area;
    }
    std::vector<int> gs;
    for (auto &e : L.ents)
        if (std::find(gs.begin(), gs.end(), e.g) == gs.end()) gs.push_back(e.g);
    // the giant step without a rotation (if any) first: its products go
    // straight into the sum
    std::stable_partition(gs.begin(), gs.end(), [](int g) { return g == 0; });
    const int n_rot = (int)std::count_if(gs.begin(), gs.end(), [](int g) { return g != 0; });
    // Giant-step lanes: the giant steps are independent up to the final sum,
    // so their rotations go round-robin over the context's side streams (each
    // with key-switching workspace of its own) and every lane keeps a partial
    // sum; the context stream adds the partial sums.  Modular sums do not
    // depend on their order, so the residues are those of one lane.  One lane
    // while timers run or the stream is captured (a captured graph stays one
    // chain of kernels).
    const int nl = (c->lanes > 1 && !c->capturing && !c->timing && n_rot > 1 && side_streams(c) == RBK_OK)
                       ? std::min(c->lanes, n_rot)
                       : 0;
    // The products of GT_MAX_G giant steps at a time, every baby step read
    // once per pass; each rotated giant step's inner sum waits in a register
    // for its rotation: one register per rotated giant step with lanes (the
    // rotations run behind the products), else GT_MAX_G used in turn on the
    // one stream.
    const int n_inner = nl ? n_rot : std::min(n_rot, GT_MAX_G);
    std::vector<u64 *> inner;
    for (int i = 0; i < n_inner; i++) {
        inner.push_back(take());
        if (!inner.back()) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
    }
    u64 *total = take();
    if (!total) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
    u64 *l_acc[RBK_LANES] = {};
    bool l_have[RBK_LANES] = {};
    for (int k = 0; k < nl; k++) {
        l_acc[k] = take();
        if (!l_acc[k]) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
    }
    const LimbMap qm{0, c->nQ, c->nQ};
    // baby-step slots: 0 is the input itself, then the hoisted rotations
    const int n_slot = 1 + nb;
    std::vector<const u64 *> bsrc(n_slot);
    std::vector<long> bstride(n_slot);
    bsrc[0] = x.d;
    bstride[0] = (long)ctw;
    for (int i = 0; i < nb; i++) {
        bsrc[1 + i] = rots + (size_t)i * ctw;
        bstride[1 + i] = (long)(nb * ctw);
    }
    auto slot_of = [&](int b) {
        return b == 0 ? 0 : 1 + (int)(std::find(babies.begin(), babies.end(), b) - babies.begin());
    };
    bool have_total = false;
    int lane = 0, n_done = 0;
    for (size_t s0 = 0; s0 < gs.size() && rc == RBK_OK; s0 += GT_MAX_G) {
        const int ng = (int)std::min<size_t>(GT_MAX_G, gs.size() - s0);
        u64 *outs[GT_MAX_G] = {};
        for (int j = 0, r = n_done; j < ng; j++) outs[j] = gs[s0 + j] == 0 ? total : inner[(r++) % n_inner];
        for (int b0 = 0; b0 < n_slot; b0 += GT_MAX_B) {
            GiantTerms T{};
            T.ng = ng;
            T.nb = std::min(GT_MAX_B, n_slot - b0);
            for (int i = 0; i < T.nb; i++) {
                T.src[i] = bsrc[b0 + i];
                T.stride[i] = bstride[b0 + i];
            }
            for (int j = 0; j < ng; j++) {
                T.out[j] = outs[j];
                T.add[j] = b0 > 0;
            }
            for (auto &e : L.ents) {
                const int j = (int)(std::find(gs.begin() + s0, gs.begin() + s0 + ng, e.g) - (gs.begin() + s0));
                const int sl = slot_of(e.b) - b0;
                if (j < ng && sl >= 0 && sl < T.nb) T.pt[j][sl] = P.d_plain[e.plain];
            }
            mac_giants_launch(c, T, lvl, n_ct, c->stream);
        }
        if (gs[s0] == 0) have_total = true;
        if (nl) {
            // the lanes' rotations start once these products are written
            if (hipEventRecord(c->side_ev[RBK_LANES], c->stream) != hipSuccess) {
                rc = rbk_set_error(RBK_EDEVICE, "fork");
                break;
            }
            for (int k = 0; k < nl && rc == RBK_OK; k++)
                if (hipStreamWaitEvent(c->side[k], c->side_ev[RBK_LANES], 0) != hipSuccess)
                    rc = rbk_set_error(RBK_EDEVICE, "fork");
            if (rc) break;
        }
        for (int j = 0; j < ng; j++) {
            const int g = gs[s0 + j];
            if (g == 0) continue;
            n_done++;
            const int64_t rk = (int64_t)g * L.n1 * L.h0;
            if (nl) {
                // the rotation on the lane's stream and workspace, into the lane's partial sum
                const int k = lane;
                std::swap(c->stream, c->side[k]);
                std::swap(c->ws, P.lane_ws[k]);
                std::swap(c->ws_words, P.lane_ws_words[k]);
                rc = l_have[k] ? rotate_add(outs[j], l_acc[k], l_acc[k], lvl, n_ct, rk)
                               : rotate(outs[j], l_acc[k], lvl, n_ct, rk);
                std::swap(c->stream, c->side[k]);
                std::swap(c->ws, P.lane_ws[k]);
                std::swap(c->ws_words, P.lane_ws_words[k]);
                if (rc) break;
                l_have[k] = true;
                lane = (lane + 1) % nl;
                continue;
            }
            rc = have_total ? rotate_add(outs[j], total, total, lvl, n_ct, rk) : rotate(outs[j], total, lvl, n_ct, rk);
            if (rc) break;
            have_total = true;
        }
    }
    // join every lane, also after a failure: later work on the context stream
    // reuses the registers and workspaces the lanes still read
    for (int k = 0; k < nl; k++) {
        hipError_t e = hipEventRecord(c->side_ev[k], c->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->side_ev[k], 0);
        if (e != hipSuccess && rc == RBK_OK) rc = rbk_set_error(RBK_EDEVICE, "lane join");
    }
    for (int k = 0; k < nl && rc == RBK_OK; k++) {
        if (!l_have[k]) continue;
        if (!have_total) {
            if (hipMemcpyAsync(total, l_acc[k], (size_t)n_ct * ctw * sizeof(u64), hipMemcpyDeviceToDevice, c->stream) !=
                hipSuccess)
                rc = RBK_EDEVICE;
            have_total = true;
        } else {
            ew_launch(c, EW_ADD, total, l_acc[k], total, 2 * n_ct, lvl + 1, qm, c->stream);
        }
    }
    for (int k = 0; k < nl; k++) give(l_acc[k]);
    if (!rc) rc = rbk_rescale_batch(c, total, x.d, lvl, n_ct);
    x.level = lvl - 1;
    for (u64 *d : inner) give(d);
    give(total);
    return rc;
}

int Runner::evalmod(Reg &x, int n_ct)
{
    const LimbMap qm{0, c->nQ, c->nQ};
    std::map<int, Reg> T;
    T[1] = x;
    std::map<std::string, Reg> regs;
    int rc = RBK_OK;
    // operand at level lv: the register itself, or a dropped copy in dst
    auto at = [&](const Reg &r, int lv, u64 *dst) -> const u64 * {
        if (r.level == lv) return r.d;
        drop(r.d, r.level, lv, dst, n_ct);
        return dst;
    };
    auto run_step = [&](const BootStep &st) -> int {
        if (st.kind == ST_PROD) {
            // T_k = 2 T_a T_b - T_c (or + constant when c = 0), exact scale via the scalar
            const int lv = st.lv;
            u64 *A = take(), *B = take(), *X = take();
            if (!A || !B || !X) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            const u64 *pa = at(T[st.a], lv, A), *pb = at(T[st.b], lv, B);
            rc = rbk_mult_relin_batch(c, pa, pb, X, lv, n_ct);
            if (rc) return rc;
            CombArgs C{};
            C.x = X;
            C.cidx = -1;
            if (st.cc == 0) C.cidx = st.sidx;
            else term(C, T[st.cc], c->N, st.sidx, 1);
            comb(C, X, lv, n_ct);
            u64 *out = take();
            if (!out) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            rc = rbk_rescale_batch(c, X, out, lv, n_ct);
            if (rc) return rc;
            T[st.k] = Reg{out, lv - 1};
            give(A);
            give(B);
            give(X);
        } else if (st.kind == ST_LEAF) {
            // sum_k s_k T_k + constant, the powers read in place at level lv
            const int lv = st.lv;
            u64 *acc = take();
            if (!acc) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            if (st.terms.size() > (size_t)COMB_MAX) return rbk_set_error(RBK_EUNSUPPORTED, "leaf with too many terms");
            CombArgs C{};
            C.x = nullptr;
            for (auto &t : st.terms) term(C, T[t.first], c->N, t.second, 0);
            C.cidx = st.cidx;
            comb(C, acc, lv, n_ct);
            u64 *out = take();
            if (!out) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            rc = rbk_rescale_batch(c, acc, out, lv, n_ct);
            if (rc) return rc;
            regs[st.reg] = Reg{out, lv - 1};
            give(acc);
        } else if (st.kind == ST_GIANT) {
            Reg q = regs[st.reg + "q"], r = regs[st.reg + "r"];
            regs.erase(st.reg + "q");
            regs.erase(st.reg + "r");
            const int lp = st.lp;
            u64 *A = take(), *B = take(), *X = take(), *Y = take();
            if (!A || !B || !X || !Y) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            const u64 *pq = at(q, lp, A), *pm = at(T[st.m], lp, B);
            rc = rbk_mult_relin_batch(c, pq, pm, X, lp, n_ct);
            if (rc) return rc;
            rc = rbk_rescale_batch(c, X, Y, lp, n_ct);
            if (rc) return rc;
            u64 *out = take();
            if (!out) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            CombArgs C{};
            C.x = nullptr;
            C.cidx = -1;
            term(C, Reg{Y, lp - 1}, c->N, -1, 0);
            term(C, r, c->N, -1, 0);
            comb(C, out, st.out, n_ct);
            regs[st.reg] = Reg{out, st.out};
            give(q.d);
            give(r.d);
            give(A);
            give(B);
            give(X);
            give(Y);
        } else {  // ST_DBL: y = 2 y^2 - 1 with the scale folded into the constant
            Reg y = regs["p"];
            const int lv = st.lv;
            u64 *A = take(), *X = take();
            if (!A || !X) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            const u64 *py = at(y, lv, A);
            rc = rbk_mult_relin_batch(c, py, py, X, lv, n_ct);
            if (rc) return rc;
            CombArgs C{};
            C.x = X;
            C.cidx = st.sidx;
            comb(C, X, lv, n_ct);
            u64 *out = take();
            if (!out) return rbk_set_error(RBK_ENOMEM, "bootstrapping registers");
            rc = rbk_rescale_batch(c, X, out, lv, n_ct);
            if (rc) return rc;
            give(y.d);
            regs["p"] = Reg{out, lv - 1};
            give(A);
            give(X);
        }
        return RBK_OK;
    };
    // EvalMod lanes: for small batches the products of one dependency depth
    // (powers T_3 and T_4; T_5 .. T_8; the giant steps of one level of the
    // evaluation tree) run on the side streams, each lane with a
    // key-switching workspace of its own; the lanes join after every depth.
    // Larger batches fill the GPU by themselves and keep the program order
    // (fewer registers alive).  The residues do not depend on the lanes.
    // One lane while timers run or the stream is captured.
    const int nl = (n_ct <= 8 && c->lanes > 1 && !c->capturing && !c->timing && side_streams(c) == RBK_OK)
                       ? c->lanes
                       : 0;
    if (!nl) {
        for (const BootStep &st : P.prog)
            if ((rc = run_step(st)) != RBK_OK) return rc;
    } else {
        // dependency depth of every step: one more than that of its deepest input
        const size_t ns = P.prog.size();
        std::vector<int> depth(ns, 0);
        std::map<int, int> dT{{1, 0}};
        std::map<std::string, int> dR;
        int max_d = 0;
        for (size_t i = 0; i < ns; i++) {
            const BootStep &st = P.prog[i];
            int d = 0;
            if (st.kind == ST_PROD) {
                d = std::max(dT[st.a], dT[st.b]);
                if (st.cc) d = std::max(d, dT[st.cc]);
                dT[st.k] = d + 1;
            } else if (st.kind == ST_LEAF) {
                for (auto &t : st.terms) d = std::max(d, dT[t.first]);
                dR[st.reg] = d + 1;
            } else if (st.kind == ST_GIANT) {
                d = std::max({dR[st.reg + "q"], dR[st.reg + "r"], dT[st.m]});
                dR[st.reg] = d + 1;
            } else {
                d = dR["p"];
                dR["p"] = d + 1;
            }
            depth[i] = d + 1;
            max_d = std::max(max_d, d + 1);
        }
        std::vector<u64 *> held_regs;
        for (int dd = 1; dd <= max_d && rc == RBK_OK; dd++) {
            std::vector<size_t> grp;
            for (size_t i = 0; i < ns; i++)
                if (depth[i] == dd) grp.push_back(i);
            if (grp.size() < 2) {
                for (size_t i : grp)
                    if ((rc = run_step(P.prog[i])) != RBK_OK) break;
                continue;
            }
            const int nq = std::min(nl, (int)grp.size());
            if (hipEventRecord(c->side_ev[RBK_LANES], c->stream) != hipSuccess) return rbk_set_error(RBK_EDEVICE, "fork");
            for (int k = 0; k < nq; k++)
                if (hipStreamWaitEvent(c->side[k], c->side_ev[RBK_LANES], 0) != hipSuccess)
                    return rbk_set_error(RBK_EDEVICE, "fork");
            held = &held_regs;
            for (size_t j = 0; j < grp.size() && rc == RBK_OK; j++) {
                const int k = (int)(j % nq);
                std::swap(c->stream, c->side[k]);
                std::swap(c->ws, P.lane_ws[k]);
                std::swap(c->ws_words, P.lane_ws_words[k]);
                rc = run_step(P.prog[grp[j]]);
                std::swap(c->stream, c->side[k]);
                std::swap(c->ws, P.lane_ws[k]);
                std::swap(c->ws_words, P.lane_ws_words[k]);
            }
            held = nullptr;
            // join every lane, also after a failure
            for (int k = 0; k < nq; k++) {
                hipError_t e = hipEventRecord(c->side_ev[k], c->side[k]);
                if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->side_ev[k], 0);
                if (e != hipSuccess && rc == RBK_OK) rc = rbk_set_error(RBK_EDEVICE, "lane join");
            }
            for (u64 *d : held_regs) free_.push_back(d);
            held_regs.clear();
        }
        if (rc) return rc;
    }
    // release the powers (T[1] is the caller's register)
    for (auto &t : T)
        if (t.first != 1) give(t.second.d);
    Reg res = regs["p"];
    if (hipMemcpyAsync(x.d, res.d, (size_t)n_ct * 2 * per(res.level) * sizeof(u64), hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
        return RBK_EDEVICE;
    x.level = res.level;
    give(res.d);
    return RBK_OK;
}

// ---------------------------------------------------------------- C ABI

static int boot_fail(int code, const char *msg);

extern "C" int rbk_boot_setup(rbk_ctx *c, const rbk_boot_params *prm)
{
    if (c && c->capturing) return boot_fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !prm) return boot_fail(RBK_EINVAL, "null argument");
    if (prm->degree < 8 || prm->degree > 255 || prm->cts_levels < 1 || prm->stc_levels < 1 || prm->K < 1 ||
        prm->cts_levels > (unsigned)(c->logN - 1) || prm->stc_levels > (unsigned)(c->logN - 1) || prm->double_angle > 8 ||
        prm->log2_rho > 20)
        return boot_fail(RBK_EINVAL, "bad bootstrapping parameters");
    boot_free(c);
    BootPlan *P = new BootPlan();
    int rc = build_plan(c, *prm, *P);
    if (rc) {
        c->boot = P;
        boot_free(c);
        return boot_fail(rc, "bootstrapping plan: chain too short or allocation failed");
    }
    c->boot = P;
    return RBK_OK;
}

extern "C" int rbk_boot_rotations(const rbk_ctx *c, int64_t *ks, int max)
{
    if (!c || !c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    const BootPlan &P = *c->boot;
    for (int i = 0; i < (int)P.rots.size() && i < max; i++) ks[i] = P.rots[i];
    return (int)P.rots.size();
}

extern "C" int rbk_boot_info(const rbk_ctx *c, int *levels, int *n_plain, int *n_scalar)
{
    if (!c || !c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    const BootPlan &P = *c->boot;
    if (levels) {
        levels[0] = P.L;
        levels[1] = P.level_evalmod;
        levels[2] = P.level_stc;
        levels[3] = P.level_out;
    }
    if (n_plain) *n_plain = (int)P.d_plain.size();
    if (n_scalar) *n_scalar = (int)P.scalars.size();
    return RBK_OK;
}

extern "C" int rbk_boot_constant_levels(const rbk_ctx *c, int *plain_levels, int *scalar_levels)
{
    if (!c || !c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    const BootPlan &P = *c->boot;
    if (plain_levels)
        for (size_t i = 0; i < P.plain_level.size(); i++) plain_levels[i] = P.plain_level[i];
    if (scalar_levels)
        for (size_t i = 0; i < P.scalar_level.size(); i++) scalar_levels[i] = P.scalar_level[i];
    return RBK_OK;
}

extern "C" int rbk_boot_export(rbk_ctx *c, uint64_t *plains, uint64_t *scalars)
{
    if (c && c->capturing) return boot_fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    BootPlan &P = *c->boot;
    const size_t N = c->N;
    if (plains) {
        size_t off = 0;
        u64 *tmp = nullptr;
        if (hipMalloc((void **)&tmp, (size_t)c->nQ * N * sizeof(u64)) != hipSuccess) return boot_fail(RBK_ENOMEM, "export");
        for (size_t i = 0; i < P.d_plain.size(); i++) {
            const int l1 = P.plain_level[i] + 1;
            (void)hipMemcpyAsync(tmp, P.d_plain[i], l1 * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream);
            std::vector<int> idx(l1);
            for (int k = 0; k < l1; k++) idx[k] = k;
            int rc = rbk_ntt(c, tmp, 1, idx.data(), l1, 1);
            if (rc) {
                (void)hipFree(tmp);
                return rc;
            }
            (void)hipMemcpyAsync(plains + off, tmp, l1 * N * sizeof(u64), hipMemcpyDeviceToHost, c->stream);
            (void)hipStreamSynchronize(c->stream);
            off += l1 * N;
        }
        (void)hipFree(tmp);
    }
    if (scalars) {
        size_t off = 0;
        for (auto &s : P.scalars) {
            std::memcpy(scalars + off, s.data(), s.size() * sizeof(u64));
            off += s.size();
        }
    }
    return RBK_OK;
}

extern "C" int rbk_boot_import(rbk_ctx *c, const uint64_t *plains, const uint64_t *scalars)
{
    if (c && c->capturing) return boot_fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    BootPlan &P = *c->boot;
    const size_t N = c->N;
    if (plains) {
        size_t off = 0;
        for (size_t i = 0; i < P.d_plain.size(); i++) {
            const int l1 = P.plain_level[i] + 1;
            for (int k = 0; k < l1; k++)
                for (size_t j = 0; j < N; j++)
                    if (plains[off + k * N + j] >= c->mod[k]) return boot_fail(RBK_EINVAL, "imported residue not below its prime");
            if (hipMemcpy(P.d_plain[i], plains + off, l1 * N * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess)
                return boot_fail(RBK_EDEVICE, "import copy");
            std::vector<int> idx(l1);
            for (int k = 0; k < l1; k++) idx[k] = k;
            int rc = rbk_ntt(c, P.d_plain[i], 1, idx.data(), l1, 0);
            if (rc) return rc;
            off += l1 * N;
        }
    }
    if (scalars) {
        size_t off = 0;
        for (size_t i = 0; i < P.scalars.size(); i++) {
            for (size_t k = 0; k < P.scalars[i].size(); k++) {
                if (scalars[off + k] >= c->mod[k]) return boot_fail(RBK_EINVAL, "imported scalar not below its prime");
                P.scalars[i][k] = scalars[off + k];
                P.scal_dirty = true;
            }
            off += P.scalars[i].size();
        }
    }
    return rbk_sync(c);
}

extern "C" int rbk_bootstrap_batch(rbk_ctx *c, const uint64_t *d_in, const double *scales_in, uint64_t *d_out,
                                   double *scales_out, int count)
{
    if (!c || !d_in || !scales_in || !d_out || count < 1) return boot_fail(RBK_EINVAL, "bad argument");
    if (!c->boot) return boot_fail(RBK_ESTATE, "bootstrapping not set up");
    BootPlan &P = *c->boot;
    if (!c->relin.data) return boot_fail(RBK_ENOKEY, "relinearisation key missing");
    if (!c->gal.count(2 * c->N - 1)) return boot_fail(RBK_ENOKEY, "conjugation key missing");
    for (int64_t k : P.rots) {
        uint64_t g = rbk_galois_elt(c, k);
        if (!c->gal.count(g)) return boot_fail(RBK_ENOKEY, "a bootstrapping rotation key is missing");
    }
    const size_t N = c->N;
    std::vector<double> dprime(count);
    std::vector<int> ex(count);
    for (int i = 0; i < count; i++) {
        int e2;
        double f = std::frexp(scales_in[i], &e2);
        if (!(scales_in[i] > 0)) return boot_fail(RBK_EINVAL, "input scale must be positive");
        ex[i] = P.dref_log2 - (f == 0.5 ? e2 - 1 : e2);
        if (ex[i] < 0) return boot_fail(RBK_EINVAL, "input scale above the bootstrapping reference scale");
        dprime[i] = std::ldexp(scales_in[i], ex[i]);
    }
    // EvalMod runs the real and imaginary halves of the batch together
    if (int rc0 = upload_scalars(c, P)) return rc0;
    Runner R{c, P, count, (size_t)2 * count * 2 * (P.L + 1) * N, {}};
    // pooled registers large enough for this run are reused; smaller ones are
    // released (a larger batch than before), new ones have this run's size
    {
        std::vector<std::pair<u64 *, size_t>> keep;
        for (auto &r : P.pool) {
            if (r.second >= R.reg_words) {
                keep.push_back(r);
                R.free_.push_back(r.first);
            } else if (c->capturing) {
                return boot_fail(RBK_ESTATE, "bootstrap registers too small during graph capture: run the call once before capturing");
            } else {
                release_buffer(c, r.first);
            }
        }
        P.pool = keep;
    }
    const LimbMap qm{0, c->nQ, c->nQ};
    int rc;
    u64 *x0 = R.take(), *tmp = R.take();
    if (!x0 || !tmp) return boot_fail(RBK_ENOMEM, "bootstrapping registers");
    // 1. pre-scale by 2^e at level 0
    for (int i = 0; i < count; i++) {
        uint64_t f = b_pow(2, (u64)ex[i], c->mod[0]);
        rc = rbk_mul_scalar(c, d_in + (size_t)i * 2 * N, &f, tmp + (size_t)i * 2 * N, 0, 2);
        if (rc) return rc;
    }
    // 2. ModRaise: inverse NTT of the level-0 limbs, centred lift, NTT of all limbs
    {
        int idx0 = 0;
        rc = rbk_ntt(c, tmp, 2 * count, &idx0, 1, 1);
        if (rc) return rc;
        modraise_lift_launch(c, tmp, x0, P.L, 2 * count, c->stream);
        std::vector<int> idx(P.L + 1);
        for (int k = 0; k <= P.L; k++) idx[k] = k;
        rc = rbk_ntt(c, x0, 2 * count, idx.data(), P.L + 1, 0);
        if (rc) return rc;
    }
    Reg x{x0, P.L};
    // 3. CoeffToSlot
    for (auto &lt : P.cts) {
        rc = R.lt(x, lt, count);
        if (rc) return rc;
    }
    // 4. real / imaginary split: re = v + conj(v), im = -i (v - conj(v)), stacked
    const int lv = P.level_evalmod;
    const size_t ctw = 2 * R.per(lv);
    u64 *conj = R.take(), *both = R.take();
    if (!conj || !both) return boot_fail(RBK_ENOMEM, "bootstrapping registers");
    rc = rotate_batch_g(c, x.d, conj, lv, count, 2 * c->N - 1);
    if (rc) return rc;
    ew_launch(c, EW_ADD, x.d, conj, both, 2 * count, lv + 1, qm, c->stream);
    ew_launch(c, EW_SUB, x.d, conj, tmp, 2 * count, lv + 1, qm, c->stream);
    monomial_half_launch(c, tmp, both + (size_t)count * ctw, 2 * count, lv, 1, c->stream);
    R.give(conj);
    // 5. EvalMod on 2*count ciphertexts
    Reg y{both, lv};
    rc = R.evalmod(y, 2 * count);
    if (rc) return rc;
    // 6. recombine: re + i im
    const int ls = P.level_stc;
    const size_t ctw2 = 2 * R.per(ls);
    monomial_half_launch(c, y.d + (size_t)count * ctw2, tmp, 2 * count, ls, 0, c->stream);
    ew_launch(c, EW_ADD, y.d, tmp, x.d, 2 * count, ls + 1, qm, c->stream);
    x.level = ls;
    R.give(both);
    // 7. SlotToCoeff
    for (auto &lt : P.stc) {
        rc = R.lt(x, lt, count);
        if (rc) return rc;
    }
    if (hipMemcpyAsync(d_out, x.d, (size_t)count * 2 * R.per(P.level_out) * sizeof(u64), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
        return boot_fail(RBK_EDEVICE, "output copy");
    R.give(x0);
    R.give(tmp);
    // the slots hold z * d' / D_ref at the arithmetic scale s_out
    for (int i = 0; i < count; i++) scales_out[i] = P.s_out * dprime[i] / std::ldexp(1.0, P.dref_log2);
    return RBK_OK;
}

extern "C" int rbk_bootstrap(rbk_ctx *c, const uint64_t *d_in, double scale_in, uint64_t *d_out, double *scale_out)
{
    return rbk_bootstrap_batch(c, d_in, &scale_in, d_out, scale_out, 1);
}

int rbk_set_error(int code, const char *msg);
static int boot_fail(int code, const char *msg) { return rbk_set_error(code, msg); }

// bytes of the plan's encoded diagonals (resident while the plan exists)
size_t boot_resident_bytes(const rbk_ctx_impl *ci)
{
    const BootPlan *P = ci->boot;
    if (!P) return 0;
    size_t w = 0;
    for (int lv : P->plain_level) w += (size_t)(lv + 1) * ci->N;
    return w * sizeof(u64);
}
