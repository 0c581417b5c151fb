// Packed local-loss MLP training step (paper Section 4, Algorithms 1 and 2)
// on the library's ciphertext operations.
//
// One step is written once, as a template over the number system it runs
// on: GpuOps executes it on the device (every operation applied to a whole
// batch of ciphertexts per launch set), LevelOps only follows levels, which
// gives the step's multiplicative depth.
//
// Device layout: a "Vec" is `count` ciphertexts (one per sample, or a single
// shared one) seen through strides, so that a ciphertext at a higher level
// is read at a lower one without copying (limbs 0..l of each polynomial),
// and a weight ciphertext multiplies every sample of a batch without being
// replicated.  Results are always written contiguously, [count][2][l+1][N].
// Device memory for results comes from a best-fit pool owned by the MLP
// object, so steps after the first allocate nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

namespace {

constexpr int MT = 256;

// ---------------------------------------------------------------- kernels

struct View {
    const u64 *d;
    long cs;  // words between ciphertexts (0: one ciphertext shared by all)
    long ps;  // words between the two polynomials
};

__device__ __forceinline__ u64 ld(const View &v, unsigned ct, unsigned poly, unsigned limb, int logN, unsigned n)
{
    return v.d[(size_t)ct * v.cs + (size_t)poly * v.ps + ((size_t)limb << logN) + n];
}

// k * 2^64 mod q for 0 <= k < 2^62 (REDC of k * 2^128 mod q)
__device__ __forceinline__ u64 to_mont_k(u64 k, const PrimeC &p) { return redc(mul_wide(k, p.r2), p.q, p.qneg); }

// (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1); grid (N/threads, L1, count)
__global__ void k_mlp_tensor(View a, View b, u64 *out, int logN, int L1, const PrimeC *pc)
{
    const unsigned n = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y, ct = blockIdx.z;
    const PrimeC p = pc[limb];
    const u64 a0 = ld(a, ct, 0, limb, logN, n), a1 = ld(a, ct, 1, limb, logN, n);
    const u64 b0 = ld(b, ct, 0, limb, logN, n), b1 = ld(b, ct, 1, limb, logN, n);
    const size_t per = (size_t)L1 << logN;
    u64 *o = out + ct * 3 * per + ((size_t)limb << logN) + n;
    o[0] = mul_mod(a0, b0, p);
    u128w s = mul_wide(a0, b1);
    acc_wide(s, mul_wide(a1, b0));
    const u64 t = redc(s, p.q, p.qneg);
    o[per] = redc(mul_wide(t, p.r2), p.q, p.qneg);
    o[2 * per] = mul_mod(a1, b1, p);
}

// a +- b over adjacent coefficient pairs (views and out 16-byte aligned);
// grid (N/(2 threads), L1, 2 count)
__global__ void k_mlp_addsub(View a, View b, u64 *out, int logN, int L1, int sub, const PrimeC *pc)
{
    const unsigned n = 2 * (blockIdx.x * blockDim.x + threadIdx.x), limb = blockIdx.y;
    const unsigned ct = blockIdx.z >> 1, poly = blockIdx.z & 1;
    const u64 q = pc[limb].q;
    const u64x2 x = ld2(&a.d[(size_t)ct * a.cs + (size_t)poly * a.ps + ((size_t)limb << logN) + n]);
    const u64x2 y = ld2(&b.d[(size_t)ct * b.cs + (size_t)poly * b.ps + ((size_t)limb << logN) + n]);
    st2(out + (((size_t)blockIdx.z * L1 + limb) << logN) + n, sub ? sub_mod(x.x, y.x, q) : add_mod(x.x, y.x, q),
        sub ? sub_mod(x.y, y.y, q) : add_mod(x.y, y.y, q));
}

// a (.) pt for a plaintext pt[L1'][N] (limbs 0..L1-1 used)
__global__ void k_mlp_pmul(View a, const u64 *pt, u64 *out, int logN, int L1, const PrimeC *pc)
{
    const unsigned n = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y;
    const unsigned ct = blockIdx.z >> 1, poly = blockIdx.z & 1;
    const PrimeC p = pc[limb];
    const u64 x = ld(a, ct, poly, limb, logN, n);
    out[(((size_t)blockIdx.z * L1 + limb) << logN) + n] = mul_mod(x, pt[((size_t)limb << logN) + n], p);
}

// ct + the constant polynomial k (|k| < 2^62): in the NTT domain k is added
// to every entry of c0
__global__ void k_mlp_addconst(View a, u64 kabs, int neg, u64 *out, int logN, int L1, const PrimeC *pc)
{
    const unsigned n = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y;
    const unsigned ct = blockIdx.z >> 1, poly = blockIdx.z & 1;
    const PrimeC p = pc[limb];
    u64 x = ld(a, ct, poly, limb, logN, n);
    if (poly == 0) {
        u128w t{to_mont_k(kabs, p), 0};
        u64 kr = redc(t, p.q, p.qneg);  // k mod q
        x = neg ? sub_mod(x, kr, p.q) : add_mod(x, kr, p.q);
    }
    out[(((size_t)blockIdx.z * L1 + limb) << logN) + n] = x;
}

constexpr int MAX_TERMS = 4;
struct Terms {
    View v[MAX_TERMS];
    u64 k[MAX_TERMS];  // |k_j| < 2^62
    int neg[MAX_TERMS];
    int n;
};

// sum_j k_j x_j: every product x (k 2^64 mod q) is below q^2, four of them
// stay below q 2^64, so one REDC ends the lazy 128-bit sum
__global__ void k_mlp_lincomb(Terms T, u64 *out, int logN, int L1, const PrimeC *pc)
{
    const unsigned n = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y;
    const unsigned ct = blockIdx.z >> 1, poly = blockIdx.z & 1;
    const PrimeC p = pc[limb];
    u128w acc{0, 0};
    for (int j = 0; j < T.n; j++) {
        u64 km = to_mont_k(T.k[j], p);
        if (T.neg[j] && km) km = p.q - km;
        acc_wide(acc, mul_wide(ld(T.v[j], ct, poly, limb, logN, n), km));
    }
    out[(((size_t)blockIdx.z * L1 + limb) << logN) + n] = redc(acc, p.q, p.qneg);
}

// sum over the count ciphertexts of a; grid (N/threads, L1, 2)
__global__ void k_mlp_batchsum(View a, int count, u64 *out, int logN, int L1, const PrimeC *pc)
{
    const unsigned n = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y, poly = blockIdx.z;
    const u64 q = pc[limb].q;
    u64 s = 0;
    for (int c = 0; c < count; c++) s = add_mod(s, ld(a, c, poly, limb, logN, n), q);
    out[(((size_t)poly * L1 + limb) << logN) + n] = s;
}

// ---------------------------------------------------------------- host side

struct MlpError {
    int code;
    std::string msg;
};

[[noreturn]] void mthrow(int code, const std::string &m) { throw MlpError{code, m}; }

void hck(hipError_t e, const char *what)
{
    if (e != hipSuccess) mthrow(RBK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void rck(int rc)
{
    if (rc) throw MlpError{rc, rbk_last_error()};
}

// best-fit pool of device buffers; a buffer is reused by later work on the
// same stream only, so stream order keeps reuse safe
// Device buffers of step results, reused best-fit.  With block-parallel
// steps two lanes issue work (the context stream and a side stream): each
// lane reuses only buffers last used by itself (stream order keeps that
// safe); a buffer both lanes used waits in `deferred` until the lanes join.
struct Pool {
    std::multimap<size_t, u64 *> free_[2];
    std::vector<std::pair<u64 *, size_t>> deferred;
    std::vector<u64 *> all_;
    ~Pool()
    {
        for (u64 *p : all_) (void)hipFree(p);
    }
    u64 *take(size_t words, size_t &cap, int lane)
    {
        auto &fl = free_[lane];
        auto it = fl.lower_bound(words);
        if (it != fl.end() && it->first <= 2 * words) {
            cap = it->first;
            u64 *p = it->second;
            fl.erase(it);
            return p;
        }
        u64 *p = nullptr;
        if (hipMalloc((void **)&p, words * sizeof(u64)) != hipSuccess) mthrow(RBK_ENOMEM, "MLP device allocation failed");
        all_.push_back(p);
        cap = words;
        return p;
    }
    void give(u64 *p, size_t cap, int lane) { free_[lane].emplace(cap, p); }
    void defer(u64 *p, size_t cap) { deferred.emplace_back(p, cap); }
    // the side lane has finished everything issued so far (the context stream waited for it)
    void joined()
    {
        for (auto &d : deferred) free_[0].emplace(d.second, d.first);
        deferred.clear();
    }
};

struct Blk {
    Pool *pool;
    u64 *d;
    size_t cap;
    bool main_use = false;   // touched by the context-stream lane
    int side_epoch = -1;     // last side-lane epoch that touched it
    const int *epoch = nullptr;  // the current (not yet joined) side epoch
    ~Blk()
    {
        const bool side_now = epoch && side_epoch == *epoch;
        if (!side_now) pool->give(d, cap, 0);        // only the context stream may still use it
        else if (!main_use) pool->give(d, cap, 1);   // only the side lane used it
        else pool->defer(d, cap);
    }
};

struct Vec {
    std::shared_ptr<Blk> blk;  // null for caller memory
    const u64 *d = nullptr;
    int lv = -1;
    long cs = 0, ps = 0;
    int count = 0;
    double s = 0;
};

enum Kind { K_W = 0, K_WSTAR = 1, K_V = 2, K_VSTAR = 3 };
struct Key {
    int kind, h, tile;
};

struct Shape {
    int k0 = 0, H = 0, o = 0, r = 0, c = 0, tiles = 1, degree = 2;
    std::vector<int> widths;
    double act[3] = {0, 0, 0};
    double gamma = 0, eta = 0, mu = 0, log2_scale = 0;
    bool literal = false, l2 = false;
    std::vector<Key> layout;

    std::pair<int, int> dims(int h) const { return {h == 1 ? k0 : widths[h - 2], widths[h - 1]}; }
    int n_tiles(int h) const { return h == 1 ? tiles : 1; }
    int pos(int kind, int h, int tile) const
    {
        for (size_t i = 0; i < layout.size(); i++)
            if (layout[i].kind == kind && layout[i].h == h && layout[i].tile == tile) return (int)i;
        return -1;
    }
};

template <class T>
struct Sample {
    std::vector<T> x;
    T ye, yr;
};

// The step (mirrors the definition used to pin it: same operations, same
// order, same constants).
template <class O>
struct Step {
    using T = typename O::T;
    O &ops;
    const Shape &sh;

    T sum_rows(T s)
    {
        for (int k = sh.r >> 1; k >= 1; k >>= 1) s = ops.rot_add(s, (int64_t)sh.c * k);
        return s;
    }
    T sum_cols(T u)
    {
        for (int k = sh.c >> 1; k >= 1; k >>= 1) u = ops.rot_add(u, k);
        u = ops.mask(u);
        for (int k = 1; k < sh.c; k <<= 1) u = ops.rot_add(u, -(int64_t)k);
        return u;
    }
    // (f(z), f'(z)); has_d false with the literal derivative or without want_d (a forward pass only)
    void activation(const T &z, T &a, T &d, bool &has_d, bool want_d = true)
    {
        const double a1 = sh.act[0], a2 = sh.act[1], a3 = sh.act[2];
        T z2 = ops.mul(z, z);
        has_d = !sh.literal && want_d;
        if (sh.degree == 2) {
            T t2 = ops.affine(z2, a2, 0.0);
            a = a1 != 0.0 ? ops.add(t2, ops.lincomb({{z, a1}}, &t2, 0.0)) : t2;
            if (has_d) d = ops.affine(z, 2.0 * a2, a1);
            return;
        }
        T z3 = ops.mul(z2, z);
        T t3 = ops.affine(z3, a3, 0.0);
        std::vector<std::pair<T, double>> terms;
        if (a2 != 0.0) terms.push_back({z2, a2});
        if (a1 != 0.0) terms.push_back({z, a1});
        a = terms.empty() ? t3 : ops.add(t3, ops.lincomb(terms, &t3, 0.0));
        if (has_d) {
            T d2 = ops.affine(z2, 3.0 * a3, 0.0);
            d = a2 != 0.0 ? ops.add(d2, ops.lincomb({{z, 2.0 * a2}}, &d2, 0.0)) : d2;
            d = ops.affine(d, 1.0, a1);
        }
    }

    static void acc(T &slot, bool &have, const T &v, O &ops)
    {
        if (!have) {
            slot = v;
            have = true;
        } else {
            slot = ops.add(slot, v);
        }
    }

    // Inference with early exit: the forward pass of blocks 1..last on one
    // (batched) sample; the output of every block's local classifier.
    std::vector<T> infer(const std::vector<T> &state, const std::vector<T> &x, int last)
    {
        std::vector<T> out;
        std::vector<T> a_in = x;
        for (int h = 1; h <= last; h++) {
            const T &Ws = state[sh.pos(K_WSTAR, h, 0)];
            T a, d;
            bool has_d = false;
            if (h % 2 == 1) {
                T p;
                bool have_p = false;
                for (int i = 0; i < sh.n_tiles(h); i++) {
                    bool hp = have_p;
                    acc(p, hp, ops.mul(a_in[i], state[sh.pos(K_W, h, i)]), ops);
                    have_p = hp;
                }
                activation(sum_rows(p), a, d, has_d, false);
                out.push_back(sum_cols(ops.mul(a, Ws)));
            } else {
                activation(sum_cols(ops.mul(a_in[0], state[sh.pos(K_W, h, 0)])), a, d, has_d, false);
                out.push_back(sum_rows(ops.mul(a, Ws)));
            }
            a_in.assign(1, a);
        }
        return out;
    }

    std::vector<T> run(const std::vector<T> &state, const std::vector<Sample<T>> &samples, int b, int t, bool boot)
    {
        const int H = sh.H;
        std::vector<std::vector<T>> grads(H + 1);
        std::vector<std::vector<char>> have_g(H + 1);
        std::vector<T> gstar(H + 1);
        std::vector<char> have_s(H + 1, 0);
        for (int h = 1; h <= H; h++) {
            grads[h].resize(sh.n_tiles(h));
            have_g[h].assign(sh.n_tiles(h), 0);
        }
        // one batched sample: every block's classifier and backward pass on
        // the side lane, next to the following block's forward pass
        const bool par = samples.size() == 1 && H > 1 && ops.parallel_ok();
        for (const Sample<T> &smp : samples) {
            std::vector<T> a_in = smp.x;
            for (int h = 1; h <= H; h++) {
                const int nt = sh.n_tiles(h);
                const T &Ws = state[sh.pos(K_WSTAR, h, 0)];
                T z, a, d, yhat, g, da;
                bool has_d = false;
                if (h % 2 == 1) {
                    T p;
                    bool have_p = false;
                    for (int i = 0; i < nt; i++) {
                        bool hp = have_p;
                        acc(p, hp, ops.mul(a_in[i], state[sh.pos(K_W, h, i)]), ops);
                        have_p = hp;
                    }
                    z = sum_rows(p);
                    activation(z, a, d, has_d);
                    if (par) ops.side_begin();
                    yhat = sum_cols(ops.mul(a, Ws));
                    g = ops.sub(yhat, ops.lincomb({{smp.ye, 1.0}}, &yhat, 0.0));
                    bool hs = have_s[h];
                    acc(gstar[h], hs, ops.bsum(ops.mul(a, g)), ops);
                    have_s[h] = hs;
                    da = sum_rows(ops.mul(g, Ws));
                } else {
                    z = sum_cols(ops.mul(a_in[0], state[sh.pos(K_W, h, 0)]));
                    activation(z, a, d, has_d);
                    if (par) ops.side_begin();
                    yhat = sum_rows(ops.mul(a, Ws));
                    g = ops.sub(yhat, ops.lincomb({{smp.yr, 1.0}}, &yhat, 0.0));
                    bool hs = have_s[h];
                    acc(gstar[h], hs, ops.bsum(ops.mul(a, g)), ops);
                    have_s[h] = hs;
                    da = sum_cols(ops.mul(g, Ws));
                }
                T dz = has_d ? ops.mul(da, d) : ops.affine(da, 2.0, 1.0);
                for (int i = 0; i < nt; i++) {
                    bool hg = have_g[h][i];
                    acc(grads[h][i], hg, ops.bsum(ops.mul(a_in[i], dz)), ops);
                    have_g[h][i] = hg;
                }
                if (par) ops.side_end();
                a_in.assign(1, a);
            }
        }
        if (par) ops.join();

        const double gm = sh.gamma, e = sh.eta, m = sh.mu;
        const double Tsc = std::pow(2.0, sh.log2_scale);
        std::vector<T> out(state.size());
        for (int h = 1; h <= H; h++) {
            for (int i = 0; i <= sh.n_tiles(h); i++) {
                const bool star = i == sh.n_tiles(h);
                const int pw = star ? sh.pos(K_WSTAR, h, 0) : sh.pos(K_W, h, i);
                const int pv = star ? sh.pos(K_VSTAR, h, 0) : sh.pos(K_V, h, i);
                const T &G = star ? gstar[h] : grads[h][i];
                const T &W = state[pw];
                std::vector<std::pair<T, double>> wt, vt;
                if (sh.l2) {
                    wt = {{W, 1.0 - gm * (1.0 + m) * e}, {G, -gm * (1.0 + m) / b}};
                    vt = {{G, 1.0 / b}, {W, e}};
                } else {
                    wt = {{W, 1.0}, {G, -gm * (1.0 + m) * (1.0 + e) / b}};
                    vt = {{G, (1.0 + e) / b}};
                }
                if (t > 1) {
                    wt.push_back({state[pv], -gm * m * m});
                    vt.push_back({state[pv], m});
                }
                out[pw] = ops.lincomb(wt, nullptr, Tsc);
                out[pv] = ops.lincomb(vt, nullptr, Tsc);
            }
        }
        if (boot) ops.bootstrap(out);
        return out;
    }
};

// levels only
struct LevelOps {
    using T = int;
    int mul(int a, int b) { return std::min(a, b) - 1; }
    int add(int a, int b) { return std::min(a, b); }
    int sub(int a, int b) { return std::min(a, b); }
    int rot_add(int a, int64_t) { return a; }
    int mask(int a) { return a - 1; }
    int affine(int a, double, double) { return a; }
    int bsum(int a) { return a; }
    int lincomb(const std::vector<std::pair<int, double>> &terms, const int *like, double)
    {
        int lv = terms[0].first;
        for (auto &t : terms) lv = std::min(lv, t.first);
        if (like) lv = std::min(lv, *like + 1);
        return lv - 1;
    }
    void bootstrap(std::vector<int> &) {}
    bool parallel_ok() { return false; }
    void side_begin() {}
    void side_end() {}
    void join() {}
};

int step_depth(const Shape &sh)
{
    LevelOps ops;
    Step<LevelOps> st{ops, sh};
    const int w = 1000, big = 1000000;
    std::vector<int> state(sh.layout.size(), w);
    Sample<int> s{std::vector<int>(sh.tiles, big), big, big};
    std::vector<int> out = st.run(state, {s}, 1, 2, false);
    return w - *std::min_element(out.begin(), out.end());
}

}  // namespace

struct rbk_mlp {
    rbk_ctx *c = nullptr;
    Shape sh;
    Pool pool;
    // block-parallel steps: the side lane's stream, its own key-switching
    // workspace, the fork / join events and the side epoch (joins so far)
    hipStream_t side = nullptr;
    u64 *side_ws = nullptr;
    size_t side_ws_words = 0;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int epoch = 0;
    bool block_parallel = true;
    // every state ciphertext lives in a buffer of its own ("home", sized for
    // the top level): a step reads the homes and copies its results into them
    // last, so the same device addresses serve every step (and the replays of
    // a captured step)
    std::vector<u64 *> home;
    std::vector<Vec> state;
    std::map<int, u64 *> masks;
    std::vector<int64_t> scalars;
    int depth = 0;

    ~rbk_mlp()
    {
        if (c) {
            (void)hipStreamSynchronize(c->stream);
            c->live_mlps--;
        }
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (side_ws) (void)hipFree(side_ws);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        state.clear();
        for (u64 *h : home) (void)hipFree(h);
        for (auto &kv : masks) (void)hipFree(kv.second);
    }
};

namespace {

struct GpuOps {
    using T = Vec;
    rbk_mlp *m;
    rbk_ctx *c;
    size_t N;
    int logN;
    unsigned thr;

    int lane = 0;   // 0: the context stream; 1: the side lane (block-parallel steps)

    explicit GpuOps(rbk_mlp *mm) : m(mm), c(mm->c), N(mm->c->N), logN(mm->c->logN)
    {
        thr = (unsigned)std::min<size_t>(MT, N);
    }

    // ---- block-parallel steps: a block's classifier and backward pass run on
    // the side lane while the next block's forward pass continues on the
    // context stream (paper Section 4.2.3: no information flows between
    // blocks in the backward pass)
    bool parallel_ok()
    {
        if (!m->block_parallel || c->capturing || c->timing) return false;
        if (!m->side) {
            if (hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess) {
                m->side = nullptr;
                return false;
            }
            if (hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) != hipSuccess)
                return false;
        }
        return true;
    }
    // swap the context's stream and key-switching workspace with the side lane's
    void swap_lane()
    {
        std::swap(c->stream, m->side);
        std::swap(c->ws, m->side_ws);
        std::swap(c->ws_words, m->side_ws_words);
        lane ^= 1;
    }
    bool forked = false;   // the side lane has work the context stream has not waited for
    void side_begin()
    {
        hck(hipEventRecord(m->ev_fork, c->stream), "fork");
        hck(hipStreamWaitEvent(m->side, m->ev_fork, 0), "fork");
        forked = true;
        swap_lane();
    }
    void side_end() { swap_lane(); }
    void join()
    {
        hck(hipEventRecord(m->ev_join, m->side), "join");
        hck(hipStreamWaitEvent(c->stream, m->ev_join, 0), "join");
        forked = false;
        m->epoch++;
        m->pool.joined();
    }
    // a step that fails half-way leaves the context on its own stream and
    // workspace, joined with the side lane
    ~GpuOps()
    {
        if (lane) swap_lane();
        if (forked) {
            if (hipEventRecord(m->ev_join, m->side) != hipSuccess ||
                hipStreamWaitEvent(c->stream, m->ev_join, 0) != hipSuccess)
                (void)hipStreamSynchronize(m->side);
            m->epoch++;
            m->pool.joined();
        }
    }
    void touch(const Vec &v)
    {
        if (!v.blk) return;
        if (lane) v.blk->side_epoch = m->epoch;
        else v.blk->main_use = true;
    }

    double q(int lv) const { return (double)c->mod[lv]; }
    size_t per(int lv) const { return (size_t)(lv + 1) * N; }

    Vec alloc(int lv, int count)
    {
        size_t cap = 0;
        const size_t words = (size_t)count * 2 * per(lv);
        u64 *d = m->pool.take(words, cap, lane);
        Vec v;
        v.blk = std::shared_ptr<Blk>(new Blk{&m->pool, d, cap});
        v.blk->epoch = &m->epoch;
        touch(v);
        v.d = d;
        v.lv = lv;
        v.ps = (long)per(lv);
        v.cs = 2 * v.ps;
        v.count = count;
        return v;
    }
    static View view(const Vec &v, int cnt) { return View{v.d, (v.count == 1 && cnt > 1) ? 0 : v.cs, v.ps}; }
    static int bcast(const Vec &a, const Vec &b)
    {
        if (a.count != b.count && a.count != 1 && b.count != 1) mthrow(RBK_EINVAL, "batch sizes do not match");
        return std::max(a.count, b.count);
    }
    dim3 grid(int lv, int z) const { return dim3((unsigned)(N / thr), (unsigned)(lv + 1), (unsigned)z); }
    void launched() { hck(hipGetLastError(), "MLP kernel launch"); }
    void record(int64_t k) { m->scalars.push_back(k); }
    static int64_t to_int(double v)
    {
        if (!(std::fabs(v) < 4611686018427387904.0)) mthrow(RBK_EINVAL, "MLP constant out of range (|k| >= 2^62)");
        return (int64_t)std::nearbyint(v);
    }

    Vec contiguous(const Vec &a)
    {
        touch(a);
        if (a.ps == (long)per(a.lv) && (a.count == 1 || a.cs == 2 * a.ps)) return a;
        Vec o = alloc(a.lv, a.count);
        for (int p = 0; p < 2; p++)
            hck(hipMemcpy2DAsync((u64 *)o.d + p * o.ps, o.cs * sizeof(u64), a.d + p * a.ps, a.cs * sizeof(u64),
                                 per(a.lv) * sizeof(u64), a.count, hipMemcpyDeviceToDevice, c->stream),
                "copy");
        o.s = a.s;
        return o;
    }
    Vec rescaled(Vec &tmp, double s)
    {
        Vec o = alloc(tmp.lv - 1, tmp.count);
        rck(rbk_rescale_batch(c, tmp.d, (u64 *)o.d, tmp.lv, tmp.count));
        o.s = s;
        return o;
    }

    Vec mul(const Vec &a, const Vec &b)
    {
        touch(a);
        touch(b);
        const int lv = std::min(a.lv, b.lv);
        if (lv < 1) mthrow(RBK_ELEVEL, "MLP step: no level left for a product");
        if (!c->relin.data) mthrow(RBK_ENOKEY, "relinearisation key not generated");
        const int cnt = bcast(a, b);
        const size_t P = per(lv);
        u64 *ws = ws_reserve(c, (size_t)cnt * 3 * P + ks_words(c, lv, cnt));
        if (!ws) mthrow(RBK_ENOMEM, "device workspace allocation failed");
        hipLaunchKernelGGL(k_mlp_tensor, grid(lv, cnt), dim3(thr), 0, c->stream, view(a, cnt), view(b, cnt), ws, logN,
                           lv + 1, c->d_pc);
        launched();
        Vec tmp = alloc(lv, cnt);
        rck(keyswitch_run(c, &c->relin, 0, ws + 2 * P, (long)(3 * P), ws, (long)(3 * P), 0, 1, (u64 *)tmp.d,
                          (long)(2 * P), lv, cnt, ws + (size_t)cnt * 3 * P));
        return rescaled(tmp, a.s * b.s / q(lv));
    }
    Vec addsub(const Vec &a, const Vec &b, int sub)
    {
        touch(a);
        touch(b);
        if (a.s != b.s) mthrow(RBK_ESCALE, "MLP step: addition of ciphertexts at different scales");
        const int lv = std::min(a.lv, b.lv), cnt = bcast(a, b);
        Vec o = alloc(lv, cnt);
        const View va = view(a, cnt), vb = view(b, cnt);
        // buffers come from whole allocations at multiples of N words
        if (((uintptr_t)va.d | (uintptr_t)vb.d | (uintptr_t)o.d) & 15 || (va.cs | va.ps | vb.cs | vb.ps) & 1)
            mthrow(RBK_EINVAL, "MLP step: unaligned operands");
        const unsigned t2 = (unsigned)std::min<size_t>(thr, N / 2);
        const dim3 g2((unsigned)(N / (2 * t2)), (unsigned)(lv + 1), (unsigned)(2 * cnt));
        hipLaunchKernelGGL(k_mlp_addsub, g2, dim3(t2), 0, c->stream, va, vb, (u64 *)o.d, logN, lv + 1, sub, c->d_pc);
        launched();
        o.s = a.s;
        return o;
    }
    Vec add(const Vec &a, const Vec &b) { return addsub(a, b, 0); }
    Vec sub(const Vec &a, const Vec &b) { return addsub(a, b, 1); }
    // a + Rot_k(a): the rotation's ModDown adds a in the same pass
    Vec rot_add(const Vec &a, int64_t k)
    {
        Vec x = contiguous(a);
        Vec o = alloc(a.lv, a.count);
        rck(rotate_add_batch_g(c, x.d, x.d, (u64 *)o.d, a.lv, a.count, rbk_galois_elt(c, k)));
        o.s = a.s;
        return o;
    }
    const u64 *mask_pt(int lv)
    {
        auto it = m->masks.find(lv);
        if (it != m->masks.end()) return it->second;
        const size_t n = N / 2;
        std::vector<double> re(n, 0.0);
        for (size_t j = 0; j < n; j += (size_t)m->sh.c) re[j] = 1.0;
        u64 *pt = nullptr;
        hck(hipMalloc((void **)&pt, per(lv) * sizeof(u64)), "mask allocation");
        m->masks[lv] = pt;
        rck(rbk_encode(c, re.data(), nullptr, n, lv, q(lv), pt));
        return pt;
    }
    Vec mask(const Vec &a)
    {
        touch(a);
        const int lv = a.lv;
        if (lv < 1) mthrow(RBK_ELEVEL, "MLP step: no level left for the mask");
        const u64 *pt = mask_pt(lv);
        Vec tmp = alloc(lv, a.count);
        hipLaunchKernelGGL(k_mlp_pmul, grid(lv, 2 * a.count), dim3(thr), 0, c->stream, view(a, a.count), pt,
                           (u64 *)tmp.d, logN, lv + 1, c->d_pc);
        launched();
        return rescaled(tmp, a.s);
    }
    Vec affine(const Vec &a, double alpha, double beta)
    {
        touch(a);
        const double s = a.s / alpha;
        if (beta == 0.0) {
            Vec r = a;
            r.s = s;
            return r;
        }
        const int64_t k = to_int(beta * s);
        record(k);
        Vec o = alloc(a.lv, a.count);
        hipLaunchKernelGGL(k_mlp_addconst, grid(a.lv, 2 * a.count), dim3(thr), 0, c->stream, view(a, a.count),
                           (u64)(k < 0 ? -k : k), k < 0 ? 1 : 0, (u64 *)o.d, logN, a.lv + 1, c->d_pc);
        launched();
        o.s = s;
        return o;
    }
    Vec lincomb(const std::vector<std::pair<Vec, double>> &terms, const Vec *like, double Tsc)
    {
        if (terms.empty() || terms.size() > (size_t)MAX_TERMS) mthrow(RBK_EINVAL, "bad linear combination");
        int lv = terms[0].first.lv, cnt = 1;
        for (auto &t : terms) {
            lv = std::min(lv, t.first.lv);
            cnt = std::max(cnt, t.first.count);
        }
        if (like) {
            lv = std::min(lv, like->lv + 1);
            Tsc = like->s;
        }
        if (lv < 1) mthrow(RBK_ELEVEL, "MLP step: no level left for a constant product");
        const double ql = q(lv);
        for (auto &t : terms) touch(t.first);
        Terms K{};
        K.n = (int)terms.size();
        for (int j = 0; j < K.n; j++) {
            const Vec &x = terms[j].first;
            if (x.count != cnt && x.count != 1) mthrow(RBK_EINVAL, "batch sizes do not match");
            const int64_t k = to_int(terms[j].second * ql * Tsc / x.s);
            record(k);
            K.v[j] = view(x, cnt);
            K.k[j] = (u64)(k < 0 ? -k : k);
            K.neg[j] = k < 0 ? 1 : 0;
        }
        Vec tmp = alloc(lv, cnt);
        hipLaunchKernelGGL(k_mlp_lincomb, grid(lv, 2 * cnt), dim3(thr), 0, c->stream, K, (u64 *)tmp.d, logN, lv + 1,
                           c->d_pc);
        launched();
        return rescaled(tmp, Tsc);
    }
    Vec bsum(const Vec &a)
    {
        touch(a);
        if (a.count == 1) return a;
        Vec o = alloc(a.lv, 1);
        hipLaunchKernelGGL(k_mlp_batchsum, grid(a.lv, 2), dim3(thr), 0, c->stream, view(a, a.count), a.count,
                           (u64 *)o.d, logN, a.lv + 1, c->d_pc);
        launched();
        o.s = a.s;
        return o;
    }
    void bootstrap(std::vector<Vec> &cts)
    {
        for (auto &x : cts) touch(x);
        if (!c->boot) mthrow(RBK_ESTATE, "bootstrapping is not set up (rbk_boot_setup)");
        int levels[4], np = 0, ns = 0;
        rck(rbk_boot_info(c, levels, &np, &ns));
        const int lo = levels[3], n = (int)cts.size();
        Vec in = alloc(0, n);
        std::vector<double> s_in(n), s_out(n);
        for (int i = 0; i < n; i++) {
            const Vec &x = cts[i];
            hck(hipMemcpy2DAsync((u64 *)in.d + (size_t)i * 2 * N, N * sizeof(u64), x.d, x.ps * sizeof(u64),
                                 N * sizeof(u64), 2, hipMemcpyDeviceToDevice, c->stream),
                "copy");
            s_in[i] = x.s;
        }
        Vec out = alloc(lo, n);
        rck(rbk_bootstrap_batch(c, in.d, s_in.data(), (u64 *)out.d, s_out.data(), n));
        for (int i = 0; i < n; i++) {
            Vec v = out;
            v.d = out.d + (size_t)i * 2 * per(lo);
            v.count = 1;
            v.s = s_out[i];
            cts[i] = v;
        }
    }
};

int mfail(const MlpError &e) { return rbk_set_error(e.code, e.msg.c_str()); }

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" int rbk_mlp_create(rbk_ctx *c, const rbk_mlp_desc *d, rbk_mlp **out)
{
    if (!c || !d || !out || (d->n_layers && !d->widths)) return rbk_set_error(RBK_EINVAL, "null argument");
    *out = nullptr;
    Shape sh;
    sh.k0 = (int)d->k0;
    sh.H = (int)d->n_layers;
    sh.o = (int)d->n_out;
    sh.r = (int)d->r;
    sh.c = (int)d->c;
    for (uint32_t i = 0; i < d->n_layers; i++) sh.widths.push_back((int)d->widths[i]);
    for (int i = 0; i < 3; i++) sh.act[i] = d->act[i];
    sh.gamma = d->gamma;
    sh.eta = d->eta;
    sh.mu = d->mu;
    sh.log2_scale = d->log2_scale;
    sh.literal = (d->flags & RBK_MLP_LITERAL_DERIV) != 0;
    sh.l2 = (d->flags & RBK_MLP_L2_DECAY) != 0;
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    if (sh.H < 1 || sh.k0 < 1 || sh.o < 1) return rbk_set_error(RBK_EINVAL, "empty MLP");
    if (!pow2(sh.r) || !pow2(sh.c) || (size_t)sh.r * sh.c != c->N / 2)
        return rbk_set_error(RBK_EINVAL, "r and c must be powers of two with r c = N/2");
    for (int w : sh.widths)
        if (w < 1) return rbk_set_error(RBK_EINVAL, "empty layer");
    sh.degree = sh.act[2] != 0.0 ? 3 : 2;
    if (!((sh.degree == 3 ? sh.act[2] : sh.act[1]) > 0.0))
        return rbk_set_error(RBK_EINVAL, "the leading activation coefficient must be positive");
    for (double v : {sh.act[0], sh.act[1], sh.act[2], sh.gamma, sh.eta, sh.mu})
        if (!std::isfinite(v)) return rbk_set_error(RBK_EINVAL, "non-finite hyperparameter");
    if (!(sh.log2_scale > 0.0 && sh.log2_scale < 62.0)) return rbk_set_error(RBK_EINVAL, "log2_scale out of (0, 62)");
    sh.tiles = (sh.k0 + sh.r - 1) / sh.r;
    for (int h = 1; h <= sh.H; h++) {
        auto dk = sh.dims(h);
        bool ok = h % 2 == 1 ? ((h == 1 || dk.first <= sh.r) && dk.second <= sh.c && sh.o <= sh.r)
                             : (dk.first <= sh.c && dk.second <= sh.r && sh.o <= sh.c);
        if (!ok) return rbk_set_error(RBK_EINVAL, ("layer " + std::to_string(h) + " does not fit the r x c packing").c_str());
    }
    for (int h = 1; h <= sh.H; h++) {
        for (int kind : {K_W, K_WSTAR, K_V, K_VSTAR}) {
            const int n = (kind == K_W || kind == K_V) ? sh.n_tiles(h) : 1;
            for (int t = 0; t < n; t++) sh.layout.push_back(Key{kind, h, t});
        }
    }
    rbk_mlp *m = new (std::nothrow) rbk_mlp;
    if (!m) return rbk_set_error(RBK_ENOMEM, "host allocation failed");
    m->c = c;
    c->live_mlps++;
    m->sh = sh;
    m->state.resize(sh.layout.size());
    m->home.assign(sh.layout.size(), nullptr);
    m->depth = step_depth(sh);
    *out = m;
    return RBK_OK;
}

extern "C" int rbk_mlp_destroy(rbk_mlp *m)
{
    delete m;
    return RBK_OK;
}

extern "C" int rbk_mlp_info(const rbk_mlp *m, int *info)
{
    if (!m || !info) return rbk_set_error(RBK_EINVAL, "null argument");
    info[0] = m->sh.tiles;
    info[1] = (int)m->sh.layout.size();
    info[2] = m->depth;
    return RBK_OK;
}

extern "C" int rbk_mlp_rotations(const rbk_mlp *m, int64_t *ks, int max)
{
    if (!m || (max > 0 && !ks)) return rbk_set_error(RBK_EINVAL, "null argument");
    std::set<int64_t> s;
    for (int k = m->sh.r >> 1; k >= 1; k >>= 1) s.insert((int64_t)m->sh.c * k);
    for (int k = m->sh.c >> 1; k >= 1; k >>= 1) {
        s.insert(k);
        s.insert(-(int64_t)k);
    }
    int i = 0;
    for (int64_t k : s) {
        if (i < max) ks[i] = k;
        i++;
    }
    return i;
}

extern "C" int rbk_mlp_set_state(rbk_mlp *m, int idx, const uint64_t *d_ct, int level, double scale)
{
    if (!m || !d_ct) return rbk_set_error(RBK_EINVAL, "null argument");
    if (idx < 0 || idx >= (int)m->state.size()) return rbk_set_error(RBK_EINVAL, "state index out of range");
    if (level < 0 || level >= m->c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    if (!(scale > 0.0)) return rbk_set_error(RBK_EINVAL, "scale must be positive");
    if (m->c->capturing) return rbk_set_error(RBK_ESTATE, "not allowed during graph capture");
    const size_t N = m->c->N, P = (size_t)(level + 1) * N;
    u64 *&h = m->home[idx];
    if (!h && hipMalloc((void **)&h, (size_t)2 * m->c->nQ * N * sizeof(u64)) != hipSuccess) {
        h = nullptr;
        return rbk_set_error(RBK_ENOMEM, "state allocation failed");
    }
    if (hipMemcpyAsync(h, d_ct, 2 * P * sizeof(u64), hipMemcpyDeviceToDevice, m->c->stream) != hipSuccess)
        return rbk_set_error(RBK_EDEVICE, "copy failed");
    Vec v;
    v.d = h;
    v.lv = level;
    v.ps = (long)P;
    v.cs = 2 * v.ps;
    v.count = 1;
    v.s = scale;
    m->state[idx] = v;
    return RBK_OK;
}

extern "C" int rbk_mlp_get_state(rbk_mlp *m, int idx, uint64_t *d_ct, int *level, double *scale)
{
    if (!m || !level || !scale) return rbk_set_error(RBK_EINVAL, "null argument");
    if (idx < 0 || idx >= (int)m->state.size()) return rbk_set_error(RBK_EINVAL, "state index out of range");
    const Vec &v = m->state[idx];
    if (!v.d) return rbk_set_error(RBK_ESTATE, "state ciphertext not set");
    *level = v.lv;
    *scale = v.s;
    if (d_ct) {
        const size_t N = m->c->N, P = (size_t)(v.lv + 1) * N;
        if (hipMemcpy2DAsync(d_ct, P * sizeof(u64), v.d, v.ps * sizeof(u64), P * sizeof(u64), 2, hipMemcpyDeviceToDevice,
                             m->c->stream) != hipSuccess)
            return rbk_set_error(RBK_EDEVICE, "copy failed");
    }
    return RBK_OK;
}

extern "C" int rbk_mlp_set_mask(rbk_mlp *m, int level, const uint64_t *d_pt)
{
    if (!m || !d_pt) return rbk_set_error(RBK_EINVAL, "null argument");
    if (level < 1 || level >= m->c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    const size_t words = (size_t)(level + 1) * m->c->N;
    u64 *&pt = m->masks[level];
    if (!pt && hipMalloc((void **)&pt, words * sizeof(u64)) != hipSuccess) {
        m->masks.erase(level);
        return rbk_set_error(RBK_ENOMEM, "mask allocation failed");
    }
    if (hipMemcpyAsync(pt, d_pt, words * sizeof(u64), hipMemcpyDeviceToDevice, m->c->stream) != hipSuccess)
        return rbk_set_error(RBK_EDEVICE, "copy failed");
    return RBK_OK;
}

extern "C" int rbk_mlp_train_step(rbk_mlp *m, const uint64_t *d_x, const uint64_t *d_y_exp, const uint64_t *d_y_rep,
                                  int b, int level, double scale, int t, uint32_t flags)
{
    if (!m || !d_x || !d_y_exp || !d_y_rep) return rbk_set_error(RBK_EINVAL, "null argument");
    if (b < 1 || t < 1) return rbk_set_error(RBK_EINVAL, "need b >= 1 and t >= 1");
    if (level < 0 || level >= m->c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    if (!(scale > 0.0)) return rbk_set_error(RBK_EINVAL, "scale must be positive");
    const Shape &sh = m->sh;
    for (size_t i = 0; i < sh.layout.size(); i++) {
        const bool is_v = sh.layout[i].kind == K_V || sh.layout[i].kind == K_VSTAR;
        if ((!is_v || t > 1) && !m->state[i].d) return rbk_set_error(RBK_ESTATE, "state ciphertext not set");
    }
    try {
        m->block_parallel = (flags & RBK_MLP_SEQUENTIAL) == 0;
        GpuOps ops(m);
        m->scalars.clear();
        const size_t P = ops.per(level);
        const long ct_x = (long)(sh.tiles * 2 * P), ct_y = (long)(2 * P);
        auto input = [&](const uint64_t *base, long cs, int count) {
            Vec v;
            v.d = base;
            v.lv = level;
            v.ps = (long)P;
            v.cs = cs;
            v.count = count;
            v.s = scale;
            return v;
        };
        std::vector<Sample<Vec>> samples;
        if (flags & RBK_MLP_PER_SAMPLE) {
            for (int i = 0; i < b; i++) {
                Sample<Vec> s;
                for (int tt = 0; tt < sh.tiles; tt++) s.x.push_back(input(d_x + i * ct_x + tt * 2 * P, ct_x, 1));
                s.ye = input(d_y_exp + i * ct_y, ct_y, 1);
                s.yr = input(d_y_rep + i * ct_y, ct_y, 1);
                samples.push_back(s);
            }
        } else {
            Sample<Vec> s;
            for (int tt = 0; tt < sh.tiles; tt++) s.x.push_back(input(d_x + tt * 2 * P, ct_x, b));
            s.ye = input(d_y_exp, ct_y, b);
            s.yr = input(d_y_rep, ct_y, b);
            samples.push_back(s);
        }
        Step<GpuOps> st{ops, sh};
        std::vector<Vec> next = st.run(m->state, samples, b, t, (flags & RBK_MLP_NO_BOOTSTRAP) == 0);
        samples.clear();
        // the new state goes into the homes (V homes may be new at t = 1)
        const size_t N = m->c->N;
        for (size_t i = 0; i < next.size(); i++) {
            const Vec &x = next[i];
            u64 *&h = m->home[i];
            if (!h) {
                if (m->c->capturing) mthrow(RBK_ESTATE, "state slot without storage during graph capture");
                hck(hipMalloc((void **)&h, (size_t)2 * m->c->nQ * N * sizeof(u64)), "state allocation");
            }
            const size_t P = (size_t)(x.lv + 1) * N;
            hck(hipMemcpy2DAsync(h, P * sizeof(u64), x.d, x.ps * sizeof(u64), P * sizeof(u64), 2,
                                 hipMemcpyDeviceToDevice, m->c->stream),
                "copy");
            Vec v;
            v.d = h;
            v.lv = x.lv;
            v.ps = (long)P;
            v.cs = 2 * v.ps;
            v.count = 1;
            v.s = x.s;
            m->state[i] = v;
        }
    } catch (const MlpError &e) {
        return mfail(e);
    } catch (const std::bad_alloc &) {
        return rbk_set_error(RBK_ENOMEM, "host allocation failed");
    }
    return RBK_OK;
}

extern "C" int rbk_mlp_infer(rbk_mlp *m, const uint64_t *d_x, int b, int level, double scale, int last,
                             uint64_t *d_out, int *levels, double *scales)
{
    if (!m || !d_x || !d_out) return rbk_set_error(RBK_EINVAL, "null argument");
    const Shape &sh = m->sh;
    if (b < 1 || last < 1 || last > sh.H) return rbk_set_error(RBK_EINVAL, "need b >= 1 and 1 <= last <= H");
    if (level < 0 || level >= m->c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    if (!(scale > 0.0)) return rbk_set_error(RBK_EINVAL, "scale must be positive");
    for (size_t i = 0; i < sh.layout.size(); i++) {
        const bool used = sh.layout[i].h <= last && (sh.layout[i].kind == K_W || sh.layout[i].kind == K_WSTAR);
        if (used && !m->state[i].d) return rbk_set_error(RBK_ESTATE, "weight ciphertext not set");
    }
    try {
        GpuOps ops(m);
        m->scalars.clear();
        const size_t P = ops.per(level), N = m->c->N;
        const long ct_x = (long)(sh.tiles * 2 * P);
        std::vector<Vec> x;
        for (int tt = 0; tt < sh.tiles; tt++) {
            Vec v;
            v.d = d_x + tt * 2 * P;
            v.lv = level;
            v.ps = (long)P;
            v.cs = ct_x;
            v.count = b;
            v.s = scale;
            x.push_back(v);
        }
        Step<GpuOps> st{ops, sh};
        std::vector<Vec> out = st.infer(m->state, x, last);
        for (int h = 0; h < last; h++) {
            const Vec &y = out[h];
            const size_t Py = (size_t)(y.lv + 1) * N;
            for (int i = 0; i < b; i++) {
                const u64 *src = y.d + (size_t)(y.count == 1 ? 0 : i) * y.cs;
                u64 *dst = d_out + ((size_t)h * b + i) * 2 * P;
                hck(hipMemcpy2DAsync(dst, Py * sizeof(u64), src, y.ps * sizeof(u64), Py * sizeof(u64), 2,
                                     hipMemcpyDeviceToDevice, m->c->stream),
                    "copy");
            }
            if (levels) levels[h] = y.lv;
            if (scales) scales[h] = y.s;
        }
        hck(hipStreamSynchronize(m->c->stream), "synchronise");   // the pooled results are released on return
    } catch (const MlpError &e) {
        return mfail(e);
    } catch (const std::bad_alloc &) {
        return rbk_set_error(RBK_ENOMEM, "host allocation failed");
    }
    return RBK_OK;
}

extern "C" int rbk_mlp_scalars(const rbk_mlp *m, int64_t *out, int max)
{
    if (!m || (max > 0 && !out)) return rbk_set_error(RBK_EINVAL, "null argument");
    const int n = (int)m->scalars.size();
    for (int i = 0; i < n && i < max; i++) out[i] = m->scalars[i];
    return n;
}

// ---------------------------------------------------------------- float64 weights in and out

namespace {

// Slot matrix (r x c, slot (i, j) at i c + j) of state slot `key` for the
// float64 matrix A (rows x cols, row-major), or the reverse.  RE-blocks (odd
// h) keep W in the row-wise format (W[i][j] at (i, j); tile t holds rows
// t r .. t r + r - 1) and W* column-wise (W*[j][i] at (i, j)); CE-blocks (even
// h) the other way round.  Velocities share the layout of their weights.
struct Placement {
    int rows, cols, row0;  // A's shape and the first row of A this slot holds
    bool transposed;       // A[a][b] sits at slot (b, a) instead of (a - row0, b)
};

Placement placement(const Shape &sh, const Key &k)
{
    const auto dk = sh.dims(k.h);
    const bool odd = k.h % 2 == 1;
    const bool is_w = k.kind == K_W || k.kind == K_V;
    Placement p;
    p.rows = is_w ? dk.first : dk.second;
    p.cols = is_w ? dk.second : sh.o;
    p.row0 = is_w ? k.tile * sh.r : 0;
    p.transposed = odd ? !is_w : is_w;
    return p;
}

// slot index of A[a][b] in the slot matrix, or -1 when this slot does not hold it
long slot_of(const Shape &sh, const Placement &p, int a, int b)
{
    if (p.transposed) return (long)b * sh.c + a;
    const int i = a - p.row0;
    if (i < 0 || i >= sh.r) return -1;
    return (long)i * sh.c + b;
}

const double *matrix_of(const Key &k, const double *const *W, const double *const *Ws, const double *const *V,
                        const double *const *Vs)
{
    const double *const *src = k.kind == K_W ? W : k.kind == K_WSTAR ? Ws : k.kind == K_V ? V : Vs;
    return src ? src[k.h - 1] : nullptr;
}

}  // namespace

extern "C" int rbk_mlp_set_weights(rbk_mlp *m, const double *const *W, const double *const *Wstar,
                                   const double *const *V, const double *const *Vstar, int level, uint64_t seed)
{
    if (!m || !W || !Wstar) return rbk_set_error(RBK_EINVAL, "null argument");
    rbk_ctx *c = m->c;
    if (level < 0 || level >= c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "not allowed during graph capture");
    const Shape &sh = m->sh;
    for (int h = 1; h <= sh.H; h++)
        if (!W[h - 1] || !Wstar[h - 1] || (V && !V[h - 1]) || (Vstar && !Vstar[h - 1]))
            return rbk_set_error(RBK_EINVAL, "null weight matrix");
    const size_t N = c->N, n = N / 2;
    const double scale = std::exp2(sh.log2_scale);
    std::vector<double> slots(n);
    u64 *buf = nullptr;
    if (hipMalloc((void **)&buf, (size_t)3 * (level + 1) * N * sizeof(u64)) != hipSuccess)
        return rbk_set_error(RBK_ENOMEM, "device allocation failed");
    u64 *pt = buf, *ct = buf + (size_t)(level + 1) * N;
    int rc = RBK_OK;
    for (size_t idx = 0; idx < sh.layout.size() && rc == RBK_OK; idx++) {
        const Key &k = sh.layout[idx];
        const Placement p = placement(sh, k);
        const double *A = matrix_of(k, W, Wstar, V, Vstar);
        std::fill(slots.begin(), slots.end(), 0.0);
        if (A)
            for (int a = 0; a < p.rows; a++)
                for (int b = 0; b < p.cols; b++) {
                    const long s = slot_of(sh, p, a, b);
                    if (s >= 0) slots[s] = A[(size_t)a * p.cols + b];
                }
        rc = rbk_encode(c, slots.data(), nullptr, n, level, scale, pt);
        if (!rc) rc = rbk_encrypt_seeded(c, pt, level, seed, idx, ct);
        if (!rc) rc = rbk_mlp_set_state(m, (int)idx, ct, level, scale);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == RBK_OK)
        rc = rbk_set_error(RBK_EDEVICE, "stream synchronisation failed");
    (void)hipFree(buf);
    return rc;
}

extern "C" int rbk_mlp_get_weights(rbk_mlp *m, double *const *W, double *const *Wstar, double *const *V,
                                   double *const *Vstar)
{
    if (!m) return rbk_set_error(RBK_EINVAL, "null argument");
    rbk_ctx *c = m->c;
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "not allowed during graph capture");
    const Shape &sh = m->sh;
    const size_t N = c->N, n = N / 2;
    std::vector<double> re(n);
    u64 *pt = nullptr;
    if (hipMalloc((void **)&pt, (size_t)3 * c->nQ * N * sizeof(u64)) != hipSuccess)
        return rbk_set_error(RBK_ENOMEM, "device allocation failed");
    u64 *ct = pt + (size_t)c->nQ * N;
    int rc = RBK_OK;
    for (size_t idx = 0; idx < sh.layout.size() && rc == RBK_OK; idx++) {
        const Key &k = sh.layout[idx];
        double *const *dst = k.kind == K_W ? W : k.kind == K_WSTAR ? Wstar : k.kind == K_V ? V : Vstar;
        if (!dst) continue;
        double *A = dst[k.h - 1];
        if (!A) continue;
        int lv = 0;
        double s = 0;
        rc = rbk_mlp_get_state(m, (int)idx, ct, &lv, &s);  // contiguous copy (state may sit at a wider stride)
        if (!rc) rc = rbk_decrypt(c, ct, lv, pt);
        if (!rc) rc = rbk_decode(c, pt, lv, s, re.data(), nullptr, n);
        if (rc) break;
        const Placement p = placement(sh, k);
        for (int a = 0; a < p.rows; a++)
            for (int b = 0; b < p.cols; b++) {
                const long s = slot_of(sh, p, a, b);
                if (s >= 0) A[(size_t)a * p.cols + b] = re[s];
            }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(pt);
    return rc;
}
