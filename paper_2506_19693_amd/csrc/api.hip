// librbk host runtime and C ABI: parameters, prime and constant tables,
// key material, workspace, and the orchestration of the kernels for every
// operation declared in include/rbk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <cmath>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

typedef unsigned __int128 u128;


static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int rbk_set_error(int code, const char *msg) { return fail(code, msg); }

#define HIPCK(x)                                                                                     \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) return fail(RBK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define HIPCK_LAUNCH() HIPCK(hipGetLastError())

bool ranges_overlap(const u64 *a, size_t a_words, const u64 *b, size_t b_words)
{
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + a_words * sizeof(u64);
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + b_words * sizeof(u64);
    return a0 < b1 && b0 < a1;
}

// ---------------------------------------------------------------- host number theory

static u64 h_mul(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

static u64 h_pow(u64 b, u64 e, u64 q)
{
    u64 r = 1;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = h_mul(r, b, q);
        b = h_mul(b, b, q);
    }
    return r;
}

static u64 h_inv(u64 a, u64 q) { return h_pow(a % q, q - 2, q); }

static u64 h_shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

static u64 h_mont(u64 x, u64 q) { return (u64)(((u128)(x % q) << 64) % q); }

// Deterministic Miller-Rabin for 64-bit n with the seven bases of Sinclair.
static bool h_is_prime(u64 n)
{
    if (n < 4) return n >= 2;
    if (n % 2 == 0) return false;
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    const u64 bases[7] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
    for (u64 a : bases) {
        a %= n;
        if (a == 0) continue;
        u64 x = h_pow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s && comp; r++) {
            x = h_mul(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

static int gen_primes(int logN, const std::vector<int> &bits, std::vector<u64> &out)
{
    const u64 step = (u64)2 << logN;
    out.clear();
    for (int b : bits) {
        if (b < logN + 2 || b > 60) return -1;
        u64 q = ((u64)1 << b) + 1;
        bool ok = false;
        while (q > step) {
            q -= step;
            if (h_is_prime(q) && std::find(out.begin(), out.end(), q) == out.end()) {
                ok = true;
                break;
            }
        }
        if (!ok) return -1;
        out.push_back(q);
    }
    return 0;
}

// smallest primitive 2N-th root of unity mod q
static u64 min_root(u64 q, int logN)
{
    const u64 N = (u64)1 << logN;
    u64 r = 0;
    for (u64 x = 2;; x++) {
        r = h_pow(x, (q - 1) >> (logN + 1), q);
        if (h_pow(r, N, q) == q - 1) break;
    }
    u64 best = r, r2 = h_mul(r, r, q), cur = r;
    for (u64 k = 1; k < N; k++) {
        cur = h_mul(cur, r2, q);
        best = std::min(best, cur);
    }
    return best;
}

static u64 neg_inv64(u64 q)
{
    u64 x = q;  // q * q = 1 mod 8 for odd q; Newton doubles the correct bits
    for (int i = 0; i < 5; i++) x *= 2 - q * x;
    return (u64)0 - x;
}

static u32 h_brv(u32 x, int bits)
{
    u32 r = 0;
    for (int i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}

// ---------------------------------------------------------------- device memory helpers

template <class T>
static int dev_alloc(rbk_ctx *c, T **p, size_t count)
{
    void *v = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e != hipSuccess) return fail(RBK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->owned.push_back(v);
    *p = (T *)v;
    return RBK_OK;
}

template <class T>
static int dev_upload(rbk_ctx *c, T **p, const std::vector<T> &h)
{
    int rc = dev_alloc(c, p, h.size());
    if (rc) return rc;
    HIPCK(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return RBK_OK;
}

// hipFree that keeps the first failure for rbk_ctx_destroy to report
void dev_free(rbk_ctx_impl *c, void *p)
{
    if (!p) return;
    hipError_t e = hipFree(p);
    if (e != hipSuccess && c->free_error == hipSuccess) c->free_error = e;
}

static void dev_release(rbk_ctx *c, void *p)
{
    if (!p) return;
    auto it = std::find(c->owned.begin(), c->owned.end(), p);
    if (it != c->owned.end()) c->owned.erase(it);
    dev_free(c, p);
}

void release_buffer(rbk_ctx_impl *c, void *p)
{
    if (!p) return;
    if (c->live_graphs > 0) {
        c->retired.push_back(p);
        return;
    }
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, p);
}

u64 *ws_reserve(rbk_ctx_impl *c, size_t words)
{
    if (words <= c->ws_words) return c->ws;
    if (c->ws_ext && c->ws == c->ws_ext) {
        // the caller's buffer (lanes swap their own workspaces in and grow those)
        fail(RBK_ENOMEM, "caller-provided workspace too small: " + std::to_string(words) + " words needed");
        return nullptr;
    }
    if (c->capturing) {
        // the captured work already points into the current workspace
        rbk_set_error(RBK_ESTATE, "workspace too small during graph capture: run the sequence once before capturing");
        return nullptr;
    }
    if (c->ws) {
        release_buffer(c, c->ws);
        c->ws = nullptr;
        c->ws_words = 0;
    }
    void *v = nullptr;
    size_t w = std::max(words, (size_t)1 << 16);
    if (hipMalloc(&v, w * sizeof(u64)) != hipSuccess) return nullptr;
    c->ws = (u64 *)v;
    c->ws_words = w;
    return c->ws;
}

char *desc_upload(rbk_ctx_impl *c, const DescBlob &b, int *rc)
{
    *rc = RBK_OK;
    if (c->capturing) {
        *rc = rbk_set_error(RBK_ESTATE, "list calls upload descriptors and cannot be captured");
        return nullptr;
    }
    const size_t n = std::max(b.h.size(), (size_t)16);
    const int k = c->desc_turn;
    c->desc_turn ^= 1;
    if (!c->desc_evt[k]) {
        if (hipEventCreateWithFlags(&c->desc_evt[k], hipEventDisableTiming) != hipSuccess) {
            c->desc_evt[k] = nullptr;
            *rc = rbk_set_error(RBK_EDEVICE, "event creation failed");
            return nullptr;
        }
    } else if (hipEventSynchronize(c->desc_evt[k]) != hipSuccess) {
        *rc = rbk_set_error(RBK_EDEVICE, "descriptor staging wait failed");
        return nullptr;
    }
    if (n > c->desc_host_bytes[k]) {
        if (c->desc_host[k]) (void)hipHostFree(c->desc_host[k]);
        c->desc_host[k] = nullptr;
        c->desc_host_bytes[k] = 0;
        const size_t w = std::max(n, (size_t)1 << 16);
        if (hipHostMalloc(&c->desc_host[k], w, hipHostMallocDefault) != hipSuccess) {
            c->desc_host[k] = nullptr;
            *rc = rbk_set_error(RBK_ENOMEM, "pinned descriptor staging allocation failed");
            return nullptr;
        }
        c->desc_host_bytes[k] = w;
    }
    if (n > c->desc_dev_bytes) {
        release_buffer(c, c->desc_dev);
        c->desc_dev = nullptr;
        c->desc_dev_bytes = 0;
        const size_t w = std::max(n, (size_t)1 << 16);
        if (hipMalloc(&c->desc_dev, w) != hipSuccess) {
            c->desc_dev = nullptr;
            *rc = rbk_set_error(RBK_ENOMEM, "descriptor arena allocation failed");
            return nullptr;
        }
        c->desc_dev_bytes = w;
    }
    std::memcpy(c->desc_host[k], b.h.data(), b.h.size());
    if (hipMemcpyAsync(c->desc_dev, c->desc_host[k], n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipEventRecord(c->desc_evt[k], c->stream) != hipSuccess) {
        *rc = rbk_set_error(RBK_EDEVICE, "descriptor upload failed");
        return nullptr;
    }
    return (char *)c->desc_dev;
}

// the side streams (default priority) and events of the multi-lane ModDown,
// created on first use on the context's device
int side_streams(rbk_ctx_impl *c)
{
    if (c->side[RBK_LANES - 1] && c->side_ev[RBK_LANES]) return RBK_OK;
    for (int k = 0; k < RBK_LANES; k++)
        if (!c->side[k] && hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking) != hipSuccess) {
            c->side[k] = nullptr;
            return rbk_set_error(RBK_EDEVICE, "side stream creation failed");
        }
    for (int k = 0; k <= RBK_LANES; k++)
        if (!c->side_ev[k] && hipEventCreateWithFlags(&c->side_ev[k], hipEventDisableTiming) != hipSuccess) {
            c->side_ev[k] = nullptr;
            return rbk_set_error(RBK_EDEVICE, "event creation failed");
        }
    return RBK_OK;
}

#define WS(ptr, words)                                                                         \
    u64 *ptr = ws_reserve(c, (words));                                                          \
    if (!ptr)                                                                                   \
        return c->capturing ? RBK_ESTATE                                                        \
                            : (c->ws_ext && c->ws == c->ws_ext ? RBK_ENOMEM                     \
                                                               : fail(RBK_ENOMEM, "device workspace allocation failed"));

// ---------------------------------------------------------------- tables

const ModUpTables &modup_tables(rbk_ctx_impl *ci, int level)
{
    rbk_ctx *c = static_cast<rbk_ctx *>(ci);
    auto it = c->modup.find(level);
    if (it != c->modup.end()) return it->second;
    ModUpTables T;
    T.level = level;
    const int L1 = level + 1, E = L1 + c->nP, alpha = c->alpha;
    T.beta = (L1 + alpha - 1) / alpha;
    std::vector<u64> A((size_t)T.beta * alpha, 0), Ash(A.size(), 0), M((size_t)T.beta * alpha * E, 0);
    auto ext_prime = [&](int e) { return e < L1 ? c->mod[e] : c->mod[c->nQ + e - L1]; };
    for (int j = 0; j < T.beta; j++) {
        int lo = j * alpha, n_in = std::min(alpha, L1 - lo);
        T.lo.push_back(lo);
        T.n_in.push_back(n_in);
        for (int i = 0; i < n_in; i++) {
            u64 qi = c->mod[lo + i];
            u64 prod = 1;
            for (int k = 0; k < n_in; k++)
                if (k != i) prod = h_mul(prod, c->mod[lo + k] % qi, qi);
            A[(size_t)j * alpha + i] = h_inv(prod, qi);
            Ash[(size_t)j * alpha + i] = h_shoup(A[(size_t)j * alpha + i], qi);
            for (int o = 0; o < E - n_in; o++) {
                int e = o < lo ? o : o + n_in;
                u64 t = ext_prime(e), pt = 1;
                for (int k = 0; k < n_in; k++)
                    if (k != i) pt = h_mul(pt, c->mod[lo + k] % t, t);
                M[((size_t)j * alpha + i) * E + o] = h_mont(pt, t);
            }
        }
    }
    if (dev_upload(c, &T.d_A, A) || dev_upload(c, &T.d_Ash, Ash) || dev_upload(c, &T.d_M, M)) {
        // leave the entry absent; callers check the pointers
        static ModUpTables empty;
        return empty;
    }
    return c->modup.emplace(level, T).first->second;
}

static int build_tables(rbk_ctx *c)
{
    const size_t N = c->N;
    const int nT = c->nT;
    c->h_pc.resize(nT);
    std::vector<u64> tw(nT * N), tws(nT * N), itw(nT * N), itws(nT * N), last(nT), lasts(nT);
    std::vector<double2> twf(nT * N, make_double2(0, 0)), itwf(nT * N, make_double2(0, 0));
    std::vector<FpC> fc(nT, FpC{0, 0, 0, 0, 0, 0, 0, 0});
    for (int p = 0; p < nT; p++) {
        u64 q = c->mod[p], psi = c->psi[p], ipsi = h_inv(psi, q);
        PrimeC &pc = c->h_pc[p];
        pc.q = q;
        pc.qneg = neg_inv64(q);
        pc.one_sh = h_shoup(1, q);
        u64 r1 = (u64)(((u128)1 << 64) % q);
        pc.r2 = h_mul(r1, r1, q);
        pc.ninv = h_inv(N % q, q);
        pc.ninv_sh = h_shoup(pc.ninv, q);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (size_t k = 1; k < N; k++) {
            pw[k] = h_mul(pw[k - 1], psi, q);
            ipw[k] = h_mul(ipw[k - 1], ipsi, q);
        }
        for (size_t k = 0; k < N; k++) {
            u32 b = h_brv((u32)k, c->logN);
            tw[p * N + k] = pw[b];
            tws[p * N + k] = h_shoup(pw[b], q);
            itw[p * N + k] = ipw[b];
            itws[p * N + k] = h_shoup(ipw[b], q);
        }
        last[p] = h_mul(itw[p * N + 1], pc.ninv, q);
        lasts[p] = h_shoup(last[p], q);
        if (q < ((u64)1 << 50)) {
            // integers below 2^50 are exact doubles; quotients are correctly rounded divisions
            const double qd = (double)q;
            for (size_t k = 0; k < N; k++) {
                twf[p * N + k] = make_double2((double)tw[p * N + k], (double)tw[p * N + k] / qd);
                itwf[p * N + k] = make_double2((double)itw[p * N + k], (double)itw[p * N + k] / qd);
            }
            fc[p] = FpC{qd, 1.0 / qd, (double)pc.ninv, (double)pc.ninv / qd, (double)last[p], (double)last[p] / qd, 1, 0};
        }
    }
    int rc = 0;
    rc |= dev_upload(c, &c->d_pc, c->h_pc);
    rc |= dev_upload(c, &c->d_tw, tw);
    rc |= dev_upload(c, &c->d_tw_sh, tws);
    rc |= dev_upload(c, &c->d_itw, itw);
    rc |= dev_upload(c, &c->d_itw_sh, itws);
    rc |= dev_upload(c, &c->d_last, last);
    rc |= dev_upload(c, &c->d_last_sh, lasts);
    rc |= dev_upload(c, &c->d_twf, twf);
    rc |= dev_upload(c, &c->d_itwf, itwf);
    rc |= dev_upload(c, &c->d_fc, fc);
    if (rc) return RBK_ENOMEM;
    c->tabs = NttTables{c->d_tw, c->d_tw_sh, c->d_itw, c->d_itw_sh, c->d_last, c->d_last_sh, c->d_pc,
                        c->d_twf, c->d_itwf, c->d_fc};
    if (dev_upload(c, &c->d_tabs, std::vector<NttTables>{c->tabs})) return RBK_ENOMEM;

    // ModDown P -> Q, P^-1, P mod q
    const int nQ = c->nQ, nP = c->nP;
    std::vector<u64> mdA(std::max(nP, 1), 0), mdAsh(mdA.size(), 0), mdM((size_t)std::max(nP, 1) * nQ, 0);
    std::vector<u64> Pinv(nQ), Pinvsh(nQ), Pmod(nQ), Pmodsh(nQ);
    for (int t = 0; t < nP; t++) {
        u64 pt = c->mod[nQ + t], prod = 1;
        for (int k = 0; k < nP; k++)
            if (k != t) prod = h_mul(prod, c->mod[nQ + k] % pt, pt);
        mdA[t] = h_inv(prod, pt);
        mdAsh[t] = h_shoup(mdA[t], pt);
        for (int i = 0; i < nQ; i++) {
            u64 qi = c->mod[i], pr = 1;
            for (int k = 0; k < nP; k++)
                if (k != t) pr = h_mul(pr, c->mod[nQ + k] % qi, qi);
            mdM[(size_t)t * nQ + i] = h_mont(pr, qi);
        }
    }
    for (int i = 0; i < nQ; i++) {
        u64 qi = c->mod[i], P = 1;
        for (int k = 0; k < nP; k++) P = h_mul(P, c->mod[nQ + k] % qi, qi);
        Pmod[i] = P;
        Pmodsh[i] = h_shoup(P, qi);
        Pinv[i] = h_inv(P, qi);
        Pinvsh[i] = h_shoup(Pinv[i], qi);
    }
    c->h_Pmod = Pmod;
    rc |= dev_upload(c, &c->d_md_A, mdA);
    rc |= dev_upload(c, &c->d_md_Ash, mdAsh);
    rc |= dev_upload(c, &c->d_md_M, mdM);
    rc |= dev_upload(c, &c->d_Pinv, Pinv);
    rc |= dev_upload(c, &c->d_Pinv_sh, Pinvsh);
    rc |= dev_upload(c, &c->d_Pmod, Pmod);
    rc |= dev_upload(c, &c->d_Pmod_sh, Pmodsh);

    // rescale tables [l][i]
    std::vector<u64> rinv((size_t)nQ * nQ, 0), rinvsh(rinv.size(), 0), rq(rinv.size(), 0);
    for (int l = 1; l < nQ; l++)
        for (int i = 0; i < l; i++) {
            u64 qi = c->mod[i];
            rinv[(size_t)l * nQ + i] = h_inv(c->mod[l] % qi, qi);
            rinvsh[(size_t)l * nQ + i] = h_shoup(rinv[(size_t)l * nQ + i], qi);
            rq[(size_t)l * nQ + i] = c->mod[l] % qi;
        }
    rc |= dev_upload(c, &c->d_rs_inv, rinv);
    rc |= dev_upload(c, &c->d_rs_inv_sh, rinvsh);
    rc |= dev_upload(c, &c->d_rs_qmod, rq);

    // slot positions for the encoder: (5^j mod 2N - 1)/2
    std::vector<int> pow5(N / 2);
    u64 x = 1;
    for (size_t j = 0; j < N / 2; j++) {
        pow5[j] = (int)((x - 1) / 2);
        x = (x * 5) % (2 * N);
    }
    rc |= dev_upload(c, &c->d_pow5, pow5);

    // bootstrapping: q_0 mod q_i and psi^(N/2) (a square root of -1) per Q prime
    std::vector<u64> q0mod(nQ), iq(nQ), iqsh(nQ);
    for (int i = 0; i < nQ; i++) {
        q0mod[i] = c->mod[0] % c->mod[i];
        iq[i] = h_pow(c->psi[i], N / 2, c->mod[i]);
        iqsh[i] = h_shoup(iq[i], c->mod[i]);
    }
    rc |= dev_upload(c, &c->d_q0mod, q0mod);
    rc |= dev_upload(c, &c->d_iq, iq);
    rc |= dev_upload(c, &c->d_iq_sh, iqsh);
    return rc ? RBK_ENOMEM : RBK_OK;
}

// ---------------------------------------------------------------- context

extern "C" const char *rbk_last_error(void) { return g_err.c_str(); }

extern "C" int rbk_ctx_create(const rbk_params *p, rbk_ctx **out)
{
    if (!p || !out) return fail(RBK_EINVAL, "null argument");
    *out = nullptr;
    if (p->log_n < 4 || p->log_n > 17) return fail(RBK_EINVAL, "log_n must be in [4, 17]");
    if (p->n_q < 1 || p->n_q + p->n_p > RBK_MAX_PRIMES) return fail(RBK_EINVAL, "bad prime counts");
    if (p->alpha < 1 || p->alpha > 16) return fail(RBK_EINVAL, "alpha must be in [1, 16]");
    if (p->n_p > 16) return fail(RBK_EINVAL, "at most 16 special primes");
    if ((p->n_q + p->alpha - 1) / p->alpha > 8) return fail(RBK_EINVAL, "at most 8 key-switching digits");
    if (p->alpha * (p->n_q + p->n_p) > 1024 || p->n_p * p->n_q > 1024)
        return fail(RBK_EINVAL, "base-conversion table too large (alpha*(n_q+n_p) and n_p*n_q must be <= 1024)");
    if (!p->q_bits || (p->n_p && !p->p_bits)) return fail(RBK_EINVAL, "null bit-size list");
    std::vector<int> bits;
    for (uint32_t i = 0; i < p->n_q; i++) bits.push_back((int)p->q_bits[i]);
    for (uint32_t i = 0; i < p->n_p; i++) bits.push_back((int)p->p_bits[i]);
    rbk_ctx *c = new rbk_ctx();
    if (gen_primes((int)p->log_n, bits, c->mod) != 0) {
        delete c;
        return fail(RBK_EINVAL, "no NTT-friendly prime for a requested bit size (need log_n+2 <= bits <= 60)");
    }
    (void)hipGetDevice(&c->device);
    if (int rc0 = noalloc_setup(c->device)) {
        delete c;
        return rc0;
    }
    c->logN = (int)p->log_n;
    c->N = (size_t)1 << c->logN;
    c->nQ = (int)p->n_q;
    c->nP = (int)p->n_p;
    c->nT = c->nQ + c->nP;
    c->alpha = (int)p->alpha;
    c->beta = (c->nQ + c->alpha - 1) / c->alpha;
    c->ntt_logC = c->logN <= 12 ? c->logN : (c->logN + 1) / 2;
    for (int i = 0; i < c->nT; i++) c->psi.push_back(min_root(c->mod[i], c->logN));
    int rc = build_tables(c);
    if (rc) {
        rbk_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return RBK_OK;
}

extern "C" int rbk_ctx_destroy(rbk_ctx *c)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c) return RBK_OK;
    if (c->live_mlps > 0) return fail(RBK_ESTATE, "destroy the MLPs built on this context first");
    (void)hipStreamSynchronize(c->stream);
    boot_free(c);
    for (int k = 0; k < KC_COUNT; k++)
        for (hipEvent_t e : c->timers[k].pending) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    for (void *p : c->owned) dev_free(c, p);
    for (void *p : c->retired) dev_free(c, p);
    if (c->ws != c->ws_ext) dev_free(c, c->ws);
    dev_free(c, c->desc_dev);
    for (int k = 0; k < RBK_LANES; k++)
        if (c->side[k]) {
            (void)hipStreamSynchronize(c->side[k]);
            (void)hipStreamDestroy(c->side[k]);
        }
    for (int k = 0; k <= RBK_LANES; k++)
        if (c->side_ev[k]) (void)hipEventDestroy(c->side_ev[k]);
    for (int k = 0; k < 2; k++) {
        if (c->desc_host[k]) (void)hipHostFree(c->desc_host[k]);
        if (c->desc_evt[k]) (void)hipEventDestroy(c->desc_evt[k]);
    }
    const hipError_t fe = c->free_error;
    delete c;
    if (fe != hipSuccess) return fail(RBK_EDEVICE, std::string("device memory release failed: ") + hipGetErrorString(fe));
    return RBK_OK;
}

extern "C" int rbk_set_stream(rbk_ctx *c, void *s)
{
    if (!c) return fail(RBK_EINVAL, "null context");
    c->stream = (hipStream_t)s;
    return RBK_OK;
}

extern "C" int rbk_sync(rbk_ctx *c)
{
    if (!c) return fail(RBK_EINVAL, "null context");
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

extern "C" int rbk_moduli(const rbk_ctx *c, uint64_t *out)
{
    if (!c || !out) return fail(RBK_EINVAL, "null argument");
    for (int i = 0; i < c->nT; i++) out[i] = c->mod[i];
    return RBK_OK;
}

extern "C" int rbk_psi(const rbk_ctx *c, uint64_t *out)
{
    if (!c || !out) return fail(RBK_EINVAL, "null argument");
    for (int i = 0; i < c->nT; i++) out[i] = c->psi[i];
    return RBK_OK;
}

extern "C" int rbk_num_digits(const rbk_ctx *c, int level)
{
    if (!c) return fail(RBK_EINVAL, "null context");
    if (level < 0 || level >= c->nQ) return fail(RBK_ELEVEL, "level out of range");
    return (level + c->alpha) / c->alpha;
}

static LimbMap qmap(const rbk_ctx *c) { return LimbMap{0, c->nQ, c->nQ}; }

static int check_level(const rbk_ctx *c, int level, int min_level = 0)
{
    if (level < min_level || level >= c->nQ) return fail(RBK_ELEVEL, "level out of range");
    return RBK_OK;
}

// workspace words of the key-switching pipeline for `count` ciphertexts at level l
size_t ks_words(const rbk_ctx *c, int level, int count)
{
    size_t L1 = level + 1, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha, N = c->N;
    size_t ext = count * beta * E * N, u = count * 2 * E * N, coef = count * L1 * N, tp = count * 2 * c->nP * N,
           conv = count * 2 * L1 * N;
    return ext + u + coef + tp + conv;
}

extern "C" int rbk_reserve(rbk_ctx *c, int level, int count)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || count < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    size_t L1 = level + 1, N = c->N;
    WS(ws, ks_words(c, level, count) + count * 3 * L1 * N + count * 2 * L1 * N);
    (void)ws;
    modup_tables(c, level);
    return RBK_OK;
}

extern "C" int rbk_workspace_words(const rbk_ctx *c, int level, int count, int n_rot, size_t *words)
{
    if (!c || !words || count < 1 || n_rot < 0) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t L1 = level + 1, N = c->N, per = L1 * N, ks = ks_words(c, level, count);
    const size_t slot = (size_t)count * 2 * (c->nP + L1) * N;   // tp + conv of one rotation's ModDown
    size_t need = std::max((size_t)count * 3 * per + ks, 2 * (size_t)count * per);   // mult_relin, rescale
    if (n_rot > 1) {
        const size_t extra = (count <= 4 && c->nP > 0) ? (size_t)std::min(n_rot, KS_MAX_ITEMS) * slot
                                                       : (size_t)(std::min(c->lanes, n_rot) - 1) * slot;
        need = std::max(need, ks + extra);
    }
    *words = need;
    return RBK_OK;
}

extern "C" int rbk_set_workspace(rbk_ctx *c, uint64_t *d_ws, size_t words)
{
    if (!c) return fail(RBK_EINVAL, "null argument");
    if (c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if ((d_ws == nullptr) != (words == 0)) return fail(RBK_EINVAL, "a buffer needs a size, no buffer none");
    // earlier calls may still use the workspace that is replaced
    HIPCK(hipStreamSynchronize(c->stream));
    if (c->ws && c->ws != c->ws_ext) release_buffer(c, c->ws);
    c->ws = d_ws;
    c->ws_words = words;
    c->ws_ext = d_ws;
    return RBK_OK;
}

// ---------------------------------------------------------------- transforms

extern "C" int rbk_ntt(rbk_ctx *c, uint64_t *d, int count, const int *idx, int nl, int inverse)
{
    if (!c || !d || !idx || count < 0 || nl < 1) return fail(RBK_EINVAL, "bad argument");
    int split = 0;
    while (split < nl && idx[split] < c->nQ) split++;
    for (int i = 0; i < nl; i++) {
        int want = i < split ? i : c->nQ + (i - split);
        if (idx[i] != want || want >= c->nT) return fail(RBK_EINVAL, "prime_idx must be 0..a-1 followed by n_q..n_q+b-1");
    }
    ntt_launch(c, d, (long)nl * c->N, count, nl, LimbMap{0, split, c->nQ}, inverse != 0, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

// ---------------------------------------------------------------- keys

static LimbMap allmap(const rbk_ctx *c) { return LimbMap{0, c->nQ, c->nQ}; }  // identity over every prime

// Randomness drawn inside the library (seeded sampling): the key stream's
// seed and the id that names the key or encryption.
struct Seeded {
    u64 seed;
    u32 id;
    u32 sub;
};

// the secret from host coefficients s, or (s null) uniform ternary from sd
static int set_secret(rbk_ctx *c, const int64_t *s, const Seeded *sd)
{
    const size_t N = c->N;
    if (!c->d_s && dev_alloc(c, &c->d_s, c->nT * N)) return RBK_ENOMEM;
    WS(ws, N);
    if (s) HIPCK(hipMemcpyAsync(ws, s, N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
    else sample_small_launch(c, (i64 *)ws, sd->seed, RBK_SAMPLE_SECRET, 0, 0, 0, c->stream);
    signed_to_limbs_launch(c, (const i64 *)ws, c->d_s, 1, c->nT, allmap(c), c->stream);
    ntt_launch(c, c->d_s, (long)c->nT * N, 1, c->nT, allmap(c), false, c->stream);
    HIPCK_LAUNCH();
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

extern "C" int rbk_set_secret(rbk_ctx *c, const int64_t *s)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !s) return fail(RBK_EINVAL, "null argument");
    return set_secret(c, s, nullptr);
}

// pk = (-a s + e, a) from host (a, e), or (a null) sampled from sd
static int keygen_public(rbk_ctx *c, const uint64_t *a, const int64_t *e, const Seeded *sd)
{
    const size_t N = c->N, nQ = c->nQ;
    if (!c->d_pk && dev_alloc(c, &c->d_pk, 2 * nQ * N)) return RBK_ENOMEM;
    WS(ws, 2 * nQ * N + N);
    u64 *ea = ws, *ee = ws + nQ * N;  // e limbs
    i64 *eraw = (i64 *)(ws + 2 * nQ * N);
    u64 *pk1 = c->d_pk + nQ * N;
    if (a) {
        HIPCK(hipMemcpyAsync(pk1, a, nQ * N * sizeof(u64), hipMemcpyHostToDevice, c->stream));
        HIPCK(hipMemcpyAsync(eraw, e, N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
    } else {
        sample_uniform_launch(c, pk1, (int)nQ, sd->seed, RBK_SAMPLE_PK_A, 0, 0, c->stream);
        sample_small_launch(c, eraw, sd->seed, RBK_SAMPLE_PK_E, 0, 0, 1, c->stream);
    }
    ntt_launch(c, pk1, (long)nQ * N, 1, (int)nQ, qmap(c), false, c->stream);
    signed_to_limbs_launch(c, eraw, ee, 1, (int)nQ, qmap(c), c->stream);
    ntt_launch(c, ee, (long)nQ * N, 1, (int)nQ, qmap(c), false, c->stream);
    ew_launch(c, EW_MUL, pk1, c->d_s, ea, 1, (int)nQ, qmap(c), c->stream);
    ew_launch(c, EW_SUB, ee, ea, c->d_pk, 1, (int)nQ, qmap(c), c->stream);
    HIPCK_LAUNCH();
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

extern "C" int rbk_keygen_public(rbk_ctx *c, const uint64_t *a, const int64_t *e)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !a || !e) return fail(RBK_EINVAL, "null argument");
    if (!c->d_s) return fail(RBK_ENOKEY, "secret key not set");
    return keygen_public(c, a, e, nullptr);
}

// generic switching key: s_from NTT domain [nT][N] (device); (a, e) from the
// host, or (a null) sampled: limb t of digit j from nonce (KEY_A, id, j 2^16 + t),
// the error of digit j from (KEY_E, id, j)
static int keygen_switch(rbk_ctx *c, DevKey &k, const u64 *s_from, const uint64_t *a, const int64_t *e,
                         const Seeded *sd = nullptr)
{
    const size_t N = c->N, nT = c->nT, beta = c->beta;
    if (!k.data && dev_alloc(c, &k.data, beta * 2 * nT * N)) return RBK_ENOMEM;
    WS(ws, 2 * beta * nT * N + beta * N + nT * N);
    u64 *da = ws, *de = ws + beta * nT * N;
    i64 *eraw = (i64 *)(ws + 2 * beta * nT * N);
    u64 *sf = ws + 2 * beta * nT * N + beta * N;
    HIPCK(hipMemcpyAsync(sf, s_from, nT * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    if (a) {
        HIPCK(hipMemcpyAsync(da, a, beta * nT * N * sizeof(u64), hipMemcpyHostToDevice, c->stream));
        HIPCK(hipMemcpyAsync(eraw, e, beta * N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
    } else {
        for (size_t j = 0; j < beta; j++) {
            sample_uniform_launch(c, da + j * nT * N, (int)nT, sd->seed, RBK_SAMPLE_KEY_A, sd->id, (u32)j, c->stream);
            sample_small_launch(c, eraw + j * N, sd->seed, RBK_SAMPLE_KEY_E, sd->id, (u32)j, 1, c->stream);
        }
    }
    ntt_launch(c, da, (long)nT * N, (int)beta, (int)nT, allmap(c), false, c->stream);
    signed_to_limbs_launch(c, eraw, de, (int)beta, (int)nT, allmap(c), c->stream);
    ntt_launch(c, de, (long)nT * N, (int)beta, (int)nT, allmap(c), false, c->stream);
    keygen_launch(c, da, de, sf, k.data, c->stream);
    HIPCK_LAUNCH();
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

static int keygen_relin(rbk_ctx *c, const uint64_t *a, const int64_t *e, const Seeded *sd)
{
    u64 *s2 = nullptr;
    if (dev_alloc(c, &s2, c->nT * c->N)) return RBK_ENOMEM;
    ew_launch(c, EW_MUL, c->d_s, c->d_s, s2, 1, c->nT, allmap(c), c->stream);
    int rc = keygen_switch(c, c->relin, s2, a, e, sd);
    (void)hipStreamSynchronize(c->stream);
    dev_release(c, s2);
    c->relin.g = 0;
    return rc;
}

extern "C" int rbk_keygen_relin(rbk_ctx *c, const uint64_t *a, const int64_t *e)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !a || !e) return fail(RBK_EINVAL, "null argument");
    if (!c->d_s) return fail(RBK_ENOKEY, "secret key not set");
    return keygen_relin(c, a, e, nullptr);
}

extern "C" uint64_t rbk_galois_elt(const rbk_ctx *c, int64_t k)
{
    if (!c) return 0;
    int64_t n = (int64_t)(c->N / 2);
    int64_t r = ((k % n) + n) % n;
    return h_pow(5, (u64)r, 2 * c->N);
}

static int keygen_galois(rbk_ctx *c, uint64_t g, const uint64_t *a, const int64_t *e, const Seeded *sd)
{
    if (g % 2 == 0 || g >= 2 * c->N || g == 1) return fail(RBK_EINVAL, "Galois element must be odd, in (1, 2N)");
    u64 *sg = nullptr;
    if (dev_alloc(c, &sg, c->nT * c->N)) return RBK_ENOMEM;
    automorph_launch(c, c->d_s, sg, 1, c->nT, g, c->stream);
    DevKey &k = c->gal[g];
    k.g = g;
    int rc = keygen_switch(c, k, sg, a, e, sd);
    (void)hipStreamSynchronize(c->stream);
    dev_release(c, sg);
    return rc;
}

extern "C" int rbk_keygen_galois(rbk_ctx *c, uint64_t g, const uint64_t *a, const int64_t *e)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !a || !e) return fail(RBK_EINVAL, "null argument");
    if (!c->d_s) return fail(RBK_ENOKEY, "secret key not set");
    return keygen_galois(c, g, a, e, nullptr);
}

extern "C" int rbk_keygen(rbk_ctx *c, uint64_t seed, int secret_hw, const int64_t *rot_steps, int n_rot, int conj)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || (n_rot > 0 && !rot_steps) || n_rot < 0) return fail(RBK_EINVAL, "bad argument");
    if (secret_hw < 0 || (size_t)secret_hw > c->N) return fail(RBK_EINVAL, "secret_hw must be in [0, N]");
    int rc;
    if (secret_hw > 0) {
        std::vector<i64> s(c->N);
        sample_ternary_hw_host(seed, c->logN, secret_hw, s.data());
        rc = set_secret(c, s.data(), nullptr);
    } else {
        const Seeded sd{seed, 0, 0};
        rc = set_secret(c, nullptr, &sd);
    }
    if (rc) return rc;
    const Seeded sd{seed, 0, 0};
    if ((rc = keygen_public(c, nullptr, nullptr, &sd))) return rc;
    if ((rc = keygen_relin(c, nullptr, nullptr, &sd))) return rc;
    std::vector<u64> gs;
    for (int i = 0; i < n_rot; i++) gs.push_back(rbk_galois_elt(c, rot_steps[i]));
    if (conj) gs.push_back(2 * c->N - 1);
    for (u64 g : gs) {
        if (g == 1 || c->gal.count(g)) continue;  // rotation by a multiple of N/2, or a repeated element
        const Seeded sg{seed, (u32)g, 0};
        if ((rc = keygen_galois(c, g, nullptr, nullptr, &sg))) return rc;
    }
    return RBK_OK;
}

static const DevKey *find_key(const rbk_ctx *c, u64 g)
{
    if (g == 0) return c->relin.data ? &c->relin : nullptr;
    auto it = c->gal.find(g);
    return it == c->gal.end() ? nullptr : &it->second;
}

extern "C" int rbk_key_export(rbk_ctx *c, uint64_t g, uint64_t *out)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !out) return fail(RBK_EINVAL, "null argument");
    const DevKey *k = find_key(c, g);
    if (!k) return fail(RBK_ENOKEY, "no such key");
    const size_t words = (size_t)c->beta * 2 * c->nT * c->N;
    WS(ws, words);
    HIPCK(hipMemcpyAsync(ws, k->data, words * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    to_mont_launch(c, ws, c->beta * 2, c->nT, allmap(c), true, c->stream);
    ntt_launch(c, ws, (long)c->nT * c->N, c->beta * 2, c->nT, allmap(c), true, c->stream);
    HIPCK_LAUNCH();
    HIPCK(hipMemcpyAsync(out, ws, words * sizeof(u64), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

// ---------------------------------------------------------------- encode / encrypt

extern "C" int rbk_encode(rbk_ctx *c, const double *re, const double *im, size_t n, int level, double scale, uint64_t *d_pt)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || (!re && n) || !d_pt) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (n > c->N / 2) return fail(RBK_EINVAL, "more slots than N/2");
    if (!(scale > 0)) return fail(RBK_EINVAL, "scale must be positive");
    const size_t N = c->N;
    WS(ws, 4 * N + 2 * N + 1);
    double *fft = (double *)ws;
    double *dre = (double *)(ws + 4 * N), *dim = (double *)(ws + 5 * N);
    int *err = (int *)(ws + 6 * N);
    if (n) HIPCK(hipMemcpyAsync(dre, re, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (n && im) HIPCK(hipMemcpyAsync(dim, im, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCK(hipMemsetAsync(err, 0, sizeof(int), c->stream));
    encode_launch(c, dre, im ? dim : nullptr, n, level, scale, d_pt, fft, err, c->stream);
    ntt_launch(c, d_pt, (long)(level + 1) * N, 1, level + 1, qmap(c), false, c->stream);
    HIPCK_LAUNCH();
    int herr = 0;
    HIPCK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    if (herr) return fail(RBK_EINVAL, "encoded coefficient reaches 2^62: scale too large for the values");
    return RBK_OK;
}

extern "C" int rbk_decode(rbk_ctx *c, const uint64_t *d_pt, int level, double scale, double *re, double *im, size_t n)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !d_pt || (!re && n)) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (n > c->N / 2) return fail(RBK_EINVAL, "more slots than N/2");
    const size_t N = c->N;
    int nl = level >= 1 ? 2 : 1;
    WS(ws, 2 * N + 4 * N + 2 * N);
    u64 *coef = ws;
    double *fft = (double *)(ws + 2 * N);
    double *dre = (double *)(ws + 6 * N), *dim = (double *)(ws + 7 * N);
    HIPCK(hipMemcpyAsync(coef, d_pt, nl * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    ntt_launch(c, coef, (long)nl * N, 1, nl, qmap(c), true, c->stream);
    decode_launch(c, coef, level, scale, dre, dim, n, fft, c->stream);
    HIPCK_LAUNCH();
    if (n) HIPCK(hipMemcpyAsync(re, dre, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (n && im) HIPCK(hipMemcpyAsync(im, dim, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

// (v, e0, e1) from the host, or (v null) sampled: nonces (ENC_V / ENC_E0 /
// ENC_E1, index low word, index high word)
static int encrypt(rbk_ctx *c, const uint64_t *d_pt, int level, const int64_t *v, const int64_t *e0, const int64_t *e1,
                   const Seeded *sd, uint64_t *d_ct)
{
    if (check_level(c, level)) return RBK_ELEVEL;
    if (!c->d_pk) return fail(RBK_ENOKEY, "public key not generated");
    const size_t N = c->N, L1 = level + 1;
    WS(ws, 3 * N + 3 * L1 * N);
    i64 *raw = (i64 *)ws;
    u64 *lv = ws + 3 * N;
    if (v) {
        HIPCK(hipMemcpyAsync(raw, v, N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
        HIPCK(hipMemcpyAsync(raw + N, e0, N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
        HIPCK(hipMemcpyAsync(raw + 2 * N, e1, N * sizeof(i64), hipMemcpyHostToDevice, c->stream));
    } else {
        sample_small_launch(c, raw, sd->seed, RBK_SAMPLE_ENC_V, sd->id, sd->sub, 0, c->stream);
        sample_small_launch(c, raw + N, sd->seed, RBK_SAMPLE_ENC_E0, sd->id, sd->sub, 1, c->stream);
        sample_small_launch(c, raw + 2 * N, sd->seed, RBK_SAMPLE_ENC_E1, sd->id, sd->sub, 1, c->stream);
    }
    signed_to_limbs_launch(c, raw, lv, 3, (int)L1, qmap(c), c->stream);
    ntt_launch(c, lv, (long)L1 * N, 3, (int)L1, qmap(c), false, c->stream);
    encrypt_launch(c, d_pt, lv, lv + L1 * N, lv + 2 * L1 * N, d_ct, level, c->stream);
    HIPCK_LAUNCH();
    // the host arrays may be released by the caller on return
    if (v) HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

extern "C" int rbk_encrypt(rbk_ctx *c, const uint64_t *d_pt, int level, const int64_t *v, const int64_t *e0,
                           const int64_t *e1, uint64_t *d_ct)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !d_pt || !v || !e0 || !e1 || !d_ct) return fail(RBK_EINVAL, "null argument");
    return encrypt(c, d_pt, level, v, e0, e1, nullptr, d_ct);
}

extern "C" int rbk_encrypt_seeded(rbk_ctx *c, const uint64_t *d_pt, int level, uint64_t seed, uint64_t index,
                                  uint64_t *d_ct)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !d_pt || !d_ct) return fail(RBK_EINVAL, "null argument");
    const Seeded sd{seed, (u32)index, (u32)(index >> 32)};
    return encrypt(c, d_pt, level, nullptr, nullptr, nullptr, &sd, d_ct);
}

// ---------------------------------------------------------------- ciphertext export / import

extern "C" int rbk_ct_export(rbk_ctx *c, const uint64_t *d_ct, int level, int npoly, uint64_t *out)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !d_ct || !out || npoly < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t words = (size_t)npoly * (level + 1) * c->N;
    WS(ws, words);
    HIPCK(hipMemcpyAsync(ws, d_ct, words * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    ntt_launch(c, ws, (long)(level + 1) * c->N, npoly, level + 1, qmap(c), true, c->stream);
    HIPCK_LAUNCH();
    HIPCK(hipMemcpyAsync(out, ws, words * sizeof(u64), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return RBK_OK;
}

extern "C" int rbk_ct_import(rbk_ctx *c, const uint64_t *in, int level, int npoly, uint64_t *d_ct)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || !d_ct || !in || npoly < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t words = (size_t)npoly * (level + 1) * c->N;
    WS(ws, 1);
    int *flag = (int *)ws;
    HIPCK(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    HIPCK(hipMemcpyAsync(d_ct, in, words * sizeof(u64), hipMemcpyHostToDevice, c->stream));
    check_residues_launch(c, d_ct, npoly, level + 1, flag, c->stream);
    HIPCK_LAUNCH();
    int herr = 0;
    HIPCK(hipMemcpyAsync(&herr, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    if (herr) return fail(RBK_EINVAL, "a residue is not below its prime");
    ntt_launch(c, d_ct, (long)(level + 1) * c->N, npoly, level + 1, qmap(c), false, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_decrypt(rbk_ctx *c, const uint64_t *d_ct, int level, uint64_t *d_pt)
{
    if (!c || !d_ct || !d_pt) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (!c->d_s) return fail(RBK_ENOKEY, "secret key not set");
    decrypt_launch(c, d_ct, d_pt, level, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

// ---------------------------------------------------------------- ring ops

static int ew(rbk_ctx *c, EwOp op, const u64 *a, const u64 *b, u64 *out, int level, int npoly)
{
    if (!c || !a || !out || (!b && op != EW_NEG)) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (npoly < 0) return fail(RBK_EINVAL, "npoly < 0");
    ew_launch(c, op, a, b, out, npoly, level + 1, qmap(c), c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_add(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *o, int l, int np) { return ew(c, EW_ADD, a, b, o, l, np); }
extern "C" int rbk_sub(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *o, int l, int np) { return ew(c, EW_SUB, a, b, o, l, np); }
extern "C" int rbk_neg(rbk_ctx *c, const uint64_t *a, uint64_t *o, int l, int np) { return ew(c, EW_NEG, a, nullptr, o, l, np); }
extern "C" int rbk_mul_poly(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *o, int l, int np) { return ew(c, EW_MUL, a, b, o, l, np); }

extern "C" int rbk_mul_plain(rbk_ctx *c, const uint64_t *ct, const uint64_t *pt, uint64_t *out, int level)
{
    if (!c || !ct || !pt || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t per = (size_t)(level + 1) * c->N;
    ew_launch(c, EW_MUL, ct, pt, out, 1, level + 1, qmap(c), c->stream);
    ew_launch(c, EW_MUL, ct + per, pt, out + per, 1, level + 1, qmap(c), c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_add_plain(rbk_ctx *c, const uint64_t *ct, const uint64_t *pt, uint64_t *out, int level)
{
    if (!c || !ct || !pt || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t per = (size_t)(level + 1) * c->N;
    ew_launch(c, EW_ADD, ct, pt, out, 1, level + 1, qmap(c), c->stream);
    if (out != ct) HIPCK(hipMemcpyAsync(out + per, ct + per, per * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    HIPCK_LAUNCH();
    return RBK_OK;
}

// Scale-checked additions: the operands must carry the same scale to a
// relative 2^-30, the result keeps scale_a.
static int scales_match(double sa, double sb, double *so)
{
    if (!(sa > 0) || !(sb > 0)) return fail(RBK_EINVAL, "scales must be positive");
    if (std::fabs(sa / sb - 1.0) >= 0x1p-30)
        return fail(RBK_ESCALE, "operands at different scales (2^" + std::to_string(std::log2(sa)) + " vs 2^" +
                                    std::to_string(std::log2(sb)) + ")");
    if (so) *so = sa;
    return RBK_OK;
}

extern "C" int rbk_add_scaled(rbk_ctx *c, const uint64_t *a, double sa, const uint64_t *b, double sb, uint64_t *o,
                              int level, double *so)
{
    if (int rc = scales_match(sa, sb, so)) return rc;
    return ew(c, EW_ADD, a, b, o, level, 2);
}

extern "C" int rbk_sub_scaled(rbk_ctx *c, const uint64_t *a, double sa, const uint64_t *b, double sb, uint64_t *o,
                              int level, double *so)
{
    if (int rc = scales_match(sa, sb, so)) return rc;
    return ew(c, EW_SUB, a, b, o, level, 2);
}

extern "C" int rbk_add_plain_scaled(rbk_ctx *c, const uint64_t *ct, double sct, const uint64_t *pt, double spt,
                                    uint64_t *out, int level, double *so)
{
    if (int rc = scales_match(sct, spt, so)) return rc;
    return rbk_add_plain(c, ct, pt, out, level);
}

static int make_scal(const rbk_ctx *c, const uint64_t *scal, int level, ScalArg &s)
{
    for (int i = 0; i <= level; i++) {
        if (scal[i] >= c->mod[i]) return fail(RBK_EINVAL, "scalar residue not below its prime");
        s.w[i] = scal[i];
        s.wsh[i] = h_shoup(scal[i], c->mod[i]);
    }
    return RBK_OK;
}

extern "C" int rbk_mul_scalar(rbk_ctx *c, const uint64_t *a, const uint64_t *scal, uint64_t *out, int level, int npoly)
{
    if (!c || !a || !scal || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    ScalArg s;
    if (make_scal(c, scal, level, s)) return RBK_EINVAL;
    mul_scalar_launch(c, a, out, npoly, level + 1, qmap(c), s, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_add_scalar(rbk_ctx *c, const uint64_t *ct, const uint64_t *scal, uint64_t *out, int level)
{
    if (!c || !ct || !scal || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    ScalArg s;
    if (make_scal(c, scal, level, s)) return RBK_EINVAL;
    add_scalar_launch(c, ct, out, level + 1, s, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_tensor(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, int level)
{
    if (!c || !a || !b || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    tensor_launch(c, a, b, out, level, 1, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_automorph(rbk_ctx *c, const uint64_t *in, uint64_t *out, int level, int npoly, uint64_t g)
{
    if (!c || !in || !out || in == out) return fail(RBK_EINVAL, "bad argument (in-place automorphism not supported)");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (g % 2 == 0 || g >= 2 * c->N) return fail(RBK_EINVAL, "Galois element must be odd and < 2N");
    automorph_launch(c, in, out, npoly, level + 1, g, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

// ---------------------------------------------------------------- key switching pipeline

// ModUp of count polynomials d (limbs 0..l at d + i*d_stride, NTT domain) into
// ext[count][beta_l][E][N] (NTT domain).  coef: count*(l+1)*N scratch.
static int modup_run(rbk_ctx *c, const u64 *d, long d_stride, u64 *ext, long ext_stride, int level, int count, u64 *coef)
{
    const size_t N = c->N;
    const int L1 = level + 1, E = L1 + c->nP;
    const ModUpTables &T = modup_tables(c, level);
    if (!T.d_M) return fail(RBK_ENOMEM, "ModUp tables");
    HIPCK(ntt_inverse_from_launch(c, d, d_stride, coef, (long)L1 * N, count, L1, qmap(c), c->stream));
    // the base conversion also places each digit's own limbs (from d, NTT domain)
    bconv_modup_launch(c, coef, (long)L1 * N, d, d_stride, ext, ext_stride, level, count, c->stream);
    for (int j = 0; j < T.beta; j++) {
        int lo = T.lo[j], n_in = T.n_in[j];
        u64 *ej = ext + (size_t)j * E * N;
        if (lo > 0) ntt_launch(c, ej, ext_stride, count, lo, LimbMap{0, L1, c->nQ}, false, c->stream);
        int hi = lo + n_in;
        if (hi < E) ntt_launch(c, ej + (size_t)hi * N, ext_stride, count, E - hi, LimbMap{hi, L1, c->nQ}, false, c->stream);
    }
    HIPCK_LAUNCH();
    return RBK_OK;
}

void ks_account(rbk_ctx_impl *c, const int *levels, int count, int key_level)
{
    const double N = (double)c->N, w = 8.0;
    for (int i = 0; i < count; i++) c->ks_bytes += 2.0 * (levels ? levels[i] + 1 : key_level + 1) * N * w;
    const int L1 = key_level + 1, beta = (L1 + c->alpha - 1) / c->alpha;
    c->ks_bytes += (double)beta * 2.0 * (L1 + c->nP) * N * w;
    c->ks_units += (unsigned long)count;
}

// ModDown of u[count][2][E][N] into out (count x [2][l+1][N] at out_stride),
// adding `add` as described in moddown_finish_launch.
static int moddown_run(rbk_ctx *c, u64 *u, const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out,
                       long out_stride, int level, int count, u64 *tp, u64 *conv)
{
    const size_t N = c->N;
    const int L1 = level + 1, E = L1 + c->nP, nP = c->nP;
    ks_account(c, nullptr, count, level);
    if (nP > 0) {
        HIPCK(hipMemcpy2DAsync(tp, nP * N * sizeof(u64), u + (size_t)L1 * N, E * N * sizeof(u64), nP * N * sizeof(u64),
                               2 * count, hipMemcpyDeviceToDevice, c->stream));
        ntt_launch(c, tp, (long)nP * N, 2 * count, nP, LimbMap{0, 0, c->nQ}, true, c->stream);
        bconv_moddown_launch(c, tp, (long)nP * N, conv, (long)L1 * N, level, 2 * count, c->stream);
        ntt_launch(c, conv, (long)L1 * N, 2 * count, L1, qmap(c), false, c->stream);
    } else {
        ew_launch(c, EW_ZERO, conv, nullptr, conv, 2 * count, L1, qmap(c), c->stream);
    }
    moddown_finish_launch(c, u, (long)2 * E * N, conv, (long)2 * L1 * N, add, add_stride, add_g, add_both, out, out_stride,
                          level, count, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

// ModDown fused with the key inner product: only the special-prime part of
// the inner product is stored; the Q part is recomputed in the final kernel.
// add2 (moddown_add2_ok only): a second addend on both polynomials, with the
// rotation form of add; it may be out itself
static int moddown_fused_run(rbk_ctx *c, const u64 *ext, long ext_stride, const DevKey *key, u64 perm_g, const u64 *add,
                             long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level, int count,
                             u64 *tp, u64 *conv, hipStream_t st = nullptr, const u64 *add2 = nullptr,
                             long add2_stride = 0)
{
    const size_t N = c->N;
    const int L1 = level + 1, nP = c->nP;
    if (!st) st = c->stream;
    if (add2 && (!moddown_add2_ok(c) || !add || add_both))
        return fail(RBK_EINVAL, "internal: second addend outside the fused ModDown");
    ks_account(c, nullptr, count, level);
    if (nP > 0) {
        moddown_head_launch(c, ext, ext_stride, key->data, tp, level, count, perm_g, st);
        bconv_moddown_launch(c, tp, (long)nP * N, conv, (long)L1 * N, level, 2 * count, st);
        moddown_tail_launch(c, ext, ext_stride, key->data, conv, add, add_stride, add_g, add_both, out, out_stride, level,
                            count, perm_g, st, add2, add2_stride);
    } else {
        ew_launch(c, EW_ZERO, conv, nullptr, conv, 2 * count, L1, qmap(c), st);
        moddown_ip_launch(c, ext, ext_stride, key->data, conv, (long)2 * L1 * N, add, add_stride, add_g, add_both, out,
                          out_stride, level, count, perm_g, st);
    }
    HIPCK_LAUNCH();
    return RBK_OK;
}

struct KsBufs {
    u64 *ext, *u, *coef, *tp, *conv;
};

static KsBufs ks_layout(const rbk_ctx *c, u64 *base, int level, int count)
{
    size_t L1 = level + 1, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha, N = c->N;
    KsBufs b;
    b.ext = base;
    b.u = b.ext + count * beta * E * N;
    b.coef = b.u + count * 2 * E * N;
    b.tp = b.coef + count * L1 * N;
    b.conv = b.tp + count * 2 * c->nP * N;
    return b;
}

extern "C" int rbk_modup(rbk_ctx *c, const uint64_t *d, uint64_t *ext, int level)
{
    if (!c || !d || !ext) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t N = c->N, L1 = level + 1, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha;
    WS(ws, L1 * N);
    return modup_run(c, d, (long)L1 * N, ext, (long)(beta * E * N), level, 1, ws);
}

extern "C" int rbk_key_inner_product(rbk_ctx *c, const uint64_t *ext, uint64_t g, uint64_t *u, int level)
{
    if (!c || !ext || !u) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const DevKey *k = find_key(c, g);
    if (!k) return fail(RBK_ENOKEY, "no such key");
    ip_launch(c, ext, 0, k->data, u, 0, level, 1, 0, c->stream);
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_moddown(rbk_ctx *c, const uint64_t *u, uint64_t *out, int level, int npoly)
{
    if (!c || !u || !out || npoly < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    // the pipeline works on pairs of polynomials; an odd count gets a zero partner
    const size_t N = c->N, L1 = level + 1, E = L1 + c->nP;
    const int pairs = (npoly + 1) / 2;
    WS(ws, pairs * 2 * E * N + pairs * 2 * c->nP * N + pairs * 2 * L1 * N + pairs * 2 * L1 * N);
    u64 *uu = ws, *tp = uu + pairs * 2 * E * N, *conv = tp + pairs * 2 * c->nP * N, *o = conv + pairs * 2 * L1 * N;
    HIPCK(hipMemcpyAsync(uu, u, npoly * E * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    if (npoly & 1) ew_launch(c, EW_ZERO, uu + npoly * E * N, nullptr, uu + npoly * E * N, 1, (int)E, qmap(c), c->stream);
    int rc = moddown_run(c, uu, nullptr, 0, 0, 0, o, (long)2 * L1 * N, level, pairs, tp, conv);
    if (rc) return rc;
    HIPCK(hipMemcpyAsync(out, o, npoly * L1 * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
    return RBK_OK;
}

// key switch of count polynomials d (at d_stride) with key g (0 = relin),
// results into out (count x [2][l+1][N] at out_stride) plus `add`.
int keyswitch_run(rbk_ctx *c, const DevKey *key, u64 perm_g, const u64 *d, long d_stride, const u64 *add,
                  long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level, int count, u64 *base,
                  const u64 *add2, long add2_stride)
{
    const size_t N = c->N, L1 = level + 1, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha;
    KsBufs b = ks_layout(c, base, level, count);
    int rc = modup_run(c, d, d_stride, b.ext, (long)(beta * E * N), level, count, b.coef);
    if (rc) return rc;
    return moddown_fused_run(c, b.ext, (long)(beta * E * N), key, perm_g, add, add_stride, add_g, add_both, out, out_stride,
                             level, count, b.tp, b.conv, nullptr, add2, add2_stride);
}

extern "C" int rbk_keyswitch(rbk_ctx *c, uint64_t g, const uint64_t *d, uint64_t *out, int level)
{
    if (!c || !d || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const DevKey *k = find_key(c, g);
    if (!k) return fail(RBK_ENOKEY, "no such key");
    const size_t L1 = level + 1, N = c->N;
    WS(ws, ks_words(c, level, 1));
    return keyswitch_run(c, k, 0, d, (long)(L1 * N), nullptr, 0, 0, 0, out, (long)(2 * L1 * N), level, 1, ws);
}

extern "C" int rbk_mult_relin_batch(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, int level, int count)
{
    if (!c || !a || !b || !out || count < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (!c->relin.data) return fail(RBK_ENOKEY, "relinearisation key not generated");
    const size_t L1 = level + 1, N = c->N, per = L1 * N;
    WS(ws, count * 3 * per + ks_words(c, level, count));
    u64 *d = ws;
    tensor_launch(c, a, b, d, level, count, c->stream);
    return keyswitch_run(c, &c->relin, 0, d + 2 * per, (long)(3 * per), d, (long)(3 * per), 0, 1, out, (long)(2 * per),
                         level, count, ws + count * 3 * per);
}

extern "C" int rbk_mult_relin(rbk_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, int level)
{
    return rbk_mult_relin_batch(c, a, b, out, level, 1);
}

size_t rescale_ws_words(const rbk_ctx *c, int level, int count)
{
    return 2 * (size_t)count * c->N * (1 + (size_t)level);
}

int rescale_check(rbk_ctx *c, const u64 *ct, u64 *out, int level, int count)
{
    if (!c || !ct || !out || count < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level, 1)) return RBK_ELEVEL;
    const size_t N = c->N, L1 = level + 1;
    // input and output have different strides: blocks of one launch would
    // overwrite limbs that others still read
    if (ranges_overlap(ct, (size_t)count * 2 * L1 * N, out, (size_t)count * 2 * level * N))
        return fail(RBK_EINVAL, "rescale: input and output overlap");
    return RBK_OK;
}

int rescale_run(rbk_ctx *c, const u64 *ct, u64 *out, int level, int count, u64 *ws)
{
    const size_t N = c->N, L1 = level + 1;
    u64 *last = ws, *lifted = ws + 2 * count * N;
    HIPCK(ntt_inverse_from_launch(c, ct + (size_t)level * N, (long)(L1 * N), last, (long)N, 2 * count, 1,
                                  LimbMap{level, c->nQ, c->nQ}, c->stream));
    if (!rescale_fused_launch(c, last, lifted, ct, out, level, 2 * count, c->stream)) {
        rescale_lift_launch(c, last, lifted, level, 2 * count, c->stream);
        ntt_launch(c, lifted, (long)level * N, 2 * count, level, qmap(c), false, c->stream);
        rescale_finish_launch(c, ct, lifted, out, level, 2 * count, c->stream);
    }
    HIPCK_LAUNCH();
    return RBK_OK;
}

extern "C" int rbk_rescale_batch(rbk_ctx *c, const uint64_t *ct, uint64_t *out, int level, int count)
{
    int rc = rescale_check(c, ct, out, level, count);
    if (rc) return rc;
    WS(ws, rescale_ws_words(c, level, count));
    return rescale_run(c, ct, out, level, count, ws);
}

extern "C" int rbk_rescale(rbk_ctx *c, const uint64_t *ct, uint64_t *out, int level)
{
    return rbk_rescale_batch(c, ct, out, level, 1);
}

// Rot for count ciphertexts [count][2][l+1][N] by the Galois element g:
// out = (sigma_g(c0), 0) + KS(sigma_g(c1)) (+ add2, count ciphertexts in the
// same layout, which may be out itself).  Only sigma_g(c1) is written out
// (the ModUp input); the ModDown reads c0 through the permutation and adds
// add2 in the same pass where the geometry allows.  An output over the
// input (rbk_rotate in place) takes the permuted copy of both polynomials.
static int rotate_run(rbk_ctx *c, const u64 *in, u64 *out, int level, int count, u64 g, const u64 *add2)
{
    const size_t L1 = level + 1, N = c->N, per = L1 * N, words = (size_t)count * 2 * per;
    if (ranges_overlap(in, words, out, words)) {
        if (add2 || (g == 1 && in != out)) return fail(RBK_EINVAL, "rotation: input and output overlap");
        if (g == 1) return RBK_OK;
        const DevKey *k = find_key(c, g);
        if (!k) return fail(RBK_ENOKEY, "no Galois key for element " + std::to_string(g));
        WS(ws, words + ks_words(c, level, count));
        automorph_launch(c, in, ws, 2 * count, (int)L1, g, c->stream);
        return keyswitch_run(c, k, 0, ws + per, (long)(2 * per), ws, (long)(2 * per), 0, 0, out, (long)(2 * per), level,
                             count, ws + words);
    }
    if (g == 1) {
        if (add2) ew_launch(c, EW_ADD, in, add2, out, 2 * count, (int)L1, qmap(c), c->stream);
        else HIPCK(hipMemcpyAsync(out, in, words * sizeof(u64), hipMemcpyDeviceToDevice, c->stream));
        HIPCK_LAUNCH();
        return RBK_OK;
    }
    const DevKey *k = find_key(c, g);
    if (!k) return fail(RBK_ENOKEY, "no Galois key for element " + std::to_string(g));
    if (add2 && !moddown_add2_ok(c)) {
        // the rotation into the workspace, then the sum
        WS(ws, words + count * per + ks_words(c, level, count));
        u64 *rot1 = ws + words;
        automorph_polys_launch(c, in + per, (long)(2 * per), rot1, (long)per, count, (int)L1, g, c->stream);
        int rc = keyswitch_run(c, k, 0, rot1, (long)per, in, (long)(2 * per), g, 0, ws, (long)(2 * per), level, count,
                               ws + words + count * per);
        if (rc) return rc;
        ew_launch(c, EW_ADD, ws, add2, out, 2 * count, (int)L1, qmap(c), c->stream);
        HIPCK_LAUNCH();
        return RBK_OK;
    }
    WS(ws, count * per + ks_words(c, level, count));
    automorph_polys_launch(c, in + per, (long)(2 * per), ws, (long)per, count, (int)L1, g, c->stream);
    return keyswitch_run(c, k, 0, ws, (long)per, in, (long)(2 * per), g, 0, out, (long)(2 * per), level, count,
                         ws + count * per, add2, (long)(2 * per));
}

int rotate_batch_g(rbk_ctx *c, const u64 *in, u64 *out, int level, int count, u64 g)
{
    return rotate_run(c, in, out, level, count, g, nullptr);
}

int rotate_add_batch_g(rbk_ctx *c, const u64 *in, const u64 *add2, u64 *out, int level, int count, u64 g)
{
    return rotate_run(c, in, out, level, count, g, add2);
}

static int rotate_g(rbk_ctx *c, const u64 *ct, u64 *out, int level, u64 g)
{
    return rotate_run(c, ct, out, level, 1, g, nullptr);
}

extern "C" int rbk_rotate_add_batch(rbk_ctx *c, const uint64_t *ct, const uint64_t *add, uint64_t *out, int level,
                                    int count, int64_t k)
{
    if (!c || !ct || !add || !out || count < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    if (((uintptr_t)ct | (uintptr_t)add | (uintptr_t)out) & 15) return fail(RBK_EINVAL, "rotate_add: unaligned buffer");
    const size_t words = (size_t)count * 2 * (level + 1) * c->N;
    if (ranges_overlap(ct, words, out, words)) return fail(RBK_EINVAL, "rotate_add: input and output overlap");
    if (add != out && ranges_overlap(add, words, out, words))
        return fail(RBK_EINVAL, "rotate_add: addend partly overlaps the output");
    return rotate_add_batch_g(c, ct, add, out, level, count, rbk_galois_elt(c, k));
}

extern "C" int rbk_rotate(rbk_ctx *c, const uint64_t *ct, uint64_t *out, int level, int64_t k)
{
    if (!c || !ct || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    return rotate_g(c, ct, out, level, rbk_galois_elt(c, k));
}

extern "C" int rbk_conjugate(rbk_ctx *c, const uint64_t *ct, uint64_t *out, int level)
{
    if (!c || !ct || !out) return fail(RBK_EINVAL, "null argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    return rotate_g(c, ct, out, level, 2 * c->N - 1);
}

extern "C" int rbk_rotate_hoisted_batch(rbk_ctx *c, const uint64_t *ct, const int64_t *ks, int n, uint64_t *outs, int level,
                                        int count)
{
    if (!c || !ct || !ks || !outs || n < 1 || count < 1) return fail(RBK_EINVAL, "bad argument");
    if (check_level(c, level)) return RBK_ELEVEL;
    const size_t L1 = level + 1, N = c->N, per = L1 * N, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha;
    std::vector<u64> gs(n);
    std::vector<const DevKey *> keys(n);
    for (int r = 0; r < n; r++) {
        gs[r] = rbk_galois_elt(c, ks[r]);
        keys[r] = gs[r] == 1 ? nullptr : find_key(c, gs[r]);
        if (gs[r] != 1 && !keys[r]) return fail(RBK_ENOKEY, "no Galois key for rotation " + std::to_string(ks[r]));
    }
    // Small batches: the rotations' ModDowns as one set of launches over
    // (rotation, ciphertext) slots (up to KS_MAX_ITEMS rotations per set), so
    // that every launch fills the GPU; larger batches fill it rotation by
    // rotation and take the lanes below
    const int n_sw = (int)std::count_if(gs.begin(), gs.end(), [](u64 g) { return g != 1; });
    if (count <= 4 && n_sw > 1 && c->nP > 0 && moddown_items_ok(c)) {
        const int gsz = std::min(n_sw, KS_MAX_ITEMS);
        const size_t tp_words = (size_t)count * 2 * c->nP * N, conv_words = (size_t)count * 2 * L1 * N;
        WS(ws, ks_words(c, level, count) + (size_t)gsz * (tp_words + conv_words));
        KsBufs b = ks_layout(c, ws, level, count);
        u64 *tpb = ws + ks_words(c, level, count), *convb = tpb + (size_t)gsz * tp_words;
        int rc = modup_run(c, ct + per, (long)(2 * per), b.ext, (long)(beta * E * N), level, count, b.coef);
        if (rc) return rc;
        std::vector<int> sw;
        for (int r = 0; r < n; r++) {
            if (gs[r] != 1) {
                sw.push_back(r);
                continue;
            }
            HIPCK(hipMemcpy2DAsync(outs + (size_t)r * 2 * per, n * 2 * per * sizeof(u64), ct, 2 * per * sizeof(u64),
                                   2 * per * sizeof(u64), count, hipMemcpyDeviceToDevice, c->stream));
        }
        for (size_t i0 = 0; i0 < sw.size(); i0 += KS_MAX_ITEMS) {
            KsItems I{};
            I.n = (int)std::min<size_t>(KS_MAX_ITEMS, sw.size() - i0);
            for (int i = 0; i < I.n; i++) {
                const int r = sw[i0 + i];
                I.key[i] = keys[r]->data;
                I.g[i] = gs[r];
                I.add_g[i] = gs[r];
                I.out_off[i] = (long)r * 2 * (long)per;
                ks_account(c, nullptr, count, level);
            }
            moddown_head_items_launch(c, b.ext, (long)(beta * E * N), I, tpb, level, count, c->stream);
            bconv_moddown_launch(c, tpb, (long)c->nP * (long)N, convb, (long)(L1 * N), level, 2 * count * I.n, c->stream);
            moddown_tail_items_launch(c, b.ext, (long)(beta * E * N), I, convb, ct, (long)(2 * per), 0, outs,
                                      (long)(n * 2 * per), level, count, c->stream);
        }
        HIPCK_LAUNCH();
        return RBK_OK;
    }
    // ModDown lanes: the rotations' independent ModDowns go round-robin over
    // RBK_LANES side streams, each with tp and conv buffers of its own, so the
    // VALU-bound kernels of one rotation (inner product + first iNTT pass,
    // base conversion) overlap the memory-bound ones of another.  One lane
    // while per-kernel timers run (overlapping kernels would not have
    // durations of their own) and while the stream is captured: buffers that
    // kernels of a captured graph with parallel branches touched were not
    // given back by hipFree (the runtime kept them for reuse at the same size)
    const int nl = (c->lanes > 1 && !c->capturing && !c->timing && n > 1 && side_streams(c) == RBK_OK)
                       ? std::min(c->lanes, n)
                       : 1;
    const size_t tp_words = (size_t)count * 2 * c->nP * N, conv_words = (size_t)count * 2 * L1 * N;
    WS(ws, ks_words(c, level, count) + (size_t)(nl - 1) * (tp_words + conv_words));
    KsBufs b = ks_layout(c, ws, level, count);
    u64 *lane_tp[RBK_LANES], *lane_conv[RBK_LANES];
    lane_tp[0] = b.tp;
    lane_conv[0] = b.conv;
    for (int k = 1; k < nl; k++) {
        lane_tp[k] = ws + ks_words(c, level, count) + (size_t)(k - 1) * (tp_words + conv_words);
        lane_conv[k] = lane_tp[k] + tp_words;
    }
    int rc = modup_run(c, ct + per, (long)(2 * per), b.ext, (long)(beta * E * N), level, count, b.coef);
    if (rc) return rc;
    if (nl > 1) {
        HIPCK(hipEventRecord(c->side_ev[RBK_LANES], c->stream));
        for (int k = 0; k < nl; k++) HIPCK(hipStreamWaitEvent(c->side[k], c->side_ev[RBK_LANES], 0));
    }
    int lane = 0;
    for (int r = 0; r < n && rc == RBK_OK; r++) {
        u64 *o = outs + (size_t)r * 2 * per;
        if (gs[r] == 1) {
            hipError_t e = hipMemcpy2DAsync(o, n * 2 * per * sizeof(u64), ct, 2 * per * sizeof(u64),
                                            2 * per * sizeof(u64), count, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) rc = fail(RBK_EDEVICE, std::string("hipMemcpy2DAsync: ") + hipGetErrorString(e));
            continue;
        }
        hipStream_t st = nl > 1 ? c->side[lane] : c->stream;
        rc = moddown_fused_run(c, b.ext, (long)(beta * E * N), keys[r], gs[r], ct, (long)(2 * per), gs[r], 0, o,
                               (long)(n * 2 * per), level, count, lane_tp[lane], lane_conv[lane], st);
        lane = (lane + 1) % nl;
    }
    // join every lane, also after a failure: the context stream must not run
    // later work on the shared workspace before a lane is done with it
    if (nl > 1)
        for (int k = 0; k < nl; k++) {
            hipError_t e = hipEventRecord(c->side_ev[k], c->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->side_ev[k], 0);
            if (e != hipSuccess && rc == RBK_OK) rc = fail(RBK_EDEVICE, std::string("lane join: ") + hipGetErrorString(e));
        }
    return rc;
}

extern "C" int rbk_rotate_hoisted(rbk_ctx *c, const uint64_t *ct, const int64_t *ks, int n, uint64_t *outs, int level)
{
    return rbk_rotate_hoisted_batch(c, ct, ks, n, outs, level, 1);
}

// ---------------------------------------------------------------- kernel timers

static const char *kc_names[KC_COUNT] = {
    "ntt_cols_fwd",      "ntt_rows_fwd",      "ntt_rows_inv",     "ntt_cols_inv",      "k_bconv_modup",
    "k_bconv_moddown",   "k_ip",              "k_moddown_finish", "k_tensor",          "k_rescale_lift+finish",
    "elementwise",       "k_ip_p",            "k_moddown_ip",     "ntt_rows_fwd+moddown_ip",
    "k_ip_p+ntt_rows_inv",
};

static hipEvent_t take_event(const rbk_ctx_impl *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void kt_begin(const rbk_ctx_impl *c, int cls, hipStream_t st)
{
    if (!c->timing) return;
    hipEvent_t e = take_event(c);
    (void)hipEventRecord(e, st);
    c->timers[cls].pending.push_back(e);
}

void kt_end(const rbk_ctx_impl *c, int cls, double bytes, hipStream_t st)
{
    if (!c->timing) return;
    hipEvent_t e = take_event(c);
    (void)hipEventRecord(e, st);
    KTimer &t = c->timers[cls];
    t.pending.push_back(e);
    t.bytes += bytes;
    t.launches++;
}

static int kt_collect(rbk_ctx *c)
{
    HIPCK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < KC_COUNT; k++) {
        KTimer &t = c->timers[k];
        for (size_t i = 0; i + 1 < t.pending.size(); i += 2) {
            float ms = 0;
            HIPCK(hipEventElapsedTime(&ms, t.pending[i], t.pending[i + 1]));
            t.ms += ms;
        }
        for (hipEvent_t e : t.pending) c->event_pool.push_back(e);
        t.pending.clear();
    }
    return RBK_OK;
}

extern "C" int rbk_set_lanes(rbk_ctx *c, int n)
{
    if (!c) return fail(RBK_EINVAL, "null context");
    if (n < 1 || n > RBK_LANES) return fail(RBK_EINVAL, "lanes out of range (1.." + std::to_string(RBK_LANES) + ")");
    c->lanes = n;
    return RBK_OK;
}

extern "C" int rbk_timer_enable(rbk_ctx *c, int on)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c) return fail(RBK_EINVAL, "null context");
    int rc = kt_collect(c);
    if (rc) return rc;
    for (int k = 0; k < KC_COUNT; k++) c->timers[k] = KTimer();
    c->ks_units = 0;
    c->ks_bytes = 0;
    c->timing = on != 0;
    return RBK_OK;
}

extern "C" int rbk_ks_stats(const rbk_ctx *c, uint64_t *n_keyswitch, double *method_bytes)
{
    if (!c) return fail(RBK_EINVAL, "null context");
    if (n_keyswitch) *n_keyswitch = c->ks_units;
    if (method_bytes) *method_bytes = c->ks_bytes;
    return RBK_OK;
}

extern "C" int rbk_timer_read(rbk_ctx *c, int cls, double *ms, uint64_t *launches, double *bytes)
{
    if (c && c->capturing) return fail(RBK_ESTATE, "not allowed during graph capture");
    if (!c || cls < 0 || cls >= KC_COUNT) return fail(RBK_EINVAL, "bad argument");
    int rc = kt_collect(c);
    if (rc) return rc;
    if (ms) *ms = c->timers[cls].ms;
    if (launches) *launches = c->timers[cls].launches;
    if (bytes) *bytes = c->timers[cls].bytes;
    return RBK_OK;
}

extern "C" const char *rbk_timer_name(int cls) { return (cls >= 0 && cls < KC_COUNT) ? kc_names[cls] : nullptr; }

// ---------------------------------------------------------------- graph capture

struct rbk_graph {
    rbk_ctx *c = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
};

extern "C" int rbk_capture_begin(rbk_ctx *c)
{
    if (!c) return fail(RBK_EINVAL, "null argument");
    if (c->capturing) return fail(RBK_ESTATE, "already capturing");
    if (c->timing) return fail(RBK_ESTATE, "disable the kernel timers before capturing");
    if (!c->stream) return fail(RBK_ESTATE, "capture needs a non-default stream (rbk_set_stream)");
    HIPCK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    return RBK_OK;
}

extern "C" int rbk_capture_end(rbk_ctx *c, rbk_graph **out)
{
    if (!c || !out) return fail(RBK_EINVAL, "null argument");
    if (!c->capturing) return fail(RBK_ESTATE, "not capturing");
    c->capturing = false;
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || !g) return fail(RBK_EDEVICE, std::string("capture failed: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(RBK_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    }
    rbk_graph *r = new (std::nothrow) rbk_graph;
    if (!r) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return fail(RBK_ENOMEM, "host allocation failed");
    }
    c->live_graphs++;
    r->c = c;
    r->g = g;
    r->e = ex;
    *out = r;
    return RBK_OK;
}

extern "C" int rbk_graph_launch(rbk_graph *g)
{
    if (!g) return fail(RBK_EINVAL, "null argument");
    if (g->c->capturing) return fail(RBK_ESTATE, "cannot launch while capturing");
    HIPCK(hipGraphLaunch(g->e, g->c->stream));
    return RBK_OK;
}

extern "C" int rbk_graph_destroy(rbk_graph *g)
{
    if (!g) return RBK_OK;
    rbk_ctx *c = g->c;
    (void)hipStreamSynchronize(c->stream);
    if (g->e) (void)hipGraphExecDestroy(g->e);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
    if (--c->live_graphs == 0) {
        for (void *p : c->retired) dev_free(c, p);
        c->retired.clear();
    }
    return RBK_OK;
}
