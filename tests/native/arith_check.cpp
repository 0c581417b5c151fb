// Host check of the inner-loop arithmetic of the transforms and of base
// conversion (paper_2506_19693_amd/csrc/wide_arith.hpp, the same functions the
// kernels call), against exact 128-bit integer arithmetic:
//  * the short Shoup quotient is at most 2 below the exact one, and its
//    product lands in [0, 4q) with the right residue;
//  * the FP64 product is exact with |a w mod p| <= (1/2 + |a| 2^-52) p for
//    |a| <= 8p (the bound the reduction points of the transforms rest on);
//  * whole forward / inverse negacyclic transforms built from the integer
//    butterflies (ranges [0, 8q) and [0, 4q)) and from the FP64 butterflies
//    (with the kernels' reduction points, |x| < 8p) give the exact transform,
//    on random and extreme inputs, every intermediate inside its range;
//  * the carry-free accumulation of up to 16 products of 60-bit values
//    equals the exact 128-bit sum.
// Built with hipcc for the host only; prints "arith ok" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_2506_19693_amd/csrc/wide_arith.hpp"

typedef uint64_t u64;
typedef unsigned __int128 u128;

static int fails = 0;
#define CHECK(c, ...)                                          \
    do {                                                       \
        if (!(c)) {                                            \
            if (fails++ < 10) {                                \
                std::printf("FAIL line %d: ", __LINE__);       \
                std::printf(__VA_ARGS__);                      \
                std::printf("\n");                             \
            }                                                  \
        }                                                      \
    } while (0)

static u64 rng_state = 0x9E3779B97F4A7C15ull;
static u64 next64()
{
    // splitmix64
    u64 z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static u64 mulm(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 powm(u64 a, u64 e, u64 q)
{
    u64 r = 1;
    for (a %= q; e; e >>= 1, a = mulm(a, a, q))
        if (e & 1) r = mulm(r, a, q);
    return r;
}
static bool is_prime(u64 n)
{
    if (n < 4) return n >= 2;
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    for (u64 a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        u64 x = powm(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool ok = false;
        for (int r = 1; r < s && !ok; r++) ok = (x = mulm(x, x, n)) == n - 1;
        if (!ok) return false;
    }
    return true;
}
static u64 ntt_prime(int bits, size_t N)
{
    for (u64 j = 1;; j++) {
        const u64 q = ((u64)1 << bits) - j * 2 * N + 1;
        if (is_prime(q)) return q;
    }
}
static unsigned brv(unsigned k, int lg)
{
    unsigned r = 0;
    for (int i = 0; i < lg; i++, k >>= 1) r = (r << 1) | (k & 1);
    return r;
}

struct Tables {
    u64 q;
    std::vector<u64> tw, itw;  // psi^brv(k), psi^-brv(k)
    u64 ninv;
};
static Tables tables(u64 q, int lg)
{
    const size_t N = (size_t)1 << lg;
    u64 psi = 0;
    for (u64 g = 2; !psi; g++) {
        const u64 c = powm(g, (q - 1) / (2 * N), q);
        if (powm(c, N, q) == q - 1) psi = c;
    }
    const u64 ipsi = powm(psi, q - 2, q);
    Tables T;
    T.q = q;
    T.tw.resize(N);
    T.itw.resize(N);
    std::vector<u64> pw(N), ipw(N);
    pw[0] = ipw[0] = 1;
    for (size_t k = 1; k < N; k++) pw[k] = mulm(pw[k - 1], psi, q), ipw[k] = mulm(ipw[k - 1], ipsi, q);
    for (size_t k = 0; k < N; k++) T.tw[k] = pw[brv((unsigned)k, lg)], T.itw[k] = ipw[brv((unsigned)k, lg)];
    T.ninv = powm(N % q, q - 2, q);
    return T;
}
static u64 shoup_q(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// exact forward transform (reference)
static std::vector<u64> ntt_exact(const Tables &T, std::vector<u64> a, int lg)
{
    const size_t N = a.size();
    const u64 q = T.q;
    for (int s = 0; s < lg; s++) {
        const size_t m = (size_t)1 << s, d = N >> (s + 1);
        for (size_t g = 0; g < m; g++)
            for (size_t j = g * 2 * d; j < g * 2 * d + d; j++) {
                const u64 u = a[j], v = mulm(a[j + d], T.tw[m + g], q);
                a[j] = (u + v) % q;
                a[j + d] = (u + q - v) % q;
            }
    }
    return a;
}

static std::vector<u64> inputs(u64 q, size_t N, int kind)
{
    std::vector<u64> a(N);
    for (size_t i = 0; i < N; i++) a[i] = kind == 0 ? next64() % q : kind == 1 ? q - 1 : (i & 1 ? q - 1 : 0);
    return a;
}

static void check_integer_transform(int bits, int lg, int kind)
{
    const size_t N = (size_t)1 << lg;
    const u64 q = ntt_prime(bits, N), q2 = 2 * q, q4 = 4 * q;
    const Tables T = tables(q, lg);
    const std::vector<u64> a = inputs(q, N, kind), want = ntt_exact(T, a, lg);
    std::vector<u64> x = a;
    for (int s = 0; s < lg; s++) {
        const size_t m = (size_t)1 << s, d = N >> (s + 1);
        for (size_t g = 0; g < m; g++) {
            const u64 w = T.tw[m + g], wsh = shoup_q(w, q);
            for (size_t j = g * 2 * d; j < g * 2 * d + d; j++) {
                wa::bfly_ct8(x[j], x[j + d], w, wsh, q, q4);
                CHECK(x[j] < 8 * q && x[j + d] < 8 * q, "forward range, %d bits", bits);
            }
        }
    }
    for (size_t i = 0; i < N; i++) {
        x[i] = wa::csub(wa::csub(wa::csub(x[i], q4), q2), q);
        CHECK(x[i] == want[i], "forward value, %d bits, N=2^%d", bits, lg);
    }
    // inverse with N^-1 folded into the last stage
    for (int s = 0; s < lg; s++) {
        const size_t d = (size_t)1 << s, m = N >> (s + 1);
        for (size_t g = 0; g < m; g++) {
            const u64 w = T.itw[m + g], wsh = shoup_q(w, q);
            const u64 lw = mulm(w, T.ninv, q), lwsh = shoup_q(lw, q), nsh = shoup_q(T.ninv, q);
            for (size_t j = g * 2 * d; j < g * 2 * d + d; j++) {
                if (s < lg - 1) {
                    wa::bfly_gs4(x[j], x[j + d], w, wsh, q, q4);
                } else {
                    const u64 sum = wa::csub(x[j] + x[j + d], q4), dd = x[j] + q4 - x[j + d];
                    x[j] = wa::shoup_lazy4(sum, T.ninv, nsh, q);
                    x[j + d] = wa::shoup_lazy4(dd, lw, lwsh, q);
                }
                CHECK(x[j] < q4 && x[j + d] < q4, "inverse range, %d bits", bits);
            }
        }
    }
    for (size_t i = 0; i < N; i++) CHECK(wa::csub(wa::csub(x[i], q2), q) == a[i], "inverse value, %d bits", bits);
}

// The FP64 twiddle of table index m formed as the row passes form it:
// tw[m] = tw[m - lo] tw[lo] for an index part lo whose bits are disjoint from
// the rest (fp_twiddle from the canonical entries).
static void gen_twiddle(const std::vector<u64> &tab, size_t m, size_t lo, u64 q, double p, double pinv, double &w,
                        double &wp)
{
    const size_t hi = m - lo;
    CHECK((hi & lo) == 0, "twiddle index split");
    const double a = (double)tab[hi], ap = a / p;
    wa::fp_twiddle((double)tab[lo], a, ap, p, pinv, w, wp);
    CHECK(std::fabs(w) <= (p - 1) / 2 && (double)(long long)w == w, "formed twiddle range");
    const long long wi = (long long)w;
    CHECK((u64)((wi % (long long)q + (long long)q) % (long long)q) == tab[m], "formed twiddle value");
}

// FP64 transform with the kernels' reduction points: with the NTT split r
// (column pass first), rounds start at stages {0, 4, r, r + 4} forward and at
// log-distances {0, 4, logC, logC + 4} inverse.  The twiddles of forward
// stages r+4.. and of inverse log-distances 0..3 (the row-pass rounds whose
// twiddles differ per butterfly) are formed from two table entries.
static void check_fp_transform(int bits, int lg, int r, int kind)
{
    const size_t N = (size_t)1 << lg;
    const int logC = lg - r;
    const u64 q = ntt_prime(bits, N);
    const Tables T = tables(q, lg);
    const double p = (double)q, pinv = 1.0 / p;
    const double lim = 8.0 * p;
    const std::vector<u64> a = inputs(q, N, kind), want = ntt_exact(T, a, lg);
    std::vector<double> x(N);
    for (size_t i = 0; i < N; i++) x[i] = wa::fp_from_u64(a[i]);
    auto reduce_all = [&] {
        for (double &v : x) {
            v = wa::fp_red(v, p, pinv);
            CHECK(std::fabs(v) <= (p - 1) / 2, "reduction range, %d bits", bits);
        }
    };
    for (int s = 0; s < lg; s++) {
        if (s == 0 || s == 4 || s == r || s == r + 4) reduce_all();
        const size_t m = (size_t)1 << s, d = N >> (s + 1);
        for (size_t g = 0; g < m; g++) {
            const u64 w = T.tw[m + g];
            double wd = (double)w, wp = (double)w / p;
            if (s >= r + 4) gen_twiddle(T.tw, m + g, g & (((size_t)1 << (s - r)) - 1), q, p, pinv, wd, wp);
            for (size_t j = g * 2 * d; j < g * 2 * d + d; j++) {
                const double t = wa::fp_mul(x[j + d], wd, wp, p), u = x[j];
                x[j] = u + t;
                x[j + d] = u - t;
                CHECK(std::fabs(x[j]) < lim && std::fabs(x[j + d]) < lim, "fp forward range, %d bits", bits);
            }
        }
    }
    for (size_t i = 0; i < N; i++) CHECK(wa::fp_to_u64(x[i], p, pinv) == want[i], "fp forward value, %d bits", bits);
    // inverse from the exact forward output
    for (size_t i = 0; i < N; i++) x[i] = wa::fp_from_u64(want[i]);
    const double ninv = (double)T.ninv, ninv_p = ninv / p;
    for (int s = 0; s < lg; s++) {
        if (s == 0 || s == 4 || s == logC || s == logC + 4) reduce_all();
        const size_t d = (size_t)1 << s, m = N >> (s + 1);
        for (size_t g = 0; g < m; g++) {
            const u64 w = T.itw[m + g], lw = mulm(w, T.ninv, q);
            double wd = (double)w, wp = wd / p;
            const double lwd = (double)lw, lwp = lwd / p;
            if (s < 4) gen_twiddle(T.itw, m + g, g & (((size_t)1 << (logC - 1 - s)) - 1), q, p, pinv, wd, wp);
            for (size_t j = g * 2 * d; j < g * 2 * d + d; j++) {
                const double u = x[j], v = x[j + d];
                if (s < lg - 1) {
                    x[j] = u + v;
                    x[j + d] = wa::fp_mul(u - v, wd, wp, p);
                } else {
                    x[j] = wa::fp_mul(u + v, ninv, ninv_p, p);
                    x[j + d] = wa::fp_mul(u - v, lwd, lwp, p);
                }
                CHECK(std::fabs(x[j]) <= lim && std::fabs(x[j + d]) <= lim, "fp inverse range, %d bits", bits);
            }
        }
    }
    for (size_t i = 0; i < N; i++) CHECK(wa::fp_to_u64(x[i], p, pinv) == a[i], "fp inverse value, %d bits", bits);
}

int main()
{
    // short quotient
    for (long it = 0; it < 4000000; it++) {
        u64 a = next64(), b = next64();
        if (it % 4 == 1) a = ~0ull - (next64() & 0xFFFF);
        if (it % 4 == 2) b = ~0ull - (next64() & 0xFFFF);
        if (it % 8 == 3) a = ~0ull, b = ~0ull;
        const u64 hi = (u64)(((u128)a * b) >> 64), ap = wa::mul_hi_approx(a, b);
        CHECK(ap <= hi && hi - ap <= 2, "short quotient %llx %llx", (unsigned long long)a, (unsigned long long)b);
    }
    for (int bits : {40, 50, 55, 60}) {
        const u64 q = ntt_prime(bits, 1 << 16);
        for (int it = 0; it < 400000; it++) {
            const u64 a = it % 3 ? next64() : ~0ull - (u64)it, w = next64() % q, wsh = shoup_q(w, q);
            const u64 r = wa::shoup_lazy4(a, w, wsh, q);
            CHECK(r < 4 * q && r % q == mulm(a % q, w, q), "shoup_lazy4, %d bits", bits);
        }
    }
    // the FP64 product lemma behind the reduction points: for exact integers
    // |a| <= 8p the result is exact (right residue) with |t| <= (1/2 + |a| 2^-52) p
    for (int bits : {30, 45, 50}) {
        const u64 q = ntt_prime(bits, 1 << 16);
        const double p = (double)q;
        for (int it = 0; it < 400000; it++) {
            const u64 w = next64() % q;
            const double wd = (double)w, wp = wd / p;
            const long long amax = 8 * (long long)q - 1;
            long long ai = (long long)(next64() % (u64)(2 * amax + 1)) - amax;
            if (it % 4 == 0) ai = it % 8 ? amax : -amax;
            const double a = (double)ai, t = wa::fp_mul(a, wd, wp, p);
            const double bound = (0.5 + std::fabs(a) * std::ldexp(1.0, -52)) * p;
            CHECK(std::fabs(t) <= bound, "fp product bound, %d bits", bits);
            const long long ti = (long long)t;
            const u64 want = mulm((u64)(ai % (long long)q + (long long)q) % q, w, q);
            CHECK((double)ti == t && (u64)((ti % (long long)q + (long long)q) % (long long)q) == want,
                  "fp product residue, %d bits", bits);
        }
    }
    // integer butterflies (the 60-bit primes of the chains), whole transforms
    for (int kind = 0; kind < 3; kind++) {
        check_integer_transform(60, 16, kind);
        check_integer_transform(55, 13, kind);
    }
    // FP64 butterflies, with the splits of the register kernels
    for (int kind = 0; kind < 3; kind++) {
        check_fp_transform(50, 16, 8, kind);
        check_fp_transform(50, 15, 7, kind);
        check_fp_transform(49, 14, 6, kind);
        check_fp_transform(40, 13, 6, kind);
        check_fp_transform(50, 14, 8, kind);
    }
    // products with formed twiddles keep the fp_mul bound
    for (int bits : {30, 45, 50}) {
        const u64 q = ntt_prime(bits, 1 << 16);
        const double p = (double)q, pinv = 1.0 / p;
        for (int it = 0; it < 400000; it++) {
            const u64 r0 = it % 5 == 0 ? q - 1 : next64() % q, a0 = it % 7 == 0 ? q - 1 : next64() % q;
            double w, wp;
            wa::fp_twiddle((double)r0, (double)a0, (double)a0 / p, p, pinv, w, wp);
            const long long wi = (long long)w;
            CHECK(std::fabs(w) <= (p - 1) / 2 && (double)wi == w, "formed twiddle range, %d bits", bits);
            CHECK((u64)((wi % (long long)q + (long long)q) % (long long)q) == mulm(r0, a0, q), "formed twiddle, %d bits",
                  bits);
            const long long amax = 8 * (long long)q - 1;
            long long ai = (long long)(next64() % (u64)(2 * amax + 1)) - amax;
            if (it % 4 == 0) ai = it % 8 ? amax : -amax;
            const double x = (double)ai, t = wa::fp_mul(x, w, wp, p);
            CHECK(std::fabs(t) <= (0.5 + std::fabs(x) * std::ldexp(1.0, -52)) * p, "formed product bound, %d bits", bits);
            const long long ti = (long long)t;
            const u64 wc = (u64)((wi % (long long)q + (long long)q) % (long long)q);
            const u64 want = mulm((u64)(ai % (long long)q + (long long)q) % q, wc, q);
            CHECK((double)ti == t && (u64)((ti % (long long)q + (long long)q) % (long long)q) == want,
                  "formed product residue, %d bits", bits);
        }
    }
    // carry-free accumulation of up to 16 products of 60-bit values
    const u64 top = ((u64)1 << 60) - 1;
    for (int it = 0; it < 200000; it++) {
        const int n = 1 + it % 16;
        wa::Acc4 acc;
        u128 want = 0;
        for (int i = 0; i < n; i++) {
            const u64 y = it % 5 == 0 ? top : next64() & top, m = it % 7 == 0 ? top : next64() & top;
            wa::acc4(acc, wa::split30(y), wa::split30(m));
            want += (u128)y * m;
        }
        const wa::Wide got = wa::acc4_value(acc);
        CHECK(got.lo == (u64)want && got.hi == (u64)(want >> 64), "accumulation, %d terms", n);
    }
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("arith ok\n");
    return 0;
}
