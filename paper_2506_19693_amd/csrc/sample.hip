// Seeded sampling of key and encryption randomness (paper Section 3: the
// secret, the uniform public polynomials and the added noise of key
// generation and encryption), drawn from one 64-bit seed on the device.
//
// Keystream: the ChaCha20 block function (RFC 8439, 20 rounds) with key
// (seed low word, seed high word, 0 x 6), a 32-bit block counter and a
// nonce (purpose, id, sub) that names the quantity.  Coefficient j of an
// N-coefficient polynomial reads the block at counter j (j + N, j + 2N, ...
// when a block yields no value), so every coefficient is one independent
// thread:
//   uniform mod q   the block's eight little-endian 64-bit words masked to
//                   bitlen(q) bits, the first below q;
//   ternary         the block's 256 2-bit fields, low bits of word 0 first,
//                   the first that is not 3 (0, 1, 2 -> 0, +1, -1);
//   Gaussian        sigma = 3.2 on |x| <= 19: w = first 64-bit word, the
//                   magnitude is the least m with (w >> 1) < T[m] for the
//                   cumulative table T[m] = floor(2^63 P(|x| <= m)), negative
//                   when m > 0 and bit 0 of w is set.
// A secret with exactly h non-zero coefficients is a sequential draw
// (host): 32-bit words of the stream (SECRET, 1, 0) in counter order, two
// per draw (position = first & (N - 1), sign = bit 0 of the second), taken
// positions skipped.
#include <cmath>
#include <vector>

#include "rbk_ctx.hpp"

namespace {

constexpr u32 SIGMA_TABLE = 20;

struct Block {
    u32 w[16];
};

__host__ __device__ __forceinline__ u32 rol(u32 v, int s) { return (v << s) | (v >> (32 - s)); }

// One ChaCha quarter round on four state words.
__host__ __device__ __forceinline__ void qround(u32 &a, u32 &b, u32 &c, u32 &d)
{
    a += b;
    d = rol(d ^ a, 16);
    c += d;
    b = rol(b ^ c, 12);
    a += b;
    d = rol(d ^ a, 8);
    c += d;
    b = rol(b ^ c, 7);
}

// RFC 8439 Section 2.3 block function: constants "expand 32-byte k", key,
// counter, nonce; ten column + diagonal double rounds; add the input.
__host__ __device__ inline Block chacha(u64 seed, u32 counter, u32 n0, u32 n1, u32 n2)
{
    const u32 init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (u32)seed, (u32)(seed >> 32), 0, 0,
                          0, 0, 0, 0, counter, n0, n1, n2};
    u32 x[16];
    for (int i = 0; i < 16; i++) x[i] = init[i];
    for (int r = 0; r < 10; r++) {
        for (int col = 0; col < 4; col++) qround(x[col], x[4 + col], x[8 + col], x[12 + col]);
        for (int dg = 0; dg < 4; dg++) qround(x[dg], x[4 + (dg + 1) % 4], x[8 + (dg + 2) % 4], x[12 + (dg + 3) % 4]);
    }
    Block b;
    for (int i = 0; i < 16; i++) b.w[i] = x[i] + init[i];
    return b;
}

__host__ __device__ inline u64 word64(const Block &b, int t) { return (u64)b.w[2 * t] | ((u64)b.w[2 * t + 1] << 32); }

struct Table20 {
    u64 t[SIGMA_TABLE];
};

// out[t][j] uniform mod prime t (t < nlimbs, prime-table order); nonce
// (purpose, id, (sub_hi << 16) | t)
__global__ void k_sample_uniform(u64 *out, const PrimeC *pc, int nlimbs, int logN, u64 seed, u32 purpose, u32 id,
                                 u32 sub_hi)
{
    const size_t N = (size_t)1 << logN;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= N * nlimbs) return;
    const int p = (int)(gid >> logN);
    const u32 j = (u32)(gid & (N - 1));
    const u64 q = pc[p].q;
    const int bits = 64 - __clzll(q);
    const u64 mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    const u32 sub = (sub_hi << 16) | (u32)p;
    for (u32 ctr = j;; ctr += (u32)N) {
        Block b = chacha(seed, ctr, purpose, id, sub);
        for (int t = 0; t < 8; t++) {
            u64 v = word64(b, t) & mask;
            if (v < q) {
                out[gid] = v;
                return;
            }
        }
    }
}

// out[j] small signed: kind 0 = uniform ternary, 1 = Gaussian
__global__ void k_sample_small(i64 *out, int logN, u64 seed, u32 purpose, u32 id, u32 sub, int kind, Table20 T)
{
    const size_t N = (size_t)1 << logN;
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    if (kind == 1) {
        Block b = chacha(seed, (u32)j, purpose, id, sub);
        const u64 w = word64(b, 0), u = w >> 1;
        int m = 0;
        while (m < (int)SIGMA_TABLE - 1 && u >= T.t[m]) m++;
        out[j] = (m > 0 && (w & 1)) ? -(i64)m : (i64)m;
        return;
    }
    for (u32 ctr = (u32)j;; ctr += (u32)N) {
        Block b = chacha(seed, ctr, purpose, id, sub);
        for (int k = 0; k < 256; k++) {
            const u32 f = (b.w[k >> 4] >> (2 * (k & 15))) & 3u;
            if (f != 3u) {
                out[j] = f == 0 ? 0 : (f == 1 ? 1 : -1);
                return;
            }
        }
    }
}

Table20 gauss_cdt()
{
    // rho(m) = exp(-m^2 / (2 sigma^2)); magnitude 0 has weight rho(0), m > 0
    // weight 2 rho(m) (both signs); cumulative sums in increasing m
    const double sigma = 3.2;
    double rho[SIGMA_TABLE], Z = 0.0, acc = 0.0;
    for (u32 m = 0; m < SIGMA_TABLE; m++) rho[m] = std::exp(-(double)(m * m) / (2.0 * sigma * sigma));
    for (u32 m = 0; m < SIGMA_TABLE; m++) Z += m == 0 ? rho[m] : 2.0 * rho[m];
    Table20 T;
    for (u32 m = 0; m + 1 < SIGMA_TABLE; m++) {
        acc += m == 0 ? rho[m] : 2.0 * rho[m];
        T.t[m] = (u64)std::floor(std::ldexp(acc / Z, 63));
    }
    T.t[SIGMA_TABLE - 1] = 1ull << 63;
    return T;
}

}  // namespace

void sample_uniform_launch(const rbk_ctx_impl *c, u64 *out, int nlimbs, u64 seed, u32 purpose, u32 id, u32 sub_hi,
                           hipStream_t st)
{
    const size_t total = c->N * (size_t)nlimbs;
    const int bs = 256;
    k_sample_uniform<<<(unsigned)((total + bs - 1) / bs), bs, 0, st>>>(out, c->d_pc, nlimbs, c->logN, seed, purpose, id,
                                                                       sub_hi);
}

void sample_small_launch(const rbk_ctx_impl *c, i64 *out, u64 seed, u32 purpose, u32 id, u32 sub, int gaussian,
                         hipStream_t st)
{
    static const Table20 T = gauss_cdt();
    const int bs = 256;
    k_sample_small<<<(unsigned)((c->N + bs - 1) / bs), bs, 0, st>>>(out, c->logN, seed, purpose, id, sub, gaussian, T);
}

void sample_ternary_hw_host(u64 seed, int logN, int h, i64 *out)
{
    const size_t N = (size_t)1 << logN;
    for (size_t j = 0; j < N; j++) out[j] = 0;
    if ((size_t)h > N) h = (int)N;
    u32 ctr = 0, words[16];
    int used = 16, set = 0;
    auto next = [&]() {
        if (used == 16) {
            Block b = chacha(seed, ctr++, RBK_SAMPLE_SECRET, 1, 0);
            for (int i = 0; i < 16; i++) words[i] = b.w[i];
            used = 0;
        }
        return words[used++];
    };
    while (set < h) {
        const u32 pos = next() & (u32)(N - 1);
        const u32 sgn = next() & 1u;
        if (out[pos]) continue;
        out[pos] = sgn ? -1 : 1;
        set++;
    }
}

// flag = 1 if any of npoly x nlimbs limbs holds a value at or above its prime
__global__ void k_check_residues(const u64 *data, size_t total, int logN, int nlimbs, const PrimeC *pc, int *flag)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int limb = (int)((i >> logN) % nlimbs);
    if (data[i] >= pc[limb].q) atomicOr(flag, 1);
}

void check_residues_launch(const rbk_ctx_impl *c, const u64 *data, int npoly, int nlimbs, int *flag, hipStream_t st)
{
    const size_t total = (size_t)npoly * nlimbs * c->N;
    const int bs = 256;
    if (total) k_check_residues<<<(unsigned)((total + bs - 1) / bs), bs, 0, st>>>(data, total, c->logN, nlimbs, c->d_pc, flag);
}

extern "C" int rbk_gauss_table(uint64_t *out)
{
    if (!out) return rbk_set_error(-1, "null argument");
    const Table20 T = gauss_cdt();
    for (u32 m = 0; m < SIGMA_TABLE; m++) out[m] = T.t[m];
    return 0;
}
