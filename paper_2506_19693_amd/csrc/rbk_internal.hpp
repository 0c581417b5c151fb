// Internal declarations shared by the HIP translation units of librbk.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "modarith.hpp"

#define RBK_MAX_PRIMES 80

__device__ __forceinline__ u32 brv_bits(u32 x, int bits) { return __brev(x) >> (32 - bits); }

// Source index of an NTT-domain automorphism X -> X^g: the value stored at
// brv(k) is a(psi^(2k+1)); after sigma_g it is a(psi^((2k+1) g)).
__device__ __forceinline__ u32 auto_src(u32 o, u64 g, int logN)
{
    u32 k = brv_bits(o, logN);
    u64 e = ((2 * (u64)k + 1) * g) & ((2ull << logN) - 1);
    return brv_bits((u32)((e - 1) >> 1), logN);
}

// Two adjacent NTT-domain coefficients (o, o+1), o even, are the values at
// psi^(2k+1) and psi^(2k+1+N) (bit reversal); an automorphism maps them to the
// two halves of one aligned pair, possibly swapped: auto_src(o+1) = auto_src(o) ^ 1.
// So the key-switch kernels read and write 16-byte pairs.
struct __attribute__((aligned(16))) u64x2 {
    u64 x, y;
};

__device__ __forceinline__ u64x2 ld2(const u64 *p) { return *reinterpret_cast<const u64x2 *>(p); }
__device__ __forceinline__ void st2(u64 *p, u64 a, u64 b)
{
    u64x2 v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<u64x2 *>(p) = v;
}
// the same, streamed: the data is not read again soon, so it bypasses the caches' retention
__device__ __forceinline__ void st2_nt(u64 *p, u64 a, u64 b)
{
    __builtin_nontemporal_store(a, p);
    __builtin_nontemporal_store(b, p + 1);
}
// the pair at source index src (even-aligned load, swapped when src is odd)
__device__ __forceinline__ u64x2 ld2_perm(const u64 *base, size_t src)
{
    u64x2 v = ld2(base + (src & ~(size_t)1));
    if (src & 1) {
        u64 t = v.x;
        v.x = v.y;
        v.y = t;
    }
    return v;
}

// Position -> prime-table index of a run of limbs.  Position p of the run is
// (pos0 + i); positions below 'split' are Q primes with the same index,
// the others are special primes P_(p - split), stored after the nQ Q primes.
// A run over the Q basis at level l uses split >= l+1; a run over the
// extended basis (q_0..q_l, p_0..p_{k-1}) uses split = l+1.
struct LimbMap {
    int pos0;
    int split;
    int nQ;
    __host__ __device__ int prime(int i) const
    {
        int p = pos0 + i;
        return p < split ? p : nQ + (p - split);
    }
};

// Per-prime constants of the floating-point butterflies (primes below 2^50):
// every value is an integer held exactly in a double, wp = fl(w / p).
struct FpC {
    double p, pinv;       // p and fl(1 / p)
    double ninv, ninv_p;  // N^-1 mod p and its quotient
    double lw, lw_p;      // psi^-brv(1) * N^-1 mod p and its quotient
    int use;              // 1 if p < 2^50 (the transform runs in FP64 for this prime)
    int pad;
};

struct NttTables {
    const u64 *tw, *tw_sh;    // [nprimes][N], psi^brv(k) and Shoup quotients
    const u64 *itw, *itw_sh;  // [nprimes][N], psi^-brv(k)
    const u64 *last, *last_sh;  // [nprimes], psi^-brv(1) * N^-1
    const PrimeC *pc;
    const double2 *twf, *itwf;  // [nprimes][N], (w, fl(w / p)) of tw / itw (FP primes only)
    const FpC *fc;              // [nprimes]
};

// A switching key on the device: beta digits of (b, a) over every prime,
// NTT domain, each residue stored times 2^64 (Montgomery form).
struct DevKey {
    u64 *data = nullptr;  // [beta][2][nT][N]
    u64 g = 0;            // Galois element, 0 for the relinearisation key
};

// One limb of one polynomial for the descriptor-list NTT: N = 2^logN
// residues at data, modulo prime `prime` of the tables at tabs (a device
// copy of a context's NttTables); logC is that context's NTT split.
struct NttItem {
    u64 *data;
    const NttTables *tabs;
    int prime;
    int logN;
    int logC;
    int pad;
};

struct rbk_ctx_impl;

// ---- launchers (defined in the .hip files) ----
void ntt_launch(const rbk_ctx_impl *c, u64 *data, long poly_stride, int npoly, int nlimbs, LimbMap map, bool inverse,
                hipStream_t st);
int ntt_item_units(int logN, bool first);
void ntt_list_launch(const NttItem *d_items, const int *d_prefix1, const int *d_prefix2, int n_items, int total1,
                     int total2, bool inverse, hipStream_t st);
