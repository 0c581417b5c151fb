// Device-side 64-bit modular arithmetic for gfx950.
//
// CDNA has no 64x64 multiplier: every wide product is built from
// v_mad_u64_u32 (32x32+64 -> 64).  Three reductions are used:
//  * Shoup's precomputed-quotient product for a fixed operand w (twiddles,
//    per-limb constants): one high product and two low products, result in
//    [0, 2q) (Harvey's lazy range);
//  * Montgomery REDC for sums of products of two variables: the fixed side of
//    every such sum is stored pre-multiplied by R = 2^64, so a whole lazy
//    128-bit dot product needs one REDC at the end;
//  * a high-word pre-reduction so REDC also accepts sums >= q * 2^64.
// All primes are below 2^61, so 4q fits a word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

struct u128w {
    u64 lo, hi;
};

// full 64x64 -> 128 product out of four 32x32 -> 64 multiply-adds
__device__ __forceinline__ u128w mul_wide(u64 a, u64 b)
{
    u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    u64 p00 = (u64)a0 * b0;
    u64 p01 = (u64)a0 * b1 + (p00 >> 32);
    u64 p10 = (u64)a1 * b0 + (u32)p01;
    u64 p11 = (u64)a1 * b1 + (p01 >> 32) + (p10 >> 32);
    u128w r;
    r.lo = (p10 << 32) | (u32)p00;
    r.hi = p11;
    return r;
}

__device__ __forceinline__ u64 mul_hi(u64 a, u64 b)
{
    u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    u64 p00 = (u64)a0 * b0;
    u64 p01 = (u64)a0 * b1 + (p00 >> 32);
    u64 p10 = (u64)a1 * b0 + (u32)p01;
    return (u64)a1 * b1 + (p01 >> 32) + (p10 >> 32);
}

__device__ __forceinline__ void acc_wide(u128w &acc, u128w p)
{
    u64 lo = acc.lo + p.lo;
    acc.hi += p.hi + (lo < p.lo ? 1 : 0);
    acc.lo = lo;
}

__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }

// a*w mod q in [0, 2q) for any a < 2^64, given wsh = floor(w * 2^64 / q)
__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wsh, u64 q)
{
    u64 qh = mul_hi(a, wsh);
    return a * w - qh * q;
}

__device__ __forceinline__ u64 shoup(u64 a, u64 w, u64 wsh, u64 q) { return csub(shoup_lazy(a, w, wsh, q), q); }

// Montgomery REDC: T * 2^-64 mod q in [0, q) for T = hi:lo < q * 2^64;
// qneg = -q^-1 mod 2^64.
__device__ __forceinline__ u64 redc(u128w T, u64 q, u64 qneg)
{
    u64 m = T.lo * qneg;
    u64 t = T.hi + mul_hi(m, q) + (T.lo != 0 ? 1 : 0);
    return csub(t, q);
}

// T * 2^-64 mod q for any 128-bit T: the high word is first reduced below q
// with a Shoup product by 1 (one_sh = floor(2^64 / q)).
__device__ __forceinline__ u64 redc_any(u128w T, u64 q, u64 qneg, u64 one_sh)
{
    T.hi = shoup(T.hi, 1, one_sh, q);
    return redc(T, q, qneg);
}

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return csub(a + q - b, q); }

// Per-prime constants, one entry per prime of the table (Q primes then P).
struct PrimeC {
    u64 q;
    u64 qneg;    // -q^-1 mod 2^64
    u64 one_sh;  // floor(2^64 / q)
    u64 r2;      // 2^128 mod q (REDC(x * r2) = x * 2^64 mod q)
    u64 ninv;    // N^-1 mod q
    u64 ninv_sh;
};

// a*b mod q for two arbitrary residues: two REDCs (a*b*2^-64, then * 2^128 * 2^-64)
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeC &p)
{
    u64 t = redc(mul_wide(a, b), p.q, p.qneg);
    return redc(mul_wide(t, p.r2), p.q, p.qneg);
}
