// Host-and-device arithmetic of the inner loops whose range arguments are
// checked by a host program against exact 128-bit integer arithmetic
// (tests/native/arith_check.cpp): the transforms' short-quotient integer
// butterflies, their FP64 butterflies for primes below 2^50, and the
// carry-free accumulation of base conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define WA_HD __host__ __device__ __forceinline__

namespace wa {

typedef uint64_t u64;
typedef uint32_t u32;

WA_HD u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }

// ---- integer butterflies with a short Shoup quotient (q < 2^61)

// floor(a * b / 2^64) minus 0, 1 or 2: a1 b1 plus the high halves of the two
// middle products; the dropped low halves and a0 b0 sum to less than 3 * 2^64
WA_HD u64 mul_hi_approx(u64 a, u64 b)
{
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p01 = (u64)a0 * b1, p10 = (u64)a1 * b0;
    return (u64)a1 * b1 + ((p01 >> 32) + (p10 >> 32));
}

// a*w mod q in [0, 4q) for any a < 2^64, given wsh = floor(w * 2^64 / q)
WA_HD u64 shoup_lazy4(u64 a, u64 w, u64 wsh, u64 q) { return a * w - mul_hi_approx(a, wsh) * q; }

// forward (Cooley-Tukey) butterfly on [0, 8q): x' = x + w y, y' = x - w y
WA_HD void bfly_ct8(u64 &x, u64 &y, u64 w, u64 wsh, u64 q, u64 q4)
{
    const u64 xx = csub(x, q4);
    const u64 t = shoup_lazy4(y, w, wsh, q);
    x = xx + t;
    y = xx + q4 - t;
}

// inverse (Gentleman-Sande) butterfly on [0, 4q): x' = x + y, y' = (x - y) w
WA_HD void bfly_gs4(u64 &x, u64 &y, u64 w, u64 wsh, u64 q, u64 q4)
{
    const u64 s = csub(x + y, q4);
    const u64 d = x + q4 - y;
    x = s;
    y = shoup_lazy4(d, w, wsh, q);
}

// ---- FP64 butterflies (p < 2^50; values are exact integers, |x| < 2^53)

// a*w mod p up to sign: (fl(a w) - qq p) + (a w - fl(a w)), qq = rint(fl(a wp)),
// wp = fl(w / p); exact, and |result| <= (1/2 + |a| 2^-52) p
WA_HD double fp_mul(double a, double w, double wp, double p)
{
    const double h = a * w;
    const double l = fma(a, w, -h);
    const double qq = rint(a * wp);
    return fma(-qq, p, h) + l;
}

// x - rint(x / p) p: exact, |result| <= (p - 1) / 2 for |x| < 2^53
WA_HD double fp_red(double x, double p, double pinv) { return fma(-rint(x * pinv), p, x); }

// A twiddle formed from two table entries: w = r a mod p with |w| <= (p-1)/2
// (r in [0, p); a canonical with ap = fl(a / p)) and wp = fl(w fl(1/p)).  The
// quotient estimate of a later fp_mul(x, w, wp, p) then carries three
// roundings of a value at most |x| / 2, an error below |x| 2^-53 * 3/4, so
// the bound (1/2 + |x| 2^-52) p of fp_mul still holds.
WA_HD void fp_twiddle(double r, double a, double ap, double p, double pinv, double &w, double &wp)
{
    w = fp_red(fp_mul(r, a, ap, p), p, pinv);
    wp = w * pinv;
}

// canonical residue (< 2^52) -> double
WA_HD double fp_from_u64(u64 v)
{
    return __builtin_bit_cast(double, v | 0x4330000000000000ull) - 4503599627370496.0;
}

// exact integer |x| < 2^53 -> canonical residue in [0, p)
WA_HD u64 fp_to_u64(double x, double p, double pinv)
{
    double r = fp_red(x, p, pinv);
    r = r < 0 ? r + p : r;
    return __builtin_bit_cast(u64, r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// ---- base conversion sums: sum_i y_i m_i for y_i, m_i < 2^60, at most 16 terms

// 30-bit halves
struct Half30 {
    u32 lo, hi;
};
WA_HD Half30 split30(u64 v) { return Half30{(u32)v & ((1u << 30) - 1), (u32)(v >> 30)}; }

// each partial product is below 2^60, so each 64-bit accumulator holds 16
// without carrying; the sum is s11 2^60 + (s01 + s10) 2^30 + s00
struct Acc4 {
    u64 s00 = 0, s01 = 0, s10 = 0, s11 = 0;
};
WA_HD void acc4(Acc4 &a, Half30 y, Half30 m)
{
    a.s00 += (u64)y.lo * m.lo;
    a.s01 += (u64)y.lo * m.hi;
    a.s10 += (u64)y.hi * m.lo;
    a.s11 += (u64)y.hi * m.hi;
}
struct Wide {
    u64 lo, hi;
};
WA_HD Wide acc4_value(const Acc4 &a)
{
    const u64 mid = a.s01 + a.s10;
    const u64 mid_c = mid < a.s01 ? 1 : 0;  // bit 64 of the middle sum
    const u64 lo1 = a.s00 + (mid << 30);
    u64 hi = (mid >> 34) + (mid_c << 30) + (lo1 < a.s00 ? 1 : 0);
    const u64 lo2 = lo1 + (a.s11 << 60);
    hi += (a.s11 >> 4) + (lo2 < lo1 ? 1 : 0);
    return Wide{lo2, hi};
}

}  // namespace wa
