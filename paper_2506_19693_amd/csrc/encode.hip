// Canonical-embedding encoder and decoder on the device (float64).
//
// Slots: slot j is the value of the plaintext polynomial at zeta^(5^j),
// zeta = exp(i pi / N), j < n = N/2 (paper Section 3 packs up to N/2 values
// per ciphertext; this order makes X -> X^(5^k) a left rotation by k).
//
// With r_j = (5^j mod 2N - 1) / 2, zeta^(5^j k) = zeta^k w^(r_j k), w = exp(2 pi i / N):
//  * encode: S_k = sum_j z_j zeta^(-5^j k) = zeta^-k * DFT_N(B)[k] where B[r_j] = z_j;
//            the real coefficients are t_k = Re(S_k)/n and t_(k+n) = Im(S_k)/n
//            (because zeta^(-5^j n) = -i), then m = round_half_even(scale * t);
//  * decode: z_j = sum_(k<n) (t_k + i t_(k+n)) zeta^k w^(r_j k)
//            = IDFT_N(C)[r_j] with C_k = (t_k + i t_(k+n)) zeta^k for k < n, 0 above.
// DFT_N is an iterative radix-2 FFT, one launch per stage.
#include "rbk_ctx.hpp"

#define FT 256

__global__ void k_fft_zero(double2 *a, size_t n)
{
    size_t i = (size_t)blockIdx.x * FT + threadIdx.x;
    if (i < n) a[i] = make_double2(0.0, 0.0);
}

__global__ void k_scatter_slots(const double *re, const double *im, size_t nslot, const int *pos, double2 *B)
{
    size_t j = (size_t)blockIdx.x * FT + threadIdx.x;
    if (j < nslot) B[pos[j]] = make_double2(re[j], im ? im[j] : 0.0);
}

__global__ void k_bitrev_copy(const double2 *in, double2 *out, int logN)
{
    size_t i = (size_t)blockIdx.x * FT + threadIdx.x;
    if (i < ((size_t)1 << logN)) out[__brev((u32)i) >> (32 - logN)] = in[i];
}

// one radix-2 decimation-in-time stage with half-size m = 2^s; sign = -1 forward
__global__ void k_fft_stage(double2 *a, int logN, int s, double sign)
{
    size_t b = (size_t)blockIdx.x * FT + threadIdx.x;
    if (b >= ((size_t)1 << (logN - 1))) return;
    size_t m = (size_t)1 << s;
    size_t grp = b >> s, j = b & (m - 1);
    size_t i0 = (grp << (s + 1)) + j, i1 = i0 + m;
    double sn, cs;
    sincospi(sign * (double)j / (double)m, &sn, &cs);
    double2 u = a[i0], v = a[i1];
    double vr = v.x * cs - v.y * sn, vi = v.x * sn + v.y * cs;
    a[i0] = make_double2(u.x + vr, u.y + vi);
    a[i1] = make_double2(u.x - vr, u.y - vi);
}

// S_k = zeta^-k F[k]; round scale * (Re, Im)/n into limbs l <= level at k and k + n
__global__ void k_encode_round(const double2 *F, u64 *pt, int logN, int L1, double scale, const PrimeC *pc, int *err)
{
    const size_t N = (size_t)1 << logN, n = N >> 1;
    size_t k = (size_t)blockIdx.x * FT + threadIdx.x;
    if (k >= n) return;
    double sn, cs;
    sincospi(-(double)k / (double)N, &sn, &cs);
    double2 f = F[k];
    double re = (f.x * cs - f.y * sn) / (double)n, im = (f.x * sn + f.y * cs) / (double)n;
    double v[2] = {rint(re * scale), rint(im * scale)};
    for (int h = 0; h < 2; h++) {
        if (!(fabs(v[h]) < 4611686018427387904.0)) {  // 2^62
            atomicOr(err, 1);
            v[h] = 0.0;
        }
        i64 m = (i64)v[h];
        u64 mag = (u64)(m < 0 ? -m : m);
        for (int l = 0; l < L1; l++) {
            u64 q = pc[l].q;
            u64 r = shoup(mag, 1, pc[l].one_sh, q);
            pt[(size_t)l * N + k + h * n] = (m < 0 && r) ? q - r : r;
        }
    }
}

void fft_run(const rbk_ctx_impl *c, double2 *a, double2 *tmp, double sign, hipStream_t st)
{
    const size_t N = c->N;
    dim3 gN((unsigned)((N + FT - 1) / FT)), gH((unsigned)((N / 2 + FT - 1) / FT));
    hipLaunchKernelGGL(k_bitrev_copy, gN, dim3(FT), 0, st, a, tmp, c->logN);
    for (int s = 0; s < c->logN; s++) hipLaunchKernelGGL(k_fft_stage, gH, dim3(FT), 0, st, tmp, c->logN, s, sign);
}

// Encode nslot values (device arrays) at 'scale' into pt [level+1][N], coefficient domain.
void encode_launch(const rbk_ctx_impl *c, const double *d_re, const double *d_im, size_t nslot, int level, double scale,
                   u64 *pt, double *fft_ws, int *err_flag, hipStream_t st)
{
    const size_t N = c->N;
    double2 *B = (double2 *)fft_ws, *F = B + N;
    dim3 gN((unsigned)((N + FT - 1) / FT));
    hipLaunchKernelGGL(k_fft_zero, gN, dim3(FT), 0, st, B, N);
    if (nslot) hipLaunchKernelGGL(k_scatter_slots, dim3((unsigned)((nslot + FT - 1) / FT)), dim3(FT), 0, st, d_re, d_im, nslot,
                                  c->d_pow5, B);
    fft_run(c, B, F, -1.0, st);
    hipLaunchKernelGGL(k_encode_round, dim3((unsigned)((N / 2 + FT - 1) / FT)), dim3(FT), 0, st, F, pt, c->logN, level + 1,
                       scale, c->d_pc, err_flag);
}

// Centred value of the plaintext from limb 0 (level 0) or from the exact CRT
// of limbs 0 and 1 (|m| < q0 q1 / 2), as a double, then C_k.
__global__ void k_decode_prep(const u64 *pt, double2 *C, int logN, int level, double inv_scale, const PrimeC *pc, u64 inv01,
                              u64 inv01_sh, u64 Qlo, u64 Qhi)
{
    const size_t N = (size_t)1 << logN, n = N >> 1;
    size_t k = (size_t)blockIdx.x * FT + threadIdx.x;
    if (k >= N) return;
    if (k >= n) { C[k] = make_double2(0.0, 0.0); return; }
    double t[2];
    for (int h = 0; h < 2; h++) {
        size_t idx = k + h * n;
        u64 x0 = pt[idx], q0 = pc[0].q;
        if (level == 0) {
            t[h] = x0 > (q0 - 1) / 2 ? -(double)(q0 - x0) : (double)x0;
        } else {
            u64 q1 = pc[1].q, x1 = pt[N + idx];
            u64 x0m = shoup(x0, 1, pc[1].one_sh, q1);
            u64 u = shoup(sub_mod(x1, x0m, q1), inv01, inv01_sh, q1);
            u128w V = mul_wide(q0, u);  // V = x0 + q0 u, exact in [0, q0 q1)
            u64 lo = V.lo + x0;
            u64 hi = V.hi + (lo < x0 ? 1 : 0);
            // centred: V > Q/2  <=>  2V > Q
            u64 dhi = (hi << 1) | (lo >> 63), dlo = lo << 1;
            bool neg = (dhi > Qhi) || (dhi == Qhi && dlo > Qlo);
            if (neg) {
                u64 rlo = Qlo - lo;
                u64 rhi = Qhi - hi - (Qlo < lo ? 1 : 0);
                t[h] = -((double)rhi * 18446744073709551616.0 + (double)rlo);
            } else {
                t[h] = (double)hi * 18446744073709551616.0 + (double)lo;
            }
        }
        t[h] *= inv_scale;
    }
    double sn, cs;
    sincospi((double)k / (double)N, &sn, &cs);
    C[k] = make_double2(t[0] * cs - t[1] * sn, t[0] * sn + t[1] * cs);
}

__global__ void k_gather_slots(const double2 *F, const int *pos, double *re, double *im, size_t nslot)
{
    size_t j = (size_t)blockIdx.x * FT + threadIdx.x;
    if (j >= nslot) return;
    double2 v = F[pos[j]];
    re[j] = v.x;
    if (im) im[j] = v.y;
}

void decode_launch(const rbk_ctx_impl *c, const u64 *pt_coef, int level, double scale, double *d_re, double *d_im,
                   size_t nslot, double *fft_ws, hipStream_t st)
{
    const size_t N = c->N;
    double2 *Cb = (double2 *)fft_ws, *F = Cb + N;
    u64 inv01 = 0, inv01_sh = 0, Qlo = 0, Qhi = 0;
    if (level >= 1) {
        u64 q0 = c->mod[0], q1 = c->mod[1];
        // q0^-1 mod q1 by Fermat
        unsigned __int128 r = 1, b = q0 % q1;
        u64 e = q1 - 2;
        while (e) {
            if (e & 1) r = (r * b) % q1;
            b = (b * b) % q1;
            e >>= 1;
        }
        inv01 = (u64)r;
        inv01_sh = (u64)((((unsigned __int128)inv01) << 64) / q1);
        unsigned __int128 Q = (unsigned __int128)q0 * q1;
        Qlo = (u64)Q;
        Qhi = (u64)(Q >> 64);
    }
    hipLaunchKernelGGL(k_decode_prep, dim3((unsigned)((N + FT - 1) / FT)), dim3(FT), 0, st, pt_coef, Cb, c->logN, level,
                       1.0 / scale, c->d_pc, inv01, inv01_sh, Qlo, Qhi);
    fft_run(c, Cb, F, 1.0, st);
    if (nslot)
        hipLaunchKernelGGL(k_gather_slots, dim3((unsigned)((nslot + FT - 1) / FT)), dim3(FT), 0, st, F, c->d_pow5, d_re,
                           d_im, nslot);
}
