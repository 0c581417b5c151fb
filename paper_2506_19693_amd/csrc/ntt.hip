// Negacyclic NTT / inverse NTT over 64-bit primes for gfx950.
//
// Convention: the forward transform of a limb a (coefficient order) writes
// a(psi^(2k+1)) to index brv(k) (Cooley-Tukey with psi merged into the
// twiddles, Longa-Naehrig 2016); the inverse (Gentleman-Sande) takes that
// order back to coefficients and folds N^-1 into its last stage.
//
// Work split: one limb is viewed as an R x C matrix (C = 2^logC contiguous
// elements per row).  Stages whose butterfly distance is >= C only mix
// elements of one column; the others only mix elements of one row.  The
// forward transform therefore runs a column pass (stages 0..r-1) then a row
// pass (stages r..n-1); the inverse runs them in the other order.  Each pass
// stages a 4096-element tile (32 KiB) through LDS: a column tile is R rows x
// (4096/R) adjacent columns, so every row segment is a 128-byte (or longer)
// coalesced run; a row tile is 4096/C whole rows.  When N <= 4096 one row
// pass does the whole transform.
//
// Value ranges follow Harvey: forward butterflies keep [0, 4q), inverse
// butterflies [0, 2q); each pass that ends a transform reduces to [0, q).
// The integer butterflies of the register passes use a quotient that may be
// up to 2 short (three 32x32 products instead of four), so their Shoup
// products land in [0, 4q) and the ranges widen to [0, 8q) forward and
// [0, 4q) inverse; with q < 2^61 every value fits a word.
#include <algorithm>

#include "rbk_internal.hpp"
#include "rbk_ctx.hpp"
#include "wide_arith.hpp"

#define NTT_TILE 4096
#define NTT_THREADS 256

__device__ __forceinline__ void bfly_ct(u64 &x, u64 &y, u64 w, u64 wsh, u64 q, u64 q2)
{
    u64 xx = csub(x, q2);
    u64 t = shoup_lazy(y, w, wsh, q);
    x = xx + t;
    y = xx + q2 - t;
}

__device__ __forceinline__ void bfly_gs(u64 &x, u64 &y, u64 w, u64 wsh, u64 q, u64 q2)
{
    u64 s = csub(x + y, q2);
    u64 d = x + q2 - y;
    x = s;
    y = shoup_lazy(d, w, wsh, q);
}

using wa::bfly_ct8;
using wa::bfly_gs4;
using wa::shoup_lazy4;

// Row pass.  Forward: stages (logN-logC) .. logN-1, output reduced to [0, q).
// Inverse: distances 1 .. C/2; if logC == logN this is the whole inverse
// (N^-1 folded into the last stage, output in [0, q)), else output in [0, 2q).
// body of one row tile; limb: the limb's first element, s: NTT_TILE words of LDS
template <bool INV>
__device__ __forceinline__ void ntt_rows_tile(u64 *limb_base, u64 *s, const NttTables &T, int pr, int logN, int logC,
                                              int rows_per_tile, int tile)
{
    const size_t N = (size_t)1 << logN;
    const PrimeC pc = T.pc[pr];
    const u64 q = pc.q, q2 = 2 * q;
    const u64 *tw = (INV ? T.itw : T.tw) + (size_t)pr * N;
    const u64 *tws = (INV ? T.itw_sh : T.tw_sh) + (size_t)pr * N;
    const int C = 1 << logC;
    const int row0 = tile * rows_per_tile;
    const int nel = rows_per_tile * C;
    u64 *g = limb_base + (size_t)row0 * C;

    for (int i = threadIdx.x; i < nel; i += NTT_THREADS) s[i] = g[i];
    __syncthreads();

    const int half = nel >> 1;
    const int hmask = (C >> 1) - 1;
    if (!INV) {
        for (int st = logN - logC; st < logN; st++) {
            const int lt = logN - 1 - st;  // log2 of the butterfly distance
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                int rl = b >> (logC - 1), kk = b & hmask;
                int grp = kk >> lt, off = kk & ((1 << lt) - 1);
                int x0 = (grp << (lt + 1)) + off;
                int gi = ((row0 + rl) << (logC - lt - 1)) + grp;
                int ti = (1 << st) + gi;
                u64 &x = s[rl * C + x0];
                u64 &y = s[rl * C + x0 + (1 << lt)];
                bfly_ct(x, y, tw[ti], tws[ti], q, q2);
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nel; i += NTT_THREADS) g[i] = csub(csub(s[i], q2), q);
    } else {
        const bool whole = (logC == logN);
        for (int lt = 0; lt < logC; lt++) {
            const int h = 1 << (logN - 1 - lt);
            const bool last = whole && (lt == logC - 1);
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                int rl = b >> (logC - 1), kk = b & hmask;
                int grp = kk >> lt, off = kk & ((1 << lt) - 1);
                int x0 = (grp << (lt + 1)) + off;
                int gi = ((row0 + rl) << (logC - lt - 1)) + grp;
                u64 &x = s[rl * C + x0];
                u64 &y = s[rl * C + x0 + (1 << lt)];
                if (!last) {
                    bfly_gs(x, y, tw[h + gi], tws[h + gi], q, q2);
                } else {
                    u64 sum = csub(x + y, q2);
                    u64 d = x + q2 - y;
                    x = shoup_lazy(sum, pc.ninv, pc.ninv_sh, q);
                    y = shoup_lazy(d, T.last[pr], T.last_sh[pr], q);
                }
            }
            __syncthreads();
        }
        if (whole)
            for (int i = threadIdx.x; i < nel; i += NTT_THREADS) g[i] = csub(s[i], q);
        else
            for (int i = threadIdx.x; i < nel; i += NTT_THREADS) g[i] = s[i];
    }
}

template <bool INV>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_rows(u64 *data, long poly_stride, LimbMap map, NttTables T, int logN,
                                                          int logC, int rows_per_tile)
{
    __shared__ u64 s[NTT_TILE];
    const int limb = blockIdx.y, poly = blockIdx.z;
    u64 *base = data + (size_t)poly * poly_stride + ((size_t)limb << logN);
    ntt_rows_tile<INV>(base, s, T, map.prime(limb), logN, logC, rows_per_tile, blockIdx.x);
}

// Whole transform of one limb of a ring of at most NTT_TILE coefficients in
// one workgroup: the limb and every twiddle (with its Shoup quotient) are
// staged in LDS first (96 KB at N = 2^12), so no stage waits on a global
// twiddle load.  Same stages and ranges as the row pass with logC = logN.
template <bool INV>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_small(u64 *data, long poly_stride, LimbMap map, NttTables T,
                                                           int logN)
{
    __shared__ u64 s[NTT_TILE], sw[NTT_TILE], sws[NTT_TILE];
    const int limb = blockIdx.y, poly = blockIdx.z;
    const int pr = map.prime(limb);
    const int N = 1 << logN;
    const PrimeC pc = T.pc[pr];
    const u64 q = pc.q, q2 = 2 * q;
    const u64 *tw = (INV ? T.itw : T.tw) + (size_t)pr * N;
    const u64 *tws = (INV ? T.itw_sh : T.tw_sh) + (size_t)pr * N;
    u64 *g = data + (size_t)poly * poly_stride + ((size_t)limb << logN);
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) {
        s[i] = g[i];
        sw[i] = tw[i];
        sws[i] = tws[i];
    }
    __syncthreads();
    const int half = N >> 1;
    if (!INV) {
        for (int st = 0; st < logN; st++) {
            const int lt = logN - 1 - st;  // log2 of the butterfly distance
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                const int grp = b >> lt, off = b & ((1 << lt) - 1);
                const int x0 = (grp << (lt + 1)) + off;
                const int ti = (1 << st) + grp;
                bfly_ct(s[x0], s[x0 + (1 << lt)], sw[ti], sws[ti], q, q2);
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < N; i += NTT_THREADS) g[i] = csub(csub(s[i], q2), q);
    } else {
        for (int lt = 0; lt < logN; lt++) {
            const int h = 1 << (logN - 1 - lt);
            const bool last = lt == logN - 1;
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                const int grp = b >> lt, off = b & ((1 << lt) - 1);
                const int x0 = (grp << (lt + 1)) + off;
                u64 &x = s[x0];
                u64 &y = s[x0 + (1 << lt)];
                if (!last) {
                    bfly_gs(x, y, sw[h + grp], sws[h + grp], q, q2);
                } else {
                    const u64 sum = csub(x + y, q2);
                    const u64 d = x + q2 - y;
                    x = shoup_lazy(sum, pc.ninv, pc.ninv_sh, q);
                    y = shoup_lazy(d, T.last[pr], T.last_sh[pr], q);
                }
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < N; i += NTT_THREADS) g[i] = csub(s[i], q);
    }
}

// Column pass over R = 2^(logN-logC) rows and 'cols' adjacent columns.
// Forward: stages 0 .. r-1, output in [0, 4q).  Inverse: distances C .. N/2,
// N^-1 folded into the last stage, output in [0, q).
template <bool INV>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_cols(u64 *data, long poly_stride, LimbMap map, NttTables T, int logN,
                                                          int logC, int logCt)
{
    __shared__ u64 s[NTT_TILE];
    const int limb = blockIdx.y, poly = blockIdx.z;
    const int pr = map.prime(limb);
    const size_t N = (size_t)1 << logN;
    const PrimeC pc = T.pc[pr];
    const u64 q = pc.q, q2 = 2 * q;
    const u64 *tw = (INV ? T.itw : T.tw) + (size_t)pr * N;
    const u64 *tws = (INV ? T.itw_sh : T.tw_sh) + (size_t)pr * N;
    const int r = logN - logC, R = 1 << r, C = 1 << logC, Ct = 1 << logCt;
    const int c0 = blockIdx.x * Ct;
    const int nel = R * Ct;
    u64 *g = data + (size_t)poly * poly_stride + (size_t)limb * N + c0;

    for (int i = threadIdx.x; i < nel; i += NTT_THREADS) {
        int row = i >> logCt, col = i & (Ct - 1);
        s[i] = g[(size_t)row * C + col];
    }
    __syncthreads();

    const int half = nel >> 1;
    if (!INV) {
        for (int st = 0; st < r; st++) {
            const int ltr = r - 1 - st;
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                int col = b & (Ct - 1), k = b >> logCt;
                int grp = k >> ltr, off = k & ((1 << ltr) - 1);
                int r0 = (grp << (ltr + 1)) + off;
                int ti = (1 << st) + grp;
                u64 &x = s[(r0 << logCt) + col];
                u64 &y = s[((r0 + (1 << ltr)) << logCt) + col];
                bfly_ct(x, y, tw[ti], tws[ti], q, q2);
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nel; i += NTT_THREADS) {
            int row = i >> logCt, col = i & (Ct - 1);
            g[(size_t)row * C + col] = s[i];
        }
    } else {
        for (int ltr = 0; ltr < r; ltr++) {
            const int h = 1 << (r - 1 - ltr);
            const bool last = (ltr == r - 1);
            for (int b = threadIdx.x; b < half; b += NTT_THREADS) {
                int col = b & (Ct - 1), k = b >> logCt;
                int grp = k >> ltr, off = k & ((1 << ltr) - 1);
                int r0 = (grp << (ltr + 1)) + off;
                u64 &x = s[(r0 << logCt) + col];
                u64 &y = s[((r0 + (1 << ltr)) << logCt) + col];
                if (!last) {
                    bfly_gs(x, y, tw[h + grp], tws[h + grp], q, q2);
                } else {
                    u64 sum = csub(x + y, q2);
                    u64 d = x + q2 - y;
                    x = shoup_lazy(sum, pc.ninv, pc.ninv_sh, q);
                    y = shoup_lazy(d, T.last[pr], T.last_sh[pr], q);
                }
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nel; i += NTT_THREADS) {
            int row = i >> logCt, col = i & (Ct - 1);
            g[(size_t)row * C + col] = csub(s[i], q);
        }
    }
}

// ---------------------------------------------------------------- radix-16 passes (13 <= logN <= 16)
//
// Each pass transforms lines of S = 2^LOGS elements (the columns of the R x C
// view in the column pass, its rows in the row pass).  A thread keeps 16
// elements of one line in registers and runs 4 butterfly stages on them
// without touching LDS; one LDS exchange regroups the elements for the
// remaining LOGS-4 stages.  Two index patterns are used:
//   strided    e = t + TPL*i   (TPL = S/16 threads per line)
//   contiguous e = 16*t + i
// Global memory is always read and written with adjacent lanes on adjacent
// addresses: in the column pass lanes run over adjacent columns, in the row
// pass over adjacent strided positions (the contiguous pattern of the row
// pass is staged through LDS).  LDS rows are padded (one slot every 16 and
// one per line) so both patterns are free of bank conflicts.

template <int LOGS>
struct Geo {
    static constexpr int S = 1 << LOGS;
    static constexpr int TPL = S / 16;
    static constexpr int LINES = 256 / TPL;
    static constexpr int LS = S + S / 16 + 1;
};

__device__ __forceinline__ int lidx(int e) { return e + (e >> 4); }

// Twiddle index of local stage s for element e of line line_id.  STG = 0: the
// table itself (forward (1 << (off+s)) + (line << s) + (e >> (LOGS-s)),
// inverse (1 << (logN-1-off-s)) + (line << (LOGS-s-1)) + (e >> (s+1))).
// STG = 1: the copy a row pass stages for its block of LINES rows starting at
// row lb: the forward stages 0..3 (2^s twiddles per row, stage s at
// LINES (2^s - 1)) or the inverse stages 4..LOGS-1 (2^(LOGS-s-1) per row,
// stage s at LINES (2^(LOGS-4) - 2^(LOGS-s))).
template <bool INV, int LOGS, int STG>
__device__ __forceinline__ int tw_index(int s, int off, int line_id, int lb, int e, int logN)
{
    constexpr int LINES = Geo<LOGS>::LINES;
    if (STG == 0) {
        if (!INV) return (1 << (off + s)) + (line_id << s) + (e >> (LOGS - s));
        return (1 << (logN - 1 - off - s)) + (line_id << (LOGS - s - 1)) + (e >> (s + 1));
    }
    if (!INV) return LINES * ((1 << s) - 1) + ((line_id - lb) << s) + (e >> (LOGS - s));
    return LINES * ((1 << (LOGS - 4)) - (1 << (LOGS - s))) + ((line_id - lb) << (LOGS - s - 1)) + (e >> (s + 1));
}

// Row passes stage the round whose twiddles repeat within a row only for
// 256-element rows: there a block's copy (15 per row, both directions) takes
// 3.75 KB beside the 35 KB tile; for shorter rows (more rows per block) it
// would cost a block per CU.
// The other round of an FP64 row pass (forward stages 4..LOGS-1, inverse
// stages 0..3) needs a distinct twiddle for almost every butterfly; those are
// formed in registers instead (GenStage): with tw[j] = psi^brv(j), an index
// m = hi + lo whose parts have disjoint bits gives tw[m] = tw[hi] tw[lo], so a
// block stages, per row, the four entries tw[hi] of its stages (A) and, for
// all rows, the entries tw[lo] for lo < 2^(LOGS-1) (R).
// TwWords: the words of LDS a pass needs for its staged twiddles (two words
// per twiddle).
template <int LOGS>
struct RowStage {
    static constexpr bool on = LOGS == 8;
    static constexpr int ENTRIES = on ? 15 * Geo<LOGS>::LINES : 0;
};
template <int LOGS>
struct GenStage {
    static constexpr int A = RowStage<LOGS>::ENTRIES;              // double2 offset of A (4 per row)
    static constexpr int R = A + 4 * Geo<LOGS>::LINES;             // double2 offset of R (doubles)
    static constexpr int END = R + (1 << (LOGS - 2));              // double2 entries in all
};
template <int LOGS, bool COLS>
struct TwWords {
    static constexpr int value = COLS ? 2 * (1 << LOGS) : 2 * GenStage<LOGS>::END;
};

// Copy into LDS the twiddles a row pass reads through tw_index<., ., 1> for
// the block of rows starting at lb: dst[k] = src[global index of entry k].
template <bool INV, int LOGS, class T>
__device__ __forceinline__ void stage_row_twiddles(T *dst, const T *src, int lb, int logN, int tid)
{
    constexpr int LINES = Geo<LOGS>::LINES;
    if (!INV) {
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int cnt = LINES << s, o = LINES * ((1 << s) - 1);
            const size_t g0 = ((size_t)1 << (logN - LOGS + s)) + ((size_t)lb << s);
            for (int w = tid; w < cnt; w += 256) dst[o + w] = src[g0 + w];
        }
    } else {
#pragma unroll
        for (int s = 4; s < LOGS; s++) {
            const int cnt = LINES << (LOGS - s - 1), o = LINES * ((1 << (LOGS - 4)) - (1 << (LOGS - s)));
            const size_t g0 = ((size_t)1 << (logN - 1 - s)) + ((size_t)lb << (LOGS - s - 1));
            for (int w = tid; w < cnt; w += 256) dst[o + w] = src[g0 + w];
        }
    }
}

// The A and R entries of GenStage for the block of rows starting at lb, from
// the direction's FP64 table: A[4 r + k] = tw[hi] of local stage k + 4
// (forward) or k (inverse) of row lb + r; R[k] = tw[k].x for k < 2^(LOGS-1).
template <bool INV, int LOGS>
__device__ __forceinline__ void stage_gen_twiddles(double2 *A, const double2 *src, int lb, int logN, int tid)
{
    constexpr int LINES = Geo<LOGS>::LINES, NS = INV ? 4 : LOGS - 4, HALF = 1 << (LOGS - 1);
    double *R = reinterpret_cast<double *>(A + 4 * LINES);
    for (int w = tid; w < LINES * NS; w += 256) {
        const int r = w / NS, k = w % NS;
        const size_t gi = INV ? ((size_t)1 << (logN - 1 - k)) + ((size_t)(lb + r) << (LOGS - 1 - k))
                              : ((size_t)1 << (logN - LOGS + 4 + k)) + ((size_t)(lb + r) << (4 + k));
        A[r * 4 + k] = src[gi];
    }
    for (int k = tid; k < HALF; k += 256) R[k] = src[k].x;
}

// NST butterfly stages on the 16 registers; register distance starts at RD0
// and halves (forward) or doubles (inverse).  Element i has line index
// ebase + estride*i.  Forward local stage s = s0+k uses twiddle
// (1 << (off+s)) + (line_id << s) + (e >> (LOGS-s)); inverse local stage
// (distance 2^s in the line) uses (1 << (logN-1-off-s)) + (line_id << (LOGS-s-1)) + (e >> (s+1)).
template <bool INV, int NST, int RD0, int LOGS, int STG = 0>
__device__ __forceinline__ void ntt_round16(u64 (&x)[16], int ebase, int estride, int s0, int off, int line_id, int logN,
                                            const u64 *tw, const u64 *tws, u64 q, u64 q4, bool fold, u64 ninv,
                                            u64 ninv_sh, u64 lw, u64 lw_sh, int lb = 0)
{
#pragma unroll
    for (int k = 0; k < NST; k++) {
        const int d = INV ? (RD0 << k) : (RD0 >> k);
        const int s = s0 + k;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int i0 = (j / d) * 2 * d + (j % d), i1 = i0 + d;
            const int e = ebase + estride * i0;
            if (!INV) {
                const int ti = tw_index<false, LOGS, STG>(s, off, line_id, lb, e, logN);
                bfly_ct8(x[i0], x[i1], tw[ti], tws[ti], q, q4);
            } else if (fold && k == NST - 1) {
                u64 sum = csub(x[i0] + x[i1], q4);
                u64 dd = x[i0] + q4 - x[i1];
                x[i0] = shoup_lazy4(sum, ninv, ninv_sh, q);
                x[i1] = shoup_lazy4(dd, lw, lw_sh, q);
            } else {
                const int ti = tw_index<true, LOGS, STG>(s, off, line_id, lb, e, logN);
                bfly_gs4(x[i0], x[i1], tw[ti], tws[ti], q, q4);
            }
        }
    }
}

// The integer row-pass round on the contiguous pattern (e = 16 t + i) whose
// twiddles differ per butterfly: forward local stages 4..LOGS-1, inverse
// 0..3.  Stage s needs 16 >> sh consecutive table entries per thread
// (sh = LOGS - s forward, s + 1 inverse); they are loaded into registers
// before the block's first barrier, pairs as one 16-byte load (the pairs
// start at even indices of a 16-byte aligned table).
template <bool INV, int LOGS>
struct PreTw {
    static constexpr int NST = INV ? 4 : LOGS - 4;
    static constexpr int S0 = INV ? 0 : 4;
};

template <bool INV, int LOGS>
__device__ __forceinline__ void prefetch_tw(u64 (&w)[15], u64 (&ws)[15], const u64 *tw, const u64 *tws, int t, int gl,
                                            int logN)
{
    int o = 0;
#pragma unroll
    for (int k = 0; k < PreTw<INV, LOGS>::NST; k++) {
        const int s = PreTw<INV, LOGS>::S0 + k, sh = INV ? s + 1 : LOGS - s, ns = 16 >> sh;
        const size_t i0 = (INV ? ((size_t)1 << (logN - 1 - s)) + ((size_t)gl << (LOGS - s - 1))
                               : ((size_t)1 << (logN - LOGS + s)) + ((size_t)gl << s)) +
                          ((size_t)t << (4 - sh));
        if (ns == 1) {
            w[o] = tw[i0];
            ws[o] = tws[i0];
        } else {
#pragma unroll
            for (int j = 0; j < ns; j += 2) {
                const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(tw + i0 + j);
                const ulonglong2 b = *reinterpret_cast<const ulonglong2 *>(tws + i0 + j);
                w[o + j] = a.x;
                w[o + j + 1] = a.y;
                ws[o + j] = b.x;
                ws[o + j + 1] = b.y;
            }
        }
        o += ns;
    }
}

template <bool INV, int LOGS>
__device__ __forceinline__ void ntt_round16_pre(u64 (&x)[16], const u64 (&w)[15], const u64 (&ws)[15], u64 q, u64 q4)
{
    constexpr int NST = PreTw<INV, LOGS>::NST;
    int o = 0;
#pragma unroll
    for (int k = 0; k < NST; k++) {
        const int d = INV ? (1 << k) : ((1 << (NST - 1)) >> k);
        const int s = PreTw<INV, LOGS>::S0 + k, sh = INV ? s + 1 : LOGS - s;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int i0 = (j / d) * 2 * d + (j % d), i1 = i0 + d, sl = o + (i0 >> sh);
            if (!INV) bfly_ct8(x[i0], x[i1], w[sl], ws[sl], q, q4);
            else bfly_gs4(x[i0], x[i1], w[sl], ws[sl], q, q4);
        }
        o += 16 >> sh;
    }
}

// ---------------------------------------------------------------- FP64 butterflies (primes below 2^50)
//
// For p < 2^50 the pass runs on the FP64 pipes: residues are integers held
// exactly in doubles and may be negative.  A product a * w mod p (w in [0, p),
// wp = fl(w / p)) is computed exactly: h = fl(a w) and l = a w - h (one FMA)
// split the product, qq = rint(fl(a wp)) estimates the quotient, and
// (h - qq p) + l is the exact integer a w - qq p (both steps are exact because
// the values are integers below 2^53).  With |a| <= k p the estimate is off by
// at most 1/2 + k/4, so the result t satisfies |t| <= (1/2 + k/4) p.
// Bounds, in units of p, for the stage sequences used here:
//  * forward (CT: x' = x + t, y' = x - t): from |x| <= 2 the next four stages
//    stay below 2 -> 3 -> 4.25 -> 5.8 -> 7.7;
//  * inverse (GS: x' = x + y, y' = (x - y) w): from |x| <= 1/2 four stages
//    stay below 1 -> 2 -> 4 -> 8;
// so every round of at most four stages starts with a reduction of its 16
// registers to |x| <= (p-1)/2 (x - rint(x / p) p, exact), and every value
// stays below 8 p < 2^53.  Between the two passes of a transform the limb is
// kept in HBM as raw double bits; the first pass reads canonical residues and
// the last one writes them back canonical in [0, p).

using wa::fp_from_u64;
using wa::fp_mul;
using wa::fp_red;
using wa::fp_to_u64;

template <int LOGS, int NST, int RD0, bool INV, int STG = 0>
__device__ __forceinline__ void fp_round16(double (&x)[16], int ebase, int estride, int s0, int off, int line_id, int logN,
                                           const double2 *twf, double p, bool fold, const FpC &fc, int lb = 0)
{
#pragma unroll
    for (int k = 0; k < NST; k++) {
        const int d = INV ? (RD0 << k) : (RD0 >> k);
        const int s = s0 + k;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int i0 = (j / d) * 2 * d + (j % d), i1 = i0 + d;
            const int e = ebase + estride * i0;
            if (!INV) {
                const int ti = tw_index<false, LOGS, STG>(s, off, line_id, lb, e, logN);
                const double2 w = twf[ti];
                const double t = fp_mul(x[i1], w.x, w.y, p);
                const double u = x[i0];
                x[i0] = u + t;
                x[i1] = u - t;
            } else if (fold && k == NST - 1) {
                const double u = x[i0], v = x[i1];
                x[i0] = fp_mul(u + v, fc.ninv, fc.ninv_p, p);
                x[i1] = fp_mul(u - v, fc.lw, fc.lw_p, p);
            } else {
                const int ti = tw_index<true, LOGS, STG>(s, off, line_id, lb, e, logN);
                const double2 w = twf[ti];
                const double u = x[i0], v = x[i1];
                x[i0] = u + v;
                x[i1] = fp_mul(u - v, w.x, w.y, p);
            }
        }
    }
}

// The GenStage round of an FP64 row pass on the contiguous pattern
// (e = 16 t + i): forward local stages 4..3+NST, inverse 0..NST-1.  The
// twiddle of element e at local stage s has index hi + lo with
// lo = e >> (LOGS - s) (forward) or e >> (s + 1) (inverse); hi is the row's
// entry A[k].  Each distinct twiddle of the thread is formed once per stage.
template <int LOGS, int NST, int RD0, bool INV>
__device__ __forceinline__ void fp_round16_gen(double (&x)[16], int t, const double2 *A, const double *R, double p,
                                               double pinv)
{
#pragma unroll
    for (int k = 0; k < NST; k++) {
        const int d = INV ? (RD0 << k) : (RD0 >> k);
        const int s = (INV ? 0 : 4) + k;
        const int sh = INV ? s + 1 : LOGS - s;                    // element -> twiddle shift, 1..4
        const double2 a = A[k];
        double w[8], wp[8];
#pragma unroll
        for (int sl = 0; sl < (16 >> sh); sl++) wa::fp_twiddle(R[(t << (4 - sh)) + sl], a.x, a.y, p, pinv, w[sl], wp[sl]);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int i0 = (j / d) * 2 * d + (j % d), i1 = i0 + d;
            const int sl = i0 >> sh;
            const double u = x[i0], v = x[i1];
            if (!INV) {
                const double tt = fp_mul(v, w[sl], wp[sl], p);
                x[i0] = u + tt;
                x[i1] = u - tt;
            } else {
                x[i0] = u + v;
                x[i1] = fp_mul(u - v, w[sl], wp[sl], p);
            }
        }
    }
}

template <int LOGS>
__device__ __forceinline__ void fp_reduce16(double (&x)[16], double p, double pinv)
{
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = fp_red(x[i], p, pinv);
}

// One pass of the register NTT in FP64 (same geometry and twiddle indexing as
// the integer pass in k_ntt16).
// twf: the twiddles of the column pass (staged) or the table; stg (row
// passes): the block's staged RowStage and GenStage entries (rows from lb)
template <int LOGS, bool INV, bool COLS, bool KEEP, bool LDSIN, class LD>
__device__ __forceinline__ void ntt16_fp(u64 *base, u64 *sm_line, const FpC &fc, const double2 *twf, const double2 *stg,
                                         int lb, int t, int gl, int logN, const LD &ld)
{
    typedef Geo<LOGS> G;
    constexpr int NST2 = LOGS - 4;
    constexpr int RS = (!COLS && RowStage<LOGS>::on) ? 1 : 0;
    const size_t N = (size_t)1 << logN;
    const size_t C = COLS ? (N >> LOGS) : (size_t)G::S;
    auto addr = [&](int e) -> size_t { return COLS ? (size_t)e * C + gl : (size_t)gl * G::S + e; };
    const int off_f = COLS ? 0 : logN - LOGS;
    const int off_i = COLS ? logN - LOGS : 0;
    const int lid = COLS ? 0 : gl;
    const double p = fc.p, pinv = fc.pinv;
    double *sl = reinterpret_cast<double *>(sm_line);
    const double2 *twr = stg;                                       // RowStage entries
    const double2 *gA = stg + GenStage<LOGS>::A + 4 * (gl - lb);    // this row's A
    const double *gR = reinterpret_cast<const double *>(stg + GenStage<LOGS>::R);
    double x[16];

    if (!INV) {
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = fp_from_u64(ld(base, addr(t + G::TPL * i)));
        } else {
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = __longlong_as_double((long long)base[addr(t + G::TPL * i)]);
        }
        fp_reduce16<LOGS>(x, p, pinv);
        fp_round16<LOGS, 4, 8, false, RS>(x, t, G::TPL, 0, off_f, lid, logN, RS ? twr : twf, p, false, fc, lb);
#pragma unroll
        for (int i = 0; i < 16; i++) sl[lidx(t + G::TPL * i)] = x[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = sl[lidx(16 * t + i)];
        fp_reduce16<LOGS>(x, p, pinv);
        if (COLS) fp_round16<LOGS, NST2, (1 << (NST2 - 1)), false>(x, 16 * t, 1, 4, off_f, lid, logN, twf, p, false, fc);
        else fp_round16_gen<LOGS, NST2, (1 << (NST2 - 1)), false>(x, t, gA, gR, p, pinv);
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(16 * t + i)] = (u64)__double_as_longlong(x[i]);
        } else {
            u64 *su = sm_line;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; i++) su[lidx(16 * t + i)] = fp_to_u64(x[i], p, pinv);
            __syncthreads();
            if (!KEEP) {
#pragma unroll
                for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = su[lidx(t + G::TPL * i)];
            }
        }
    } else {
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = __longlong_as_double((long long)base[addr(16 * t + i)]);
        } else {
            u64 *su = sm_line;
            if (!LDSIN) {
#pragma unroll
                for (int i = 0; i < 16; i++) su[lidx(t + G::TPL * i)] = ld(base, addr(t + G::TPL * i));
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = fp_from_u64(su[lidx(16 * t + i)]);
            __syncthreads();
        }
        fp_reduce16<LOGS>(x, p, pinv);
        if (COLS) fp_round16<LOGS, 4, 1, true>(x, 16 * t, 1, 0, off_i, lid, logN, twf, p, false, fc);
        else fp_round16_gen<LOGS, 4, 1, true>(x, t, gA, gR, p, pinv);
#pragma unroll
        for (int i = 0; i < 16; i++) sl[lidx(16 * t + i)] = x[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = sl[lidx(t + G::TPL * i)];
        fp_reduce16<LOGS>(x, p, pinv);
        fp_round16<LOGS, NST2, (16 >> NST2), true, RS>(x, t, G::TPL, 4, off_i, lid, logN, RS ? twr : twf, p, COLS, fc, lb);
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = fp_to_u64(x[i], p, pinv);
        } else {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = (u64)__double_as_longlong(x[i]);
        }
    }
}

// One tile (4096 elements: LINES lines of S) of one pass over the limb at
// base (prime pr of the tables T).  sm: LINES * LS words of LDS; smtw:
// TwWords<LOGS, COLS> words of LDS for staged twiddles.  A column pass uses
// only the twiddles 1 .. 2^LOGS - 1 (the same for every column of the limb),
// so the block stages them in LDS once instead of every thread loading them
// from memory.  A row pass stages the round whose twiddles depend on the row
// (forward stages 0..3, inverse stages 4..LOGS-1): the block's rows use a
// contiguous range of each stage's table, which is read once per block.
// KEEP (forward row pass only): the canonical outputs stay in the LDS tile
// (element e of the block's row line at sm[line LS + lidx(e)], visible to the
// whole block) instead of being stored.
// LDSIN (inverse row pass only): the caller has written the canonical inputs
// to the LDS tile in that layout; they are not loaded from base.
// LD (the first pass: forward column, inverse row): ld(base, pos) supplies
// the canonical input at position pos of the limb (default: base[pos]); the
// outputs go to base.
struct PlainLd {
    __device__ u64 operator()(const u64 *base, size_t pos) const { return base[pos]; }
};

template <int LOGS, bool INV, bool COLS, bool KEEP = false, bool LDSIN = false, class LD = PlainLd>
__device__ __forceinline__ void ntt16_tile(u64 *base, u64 *sm, u64 *smtw, const NttTables &T, int pr, int tile, int logN,
                                           const LD &ld = LD())
{
    static_assert(!KEEP || (!INV && !COLS), "only the forward row pass keeps its outputs");
    static_assert(!LDSIN || (INV && !COLS), "only the inverse row pass takes its inputs from LDS");
    typedef Geo<LOGS> G;
    constexpr int NST2 = LOGS - 4;
    const size_t N = (size_t)1 << logN;
    const int tid = threadIdx.x;
    int line, t;
    if (COLS) {
        line = tid % G::LINES;
        t = tid / G::LINES;
    } else {
        t = tid % G::TPL;
        line = tid / G::TPL;
    }
    const int gl = tile * G::LINES + line;                // column (COLS) or row index
    const FpC fc = T.fc[pr];
    const int lb = tile * G::LINES;                        // first line of the block
    if (fc.use) {
        const double2 *twf = (INV ? T.itwf : T.twf) + (size_t)pr * N;
        double2 *st = reinterpret_cast<double2 *>(smtw);
        if (COLS) {
            for (int k = tid; k < G::S; k += 256) st[k] = twf[k];
            twf = st;
            __syncthreads();
        } else {
            if (RowStage<LOGS>::on) stage_row_twiddles<INV, LOGS>(st, twf, lb, logN, tid);
            stage_gen_twiddles<INV, LOGS>(st + GenStage<LOGS>::A, twf, lb, logN, tid);
            __syncthreads();
        }
        ntt16_fp<LOGS, INV, COLS, KEEP, LDSIN>(base, sm + line * G::LS, fc, twf, st, lb, t, gl, logN, ld);
        return;
    }
    const PrimeC pc = T.pc[pr];
    const u64 q = pc.q, q2 = 2 * q, q4 = 4 * q;
    const u64 *tw = (INV ? T.itw : T.tw) + (size_t)pr * N;
    const u64 *tws = (INV ? T.itw_sh : T.tw_sh) + (size_t)pr * N;
    // staged copies: for a column pass every twiddle it uses, for a row pass
    // the round whose twiddles repeat within a row (twr / twsr)
    u64 ipw[15], ipws[15];
    if (INV && !COLS) prefetch_tw<true, LOGS>(ipw, ipws, tw, tws, t, gl, logN);
    constexpr int TH = TwWords<LOGS, COLS>::value / 2;
    constexpr int RS = (!COLS && RowStage<LOGS>::on) ? 1 : 0;
    const u64 *twr = RS ? smtw : tw, *twsr = RS ? smtw + TH : tws;
    if (COLS) {
        for (int k = tid; k < G::S; k += 256) {
            smtw[k] = tw[k];
            smtw[TH + k] = tws[k];
        }
        tw = smtw;
        tws = smtw + TH;
        __syncthreads();
    } else if (RS) {
        stage_row_twiddles<INV, LOGS>(smtw, tw, lb, logN, tid);
        stage_row_twiddles<INV, LOGS>(smtw + TH, tws, lb, logN, tid);
        __syncthreads();
    }
    const size_t C = COLS ? (N >> LOGS) : (size_t)G::S;   // row length of the R x C view
    u64 *sl = sm + line * G::LS;
    auto addr = [&](int e) -> size_t { return COLS ? (size_t)e * C + gl : (size_t)gl * G::S + e; };
    const int off_f = COLS ? 0 : logN - LOGS;             // forward: global stage offset
    const int off_i = COLS ? logN - LOGS : 0;             // inverse: global log-distance offset
    const int lid = COLS ? 0 : gl;
    u64 x[16];

    u64 pw[15], pws[15];                                 // row passes: prefetched twiddles
    if (!INV) {
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = ld(base, addr(t + G::TPL * i));
        if (!COLS) prefetch_tw<false, LOGS>(pw, pws, tw, tws, t, gl, logN);
        ntt_round16<false, 4, 8, LOGS, RS>(x, t, G::TPL, 0, off_f, lid, logN, RS ? twr : tw, RS ? twsr : tws, q, q4, false,
                                           0, 0, 0, 0, lb);
#pragma unroll
        for (int i = 0; i < 16; i++) sl[lidx(t + G::TPL * i)] = x[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = sl[lidx(16 * t + i)];
        if (COLS)
            ntt_round16<false, NST2, (1 << (NST2 - 1)), LOGS>(x, 16 * t, 1, 4, off_f, lid, logN, tw, tws, q, q4, false, 0, 0,
                                                              0, 0);
        else
            ntt_round16_pre<false, LOGS>(x, pw, pws, q, q4);
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(16 * t + i)] = x[i];
        } else {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; i++) sl[lidx(16 * t + i)] = csub(csub(csub(x[i], q4), q2), q);
            __syncthreads();
            if (!KEEP) {
#pragma unroll
                for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = sl[lidx(t + G::TPL * i)];
            }
        }
    } else {
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = base[addr(16 * t + i)];
        } else {
            if (!LDSIN) {
#pragma unroll
                for (int i = 0; i < 16; i++) sl[lidx(t + G::TPL * i)] = ld(base, addr(t + G::TPL * i));
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; i++) x[i] = sl[lidx(16 * t + i)];
            __syncthreads();
        }
        if (COLS) ntt_round16<true, 4, 1, LOGS>(x, 16 * t, 1, 0, off_i, lid, logN, tw, tws, q, q4, false, 0, 0, 0, 0);
        else ntt_round16_pre<true, LOGS>(x, ipw, ipws, q, q4);
#pragma unroll
        for (int i = 0; i < 16; i++) sl[lidx(16 * t + i)] = x[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = sl[lidx(t + G::TPL * i)];
        ntt_round16<true, NST2, (16 >> NST2), LOGS, RS>(x, t, G::TPL, 4, off_i, lid, logN, RS ? twr : tw, RS ? twsr : tws, q,
                                                        q4, COLS, pc.ninv, pc.ninv_sh, T.last[pr], T.last_sh[pr], lb);
        if (COLS) {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = csub(csub(x[i], q2), q);
        } else {
#pragma unroll
            for (int i = 0; i < 16; i++) base[addr(t + G::TPL * i)] = x[i];
        }
    }
}

template <int LOGS, bool INV, bool COLS>
__global__ __launch_bounds__(256) void k_ntt16(u64 *data, long poly_stride, LimbMap map, NttTables T, int logN)
{
    __shared__ u64 sm[Geo<LOGS>::LINES * Geo<LOGS>::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, COLS>::value];
    const int limb = blockIdx.z, poly = blockIdx.y;
    u64 *base = data + (size_t)poly * poly_stride + ((size_t)limb << logN);
    ntt16_tile<LOGS, INV, COLS>(base, sm, smtw, T, map.prime(limb), blockIdx.x, logN);
}

// Descriptor-list form: a persistent grid walks the (item, tile) units of a
// list of limbs that may belong to different ring degrees, primes and
// contexts.  FIRST selects the first pass of the transform (the column pass
// of a forward transform, the row pass of an inverse one); the caller
// launches FIRST, then the second pass, over the same list.
// Items with N <= 4096 take one row pass over the whole limb (in the first
// launch); they have no units in the second.
template <bool INV, bool FIRST>
__global__ __launch_bounds__(256) void k_ntt16_list(const NttItem *items, const int *prefix, int n_items, int total)
{
    constexpr bool COLS = INV ? !FIRST : FIRST;
    // the largest tile of the three geometries and of the one-pass row tile
    // (tile and staged twiddles of one geometry, one array: the staged part
    // starts at the end of that geometry's tile)
    constexpr int W6 = Geo<6>::LINES * Geo<6>::LS, W7 = Geo<7>::LINES * Geo<7>::LS, W8 = Geo<8>::LINES * Geo<8>::LS;
    constexpr int A6 = W6 + TwWords<6, COLS>::value, A7 = W7 + TwWords<7, COLS>::value, A8 = W8 + TwWords<8, COLS>::value;
    constexpr int A67 = A6 > A7 ? A6 : A7, A678 = A67 > A8 ? A67 : A8;
    static_assert(W6 % 2 == 0 && W7 % 2 == 0 && W8 % 2 == 0, "staged twiddles must stay 16-byte aligned");
    __shared__ __attribute__((aligned(16))) u64 sm[A678 > NTT_TILE ? A678 : NTT_TILE];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        // the item holding unit u: prefix[it] <= u < prefix[it + 1]
        int lo = 0, hi = n_items - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const NttItem it = items[lo];
        const int tile = u - prefix[lo];
        if (it.logN <= 12) {
            ntt_rows_tile<INV>(it.data, sm, *it.tabs, it.prime, it.logN, it.logN, 1, 0);
            __syncthreads();
            continue;
        }
        const int logs = COLS ? it.logN - it.logC : it.logC;
        switch (logs) {
        case 6: ntt16_tile<6, INV, COLS>(it.data, sm, sm + W6, *it.tabs, it.prime, tile, it.logN); break;
        case 7: ntt16_tile<7, INV, COLS>(it.data, sm, sm + W7, *it.tabs, it.prime, tile, it.logN); break;
        default: ntt16_tile<8, INV, COLS>(it.data, sm, sm + W8, *it.tabs, it.prime, tile, it.logN); break;
        }
        __syncthreads();  // the next unit reuses the LDS tile
    }
}

template <int LOGS, bool INV, bool COLS>
static void launch16(u64 *data, long poly_stride, int npoly, int nlimbs, LimbMap map, const NttTables &T, int logN,
                     hipStream_t st)
{
    // limbs outermost: the blocks in flight share one prime's twiddles
    dim3 grid((unsigned)(((size_t)1 << logN) / 4096), npoly, nlimbs);
    hipLaunchKernelGGL((k_ntt16<LOGS, INV, COLS>), grid, dim3(256), 0, st, data, poly_stride, map, T, logN);
}

template <bool INV, bool COLS>
static void launch16_logs(int logs, u64 *data, long poly_stride, int npoly, int nlimbs, LimbMap map, const NttTables &T,
                          int logN, hipStream_t st)
{
    switch (logs) {
    case 6: launch16<6, INV, COLS>(data, poly_stride, npoly, nlimbs, map, T, logN, st); break;
    case 7: launch16<7, INV, COLS>(data, poly_stride, npoly, nlimbs, map, T, logN, st); break;
    default: launch16<8, INV, COLS>(data, poly_stride, npoly, nlimbs, map, T, logN, st); break;
    }
}

// ---------------------------------------------------------------- ModDown: last NTT pass fused with the epilogue
//
// The ModDown of a key switch converts the special-prime part to the Q basis
// (conv, coefficient domain), transforms it and combines it with the Q part
// of the key inner product: out_p = (sum_j d_j key_{j,p} - NTT(conv_p)) P^-1
// (+ the addends).  Here the forward row pass of conv_p (after its column
// pass) leaves its canonical outputs in its LDS tile and the same block
// applies that epilogue, so the transformed conv is never written to and read
// back from memory.  One block per (row tile, limb, ciphertext, polynomial).  Blocks
// are numbered so that each XCD (blocks b, b+8, ...) walks a contiguous range
// in which all ciphertexts and both polynomials of one (limb, tile) follow
// each other: the tile's key words and ModUp digits are then re-read from
// that XCD's L2.
// ADD: 0 no addend; 1 `add` on polynomial 0 (read through add_g); 2 `add` on
// both; 3 as 1, plus `add2` on both polynomials read in place (a rotation
// added to a ciphertext).  add2 may be `out` itself: every position of add2 is
// read by the thread that writes the same position of out.
template <int LOGS, int BETA, int ADD>
__global__ __launch_bounds__(256, 4) void k_ntt_rows_md(const u64 *__restrict__ ext, long ext_stride, KsItems I,
                                                    u64 *conv, long conv_stride, const u64 *__restrict__ add,
                                                    long add_stride, const u64 *add2, long add2_stride, u64 *out,
                                                    long out_stride, NttTables T, int logN, int L1, int E, int nT,
                                                    int count, const u64 *Pinv, const u64 *Pinv_sh)
{
    typedef Geo<LOGS> G;
    __shared__ u64 sm[G::LINES * G::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, false>::value];
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned u = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const unsigned slots = (unsigned)count * (unsigned)I.n;         // (item, ciphertext) slots of conv
    const int poly = (int)(u % 2);
    const int cs = (int)((u / 2) % slots), item = cs / count, ct = cs % count;
    const unsigned rest = u / (2u * slots);
    const unsigned tiles = 1u << (logN - 12);
    const int tile = (int)(rest % tiles), limb = (int)(rest / tiles);
    const size_t N = (size_t)1 << logN, per = (size_t)L1 * N, li = (size_t)limb * N;
    const u64 g = I.g[item], add_g = I.add_g[item], *key = I.key[item];
    out += I.out_off[item];

    ntt16_tile<LOGS, false, false, true>(conv + cs * conv_stride + poly * per + li, sm, smtw, T, limb, tile, logN);

    // the transformed tile (4096 consecutive positions of the limb) is in
    // LDS; each thread finishes 8 adjacent pairs, lanes on adjacent pairs
    const size_t tbase = (size_t)tile * 4096;
    const PrimeC p = T.pc[limb];
    const u64 pinv = Pinv[limb], pinv_sh = Pinv_sh[limb];
    const u64 *x = ext + ct * ext_stride + li;
    const u64 *kp = key + ((size_t)poly * nT + limb) * N;              // digit j at + j 2 nT N
    const bool do_add = (ADD >= 1 && poly == 0) || (ADD == 2 && poly == 1);
    const u64 *ad = ADD ? add + ct * add_stride + poly * per + li : nullptr;
    const u64 *ad2 = ADD == 3 ? add2 + ct * add2_stride + poly * per + li : nullptr;
    u64 *o = out + ct * out_stride + poly * per + li;
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const int e = 2 * (int)threadIdx.x + 512 * m;                  // even position in the tile
        const size_t pos = tbase + e;
        const size_t src = g ? auto_src((u32)pos, g, logN) : pos;
        u64x2 d[BETA], kw[BETA];
#pragma unroll
        for (int j = 0; j < BETA; j++) {
            d[j] = ld2_perm(x + (size_t)j * E * N, src);
            kw[j] = ld2(kp + (size_t)j * 2 * nT * N + pos);
        }
        u64x2 a = {0, 0};
        if (ADD && do_add) a = ld2_perm(ad, add_g ? auto_src((u32)pos, add_g, logN) : pos);
        const u64 *cl = sm + (e >> LOGS) * G::LS;
        const int cc = e & (G::S - 1);
        const u64 c0 = cl[lidx(cc)], c1 = cl[lidx(cc + 1)];
        u128w s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++) {
            acc_wide(s0, mul_wide(d[j].x, kw[j].x));
            acc_wide(s1, mul_wide(d[j].y, kw[j].y));
        }
        // beta <= 8 products below q^2: every sum is below q 2^64, a plain REDC suffices
        u64 v0 = shoup(sub_mod(redc(s0, p.q, p.qneg), c0, p.q), pinv, pinv_sh, p.q);
        u64 v1 = shoup(sub_mod(redc(s1, p.q, p.qneg), c1, p.q), pinv, pinv_sh, p.q);
        if (ADD && do_add) {
            v0 = add_mod(v0, a.x, p.q);
            v1 = add_mod(v1, a.y, p.q);
        }
        if (ADD == 3) {
            const u64x2 a2 = ld2(ad2 + pos);
            v0 = add_mod(v0, a2.x, p.q);
            v1 = add_mod(v1, a2.y, p.q);
        }
        st2_nt(o + pos, v0, v1);
    }
}

static bool ntt_rows_md_ok(const rbk_ctx_impl *c)
{
    const int logN = c->logN, logC = c->ntt_logC, r = logN - logC;
    return logN >= 13 && logN <= 16 && r >= 6 && r <= 8 && logC >= 6 && logC <= 8;
}

static void ntt_cols_fwd_launch(const rbk_ctx_impl *c, u64 *data, long poly_stride, int npoly, int nlimbs, LimbMap map,
                                hipStream_t st)
{
    if (npoly <= 0 || nlimbs <= 0) return;
    const int logN = c->logN, r = logN - c->ntt_logC;
    kt_begin(c, KC_NTT_COLS_FWD, st);
    launch16_logs<false, true>(r, data, poly_stride, npoly, nlimbs, map, c->tabs, logN, st);
    kt_end(c, KC_NTT_COLS_FWD, 2.0 * npoly * nlimbs * c->N * sizeof(u64), st);
}

static void ntt_rows_md_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *conv,
                               long conv_stride, const u64 *add, long add_stride, int add_both, const u64 *add2,
                               long add2_stride, u64 *out, long out_stride, int level, int count, hipStream_t st)
{
    const int L1 = level + 1, E = L1 + c->nP, logN = c->logN, logC = c->ntt_logC;
    const int beta_l = (L1 + c->alpha - 1) / c->alpha;
    // a second addend goes with the rotation form (c0's addend only)
    const int addm = add2 ? 3 : add ? (add_both ? 2 : 1) : 0;
    const dim3 grid((unsigned)(((size_t)1 << logN) / 4096 * 2 * (size_t)count * I.n * L1));
    kt_begin(c, KC_NTT_ROWS_MD, st);
#define RMD_LAUNCH(LG, B, A)                                                                                     \
    hipLaunchKernelGGL((k_ntt_rows_md<LG, B, A>), grid, dim3(256), 0, st, ext, ext_stride, I, conv, conv_stride, add,   \
                       add_stride, add2, add2_stride, out, out_stride, c->tabs, logN, L1, E, c->nT, count, c->d_Pinv,   \
                       c->d_Pinv_sh)
#define RMD_ADD(LG, B)                                                                                          \
    do {                                                                                                        \
        if (addm == 0) RMD_LAUNCH(LG, B, 0);                                                                    \
        else if (addm == 1) RMD_LAUNCH(LG, B, 1);                                                               \
        else if (addm == 2) RMD_LAUNCH(LG, B, 2);                                                               \
        else RMD_LAUNCH(LG, B, 3);                                                                              \
    } while (0)
#define RMD_BETA(LG)                                                                                            \
    switch (beta_l) {                                                                                           \
    case 1: RMD_ADD(LG, 1); break;                                                                              \
    case 2: RMD_ADD(LG, 2); break;                                                                              \
    case 3: RMD_ADD(LG, 3); break;                                                                              \
    case 4: RMD_ADD(LG, 4); break;                                                                              \
    case 5: RMD_ADD(LG, 5); break;                                                                              \
    case 6: RMD_ADD(LG, 6); break;                                                                              \
    case 7: RMD_ADD(LG, 7); break;                                                                              \
    default: RMD_ADD(LG, 8); break;                                                                             \
    }
    switch (logC) {
    case 6: RMD_BETA(6); break;
    case 7: RMD_BETA(7); break;
    default: RMD_BETA(8); break;
    }
#undef RMD_BETA
#undef RMD_ADD
#undef RMD_LAUNCH
    // algorithmic bytes: conv (after its column pass) and the ModUp digits
    // read, the outputs written, the addends read, each item's key words read once
    const int add_words = addm == 3 ? 3 : addm;
    const double words = (double)count * I.n * L1 * (beta_l + 2 + 2 + add_words) + 2.0 * I.n * beta_l * L1;
    kt_end(c, KC_NTT_ROWS_MD, words * c->N * sizeof(u64), st);
}

// ---------------------------------------------------------------- ModDown: inner product fused with the first iNTT pass
//
// The special-prime part of the key inner product, tp_p = sum_j d_j key_{j,p}
// on the special primes, is only read by the inverse NTT that starts the
// ModDown.  Its first (row) pass computes the tile in LDS instead of loading
// it (adjacent pairs, as in k_ntt_rows_md), so tp is written once, by the row
// pass.  Blocks per (row tile, special prime, ciphertext, polynomial),
// numbered per XCD as in k_ntt_rows_md.
template <int LOGS, int BETA>
__global__ __launch_bounds__(256, 4) void k_ntt_rows_ip(const u64 *__restrict__ ext, long ext_stride, KsItems I,
                                                       u64 *tp, NttTables T, int logN, int L1, int E, int nT, int nQ,
                                                       int nP, int count)
{
    typedef Geo<LOGS> G;
    __shared__ u64 sm[G::LINES * G::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, false>::value];
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned u = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const unsigned slots = (unsigned)count * (unsigned)I.n;         // (item, ciphertext) slots of tp
    const int poly = (int)(u % 2);
    const int cs = (int)((u / 2) % slots), item = cs / count, ct = cs % count;
    const unsigned rest = u / (2u * slots);
    const unsigned tiles = 1u << (logN - 12);
    const int tile = (int)(rest % tiles), k = (int)(rest / tiles);
    const u64 g = I.g[item], *key = I.key[item];
    const size_t N = (size_t)1 << logN, tbase = (size_t)tile * 4096;
    const int pr = nQ + k;
    const PrimeC p = T.pc[pr];
    const u64 *x = ext + ct * ext_stride + (size_t)(L1 + k) * N;     // digit j at + j E N
    const u64 *kp = key + ((size_t)poly * nT + pr) * N;              // digit j at + j 2 nT N
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const int e = 2 * (int)threadIdx.x + 512 * m;                // even position in the tile
        const size_t pos = tbase + e;
        const size_t src = g ? auto_src((u32)pos, g, logN) : pos;
        u64x2 d[BETA], kw[BETA];
#pragma unroll
        for (int j = 0; j < BETA; j++) {
            d[j] = ld2_perm(x + (size_t)j * E * N, src);
            kw[j] = ld2(kp + (size_t)j * 2 * nT * N + pos);
        }
        u128w s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int j = 0; j < BETA; j++) {
            acc_wide(s0, mul_wide(d[j].x, kw[j].x));
            acc_wide(s1, mul_wide(d[j].y, kw[j].y));
        }
        // beta <= 8 products below p^2: every sum is below p 2^64, a plain REDC suffices
        u64 *row = sm + (e >> LOGS) * G::LS;
        const int cc = e & (G::S - 1);
        row[lidx(cc)] = redc(s0, p.q, p.qneg);
        row[lidx(cc + 1)] = redc(s1, p.q, p.qneg);
    }
    ntt16_tile<LOGS, true, false, false, true>(tp + (((size_t)cs * 2 + poly) * nP + k) * N, sm, smtw, T, pr, tile, logN);
}

static void ntt_rows_ip_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *tp,
                               int level, int count, hipStream_t st)
{
    const int L1 = level + 1, E = L1 + c->nP, logN = c->logN, logC = c->ntt_logC;
    const int beta_l = (L1 + c->alpha - 1) / c->alpha;
    const dim3 grid((unsigned)(((size_t)1 << logN) / 4096 * 2 * (size_t)count * I.n * c->nP));
    kt_begin(c, KC_NTT_ROWS_IP, st);
#define RIP_LAUNCH(LG, B)                                                                                       \
    hipLaunchKernelGGL((k_ntt_rows_ip<LG, B>), grid, dim3(256), 0, st, ext, ext_stride, I, tp, c->tabs, logN, L1, E,   \
                       c->nT, c->nQ, c->nP, count)
#define RIP_BETA(LG)                                                                                            \
    switch (beta_l) {                                                                                           \
    case 1: RIP_LAUNCH(LG, 1); break;                                                                           \
    case 2: RIP_LAUNCH(LG, 2); break;                                                                           \
    case 3: RIP_LAUNCH(LG, 3); break;                                                                           \
    case 4: RIP_LAUNCH(LG, 4); break;                                                                           \
    case 5: RIP_LAUNCH(LG, 5); break;                                                                           \
    case 6: RIP_LAUNCH(LG, 6); break;                                                                           \
    case 7: RIP_LAUNCH(LG, 7); break;                                                                           \
    default: RIP_LAUNCH(LG, 8); break;                                                                          \
    }
    switch (logC) {
    case 6: RIP_BETA(6); break;
    case 7: RIP_BETA(7); break;
    default: RIP_BETA(8); break;
    }
#undef RIP_BETA
#undef RIP_LAUNCH
    // algorithmic bytes: the digits' special-prime limbs and each item's key
    // words read once, tp written once
    const double words = (double)count * I.n * c->nP * (beta_l + 2) + 2.0 * I.n * beta_l * c->nP;
    kt_end(c, KC_NTT_ROWS_IP, words * c->N * sizeof(u64), st);
}

static KsItems one_item(const u64 *key, u64 g, u64 add_g)
{
    KsItems I{};
    I.key[0] = key;
    I.g[0] = g;
    I.add_g[0] = add_g;
    I.out_off[0] = 0;
    I.n = 1;
    return I;
}

bool moddown_items_ok(const rbk_ctx_impl *c) { return ntt_rows_md_ok(c); }

void moddown_head_items_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *tp,
                               int level, int count, hipStream_t st)
{
    const int nP = c->nP;
    const LimbMap pm{0, 0, c->nQ};
    ntt_rows_ip_launch(c, ext, ext_stride, I, tp, level, count, st);
    kt_begin(c, KC_NTT_COLS_INV, st);
    launch16_logs<true, true>(c->logN - c->ntt_logC, tp, (long)nP * c->N, 2 * count * I.n, nP, pm, c->tabs, c->logN, st);
    kt_end(c, KC_NTT_COLS_INV, 2.0 * 2 * count * I.n * nP * c->N * sizeof(u64), st);
}

void moddown_head_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *tp, int level,
                         int count, u64 g, hipStream_t st)
{
    const int nP = c->nP;
    const LimbMap pm{0, 0, c->nQ};
    if (ntt_rows_md_ok(c)) {
        moddown_head_items_launch(c, ext, ext_stride, one_item(key, g, 0), tp, level, count, st);
        return;
    }
    ip_p_launch(c, ext, ext_stride, key, tp, level, count, g, st);
    ntt_launch(c, tp, (long)nP * c->N, 2 * count, nP, pm, true, st);
}

// ---------------------------------------------------------------- rescale: NTT of the lifted last limb, fused at both ends
//
// Rescale lifts each polynomial's last limb (coefficient domain, centred)
// to the other limbs, transforms the lifts and finishes with
// out = (in - NTT(lift)) q_l^-1.  The column pass computes the lift of its
// inputs from the last limb itself (LiftLd), and the row pass leaves its
// outputs in LDS for the same block to finish, so the lifted limbs are
// written and read once, between the two passes.
struct LiftLd {
    const u64 *last;  // the polynomial's last limb, coefficient domain
    u64 q, one_sh, qmod, half;  // target prime, floor(2^64/q), q_l mod q, (q_l - 1) / 2
    __device__ u64 operator()(const u64 *, size_t pos) const
    {
        const u64 x = last[pos];
        const u64 xm = shoup(x, 1, one_sh, q);
        return x <= half ? xm : sub_mod(xm, qmod, q);
    }
};

template <int LOGS>
__global__ __launch_bounds__(256) void k_ntt_cols_lift(const u64 *last, u64 *lifted, NttTables T, const u64 *qmod,
                                                       int logN, int level)
{
    __shared__ u64 sm[Geo<LOGS>::LINES * Geo<LOGS>::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, true>::value];
    const int limb = blockIdx.z, poly = blockIdx.y;
    const size_t N = (size_t)1 << logN;
    const PrimeC p = T.pc[limb];
    const LiftLd ld{last + (size_t)poly * N, p.q, p.one_sh, qmod[limb], (T.pc[level].q - 1) / 2};
    ntt16_tile<LOGS, false, true, false, false, LiftLd>(lifted + ((size_t)poly * level + limb) * N, sm, smtw, T, limb,
                                                        blockIdx.x, logN, ld);
}

template <int LOGS>
__global__ __launch_bounds__(256) void k_ntt_rows_rs(const u64 *lifted, const u64 *__restrict__ in, u64 *__restrict__ out,
                                                     NttTables T, const u64 *inv, const u64 *inv_sh, int logN, int level)
{
    typedef Geo<LOGS> G;
    __shared__ u64 sm[G::LINES * G::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, false>::value];
    const int limb = blockIdx.z, poly = blockIdx.y, tile = blockIdx.x;
    const size_t N = (size_t)1 << logN, li = (size_t)limb * N;
    ntt16_tile<LOGS, false, false, true>(const_cast<u64 *>(lifted) + (size_t)poly * level * N + li, sm, smtw, T, limb, tile,
                                         logN);
    const u64 q = T.pc[limb].q, w = inv[limb], wsh = inv_sh[limb];
    const u64 *x = in + (size_t)poly * (level + 1) * N + li;
    u64 *o = out + (size_t)poly * level * N + li;
    const size_t tbase = (size_t)tile * 4096;
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const int e = 2 * (int)threadIdx.x + 512 * m;              // even position in the tile
        const size_t pos = tbase + e;
        const u64x2 v = ld2(x + pos);
        const u64 *cl = sm + (e >> LOGS) * G::LS;
        const int cc = e & (G::S - 1);
        st2(o + pos, shoup(sub_mod(v.x, cl[lidx(cc)], q), w, wsh, q), shoup(sub_mod(v.y, cl[lidx(cc + 1)], q), w, wsh, q));
    }
}

bool rescale_fused_launch(const rbk_ctx_impl *c, const u64 *last, u64 *lifted, const u64 *in, u64 *out, int level,
                          int npoly, hipStream_t st)
{
    if (!ntt_rows_md_ok(c) || level < 1 || npoly < 1) return false;
    if (((uintptr_t)in | (uintptr_t)out) & 15) return false;  // the finish moves 16-byte pairs
    const int logN = c->logN, logC = c->ntt_logC, r = logN - logC;
    const size_t N = c->N;
    const u64 *qmod = c->d_rs_qmod + (size_t)level * c->nQ;
    const u64 *inv = c->d_rs_inv + (size_t)level * c->nQ, *inv_sh = c->d_rs_inv_sh + (size_t)level * c->nQ;
    const dim3 grid((unsigned)(N / 4096), npoly, level);
    const double bytes = 2.0 * npoly * level * N * sizeof(u64);
    kt_begin(c, KC_NTT_COLS_FWD, st);
    switch (r) {
    case 6: hipLaunchKernelGGL(k_ntt_cols_lift<6>, grid, dim3(256), 0, st, last, lifted, c->tabs, qmod, logN, level); break;
    case 7: hipLaunchKernelGGL(k_ntt_cols_lift<7>, grid, dim3(256), 0, st, last, lifted, c->tabs, qmod, logN, level); break;
    default: hipLaunchKernelGGL(k_ntt_cols_lift<8>, grid, dim3(256), 0, st, last, lifted, c->tabs, qmod, logN, level); break;
    }
    kt_end(c, KC_NTT_COLS_FWD, bytes / 2 + (double)npoly * N * sizeof(u64), st);
    kt_begin(c, KC_RESCALE, st);
    switch (logC) {
    case 6: hipLaunchKernelGGL(k_ntt_rows_rs<6>, grid, dim3(256), 0, st, lifted, in, out, c->tabs, inv, inv_sh, logN, level); break;
    case 7: hipLaunchKernelGGL(k_ntt_rows_rs<7>, grid, dim3(256), 0, st, lifted, in, out, c->tabs, inv, inv_sh, logN, level); break;
    default: hipLaunchKernelGGL(k_ntt_rows_rs<8>, grid, dim3(256), 0, st, lifted, in, out, c->tabs, inv, inv_sh, logN, level); break;
    }
    kt_end(c, KC_RESCALE, 3.0 * npoly * level * N * sizeof(u64), st);
    return true;
}

// ---------------------------------------------------------------- inverse NTT out of place
//
// The first (row) pass reads the limbs from src and writes dst; the column
// pass then runs in place on dst.  Saves the copy an in-place transform of a
// buffer that must survive would need.
struct OffsetLd {
    const u64 *src;  // the limb's first element in the source buffer
    __device__ u64 operator()(const u64 *, size_t pos) const { return src[pos]; }
};

template <int LOGS>
__global__ __launch_bounds__(256) void k_ntt16_inv_from(const u64 *src, long src_stride, u64 *dst, long dst_stride,
                                                        LimbMap map, NttTables T, int logN)
{
    __shared__ u64 sm[Geo<LOGS>::LINES * Geo<LOGS>::LS];
    __shared__ __attribute__((aligned(16))) u64 smtw[TwWords<LOGS, false>::value];
    const int limb = blockIdx.z, poly = blockIdx.y;
    const size_t off = ((size_t)limb << logN);
    const OffsetLd ld{src + poly * src_stride + off};
    ntt16_tile<LOGS, true, false, false, false, OffsetLd>(dst + poly * dst_stride + off, sm, smtw, T, map.prime(limb),
                                                          blockIdx.x, logN, ld);
}

hipError_t ntt_inverse_from_launch(const rbk_ctx_impl *c, const u64 *src, long src_stride, u64 *dst, long dst_stride,
                                   int npoly, int nlimbs, LimbMap map, hipStream_t st)
{
    if (npoly <= 0 || nlimbs <= 0) return hipSuccess;
    const int logN = c->logN, logC = c->ntt_logC, r = logN - logC;
    if (!ntt_rows_md_ok(c)) {
        const hipError_t e =
            hipMemcpy2DAsync(dst, dst_stride * sizeof(u64), src, src_stride * sizeof(u64), (size_t)nlimbs * c->N * sizeof(u64),
                             npoly, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        ntt_launch(c, dst, dst_stride, npoly, nlimbs, map, true, st);
        return hipSuccess;
    }
    // chunks of whole polynomials, both passes per chunk (as ntt_launch)
    int ppc = npoly;
    if (c->ntt_chunk > 0 && (long)npoly * nlimbs > c->ntt_chunk) ppc = std::max(1, c->ntt_chunk / nlimbs);
    const double bytes = 2.0 * nlimbs * c->N * sizeof(u64);
    for (int p0 = 0; p0 < npoly; p0 += ppc) {
        const int np = std::min(ppc, npoly - p0);
        const u64 *s = src + (size_t)p0 * src_stride;
        u64 *d = dst + (size_t)p0 * dst_stride;
        const dim3 grid((unsigned)(((size_t)1 << logN) / 4096), np, nlimbs);
        kt_begin(c, KC_NTT_ROWS_INV, st);
        switch (logC) {
        case 6: hipLaunchKernelGGL(k_ntt16_inv_from<6>, grid, dim3(256), 0, st, s, src_stride, d, dst_stride, map, c->tabs, logN); break;
        case 7: hipLaunchKernelGGL(k_ntt16_inv_from<7>, grid, dim3(256), 0, st, s, src_stride, d, dst_stride, map, c->tabs, logN); break;
        default: hipLaunchKernelGGL(k_ntt16_inv_from<8>, grid, dim3(256), 0, st, s, src_stride, d, dst_stride, map, c->tabs, logN); break;
        }
        kt_end(c, KC_NTT_ROWS_INV, bytes * np, st);
        kt_begin(c, KC_NTT_COLS_INV, st);
        launch16_logs<true, true>(r, d, dst_stride, np, nlimbs, map, c->tabs, logN, st);
        kt_end(c, KC_NTT_COLS_INV, bytes * np, st);
    }
    return hipSuccess;
}

void moddown_tail_items_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *conv,
                               const u64 *add, long add_stride, int add_both, u64 *out, long out_stride, int level,
                               int count, hipStream_t st, const u64 *add2, long add2_stride)
{
    const int L1 = level + 1;
    const size_t N = c->N;
    const LimbMap qm{0, c->nQ, c->nQ};
    ntt_cols_fwd_launch(c, conv, (long)(L1 * N), 2 * count * I.n, L1, qm, st);
    ntt_rows_md_launch(c, ext, ext_stride, I, conv, (long)(2 * L1 * N), add, add_stride, add_both, add2, add2_stride, out,
                       out_stride, level, count, st);
}

bool moddown_add2_ok(const rbk_ctx_impl *c) { return c->nP > 0 && ntt_rows_md_ok(c); }

void moddown_tail_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *conv,
                         const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level,
                         int count, u64 g, hipStream_t st, const u64 *add2, long add2_stride)
{
    const int L1 = level + 1;
    const size_t N = c->N;
    const LimbMap qm{0, c->nQ, c->nQ};
    if (ntt_rows_md_ok(c)) {
        moddown_tail_items_launch(c, ext, ext_stride, one_item(key, g, add_g), conv, add, add_stride, add_both, out,
                                  out_stride, level, count, st, add2, add2_stride);
        return;
    }
    ntt_launch(c, conv, (long)(L1 * N), 2 * count, L1, qm, false, st);
    moddown_ip_launch(c, ext, ext_stride, key, conv, (long)(2 * L1 * N), add, add_stride, add_g, add_both, out, out_stride,
                      level, count, g, st);
}

void ntt_launch(const rbk_ctx_impl *c, u64 *data, long poly_stride, int npoly, int nlimbs, LimbMap map, bool inverse,
                hipStream_t st)
{
    if (npoly <= 0 || nlimbs <= 0) return;
    const int logN = c->logN, logC = c->ntt_logC;
    const int r = logN - logC;
    NttTables T = c->tabs;
    const double bytes = 2.0 * npoly * nlimbs * c->N * sizeof(u64);  // one read and one write of every limb
    if (r == 0) {
        dim3 grid(1, nlimbs, npoly);
        int cls = inverse ? KC_NTT_ROWS_INV : KC_NTT_ROWS_FWD;
        kt_begin(c, cls, st);
        if (inverse)
            hipLaunchKernelGGL(k_ntt_small<true>, grid, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN);
        else
            hipLaunchKernelGGL(k_ntt_small<false>, grid, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN);
        kt_end(c, cls, bytes, st);
        return;
    }
    if (logN >= 13 && logN <= 16 && r >= 6 && r <= 8 && logC >= 6 && logC <= 8) {
        // chunks of whole polynomials, both passes per chunk
        int ppc = npoly;
        if (c->ntt_chunk > 0 && (long)npoly * nlimbs > c->ntt_chunk) ppc = std::max(1, c->ntt_chunk / nlimbs);
        for (int p0 = 0; p0 < npoly; p0 += ppc) {
            const int np = std::min(ppc, npoly - p0);
            u64 *d = data + (size_t)p0 * poly_stride;
            const double cb = bytes * np / npoly;
            if (!inverse) {
                kt_begin(c, KC_NTT_COLS_FWD, st);
                launch16_logs<false, true>(r, d, poly_stride, np, nlimbs, map, T, logN, st);
                kt_end(c, KC_NTT_COLS_FWD, cb, st);
                kt_begin(c, KC_NTT_ROWS_FWD, st);
                launch16_logs<false, false>(logC, d, poly_stride, np, nlimbs, map, T, logN, st);
                kt_end(c, KC_NTT_ROWS_FWD, cb, st);
            } else {
                kt_begin(c, KC_NTT_ROWS_INV, st);
                launch16_logs<true, false>(logC, d, poly_stride, np, nlimbs, map, T, logN, st);
                kt_end(c, KC_NTT_ROWS_INV, cb, st);
                kt_begin(c, KC_NTT_COLS_INV, st);
                launch16_logs<true, true>(r, d, poly_stride, np, nlimbs, map, T, logN, st);
                kt_end(c, KC_NTT_COLS_INV, cb, st);
            }
        }
        return;
    }
    const int rows_per_tile = NTT_TILE >> logC;       // row pass
    const int logCt = 12 - r;                          // column pass: 4096 / R columns
    dim3 grow((1 << r) / rows_per_tile, nlimbs, npoly);
    dim3 gcol((1 << logC) >> logCt, nlimbs, npoly);
    if (!inverse) {
        kt_begin(c, KC_NTT_COLS_FWD, st);
        hipLaunchKernelGGL(k_ntt_cols<false>, gcol, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN, logC, logCt);
        kt_end(c, KC_NTT_COLS_FWD, bytes, st);
        kt_begin(c, KC_NTT_ROWS_FWD, st);
        hipLaunchKernelGGL(k_ntt_rows<false>, grow, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN, logC,
                           rows_per_tile);
        kt_end(c, KC_NTT_ROWS_FWD, bytes, st);
    } else {
        kt_begin(c, KC_NTT_ROWS_INV, st);
        hipLaunchKernelGGL(k_ntt_rows<true>, grow, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN, logC,
                           rows_per_tile);
        kt_end(c, KC_NTT_ROWS_INV, bytes, st);
        kt_begin(c, KC_NTT_COLS_INV, st);
        hipLaunchKernelGGL(k_ntt_cols<true>, gcol, dim3(NTT_THREADS), 0, st, data, poly_stride, map, T, logN, logC, logCt);
        kt_end(c, KC_NTT_COLS_INV, bytes, st);
    }
}

// units of an item in the first / second launch of a list transform
int ntt_item_units(int logN, bool first)
{
    if (logN <= 12) return first ? 1 : 0;
    return 1 << (logN - 12);
}

void ntt_list_launch(const NttItem *d_items, const int *d_prefix1, const int *d_prefix2, int n_items, int total1,
                     int total2, bool inverse, hipStream_t st)
{
    // persistent grid: four resident blocks per compute unit
    const int cap = 4 * 256;
    if (total1 > 0) {
        dim3 g1(std::min(total1, cap));
        if (inverse) hipLaunchKernelGGL((k_ntt16_list<true, true>), g1, dim3(256), 0, st, d_items, d_prefix1, n_items, total1);
        else hipLaunchKernelGGL((k_ntt16_list<false, true>), g1, dim3(256), 0, st, d_items, d_prefix1, n_items, total1);
    }
    if (total2 > 0) {
        dim3 g2(std::min(total2, cap));
        if (inverse) hipLaunchKernelGGL((k_ntt16_list<true, false>), g2, dim3(256), 0, st, d_items, d_prefix2, n_items, total2);
        else hipLaunchKernelGGL((k_ntt16_list<false, false>), g2, dim3(256), 0, st, d_items, d_prefix2, n_items, total2);
    }
}
