// Register-resident tridiagonal line solver for one workgroup (device code).
//
// One line of up to NT*C points lives in the registers of NT threads, C
// consecutive points per thread.  A solve is two first-order linear
// recurrences (forward elimination, back substitution with the precomputed
// LU factors of the constant matrix).  Each recurrence runs as
//   1. a local pass over the thread's C points with zero inflow,
//   2. a scan of the chunk carries inside the wavefront: four DPP row-shift
//      levels and three readlane row totals (the multipliers are precomputed
//      constants, so a level is one lane move and one FMA),
//   3. one LDS exchange of the W wave aggregates and a short Horner loop,
//   4. a second local pass from the true carry.
// So a solve costs two workgroup barriers.  For cyclic matrices the
// Sherman-Morrison correction needs x_0 and x_{M-1}; both are the totals of
// the scans, which every thread already has after step 3, so the correction
// costs no extra barrier.
#pragma once

#include "pit_internal.hpp"

namespace pit {

// ---- cross-lane helpers (DPP row shifts, whole-wave shifts, readlane) ----
// DPP controls: row_shr:s = 0x110+s, row_shl:s = 0x100+s, wave_shr:1 = 0x138,
// wave_shl:1 = 0x130.  With bound_ctrl set, a lane whose source is outside
// the row (or the wave) reads 0.
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Inclusive scan of the affine carries inside one wavefront, lanes in
// increasing order: four DPP levels inside each 16-lane row, then the three
// lower row totals (read with readlane) added with their precomputed
// multipliers.  m[0..3]: in-row level multipliers, m[4..6]: row-total
// multipliers (0 where not applicable).
template <typename T>
__device__ __forceinline__ T scan_up(T v, const T (&m)[7])
{
    v = fma(m[0], dpp<0x111>(v), v);
    v = fma(m[1], dpp<0x112>(v), v);
    v = fma(m[2], dpp<0x114>(v), v);
    v = fma(m[3], dpp<0x118>(v), v);
    const T t0 = readlane(v, 15), t1 = readlane(v, 31), t2 = readlane(v, 47);
    return fma(m[6], t2, fma(m[5], t1, fma(m[4], t0, v)));
}

// The same in decreasing lane order (row_shl, row totals at lanes 16/32/48).
template <typename T>
__device__ __forceinline__ T scan_down(T v, const T (&m)[7])
{
    v = fma(m[0], dpp<0x101>(v), v);
    v = fma(m[1], dpp<0x102>(v), v);
    v = fma(m[2], dpp<0x104>(v), v);
    v = fma(m[3], dpp<0x108>(v), v);
    const T t1 = readlane(v, 16), t2 = readlane(v, 32), t3 = readlane(v, 48);
    return fma(m[4], t1, fma(m[5], t2, fma(m[6], t3, v)));
}

template <typename T, int NT, int C>
struct LineSolver {
    static constexpr int W = NT / kWave;
    static_assert(NT % kWave == 0 && W <= kMaxWaves, "bad line shape");

    T lm[C], iu[C], cm[C], z[C];
    T wf[kScanConsts], wb[kScanConsts];
    T qf, qb;
    T inv_den, bg, iu_last;
    int cyclic;
    // LDS: [0,W) forward aggregates, [W,2W) backward aggregates,
    //      [2W,3W) pwf, [3W,4W) pwb
    T *sh;

    __device__ __forceinline__ void load(const LineTab<T> &tb, T *lds)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            lm[k] = tb.lm[k * NT + t];
            iu[k] = tb.iu[k * NT + t];
            cm[k] = tb.cm[k * NT + t];
            z[k] = tb.z[k * NT + t];
        }
#pragma unroll
        for (int l = 0; l < kScanConsts; ++l) {
            wf[l] = tb.wf[l * NT + t];
            wb[l] = tb.wb[l * NT + t];
        }
        qf = tb.qf[t];
        qb = tb.qb[t];
        inv_den = tb.inv_den;
        bg = tb.bg;
        iu_last = tb.iu_last;
        cyclic = tb.cyclic;
        sh = lds;
        if (t < W) {
            sh[2 * W + t] = tb.pwf[t];
            sh[3 * W + t] = tb.pwb[t];
        }
        __syncthreads();
    }

    // Solve A x = d; d is overwritten by x.
    __device__ __forceinline__ void solve(T (&d)[C])
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;

        // ---- forward elimination: y_j = d_j + lm_j y_{j-1} ----
        T e = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) e = fma(lm[k], e, d[k]);
        T v = scan_up(e, wf);
        T cw = T(0), ytot;
        if constexpr (W > 1) {
            if (lane == kWave - 1) sh[w] = v;
            __syncthreads();
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if (q == w) cw = acc;
                acc = fma(sh[2 * W + q], acc, sh[q]);
            }
            ytot = acc;
        } else {
            ytot = readlane(v, kWave - 1);
        }
        const T prev = dpp<0x138>(v);  // wave_shr:1, lane 0 reads 0
        T y = fma(qf, cw, prev);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            y = fma(lm[k], y, d[k]);
            d[k] = y;
        }

        // ---- back substitution: x_j = iu_j y_j + cm_j x_{j+1} ----
        T b = T(0);
#pragma unroll
        for (int k = C - 1; k >= 0; --k) b = fma(cm[k], b, iu[k] * d[k]);
        v = scan_down(b, wb);
        T cb = T(0), xtot;
        if constexpr (W > 1) {
            if (lane == 0) sh[W + w] = v;
            __syncthreads();
            T acc = T(0);
#pragma unroll
            for (int q = W - 1; q >= 0; --q) {
                if (q == w) cb = acc;
                acc = fma(sh[3 * W + q], acc, sh[W + q]);
            }
            xtot = acc;
        } else {
            xtot = readlane(v, 0);
        }
        const T next = dpp<0x130>(v);  // wave_shl:1, lane 63 reads 0
        T x = fma(qb, cb, next);
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            x = fma(cm[k], x, iu[k] * d[k]);
            d[k] = x;
        }

        // ---- Sherman-Morrison correction for the periodic case ----
        if (cyclic) {
            const T xlast = iu_last * ytot;  // cm_{M-1} = 0
            const T phi = (xtot + bg * xlast) * inv_den;
#pragma unroll
            for (int k = 0; k < C; ++k) d[k] = fma(-phi, z[k], d[k]);
        }
    }
};

}  // namespace pit
