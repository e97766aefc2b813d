// Register-resident tridiagonal line solver for one workgroup (device code).
//
// One line of up to NT*C points lives in the registers of NT threads, C
// consecutive points per thread.  A solve is two first-order linear
// recurrences (forward elimination, back substitution with the precomputed
// LU factors of the constant matrix).  Each recurrence runs as
//   1. a local pass over the thread's C points with zero inflow,
//   2. a Kogge-Stone scan of the chunk carries inside the wavefront (the
//      multipliers are precomputed constants, so a level is one shuffle and
//      one FMA),
//   3. one LDS exchange of the W wave aggregates and a short Horner loop,
//   4. a second local pass from the true carry.
// So a solve costs two workgroup barriers.  For cyclic matrices the
// Sherman-Morrison correction needs x_0 and x_{M-1}; both are the totals of
// the scans, which every thread already has after step 3, so the correction
// costs no extra barrier.
#pragma once

#include "pit_internal.hpp"

namespace pit {

template <typename T>
__device__ __forceinline__ T shfl_up1(T v, int d)
{
    return __shfl_up(v, d, kWave);
}
template <typename T>
__device__ __forceinline__ T shfl_down1(T v, int d)
{
    return __shfl_down(v, d, kWave);
}

template <typename T, int NT, int C>
struct LineSolver {
    static constexpr int W = NT / kWave;
    static_assert(NT % kWave == 0 && W <= kMaxWaves, "bad line shape");

    T lm[C], iu[C], cm[C], z[C];
    T wf[kLevels], wb[kLevels];
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
        for (int l = 0; l < kLevels; ++l) {
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
        T v = e;
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            T o = shfl_up1(v, 1 << l);
            v = fma(wf[l], o, v);  // wf = 0 where the source lane is outside the wave
        }
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
            ytot = __shfl(v, kWave - 1, kWave);
        }
        T prev = shfl_up1(v, 1);
        if (lane == 0) prev = T(0);
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
        v = b;
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            T o = shfl_down1(v, 1 << l);
            v = fma(wb[l], o, v);
        }
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
            xtot = __shfl(v, 0, kWave);
        }
        T next = shfl_down1(v, 1);
        if (lane == kWave - 1) next = T(0);
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
