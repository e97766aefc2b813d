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

// CYC = false drops the periodic (Sherman-Morrison) part: no z vector in
// registers and no correction.
template <typename T, int NT, int C, bool CYC = true>
struct LineSolver {
    static constexpr int W = NT / kWave;
    static_assert(NT % kWave == 0 && W <= kMaxWaves, "bad line shape");
    // LDS slots (units of T)
    static constexpr int kAggF = 0, kAggB = W, kPwf = 2 * W, kPwb = 3 * W, kRfw = 4 * W, kUFirst = 5 * W,
                         kULast = 6 * W, kUWrap = 7 * W;
    static constexpr int kLds = 7 * W + 2;

    T lm[C], iu[C], cm[C], z[C];
    T wf[kScanConsts], wb[kScanConsts];
    T qf, qb, rf, rfw0;
    T inv_den, bg, iu_last;
    int cyclic;
    T *sh;

    // Loads the thread's constants.  With one wavefront per line (W == 1) the
    // solver uses no LDS and no barrier, so several waves of a workgroup can
    // each own an independent line (lds may then be null).
    __device__ __forceinline__ void load(const LineTab<T> &tb, T *lds)
    {
        const int t = threadIdx.x & (NT - 1);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            lm[k] = tb.lm[k * NT + t];
            iu[k] = tb.iu[k * NT + t];
            cm[k] = tb.cm[k * NT + t];
            if constexpr (CYC) z[k] = tb.z[k * NT + t];
        }
#pragma unroll
        for (int l = 0; l < kScanConsts; ++l) {
            wf[l] = tb.wf[l * NT + t];
            wb[l] = tb.wb[l * NT + t];
        }
        qf = tb.qf[t];
        qb = tb.qb[t];
        rf = tb.rf[t];
        rfw0 = tb.rfw[0];
        inv_den = tb.inv_den;
        bg = tb.bg;
        iu_last = tb.iu_last;
        cyclic = tb.cyclic;
        sh = lds;
        if constexpr (W > 1) {
            if (t < W) {
                sh[kPwf + t] = tb.pwf[t];
                sh[kPwb + t] = tb.pwb[t];
                sh[kRfw + t] = tb.rfw[t];
            }
            __syncthreads();
        }
    }

    // ---- forward elimination y_j = d_j + lm_j y_{j-1}: local pass + in-wave scan ----
    __device__ __forceinline__ T fwd_scan(const T (&d)[C]) const
    {
        T e = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) e = fma(lm[k], e, d[k]);
        return scan_up(e, wf);
    }

    // second local pass from the carry c = y_{tC-1}; d is overwritten by y
    __device__ __forceinline__ void fwd_pass2(T (&d)[C], T c) const
    {
        T y = c;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            y = fma(lm[k], y, d[k]);
            d[k] = y;
        }
    }

    // ---- back substitution x_j = iu_j y_j + cm_j x_{j+1}, then the periodic
    // correction; ytot is the forward value at point M-1 ----
    __device__ __forceinline__ void backward(T (&d)[C], T ytot)
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        T b = T(0);
#pragma unroll
        for (int k = C - 1; k >= 0; --k) b = fma(cm[k], b, iu[k] * d[k]);
        T v = scan_down(b, wb);
        T cb = T(0), xtot;
        if constexpr (W > 1) {
            if (lane == 0) sh[kAggB + w] = v;
            __syncthreads();
            T acc = T(0);
#pragma unroll
            for (int q = W - 1; q >= 0; --q) {
                if (q == w) cb = acc;
                acc = fma(sh[kPwb + q], acc, sh[kAggB + q]);
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
        if (CYC && cyclic) {  // Sherman-Morrison correction
            const T xlast = iu_last * ytot;  // cm_{M-1} = 0
            const T phi = (xtot + bg * xlast) * inv_den;
#pragma unroll
            for (int k = 0; k < C; ++k) d[k] = fma(-phi, z[k], d[k]);
        }
    }

    // Solve A x = d; d is overwritten by x.
    __device__ __forceinline__ void solve(T (&d)[C])
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        const T v = fwd_scan(d);
        T cw = T(0), ytot;
        if constexpr (W > 1) {
            if (lane == kWave - 1) sh[kAggF + w] = v;
            __syncthreads();
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if (q == w) cw = acc;
                acc = fma(sh[kPwf + q], acc, sh[kAggF + q]);
            }
            ytot = acc;
        } else {
            ytot = readlane(v, kWave - 1);
        }
        const T prev = dpp<0x138>(v);  // wave_shr:1, lane 0 reads 0
        fwd_pass2(d, fma(qf, cw, prev));
        backward(d, ytot);
    }

    // One step in increment form:  u <- u + A^{-1} r,  with
    //   r_j = pl (u_{j-1} - u_j) + pu (u_{j+1} - u_j) - pr u_j    (= dt L u, written
    // with differences so that a constant field gives exactly 0).  Neighbour
    // values inside a wavefront come from DPP; the two neighbours across wave
    // edges and the periodic wrap (point 0 <-> point M-1) are exchanged in the
    // forward scan's LDS round and enter as late right-hand-side terms: their
    // effect on the carries is linear (multipliers rf_t and rfw_w), so no extra
    // barrier is needed and every copy of a neighbour value is exact.
    __device__ __forceinline__ void step_delta(T (&u)[C], T (&lo)[C], T pl, T pu, T pr, int M, int periodic)
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        const int j0 = t * C;
        const T uprev = dpp<0x138>(u[C - 1]);  // lane-1's last point (lane 0 reads 0)
        const T unext = dpp<0x130>(u[0]);      // lane+1's first point (lane 63 reads 0)
        T d[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const T left = (k == 0) ? uprev : u[k - 1];
            const T right = (k == C - 1) ? unext : u[k + 1];
            const T r = fma(pl, left - u[k], fma(pu, right - u[k], -pr * u[k]));
            d[k] = (j0 + k < M) ? r : T(0);
        }
        // value of point M-1 (owner only)
        T uwrap = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k)
            if (j0 + k == M - 1) uwrap = u[k];
        const int owner_last = (M - 1) / C;   // thread holding point M-1
        const int wstar = owner_last / kWave; // its wave
        const T v = fwd_scan(d);
        T cw = T(0), ytot, dL = T(0), dR = T(0), dM = T(0);
        if constexpr (W > 1) {
            if (lane == kWave - 1) {
                sh[kAggF + w] = v;
                sh[kULast + w] = u[C - 1];
            }
            if (lane == 0) sh[kUFirst + w] = u[0];
            if (t == owner_last) sh[kUWrap] = uwrap;
            __syncthreads();
            const T u0 = sh[kUFirst];
            const T uM = sh[kUWrap];
            if (periodic) dM = pu * u0;
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int Pq = q * kWave * C, Qq = Pq + kWave * C - 1;
                T l = T(0), r = T(0);
                if (Pq < M) l = pl * ((q > 0) ? sh[kULast + q - 1] : (periodic ? uM : T(0)));
                if (Qq < M - 1) r = pu * sh[kUFirst + q + 1];
                if (q == w) {
                    cw = acc;
                    dL = l;
                    dR = r;
                }
                T agg = sh[kAggF + q] + fma(sh[kRfw + q], l, r);
                if (q == wstar) agg += dM;
                acc = fma(sh[kPwf + q], acc, agg);
            }
            ytot = acc;
        } else {
            const T u0 = readlane(u[0], 0);
            const T uM = readlane(uwrap, owner_last);
            if (periodic) {
                dM = pu * u0;
                dL = pl * uM;
            }
            ytot = readlane(v, kWave - 1) + fma(rfw0, dL, dM);
        }
        const T prev = dpp<0x138>(v);
        const T c = (lane == 0) ? cw : fma(rf, dL, fma(qf, cw, prev));
        // complete the right-hand side with the late terms
        if (lane == 0 && j0 < M) d[0] += dL;
        if (lane == kWave - 1 && j0 + C - 1 < M - 1) d[C - 1] += dR;
#pragma unroll
        for (int k = 0; k < C; ++k)
            if (j0 + k == M - 1) d[k] += dM;
        fwd_pass2(d, c);
        backward(d, ytot);
        // u + lo += d, compensated: the state is the unevaluated sum u + lo
        // and the rounding error of every update is carried in lo (TwoSum),
        // so many small increments do not drift by the state's rounding.
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const T y = d[k] + lo[k];
            const T s = u[k] + y;
            const T bb = s - u[k];
            lo[k] = (u[k] - (s - bb)) + (y - bb);
            u[k] = s;
        }
    }
};

}  // namespace pit
