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

#include "check.hpp"
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

// The tables of slice n (a time-dependent operator, constant on each slice);
// the shared table itself when there is one for every slice.  The branch is
// uniform (a kernel argument).
template <typename T>
__device__ __forceinline__ LineTab<T> line_tab_slice(const LineTab<T> &tb, int n)
{
    if (tb.sstride == 0) return tb;
    LineTab<T> t = tb;
    const long o = (long)n * tb.sstride;
    t.lm += o;
    t.iu += o;
    t.cm += o;
    t.z += o;
    t.wf += o;
    t.wb += o;
    t.qf += o;
    t.qb += o;
    t.pwf += o;
    t.pwb += o;
    t.rfw += o;
    t.rf += o;
    const T *sc = tb.sscal + (long)kSliceScalars * n;
    t.inv_den = sc[0];
    t.bg = sc[1];
    t.iu_last = sc[2];
    t.na = sc[3];
    t.nc = sc[4];
    return t;
}

// Hook points of a solve.  A caller that has global memory instructions to
// issue while a line is being solved (a sweep writing the previous slice and
// reading the next one) passes a callable, run at twelve fixed points of
// solve_to: 0 at the start, 1 halfway through the forward local pass, 2 after
// the in-wave forward scan, 3 after posting the wave aggregate (before the
// barrier), 4 after the cross-wave combination, 5 halfway through and 6 after
// the forward second pass, 7 halfway through the backward local pass, 8 after
// the in-wave backward scan, 9 after posting (before the barrier), 10 after
// the combination and 11 after the backward second pass (before the periodic
// correction).  Every point is reached exactly once per solve, whatever the
// shape.  Spread over those points, a wave's 1 KiB loads and stores drain
// through the compute unit's memory pipeline while the wave waits on its FMA
// chains and barriers; issued back to back (sixteen per wave at the end of a
// slice) they stall every wave until the pipeline has taken them all.  The
// scheduling fences keep the compiler from bunching them again.  NoHook
// compiles to nothing.
struct NoHook {
    static constexpr bool kActive = false;
    __device__ void operator()(int) const {}
};
template <class F>
struct Hook {
    static constexpr bool kActive = true;
    F f;
    __device__ __forceinline__ void operator()(int p) { f(p); }
};
template <class F>
__device__ __forceinline__ Hook<F> make_hook(F f)
{
    return Hook<F>{f};
}
template <class H>
__device__ __forceinline__ void at(H &h, int p)
{
    if constexpr (H::kActive) {
        __builtin_amdgcn_sched_barrier(0);
        h(p);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// CYC = false drops the periodic (Sherman-Morrison) part: no z vector in
// registers and no correction.  CP selects the compact tables (only iu per
// point; see pit_internal.hpp), which the longest FP64 lines need.  FP32
// tables take half the registers and keep the register form.
template <typename T, int NT, int C, bool CYC = true, bool CP = line_compact(NT, C) && sizeof(T) == 8>
struct LineSolver {
    static constexpr int W = NT / kWave;
    static_assert(NT % kWave == 0 && W <= kMaxWaves, "bad line shape");
    static_assert(!CP || W > 1, "the compact form hands y_{M-1} over in LDS");
    // z in LDS instead of registers (lines longer than kCompactAbove points)
    static constexpr bool kZLds = line_compact(NT, C) && CYC;
    // The wave aggregates are combined by a DPP scan over lanes 0..W-1 (lane q
    // holds wave q's aggregate) instead of a Horner loop over W LDS values in
    // every thread, whose unrolled selects and per-wave masks cost registers
    // (at 16 waves more than a 1024-thread workgroup has) and instructions.
    // FP32 (the increment-form step, with its per-wave late terms) from 4
    // waves on: 15% off the batched fine applies.  FP64 from 16 waves: at 4
    // and 8 waves its Horner loop was as fast or slightly faster.
    static constexpr bool kLaneComb = W > (sizeof(T) == 8 ? 8 : 2);
    static constexpr int kCombLevels = W > 8 ? 4 : W > 4 ? 3 : W > 2 ? 2 : 1;
    // LDS slots (units of T)
    static constexpr int kAggF = 0, kAggB = W, kPwf = 2 * W, kPwb = 3 * W, kRfw = 4 * W, kUFirst = 5 * W,
                         kULast = 6 * W, kUWrap = 7 * W, kYLast = 7 * W + 1, kMf = 7 * W + 2,
                         kMb = kMf + (kLaneComb ? 4 * 16 : 0), kZ = kMb + (kLaneComb ? 4 * 16 : 0);
    static constexpr int kLds = kZ + (kZLds ? NT * C : 0);

    T lm[C], iu[C], cm[C], z[C];
    T wf[kScanConsts], wb[kScanConsts];
    T qf, qb, rf, rfw0;
    T inv_den, bg, iu_last;
    T iup, na, nc;  // compact: iu of the point before the chunk, -a, -c
    int cyclic, M;
    T *sh;

    // Loads the thread's constants.  With one wavefront per line (W == 1) the
    // solver uses no LDS and no barrier, so several waves of a workgroup can
    // each own an independent line (lds may then be null).
    __device__ __forceinline__ void load(const LineTab<T> &tb, T *lds)
    {
        const int t = threadIdx.x & (NT - 1);
        cyclic = tb.cyclic;
        sh = lds;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            iu[k] = tb.iu[k * NT + t];
            if constexpr (!CP) {
                lm[k] = tb.lm[k * NT + t];
                cm[k] = tb.cm[k * NT + t];
            }
            if constexpr (CYC && !kZLds) z[k] = tb.z[k * NT + t];
            if constexpr (kZLds)
                if (cyclic) sh[kZ + k * NT + t] = tb.z[k * NT + t];
        }
        if constexpr (CP) {
            iup = (t > 0) ? tb.iu[(C - 1) * NT + t - 1] : T(0);
            na = tb.na;
            nc = tb.nc;
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
        M = tb.M;
        if constexpr (W > 1) {
            if (t < W) {
                sh[kPwf + t] = tb.pwf[t];
                sh[kPwb + t] = tb.pwb[t];
                sh[kRfw + t] = tb.rfw[t];
            }
            if constexpr (kLaneComb) {
                // level multipliers of the lane scans over the waves:
                //   up:   prod pwf over waves q-s+1..q   (0 if q < s)
                //   down: prod pwb over waves q..q+s-1   (0 if q+s > W-1)
                if (t < 16) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int s = 1 << i;
                        T f = T(0), b = T(0);
                        if (t < W && t >= s) {
                            f = T(1);
                            for (int q = t - s + 1; q <= t; ++q) f *= tb.pwf[q];
                        }
                        if (t + s <= W - 1) {
                            b = T(1);
                            for (int q = t; q < t + s; ++q) b *= tb.pwb[q];
                        }
                        sh[kMf + 16 * i + t] = f;
                        sh[kMb + 16 * i + t] = b;
                    }
                }
            }
            __syncthreads();
        }
    }

    // Inclusive scans over the wave aggregates held in lanes 0..W-1 (other
    // lanes carry 0 and are ignored): up combines waves 0..q into lane q, down
    // waves q..W-1.
    __device__ __forceinline__ T lane_scan_up(T g, int lane) const
    {
        const int q = lane & 15;
        T v = (lane < W) ? g : T(0);
        v = fma(sh[kMf + q], dpp<0x111>(v), v);
        if constexpr (kCombLevels > 1) v = fma(sh[kMf + 16 + q], dpp<0x112>(v), v);
        if constexpr (kCombLevels > 2) v = fma(sh[kMf + 32 + q], dpp<0x114>(v), v);
        if constexpr (kCombLevels > 3) v = fma(sh[kMf + 48 + q], dpp<0x118>(v), v);
        return v;
    }
    __device__ __forceinline__ T lane_scan_down(T g, int lane) const
    {
        const int q = lane & 15;
        T v = (lane < W) ? g : T(0);
        v = fma(sh[kMb + q], dpp<0x101>(v), v);
        if constexpr (kCombLevels > 1) v = fma(sh[kMb + 16 + q], dpp<0x102>(v), v);
        if constexpr (kCombLevels > 2) v = fma(sh[kMb + 32 + q], dpp<0x104>(v), v);
        if constexpr (kCombLevels > 3) v = fma(sh[kMb + 48 + q], dpp<0x108>(v), v);
        return v;
    }

    // ---- forward elimination y_j = d_j + lm_j y_{j-1}: local pass + in-wave scan ----
    template <class H = NoHook>
    __device__ __forceinline__ T fwd_scan(const T (&d)[C], H h = H{}) const
    {
        T e = d[0];
#pragma unroll
        for (int k = 1; k < C; ++k) {
            e = CP ? fma(na, iu[k - 1] * e, d[k]) : fma(lm[k], e, d[k]);
            if (k == C / 2) at(h, 1);
        }
        if constexpr (C < 2) at(h, 1);
        return scan_up(e, wf);
    }

    // second local pass from the carry c = y_{tC-1}; d is overwritten by y
    __device__ __forceinline__ void fwd_pass2(T (&d)[C], T c) const
    {
        T y = c;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if constexpr (CP) y = fma(na, (k == 0 ? iup : iu[k - 1]) * y, d[k]);
            else y = fma(lm[k], y, d[k]);
            d[k] = y;
        }
    }

    // the same out of place: out = y from in (in may be out)
    template <class H>
    __device__ __forceinline__ void fwd_pass2_to(const T (&in)[C], T (&out)[C], T c, H &h) const
    {
        T y = c;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if constexpr (CP) y = fma(na, (k == 0 ? iup : iu[k - 1]) * y, in[k]);
            else y = fma(lm[k], y, in[k]);
            out[k] = y;
            if (k == C / 2) at(h, 5);
        }
    }

    // one backward step x = iu_k y + cm_k x_next
    __device__ __forceinline__ T bstep(int k, T x, T y) const
    {
        if constexpr (CP) return iu[k] * fma(nc, x, y);
        else return fma(cm[k], x, iu[k] * y);
    }

    // ---- back substitution x_j = iu_j y_j + cm_j x_{j+1}, then the periodic
    // correction; ytot is the forward value at point M-1 ----
    template <class H = NoHook>
    __device__ __forceinline__ void backward(T (&d)[C], T ytot, H h = H{})
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        T b = iu[C - 1] * d[C - 1];
#pragma unroll
        for (int k = C - 2; k >= 0; --k) {
            b = bstep(k, b, d[k]);
            if (k == C / 2 - 1) at(h, 7);
        }
        if constexpr (C < 2) at(h, 7);
        T v = scan_down(b, wb);
        at(h, 8);
        T cb = T(0), xtot;
        if constexpr (W > 1) {
            if (lane == 0) sh[kAggB + w] = v;
            if constexpr (CP && CYC) {  // y_{M-1}: the forward total is not it here
                if (cyclic) {
                    const int j0 = t * C;
#pragma unroll
                    for (int k = 0; k < C; ++k)
                        if (j0 + k == M - 1) sh[kYLast] = d[k];
                }
            }
            at(h, 9);
            __syncthreads();
            if constexpr (CP && CYC) ytot = sh[kYLast];
            if constexpr (kLaneComb) {
                const T S = lane_scan_down(sh[kAggB + (lane & (W - 1))], lane);
                const int wu = __builtin_amdgcn_readfirstlane(w);
                const T nx = readlane(S, min(wu + 1, W - 1));
                cb = (wu < W - 1) ? nx : T(0);
                xtot = readlane(S, 0);
            } else {
                T acc = T(0);
#pragma unroll
                for (int q = W - 1; q >= 0; --q) {
                    if (q == w) cb = acc;
                    acc = fma(sh[kPwb + q], acc, sh[kAggB + q]);
                }
                xtot = acc;
            }
        } else {
            at(h, 9);
            xtot = readlane(v, 0);
        }
        at(h, 10);
        const T next = dpp<0x130>(v);  // wave_shl:1, lane 63 reads 0
        T x = fma(qb, cb, next);
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            x = bstep(k, x, d[k]);
            d[k] = x;
        }
        at(h, 11);
        if (CYC && cyclic) {  // Sherman-Morrison correction
            const T xlast = iu_last * ytot;  // x_{M-1} = iu_{M-1} y_{M-1}: nothing lies beyond it
            const T phi = (xtot + bg * xlast) * inv_den;
#pragma unroll
            for (int k = 0; k < C; ++k) d[k] = fma(-phi, kZLds ? sh[kZ + k * NT + t] : z[k], d[k]);
        }
    }

    // Solve A x = d; d is overwritten by x.
    __device__ __forceinline__ void solve(T (&d)[C]) { solve_to(d, d); }

    // Solve A out = in (in may be out; otherwise in is left as it was), with
    // the caller's hook run at the twelve points listed above NoHook.
    template <class H = NoHook>
    __device__ __forceinline__ void solve_to(const T (&in)[C], T (&out)[C], H h = H{})
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        at(h, 0);
        const T v = fwd_scan(in, h);
        at(h, 2);
        T cw = T(0), ytot;
        if constexpr (W > 1) {
            if (lane == kWave - 1) sh[kAggF + w] = v;
            at(h, 3);
            __syncthreads();
            if constexpr (kLaneComb) {
                const T S = lane_scan_up(sh[kAggF + (lane & (W - 1))], lane);
                const int wu = __builtin_amdgcn_readfirstlane(w);
                const T pv = readlane(S, max(wu - 1, 0));
                cw = (wu > 0) ? pv : T(0);
                ytot = readlane(S, W - 1);
            } else {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    if (q == w) cw = acc;
                    acc = fma(sh[kPwf + q], acc, sh[kAggF + q]);
                }
                ytot = acc;
            }
        } else {
            at(h, 3);
            ytot = readlane(v, kWave - 1);
        }
        at(h, 4);
        const T prev = dpp<0x138>(v);  // wave_shr:1, lane 0 reads 0
        fwd_pass2_to(in, out, fma(qf, cw, prev), h);
        at(h, 6);
        backward(out, ytot, h);
    }

    // One step in increment form:  u <- u + A^{-1} r,  with
    //   r_j = pd (u_{j-1} - 2 u_j + u_{j+1}) + pa (u_{j-1} - u_{j+1}) - pr u_j
    // (= dt L u: pd = dt nu/h^2, pa = dt a/(2h), pr = dt r).  The diffusion
    // part is written with differences, so a constant field gives exactly 0,
    // and the advection coefficient is rounded on its own: rounded as part of
    // dt (nu/h^2 +- a/(2h)), where the diffusion part is far larger, it would
    // lose most of its digits and the field would be advected at a visibly
    // wrong speed.  Neighbour values inside a wavefront come from DPP; a
    // neighbour across a wave edge or the periodic wrap (point 0 <-> point
    // M-1) is exchanged in the forward scan's LDS round and enters as a late
    // right-hand-side term, itself a difference with the point's own value:
    // its effect on the carries is linear (multipliers rf_t and rfw_w), so no
    // extra barrier is needed.  Pads (points M..) have a zero right-hand side.
    __device__ __forceinline__ void step_delta(T (&u)[C], T (&lo)[C], T pd, T pa, T pr, int M, int periodic)
    {
        const int t = threadIdx.x;
        const int lane = t & (kWave - 1);
        const int w = t / kWave;
        const int j0 = t * C;
        const T uprev = dpp<0x138>(u[C - 1]);  // lane-1's last point (lane 0 reads 0)
        const T unext = dpp<0x130>(u[0]);      // lane+1's first point (lane 63 reads 0)
        // A left or right neighbour outside the wave (or across the periodic
        // wrap) is a late term; one outside a Dirichlet line is the boundary
        // value 0, read in-wave (DPP and the zero pads supply it).
        const bool left_late = lane == 0 && (w > 0 || periodic);
        T d[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int j = j0 + k;
            const bool ll = k == 0 && left_late;
            const bool rl = (periodic && j == M - 1) || (k == C - 1 && lane == kWave - 1 && j < M - 1);
            const T left = ll ? u[k] : ((k == 0) ? uprev : u[k - 1]);
            const T right = rl ? u[k] : ((k == C - 1) ? unext : u[k + 1]);
            const T al = ll ? T(0) : left, ar = rl ? T(0) : right;
            const T v = fma(pd, (left - u[k]) + (right - u[k]), fma(pa, al - ar, -pr * u[k]));
            d[k] = (j < M) ? v : T(0);
        }
        // point M-1: its thread, its index in that thread's chunk, its wave
        // (all uniform, so u_{M-1} is read with one readlane of one register)
        const int owner_last = (M - 1) / C;
        const int kk = (M - 1) - owner_last * C;
        const int wstar = owner_last / kWave;
        const int wu = __builtin_amdgcn_readfirstlane(w);
        const T v = fwd_scan(d);
        T cw = T(0), ytot, dL = T(0), dR = T(0), dM = T(0);
        if constexpr (W > 1) {
            if (lane == kWave - 1) {
                sh[kAggF + w] = v;
                sh[kULast + w] = u[C - 1];
            }
            if (lane == 0) sh[kUFirst + w] = u[0];
            if (wu == wstar) {
                T val = T(0);
#pragma unroll
                for (int k = 0; k < C; ++k)
                    if (k == kk) val = readlane(u[k], owner_last & (kWave - 1));
                if (lane == 0) sh[kUWrap] = val;
            }
            __syncthreads();
            const T u0 = sh[kUFirst];
            const T uM = sh[kUWrap];
            if (periodic) dM = fma(pd, u0 - uM, -pa * u0);
            // wave q's late terms: l at its first point Pq, r at its last Qq
            auto late = [&](int q, T &l, T &r) {
                const int Pq = q * kWave * C, Qq = Pq + kWave * C - 1;
                l = T(0);
                r = T(0);
                if (Pq < M && (q > 0 || periodic)) {
                    const T ul = (q > 0) ? sh[kULast + q - 1] : uM;
                    l = fma(pd, ul - sh[kUFirst + q], pa * ul);
                }
                if (Qq < M - 1) {
                    const T ur = sh[kUFirst + q + 1];
                    r = fma(pd, ur - sh[kULast + q], -pa * ur);
                }
            };
            if constexpr (kLaneComb) {  // lane q assembles wave q's terms
                const int q = lane & (W - 1);
                T l, r;
                late(q, l, r);
                T agg = sh[kAggF + q] + fma(sh[kRfw + q], l, r);
                if (q == wstar) agg += dM;
                const T S = lane_scan_up(agg, lane);
                const T pv = readlane(S, max(wu - 1, 0));
                cw = (wu > 0) ? pv : T(0);
                dL = readlane(l, wu);
                dR = readlane(r, wu);
                ytot = readlane(S, W - 1);
            } else {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    T l, r;
                    late(q, l, r);
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
            }
        } else {
            const T u0 = readlane(u[0], 0);
            T uM = T(0);
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (k == kk) uM = readlane(u[k], owner_last);
            if (periodic) {
                dM = fma(pd, u0 - uM, -pa * u0);
                dL = fma(pd, uM - u0, pa * uM);
            }
            ytot = readlane(v, kWave - 1) + fma(rfw0, dL, dM);
        }
        const T prev = dpp<0x138>(v);
        const T c = (lane == 0) ? cw : fma(rf, dL, fma(qf, cw, prev));
        // complete the right-hand side with the late terms
        if (lane == 0 && j0 < M) d[0] += dL;
        if (lane == kWave - 1 && j0 + C - 1 < M - 1) d[C - 1] += dR;
        if (t == owner_last) d[__builtin_amdgcn_readfirstlane(kk)] += dM;
        fwd_pass2(d, c);
        backward(d, ytot);
        // u + lo += d, compensated: the state is the unevaluated sum u + lo
        // and the rounding error of every update is carried in lo, so many
        // small increments do not drift by the state's rounding.  The error
        // term is Fast2Sum's, exact whenever |increment| <= |u| (the regime
        // where drift builds up); otherwise it is an ordinary rounding.
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const T y = d[k] + lo[k];
            const T s = u[k] + y;
            lo[k] = y - (s - u[k]);
            u[k] = s;
        }
    }
};

}  // namespace pit
