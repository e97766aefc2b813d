// 2D PR-ADI half-steps with per-line operators (velocity field), FP64.
//
// One thread per line (row for the x half-step, column for the y half-step,
// grid.y = slice) runs the Thomas recurrences of its line with the
// precomputed pivots.  Column threads of a wavefront touch consecutive
// addresses at every point of their walk; row threads touch one point of 64
// rows per step and reuse each fetched 128-byte line over the next 15 steps
// from L1.  The walks are unrolled so that the loads of several points
// (which depend on the index only) are in flight at once; on small grids the
// launches are bound by that latency.
#include "vel2d.hpp"

namespace pit {

constexpr int kVelThreads = 64;

// EXPL: explicit part on (the half-step) or off (a plain solve).  Neighbour
// loads are unconditional from a clamped (in-line) index and then masked, so
// the walk has no branches and the loads of an unrolled stretch overlap.
template <bool EXPL>
__global__ __launch_bounds__(kVelThreads) void k_vel_x(VelTab t, const double *__restrict__ in, long in_off,
                                                        double *__restrict__ out, long out_off, int Mx, int My)
{
    const int j = blockIdx.x * kVelThreads + threadIdx.x;
    if (j >= My) return;
    const long np = (long)Mx * My;
    const double *u = in + (in_off + blockIdx.y) * np;
    double *o = out + (out_off + blockIdx.y) * np;
    const long row = (long)j * Mx;
    // the tables are read-only and never overlap the fields
    const double *__restrict__ xw = t.xw;
    const double *__restrict__ xc = t.xc;
    const double *__restrict__ ylo = t.ylo;
    const double *__restrict__ yup = t.yup;
    const double a = t.xa[j], ydi = t.ydi;
    const bool has_m = j > 0, has_q = j < My - 1;
    const long om = has_m ? Mx : 0, oq = has_q ? Mx : 0;
    double d = 0.0;
#pragma unroll 8
    for (int i = 0; i < Mx; ++i) {
        const long q = row + i;
        double r = u[q];
        if constexpr (EXPL) {
            const double um = u[q - om], uq = u[q + oq];
            const double cm = has_m ? um : 0.0, cq = has_q ? uq : 0.0;
            r = r + ylo[i] * cm + ydi * r + yup[i] * cq;
        }
        d = (r - a * d) * xw[q];
        o[q] = d;
    }
    double x = d;
#pragma unroll 8
    for (int i = Mx - 2; i >= 0; --i) {
        const long q = row + i;
        x = o[q] - xc[q] * x;
        o[q] = x;
    }
}

template <bool EXPL>
__global__ __launch_bounds__(kVelThreads) void k_vel_y(VelTab t, const double *__restrict__ in, long in_off,
                                                        double *out, long out_off, const double *base,
                                                        long base_off, double sign, double *__restrict__ wk,
                                                        int Mx, int My)
{
    const int i = blockIdx.x * kVelThreads + threadIdx.x;
    if (i >= Mx) return;
    const long np = (long)Mx * My;
    const double *u = in + (in_off + blockIdx.y) * np;
    double *o = out + (out_off + blockIdx.y) * np;
    double *w = wk + (long)blockIdx.y * np;
    const double *b = base ? base + (base_off + blockIdx.y) * np : nullptr;
    const double *__restrict__ yw = t.yw;
    const double *__restrict__ yc = t.yc;
    const double *__restrict__ xlo = t.xlo;
    const double *__restrict__ xup = t.xup;
    const double a = t.ya[i], xdi = t.xdi;
    const bool has_m = i > 0, has_q = i < Mx - 1;
    const long om = has_m ? 1 : 0, oq = has_q ? 1 : 0;
    double d = 0.0;
#pragma unroll 8
    for (int j = 0; j < My; ++j) {
        const long q = (long)j * Mx + i;
        double r = u[q];
        if constexpr (EXPL) {
            const double um = u[q - om], uq = u[q + oq];
            const double cm = has_m ? um : 0.0, cq = has_q ? uq : 0.0;
            r = r + xlo[j] * cm + xdi * r + xup[j] * cq;
        }
        d = (r - a * d) * yw[q];
        w[q] = d;
    }
    double x = d;
    {
        const long q = (long)(My - 1) * Mx + i;
        o[q] = b ? b[q] + sign * x : x;
    }
#pragma unroll 8
    for (int j = My - 2; j >= 0; --j) {
        const long q = (long)j * Mx + i;
        x = w[q] - yc[q] * x;
        o[q] = b ? b[q] + sign * x : x;
    }
}

// ---------------------------------------------------------------------------
// Slices that fit in LDS: one workgroup keeps a whole slice on chip for all
// its steps.  LDS holds the fields U, S and W and, when they fit as well,
// the four point tables and the six line vectors (copied in once per launch).
// Each field has a ring of zero ghost points (point (i, j) at (j+1) P + i+1,
// odd pitch P >= Mx + 2, so that row threads at stride P hit distinct banks):
// the explicit part then reads its neighbours without masks.  A step is the
// x half-step (row threads: U -> S, the forward values in W), a barrier, the
// y half-step (column threads: S -> U) and a barrier.  No walk reads a field
// it writes, so the loads of an unrolled stretch issue ahead of the
// recurrence; one wavefront does all the walks of a slice of up to 64 lines
// per axis, so the step is bound by its instruction count per point.
// ---------------------------------------------------------------------------

// At most this many lines per axis (one thread per line, one workgroup).
constexpr int kVelLdsLines = 512;

// Where the walks read their tables (point tables with row pitch tp).
struct VelView {
    const double *xw, *xc, *yw, *yc;
    const double *xa, *xlo, *xup, *ya, *ylo, *yup;
    int tp;
};

__host__ __device__ inline int vel_pitch(int Mx) { return (Mx + 2) | 1; }
__host__ __device__ inline long vel_field(int Mx, int My) { return (long)(My + 2) * vel_pitch(Mx); }
// LDS index of interior point q = j Mx + i (slices of at most 512 x 512
// points: 32-bit arithmetic).
__device__ __forceinline__ int vel_at(int q, int Mx, int P)
{
    const int j = q / Mx;
    return (j + 1) * P + (q - j * Mx) + 1;
}

// One line: n points at field stride fs and table stride ts.  The explicit
// part at point e is c + lo[e] cm + di c + up[e] cq (cm, cq the neighbours
// across the line, ghosts outside), then the Thomas passes with pivots w,
// cc; the forward values go to fw, the solution to o.
__device__ __forceinline__ void vel_walk(const double *__restrict__ cp, const double *__restrict__ mp,
                                         const double *__restrict__ qp, double *__restrict__ fw,
                                         double *__restrict__ o, const double *__restrict__ w,
                                         const double *__restrict__ cc, const double *__restrict__ lo,
                                         const double *__restrict__ up, double a, double di, int n, int fs, int ts)
{
    double d = 0.0;
#pragma unroll 8
    for (int e = 0; e < n; ++e) {
        const double c0 = cp[e * fs];
        const double r = c0 + lo[e] * mp[e * fs] + di * c0 + up[e] * qp[e * fs];
        d = (r - a * d) * w[e * ts];
        fw[e * fs] = d;
    }
    double x = d;
    o[(n - 1) * fs] = x;
#pragma unroll 8
    for (int e = n - 2; e >= 0; --e) {
        x = fw[e * fs] - cc[e * ts] * x;
        o[e * fs] = x;
    }
}

__device__ __forceinline__ void vel_step_lds(const VelView &v, double xdi, double ydi, double *U, double *S,
                                             double *W, int Mx, int My, int P)
{
    // The line index and the pitch pass through an empty asm once per step:
    // otherwise the compiler hoists every address of both walks out of the
    // loop over steps and keeps them all live (register spills).
    int k = threadIdx.x;
    asm volatile("" : "+v"(k));
    asm volatile("" : "+s"(P));
    if (k < My) {  // row k: S = X^{-1} (I + th Ly) U
        const int j = k;
        const long r0 = (long)(j + 1) * P + 1;
        vel_walk(U + r0, U + r0 - P, U + r0 + P, W + r0, S + r0, v.xw + j * v.tp, v.xc + j * v.tp, v.ylo, v.yup,
                 v.xa[j], ydi, Mx, 1, 1);
    }
    __syncthreads();
    if (k < Mx) {  // column k: U = Y^{-1} (I + th Lx) S
        const int i = k;
        const long c0 = P + i + 1;
        vel_walk(S + c0, S + c0 - 1, S + c0 + 1, W + c0, U + c0, v.yw + i, v.yc + i, v.xlo, v.xup, v.ya[i], xdi, My,
                 P, v.tp);
    }
    __syncthreads();
}

// TAB: copy the tables into LDS behind the three fields (the caller's
// barrier publishes them); else read them in place.
template <bool TAB>
__device__ __forceinline__ VelView vel_stage(const VelTab &t, double *sh, int Mx, int My, int P)
{
    if constexpr (!TAB) {
        return VelView{t.xw, t.xc, t.yw, t.yc, t.xa, t.xlo, t.xup, t.ya, t.ylo, t.yup, Mx};
    } else {
        const int tpl = My * P, np = Mx * My;
        double *T = sh + 3 * vel_field(Mx, My);
        for (int q = threadIdx.x; q < np; q += blockDim.x) {
            const int jq = q / Mx, l = jq * P + (q - jq * Mx);
            T[l] = t.xw[q];
            T[tpl + l] = t.xc[q];
            T[2 * tpl + l] = t.yw[q];
            T[3 * tpl + l] = t.yc[q];
        }
        double *L = T + 4 * tpl, *C = L + 3 * My;
        for (int q = threadIdx.x; q < My; q += blockDim.x) {
            L[q] = t.xa[q];
            L[My + q] = t.xlo[q];
            L[2 * My + q] = t.xup[q];
        }
        for (int q = threadIdx.x; q < Mx; q += blockDim.x) {
            C[q] = t.ya[q];
            C[Mx + q] = t.ylo[q];
            C[2 * Mx + q] = t.yup[q];
        }
        return VelView{T, T + tpl, T + 2 * tpl, T + 3 * tpl, L, L + My, L + 2 * My, C, C + Mx, C + 2 * Mx, P};
    }
}

// U = slice u (interior), ghosts of U and S zero.
__device__ __forceinline__ void vel_load_field(double *U, double *S, const double *u, int Mx, int My, int P)
{
    const int fp = (int)vel_field(Mx, My);
    for (int l = threadIdx.x; l < fp; l += blockDim.x) {
        const int jj = l / P - 1, ii = l - (jj + 1) * P - 1;
        const bool in = jj >= 0 && jj < My && ii >= 0 && ii < Mx;
        U[l] = in ? u[(long)jj * Mx + ii] : 0.0;
        S[l] = 0.0;
    }
}

// All-at-once apply on `ns` slices: out_{s+out_off} = base_{s+out_off} + sign F(in_{s+in_off})
// (base NULL: F(in)), F = m steps, one workgroup per slice.
template <bool TAB>
__global__ __launch_bounds__(kVelLdsLines) void k_vel_apply_lds(VelTab t, const double *__restrict__ in, long in_off,
                                                                 double *out, long out_off, const double *base,
                                                                 long base_off, double sign, int m, int Mx, int My)
{
    extern __shared__ double sh[];
    const int P = vel_pitch(Mx);
    const long fp = vel_field(Mx, My);
    double *U = sh, *S = sh + fp, *W = sh + 2 * fp;
    const VelView v = vel_stage<TAB>(t, sh, Mx, My, P);
    const int np = Mx * My;
    vel_load_field(U, S, in + (in_off + blockIdx.x) * np, Mx, My, P);
    __syncthreads();
    for (int s = 0; s < m; ++s) vel_step_lds(v, t.xdi, t.ydi, U, S, W, Mx, My, P);
    double *o = out + (out_off + blockIdx.x) * np;
    const double *b = base ? base + (base_off + blockIdx.x) * np : nullptr;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const double x = U[vel_at(q, Mx, P)];
        o[q] = b ? b[q] + sign * x : x;
    }
}

// Values of v_n each thread loads ahead of the walks of slice n.
constexpr int kVelPre = 16;

// Coarse sweep z_0 = v_0, z_n = v_n + G(z_{n-1}) (G = c steps) by one
// workgroup marching the slices; v == z is allowed.  Each slice first issues
// the loads of v_n and the stores of z_{n-1} (from LDS), then walks: both
// transfers overlap the walks.
template <bool TAB>
__global__ __launch_bounds__(kVelLdsLines) void k_vel_sweep_lds(VelTab t, const double *v, double *z, int N, int c,
                                                                 int Mx, int My)
{
    extern __shared__ double sh[];
    const int P = vel_pitch(Mx);
    const long fp = vel_field(Mx, My);
    double *U = sh, *S = sh + fp, *W = sh + 2 * fp;
    const VelView w = vel_stage<TAB>(t, sh, Mx, My, P);
    const int np = Mx * My, bd = blockDim.x, tid = threadIdx.x;
    vel_load_field(U, S, v, Mx, My, P);
    if (z != v)
        for (int q = tid; q < np; q += bd) z[q] = v[q];
    // this thread's first kVelPre points and their LDS indices
    int at[kVelPre];
#pragma unroll
    for (int k = 0; k < kVelPre; ++k) {
        const int q = tid + k * bd;
        at[k] = q < np ? vel_at(q, Mx, P) : 0;
    }
    // z_s = U (this thread's points)
    auto store = [&](double *zs) {
#pragma unroll
        for (int k = 0; k < kVelPre; ++k) {
            const int q = tid + k * bd;
            if (q < np) zs[q] = U[at[k]];
        }
        for (int q = tid + kVelPre * bd; q < np; q += bd) zs[q] = U[vel_at(q, Mx, P)];
    };
    __syncthreads();
    for (int n = 1; n < N; ++n) {
        const double *vn = v + (long)n * np;
        // branch-free: points past the slice reload its last point
        double pre[kVelPre];
#pragma unroll
        for (int k = 0; k < kVelPre; ++k) pre[k] = vn[min(tid + k * bd, np - 1)];
        if (n > 1) store(z + (long)(n - 1) * np);
        for (int s = 0; s < c; ++s) vel_step_lds(w, t.xdi, t.ydi, U, S, W, Mx, My, P);
#pragma unroll
        for (int k = 0; k < kVelPre; ++k)
            if (tid + k * bd < np) U[at[k]] += pre[k];
        for (int q = tid + kVelPre * bd; q < np; q += bd) U[vel_at(q, Mx, P)] += vn[q];
        __syncthreads();
    }
    if (N > 1) store(z + (long)(N - 1) * np);
}

size_t vel_lds_bytes(int Mx, int My, bool tab)
{
    const size_t fp = (size_t)vel_field(Mx, My), tpl = (size_t)My * vel_pitch(Mx);
    return sizeof(double) * (3 * fp + (tab ? 4 * tpl + 3 * ((size_t)Mx + My) : 0));
}

// Lines per axis fit one workgroup; at least four wavefronts for the copies.
static int vel_lds_threads(int Mx, int My)
{
    const int lines = Mx > My ? Mx : My;
    const int t = ((lines + 63) / 64) * 64;
    return t < 256 ? 256 : t;
}

int vel_lds_mode(int Mx, int My)
{
    if (Mx < 1 || My < 1 || (Mx > My ? Mx : My) > kVelLdsLines) return 0;
    if (vel_lds_bytes(Mx, My, true) <= kVelLdsMax) return 2;
    return vel_lds_bytes(Mx, My, false) <= kVelLdsMax ? 1 : 0;
}

// Raise the dynamic LDS limit of a kernel once.
template <bool TAB>
static hipError_t apply_lds_attr()
{
    static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vel_apply_lds<TAB>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kVelLdsMax);
    return e;
}
template <bool TAB>
static hipError_t sweep_lds_attr()
{
    static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vel_sweep_lds<TAB>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kVelLdsMax);
    return e;
}

hipError_t launch_vel_apply_lds(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                                const double *base, long base_off, double sign, int ns, int m, int Mx, int My,
                                hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const int mode = vel_lds_mode(Mx, My);
    if (mode == 0) return hipErrorInvalidValue;
    const bool tab = mode == 2;
    const hipError_t e = tab ? apply_lds_attr<true>() : apply_lds_attr<false>();
    if (e != hipSuccess) return e;
    const dim3 grid(ns), block(vel_lds_threads(Mx, My));
    const size_t lds = vel_lds_bytes(Mx, My, tab);
    if (tab)
        hipLaunchKernelGGL(k_vel_apply_lds<true>, grid, block, lds, st, t, in, in_off, out, out_off, base, base_off,
                           sign, m, Mx, My);
    else
        hipLaunchKernelGGL(k_vel_apply_lds<false>, grid, block, lds, st, t, in, in_off, out, out_off, base, base_off,
                           sign, m, Mx, My);
    return hipGetLastError();
}

hipError_t launch_vel_sweep_lds(const VelTab &t, const double *v, double *z, int N, int c, int Mx, int My,
                                hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    const int mode = vel_lds_mode(Mx, My);
    if (mode == 0) return hipErrorInvalidValue;
    const bool tab = mode == 2;
    const hipError_t e = tab ? sweep_lds_attr<true>() : sweep_lds_attr<false>();
    if (e != hipSuccess) return e;
    const dim3 block(vel_lds_threads(Mx, My));
    const size_t lds = vel_lds_bytes(Mx, My, tab);
    if (tab) hipLaunchKernelGGL(k_vel_sweep_lds<true>, dim3(1), block, lds, st, t, v, z, N, c, Mx, My);
    else hipLaunchKernelGGL(k_vel_sweep_lds<false>, dim3(1), block, lds, st, t, v, z, N, c, Mx, My);
    return hipGetLastError();
}

hipError_t launch_vel_x(const VelTab &t, const double *in, long in_off, double *out, long out_off, int ns,
                        int Mx, int My, int expl, hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const dim3 grid((My + kVelThreads - 1) / kVelThreads, ns);
    if (expl) hipLaunchKernelGGL(k_vel_x<true>, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, Mx, My);
    else hipLaunchKernelGGL(k_vel_x<false>, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, Mx, My);
    return hipGetLastError();
}

hipError_t launch_vel_y(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                        const double *base, long base_off, double sign, double *wk, int ns, int Mx, int My,
                        int expl, hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const dim3 grid((Mx + kVelThreads - 1) / kVelThreads, ns);
    if (expl)
        hipLaunchKernelGGL(k_vel_y<true>, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, base, base_off,
                           sign, wk, Mx, My);
    else
        hipLaunchKernelGGL(k_vel_y<false>, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, base,
                           base_off, sign, wk, Mx, My);
    return hipGetLastError();
}

}  // namespace pit
