// 2D PR-ADI with per-line operators (velocity field), FP64.
//
// One thread per line (row for the x half-step, column for the y half-step)
// runs the Thomas recurrences of its line with the precomputed pivots.  Two
// forms: slices that fit in LDS run whole on chip for all their steps (the
// kernels at the end of this file); larger slices take one launch per
// half-step over all slices (grid.y = slice) with the fields in HBM, where
// column threads of a wavefront touch consecutive addresses at every point
// of their walk and row threads touch one point of 64 rows per step and
// reuse each fetched 128-byte line over the next 15 steps from L1.  The walks
// are unrolled so that the loads of several points (which depend on the
// index only) are in flight at once.
#include "check.hpp"
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
// its steps.  LDS holds three fields and, when they fit as well, the four
// point tables and the six line vectors (copied in once per launch):
//   U   the slice, row-major: point (i, j) at (j+1) P + i+1;
//   S   the x half-step's result, transposed: point (i, j) at (i+1) Q + j+1;
//   W   the forward values of the walk in progress (either layout);
// with a ring of zero ghost points around U and S, so the explicit parts read
// their neighbours without masks, and odd pitches P >= Mx + 2, Q >= My + 2,
// so that threads at stride P or Q hit distinct banks.  Row thread j reads
// rows j-1, j, j+1 of U and column thread i rows i-1, i, i+1 of S: every
// load of a walk is contiguous along the walk (immediate offsets, paired
// loads) and only the solution is stored across the other layout.  The y
// tables are staged transposed for the same reason.  A step is the x
// half-step (row threads: U -> S), a barrier, the y half-step (column
// threads: S -> U) and a barrier.  One wavefront does all the walks of a
// slice of up to 64 lines per axis, so a step is bound by its instruction
// count per point.
// ---------------------------------------------------------------------------

// At most this many lines per axis (one thread per line, one workgroup).
constexpr int kVelLdsLines = 512;

// LDS layout of one slice, in doubles.
struct VelLds {
    int P, Q;      // row pitch of U (and the x tables), of S (and the y tables)
    int s, w, t;   // offsets of S, W, the tables (U at 0)
    int total;     // doubles without tables (fields only) or with them
};
__host__ __device__ inline VelLds vel_lds_layout(int Mx, int My, bool tab)
{
    VelLds l;
    l.P = (Mx + 2) | 1;
    l.Q = (My + 2) | 1;
    const int fu = (My + 2) * l.P, fs = (Mx + 2) * l.Q;
    l.s = fu;
    l.w = fu + fs;
    l.t = l.w + (fu > fs ? fu : fs);
    l.total = l.t + (tab ? 2 * My * l.P + 2 * Mx * l.Q + 3 * (Mx + My) : 0);
    return l;
}
// LDS index in U of interior point q = j Mx + i (32-bit: slices of at most
// 512 x 512 points).
__device__ __forceinline__ int vel_at(int q, int Mx, int P)
{
    const int j = q / Mx;
    return (j + 1) * P + (q - j * Mx) + 1;
}

// Where the walks read their tables: x tables of row j at xw + j tp + i,
// y tables of column i at yw + i yq + j ys.
struct VelView {
    const double *xw, *xc, *yw, *yc;
    const double *xa, *xlo, *xup, *ya, *ylo, *yup;
    int tp, yq, ys;
};

// One line of n points: the Thomas passes with pivots w, cc (table stride
// ts) on the right-hand side rp (contiguous); the forward values go to fw
// (contiguous; fw may be rp itself), the solution to o at stride fo.  Both
// passes go in blocks of KB points with two register sets used in turn: the
// loads of one block are issued before the recurrence of the other runs, so
// their latency is hidden behind it.  In that order every right-hand-side
// value is read a block before its forward value overwrites it.
__device__ __forceinline__ void vel_walk(const double *rp, double *fw, double *__restrict__ o,
                                         const double *__restrict__ w, const double *__restrict__ cc, double a,
                                         int n, int fo, int ts)
{
    constexpr int KB = 8;
    // ---- forward: d_e = (r_e - a d_{e-1}) w_e
    double d = 0.0;
    {
        double ra[KB], wa[KB], rb[KB], wb[KB];
        auto load = [&](int e0, double (&r)[KB], double (&wv)[KB]) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                r[k] = rp[e0 + k];
                wv[k] = w[(e0 + k) * ts];
            }
        };
        auto run = [&](int e0, const double (&r)[KB], const double (&wv)[KB]) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                d = (r[k] - a * d) * wv[k];
                fw[e0 + k] = d;
            }
        };
        const int nb = n / KB;
        if (nb > 0) load(0, ra, wa);
        int b = 0;
        for (; b + 1 < nb; b += 2) {
            load((b + 1) * KB, rb, wb);
            run(b * KB, ra, wa);
            if (b + 2 < nb) load((b + 2) * KB, ra, wa);
            run((b + 1) * KB, rb, wb);
        }
        if (b < nb) run(b * KB, ra, wa);
        for (int e = nb * KB; e < n; ++e) {
            d = (rp[e] - a * d) * w[e * ts];
            fw[e] = d;
        }
    }
    // ---- backward over e = n-2 .. 0: x_e = d_e - cc_e x_{e+1}
    double x = d;
    o[(n - 1) * fo] = x;
    {
        double fa[KB], ca[KB], fb[KB], cb[KB];
        auto load = [&](int e0, double (&f)[KB], double (&cv)[KB]) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                f[k] = fw[e0 - k];
                cv[k] = cc[(e0 - k) * ts];
            }
        };
        auto run = [&](int e0, const double (&f)[KB], const double (&cv)[KB]) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                x = f[k] - cv[k] * x;
                o[(e0 - k) * fo] = x;
            }
        };
        const int nb = (n - 1) / KB;
        if (nb > 0) load(n - 2, fa, ca);
        int b = 0;
        for (; b + 1 < nb; b += 2) {
            load(n - 2 - (b + 1) * KB, fb, cb);
            run(n - 2 - b * KB, fa, ca);
            if (b + 2 < nb) load(n - 2 - (b + 2) * KB, fa, ca);
            run(n - 2 - (b + 1) * KB, fb, cb);
        }
        if (b < nb) run(n - 2 - b * KB, fa, ca);
        for (int e = n - 2 - nb * KB; e >= 0; --e) {
            x = fw[e] - cc[e * ts] * x;
            o[e * fo] = x;
        }
    }
}

// The explicit parts of a PR-ADI step, by all threads (wavefronts over the
// lines, lanes along them), into W in the layout the next walk reads:
//   x half-step, row-major:  W(i, j) = U + ylo[i] U(i, j-1) + ydi U + yup[i] U(i, j+1)
//   y half-step, transposed: W(i, j) = S + xlo[j] S(i-1, j) + xdi S + xup[j] S(i+1, j)
// (the ghost rows of U and S supply the zeros outside).
__device__ __forceinline__ void vel_rhs_x(const VelView &v, double ydi, const double *__restrict__ U,
                                          double *__restrict__ W, int Mx, int My, int P)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll 2
    for (int j = threadIdx.x >> 6; j < My; j += nw)
        for (int i = lane; i < Mx; i += 64) {
            const int l = (j + 1) * P + i + 1;
            const double c0 = U[l];
            W[l] = c0 + v.ylo[i] * U[l - P] + ydi * c0 + v.yup[i] * U[l + P];
        }
}

__device__ __forceinline__ void vel_rhs_y(const VelView &v, double xdi, const double *__restrict__ S,
                                          double *__restrict__ W, int Mx, int My, int Q)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll 2
    for (int i = threadIdx.x >> 6; i < Mx; i += nw)
        for (int j = lane; j < My; j += 64) {
            const int l = (i + 1) * Q + j + 1;
            const double c0 = S[l];
            W[l] = c0 + v.xlo[j] * S[l - Q] + xdi * c0 + v.xup[j] * S[l + Q];
        }
}

// One step: x half-step (row threads: the right-hand side -> S), barrier,
// y half-step (column threads: -> U), barrier.  EXPL: the PR-ADI explicit
// parts go first into W (a parallel pass and a barrier each) and the walks
// solve in place on W; else the walks read U and S directly.
template <bool EXPL>
__device__ __forceinline__ void vel_step_lds(const VelView &v, double xdi, double ydi, double *U, double *S,
                                             double *W, int Mx, int My, int P, int Q)
{
    // The line index and the pitches pass through an empty asm once per
    // step: otherwise the compiler hoists every address of both walks out
    // of the loop over steps and keeps them all live (register spills).
    int k = threadIdx.x;
    asm volatile("" : "+v"(k));
    asm volatile("" : "+s"(P));
    asm volatile("" : "+s"(Q));
    if constexpr (EXPL) {
        vel_rhs_x(v, ydi, U, W, Mx, My, P);
        __syncthreads();
    }
    if (k < My) {  // row k: S = X^{-1} (I + th Ly) U
        const int j = k;
        const int r0 = (j + 1) * P + 1;
        vel_walk(EXPL ? W + r0 : U + r0, W + r0, S + Q + j + 1, v.xw + j * v.tp, v.xc + j * v.tp, v.xa[j], Mx, Q,
                 1);
    }
    __syncthreads();
    if constexpr (EXPL) {
        vel_rhs_y(v, xdi, S, W, Mx, My, Q);
        __syncthreads();
    }
    if (k < Mx) {  // column k: U = Y^{-1} (I + th Lx) S
        const int i = k;
        const int c0 = (i + 1) * Q + 1;
        vel_walk(EXPL ? W + c0 : S + c0, W + c0, U + P + i + 1, v.yw + i * v.yq, v.yc + i * v.yq, v.ya[i], My, P,
                 v.ys);
    }
    __syncthreads();
}

// TAB: copy the tables into LDS behind the fields (the y tables
// transposed; the caller's barrier publishes them); else read them in place.
template <bool TAB>
__device__ __forceinline__ VelView vel_stage(const VelTab &t, double *sh, int Mx, int My, const VelLds &L)
{
    if constexpr (!TAB) {
        return VelView{t.xw, t.xc, t.yw, t.yc, t.xa, t.xlo, t.xup, t.ya, t.ylo, t.yup, Mx, 1, Mx};
    } else {
        const int P = L.P, Q = L.Q, np = Mx * My;
        double *XW = sh + L.t, *XC = XW + My * P, *YW = XC + My * P, *YC = YW + Mx * Q;
        for (int q = threadIdx.x; q < np; q += blockDim.x) {
            const int j = q / Mx, i = q - j * Mx;
            XW[j * P + i] = t.xw[q];
            XC[j * P + i] = t.xc[q];
            YW[i * Q + j] = t.yw[q];
            YC[i * Q + j] = t.yc[q];
        }
        double *R = YC + Mx * Q, *C = R + 3 * My;
        for (int q = threadIdx.x; q < My; q += blockDim.x) {
            R[q] = t.xa[q];
            R[My + q] = t.xlo[q];
            R[2 * My + q] = t.xup[q];
        }
        for (int q = threadIdx.x; q < Mx; q += blockDim.x) {
            C[q] = t.ya[q];
            C[Mx + q] = t.ylo[q];
            C[2 * Mx + q] = t.yup[q];
        }
        return VelView{XW, XC, YW, YC, R, R + My, R + 2 * My, C, C + Mx, C + 2 * Mx, P, Q, 1};
    }
}

// U = slice u (interior) with zero ghosts; S all zero (its ghosts stay so).
__device__ __forceinline__ void vel_load_field(double *U, double *S, const double *u, int Mx, int My,
                                               const VelLds &L)
{
    const int P = L.P, fu = (My + 2) * P, fs = (Mx + 2) * L.Q;
    for (int l = threadIdx.x; l < fu; l += blockDim.x) {
        const int jj = l / P - 1, ii = l - (jj + 1) * P - 1;
        const bool in = jj >= 0 && jj < My && ii >= 0 && ii < Mx;
        U[l] = in ? u[jj * Mx + ii] : 0.0;
    }
    for (int l = threadIdx.x; l < fs; l += blockDim.x) S[l] = 0.0;
}

// All-at-once apply on `ns` slices: out_{s+out_off} = base_{s+out_off} + sign F(in_{s+in_off})
// (base NULL: F(in)), F = m steps, one workgroup per slice.
template <bool TAB, bool EXPL>
__global__ __launch_bounds__(kVelLdsLines) void k_vel_apply_lds(VelTab t, const double *__restrict__ in, long in_off,
                                                                 double *out, long out_off, const double *base,
                                                                 long base_off, double sign, int m, int Mx, int My)
{
    extern __shared__ double sh[];
    const VelLds L = vel_lds_layout(Mx, My, TAB);
    poison_lds(sh, (int)L.total);
    double *U = sh, *S = sh + L.s, *W = sh + L.w;
    const VelView v = vel_stage<TAB>(t, sh, Mx, My, L);
    const int np = Mx * My;
    vel_load_field(U, S, in + (in_off + blockIdx.x) * np, Mx, My, L);
    __syncthreads();
    for (int s = 0; s < m; ++s) vel_step_lds<EXPL>(v, t.xdi, t.ydi, U, S, W, Mx, My, L.P, L.Q);
    double *o = out + (out_off + blockIdx.x) * np;
    const double *b = base ? base + (base_off + blockIdx.x) * np : nullptr;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const double x = U[vel_at(q, Mx, L.P)];
        o[q] = b ? b[q] + sign * x : x;
    }
}

// Values of v_n each thread loads ahead of the walks of slice n.
constexpr int kVelPre = 8;

// Coarse sweep z_0 = v_0, z_n = v_n + G(z_{n-1}) (G = c steps) by one
// workgroup marching the slices; v == z is allowed.  Each slice first issues
// the loads of v_n and the stores of z_{n-1} (from LDS), then walks: both
// transfers overlap the walks.
template <bool TAB, bool EXPL>
__global__ __launch_bounds__(kVelLdsLines) void k_vel_sweep_lds(VelTab t, const double *v, double *z, int N, int c,
                                                                 int Mx, int My)
{
    extern __shared__ double sh[];
    const VelLds L = vel_lds_layout(Mx, My, TAB);
    poison_lds(sh, (int)L.total);
    const int P = L.P;
    double *U = sh, *S = sh + L.s, *W = sh + L.w;
    const VelView w = vel_stage<TAB>(t, sh, Mx, My, L);
    const int np = Mx * My, bd = blockDim.x, tid = threadIdx.x;
    vel_load_field(U, S, v, Mx, My, L);
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
        for (int s = 0; s < c; ++s) vel_step_lds<EXPL>(w, t.xdi, t.ydi, U, S, W, Mx, My, P, L.Q);
#pragma unroll
        for (int k = 0; k < kVelPre; ++k)
            if (tid + k * bd < np) U[at[k]] += pre[k];
        for (int q = tid + kVelPre * bd; q < np; q += bd) U[vel_at(q, Mx, P)] += vn[q];
        __syncthreads();
    }
    if (N > 1) store(z + (long)(N - 1) * np);
}

size_t vel_lds_bytes(int Mx, int My, bool tab) { return sizeof(double) * (size_t)vel_lds_layout(Mx, My, tab).total; }

// Lines per axis fit one workgroup; at least four wavefronts for the copies.
static int vel_lds_threads(int Mx, int My)
{
    const int lines = Mx > My ? Mx : My;
    const int t = ((lines + 63) / 64) * 64;
    return t < 256 ? 256 : t;
}

// The sweep adds v_n and stores z_n every slice, and a PR-ADI step has its
// explicit parts computed by all threads: there all kVelLdsLines threads
// share that work (the walks use one thread per line).
static int vel_wide_threads(int Mx, int My)
{
    return kVelLdsLines > vel_lds_threads(Mx, My) ? kVelLdsLines : vel_lds_threads(Mx, My);
}

int vel_lds_mode(int Mx, int My)
{
    if (Mx < 1 || My < 1 || (Mx > My ? Mx : My) > kVelLdsLines) return 0;
    if (vel_lds_bytes(Mx, My, true) <= kVelLdsMax) return 2;
    return vel_lds_bytes(Mx, My, false) <= kVelLdsMax ? 1 : 0;
}

// Raise the dynamic LDS limit of a kernel once.
template <bool TAB, bool EXPL>
static hipError_t apply_lds_attr()
{
    static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vel_apply_lds<TAB, EXPL>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kVelLdsMax);
    return e;
}
template <bool TAB, bool EXPL>
static hipError_t sweep_lds_attr()
{
    static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vel_sweep_lds<TAB, EXPL>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kVelLdsMax);
    return e;
}

template <bool TAB, bool EXPL>
static hipError_t apply_lds(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                            const double *base, long base_off, double sign, int ns, int m, int Mx, int My,
                            hipStream_t st)
{
    const hipError_t e = apply_lds_attr<TAB, EXPL>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_vel_apply_lds<TAB, EXPL>), dim3(ns), dim3(EXPL ? vel_wide_threads(Mx, My) : vel_lds_threads(Mx, My)),
                       vel_lds_bytes(Mx, My, TAB), st, t, in, in_off, out, out_off, base, base_off, sign, m, Mx, My);
    return hipGetLastError();
}

template <bool TAB, bool EXPL>
static hipError_t sweep_lds(const VelTab &t, const double *v, double *z, int N, int c, int Mx, int My,
                            hipStream_t st)
{
    const hipError_t e = sweep_lds_attr<TAB, EXPL>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_vel_sweep_lds<TAB, EXPL>), dim3(1), dim3(vel_wide_threads(Mx, My)),
                       vel_lds_bytes(Mx, My, TAB), st, t, v, z, N, c, Mx, My);
    return hipGetLastError();
}

hipError_t launch_vel_apply_lds(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                                const double *base, long base_off, double sign, int ns, int m, int Mx, int My,
                                hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const int mode = vel_lds_mode(Mx, My);
    if (mode == 0) return hipErrorInvalidValue;
    if (mode == 2)
        return t.expl ? apply_lds<true, true>(t, in, in_off, out, out_off, base, base_off, sign, ns, m, Mx, My, st)
                      : apply_lds<true, false>(t, in, in_off, out, out_off, base, base_off, sign, ns, m, Mx, My, st);
    return t.expl ? apply_lds<false, true>(t, in, in_off, out, out_off, base, base_off, sign, ns, m, Mx, My, st)
                  : apply_lds<false, false>(t, in, in_off, out, out_off, base, base_off, sign, ns, m, Mx, My, st);
}

hipError_t launch_vel_sweep_lds(const VelTab &t, const double *v, double *z, int N, int c, int Mx, int My,
                                hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    const int mode = vel_lds_mode(Mx, My);
    if (mode == 0) return hipErrorInvalidValue;
    if (mode == 2)
        return t.expl ? sweep_lds<true, true>(t, v, z, N, c, Mx, My, st) : sweep_lds<true, false>(t, v, z, N, c, Mx, My, st);
    return t.expl ? sweep_lds<false, true>(t, v, z, N, c, Mx, My, st) : sweep_lds<false, false>(t, v, z, N, c, Mx, My, st);
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
