// 1D fine propagator and coarse sweep kernels (FP64 state).
//
// Fine apply (Sec. 2, eq. (algebraiclinearsystem)): one workgroup per slice;
// the slice state stays in registers for all m implicit steps, so HBM sees
// only the slice in and the result out.
//   IE step:  u <- A^{-1} u,               A = I - dt L
//   CN step:  u <- 2 A^{-1} u - u,         A = I - dt/2 L
//   (the CN right-hand side (I + dt/2 L) u equals 2u - A u).
// Coarse sweep (Sec. 3, eq. (eqinverse), solved sequentially by forward
// substitution): one workgroup marches n = 1..N-1 with z_{n-1} in registers,
// prefetching v_n while it runs the c coarse steps.
#include "line1d.hpp"

namespace pit {

// Thread t owns points t*C .. t*C+C-1 of a line of M points.  Two slice
// layouts exist:
//   natural  (TR = false): point j of a slice at j, slice stride M (the ABI
//            layout).  Loads are branch-free: the index is clamped into the
//            line and padding points j >= M are zeroed where the value is
//            used, so a prefetched register is not merged across control
//            flow (that would force an early wait on the load).
//   chunked  (TR = true):  point t*C+k at chunk_pos(NT, C, t, k): the
//            thread's points in pairs, pair g of all threads side by side
//            (C = 1: point t at t).  Slice stride NT*C, padding stored as
//            zeros.  Every load and store moves 16 bytes per lane and is
//            contiguous across the wavefront; pit_solve keeps its block
//            vectors in this layout.  On one CU the cost of a slice's loads
//            and stores is set by the number of memory instructions, not by
//            bytes, so the pairs halve it against one point per access.
typedef double pit_d2 __attribute__((ext_vector_type(2)));

template <int NT, int C, bool TR>
__device__ __forceinline__ void load_chunk(const double *__restrict__ src, int t, int M, double (&u)[C])
{
    if constexpr (TR && chunk_width(C) == 2) {
        const pit_d2 *s2 = reinterpret_cast<const pit_d2 *>(src);
#pragma unroll
        for (int g = 0; g < C / 2; ++g) {
            const pit_d2 x = s2[g * NT + t];
            u[2 * g] = x.x;
            u[2 * g + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) u[k] = TR ? src[k * NT + t] : src[min(t * C + k, M - 1)];
    }
}

template <int C>
__device__ __forceinline__ void zero_pads(int t, int M, double (&u)[C])
{
    const int j0 = t * C;
#pragma unroll
    for (int k = 0; k < C; ++k) u[k] = (j0 + k < M) ? u[k] : 0.0;
}

template <int NT, int C, bool TR>
__device__ __forceinline__ void store_chunk(double *__restrict__ dst, int t, int M, const double (&u)[C])
{
    if constexpr (TR && chunk_width(C) == 2) {
        pit_d2 *d2 = reinterpret_cast<pit_d2 *>(dst);
#pragma unroll
        for (int g = 0; g < C / 2; ++g) {
            pit_d2 x;
            x.x = u[2 * g];
            x.y = u[2 * g + 1];
            d2[g * NT + t] = x;
        }
    } else if constexpr (TR) {
#pragma unroll
        for (int k = 0; k < C; ++k) dst[k * NT + t] = u[k];
    } else {
        const int j0 = t * C;
        if (j0 + C <= M) {
#pragma unroll
            for (int k = 0; k < C; ++k) dst[j0 + k] = u[k];
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (j0 + k < M) dst[j0 + k] = u[k];
        }
    }
}

// Fine apply of one slice: y_n = lam_n - F(lam_{n-1}) (or F(lam_n) when
// raw); ld is the slice stride of lam and y.  Shared by the single-instance
// kernel and the multi-instance one, so an instance computes the same bits in
// either.
template <int NT, int C, int SCHEME, bool TR>
__device__ __forceinline__ void fine1d_f64_slice(const LineTab<double> &tb, const double *__restrict__ lam,
                                                 double *__restrict__ y, int M, long ld, int m, int raw, int n,
                                                 double *lds)
{
    const int t = threadIdx.x;
    if (!raw && n == 0) {  // y_0 = lam_0
        for (long j = t; j < ld; j += NT) y[j] = lam[j];
        return;
    }
    LineSolver<double, NT, C> S;
    S.load(line_tab_slice(tb, raw ? n : n - 1), lds);  // the propagator of the slice it advances
    double u[C];
    load_chunk<NT, C, TR>(lam + (size_t)(raw ? n : n - 1) * ld, t, M, u);
    zero_pads<C>(t, M, u);
    for (int s = 0; s < m; ++s) {
        if constexpr (SCHEME == SCHEME_IE) {
            S.solve(u);
        } else {
            double w[C];
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = u[k];
            S.solve(w);
#pragma unroll
            for (int k = 0; k < C; ++k) u[k] = fma(2.0, w[k], -u[k]);
        }
    }
    if (!raw) {
        double own[C];
        load_chunk<NT, C, TR>(lam + (size_t)n * ld, t, M, own);
#pragma unroll
        for (int k = 0; k < C; ++k) u[k] = own[k] - u[k];
        zero_pads<C>(t, M, u);
    }
    store_chunk<NT, C, TR>(y + (size_t)n * ld, t, M, u);
}

template <int NT, int C, int SCHEME, bool TR>
__global__ __launch_bounds__(NT) void k_fine1d_f64(LineTab<double> tb, const double *__restrict__ lam,
                                                   double *__restrict__ y, int N, int M, long ld, int m,
                                                   int raw, int n0)
{
    __shared__ double lds[LineSolver<double, NT, C>::kLds];
    poison_lds(lds, LineSolver<double, NT, C>::kLds);
    fine1d_f64_slice<NT, C, SCHEME, TR>(tb, lam, y, M, ld, m, raw, n0 + blockIdx.x, lds);
}

// Fine apply with an FP32 propagator: the slice state is an FP32 pair
// (value + compensation) and every step is taken in increment form
// (LineSolver::step_delta), so rounding the step matrix to FP32 perturbs only
// the increment, and the state's own rounding is carried in the compensation;
// lam and y are FP64 and the subtraction y_n = lam_n - F(lam_{n-1}) is done in
// FP64.
template <int NT, int C, bool TR>
__device__ __forceinline__ void fine1d_f32_slice(const LineTab<float> &tb, const double *__restrict__ lam,
                                                 double *__restrict__ y, int M, long ld, int m, float pd,
                                                 float pa, float pr, int periodic, int raw, int n, float *lds)
{
    const int t = threadIdx.x;
    if (!raw && n == 0) {  // y_0 = lam_0
        for (long j = t; j < ld; j += NT) y[j] = lam[j];
        return;
    }
    LineSolver<float, NT, C> S;
    const int sl = raw ? n : n - 1;  // the slice whose propagator it applies
    S.load(line_tab_slice(tb, sl), lds);
    if (tb.sstride) pd = tb.sscal[kSliceScalars * sl + 5];
    double ud[C];
    load_chunk<NT, C, TR>(lam + (size_t)(raw ? n : n - 1) * ld, t, M, ud);
    zero_pads<C>(t, M, ud);
    float u[C], lo[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        u[k] = (float)ud[k];
        lo[k] = (float)(ud[k] - (double)u[k]);
    }
    for (int s = 0; s < m; ++s) S.step_delta(u, lo, pd, pa, pr, M, periodic);
#pragma unroll
    for (int k = 0; k < C; ++k) ud[k] = (double)u[k] + (double)lo[k];
    if (!raw) {
        double own[C];
        load_chunk<NT, C, TR>(lam + (size_t)n * ld, t, M, own);
#pragma unroll
        for (int k = 0; k < C; ++k) ud[k] = own[k] - ud[k];
        zero_pads<C>(t, M, ud);
    }
    store_chunk<NT, C, TR>(y + (size_t)n * ld, t, M, ud);
}

template <int NT, int C, bool TR>
__global__ __launch_bounds__(NT) void k_fine1d_f32(LineTab<float> tb, const double *__restrict__ lam,
                                                   double *__restrict__ y, int N, int M, long ld, int m,
                                                   float pd, float pa, float pr, int periodic, int raw, int n0)
{
    __shared__ float lds[LineSolver<float, NT, C>::kLds];
    poison_lds(lds, LineSolver<float, NT, C>::kLds);
    fine1d_f32_slice<NT, C, TR>(tb, lam, y, M, ld, m, pd, pa, pr, periodic, raw, n0 + blockIdx.x, lds);
}

// One coarse slice step of the sweep: u <- G(u) + v_n (pads stay 0).
template <int NT, int C, int SCHEME>
__device__ __forceinline__ void coarse_step(LineSolver<double, NT, C> &S, double (&u)[C], const double (&vn)[C],
                                            int c, int t, int M)
{
    for (int s = 0; s < c; ++s) {
        if constexpr (SCHEME == SCHEME_IE) {
            S.solve(u);
        } else {
            double w[C];
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = u[k];
            S.solve(w);
#pragma unroll
            for (int k = 0; k < C; ++k) u[k] = fma(2.0, w[k], -u[k]);
        }
    }
    const int j0 = t * C;
#pragma unroll
    for (int k = 0; k < C; ++k) u[k] = (j0 + k < M) ? u[k] + vn[k] : 0.0;
}

// Implicit-Euler sweep with the slice's global traffic spread over the
// solves (chunked layout, point pairs).  The first solve of slice n runs out
// of place, so u keeps z_{n-1} through it and z_{n-1} is stored from u at its
// hook points; v_n is then loaded into u at the second solve's hook points
// (c >= 2; with c = 1 after the stores, in the backward half of the one
// solve), and z_n = w + v_n.  The same registers as a one-buffer prefetch,
// but no wave issues sixteen 1 KiB accesses back to back.  A touch of v_{n+2}
// (one element of each thread's chunk) makes the loads L2 hits.  Hook plans
// (measured on the 4096-point line, 256 threads): pair g of the P pairs a
// thread holds takes slot s = 8g/P; its store goes at hook s + (s > 0) +
// (s > 3) of the first solve, its load at the same hook of the second, the
// touch at hook 10 of the first; with c = 1 stores at hook s, loads at hook
// 8 + s/2, the touch at the start of the slice.
template <int NT, int C, bool ONE>
__device__ __forceinline__ void sweep1d_ie_spread(const LineTab<double> &tb, const double *v, double *z, int N,
                                                  int M, long ld, int c, double *lds)
{
    static_assert(chunk_width(C) == 2, "point pairs");
    constexpr int P = C / 2;  // pairs per thread
    const int t = threadIdx.x;
    LineSolver<double, NT, C> S;
    S.load(tb, lds);
    double u[C], w[C];
    load_chunk<NT, C, true>(v, t, M, u);
    zero_pads<C>(t, M, u);
    const long tofs = min(t * C, NT * C - 1);
    for (int n = 1; n < N; ++n) {
        pit_d2 *zp = reinterpret_cast<pit_d2 *>(z + (size_t)(n - 1) * ld);
        const pit_d2 *vn = reinterpret_cast<const pit_d2 *>(v + (size_t)n * ld);
        const double *vt = v + (size_t)min(n + 2, N - 1) * ld + tofs;
        auto store_pair = [&](int g) {
            pit_d2 x;
            x.x = u[2 * g];
            x.y = u[2 * g + 1];
            zp[g * NT + t] = x;
        };
        auto load_pair = [&](int g) {
            const pit_d2 x = vn[g * NT + t];
            u[2 * g] = x.x;
            u[2 * g + 1] = x.y;
        };
        double touch = 0.0;
        if constexpr (ONE) {
            touch = *vt;
            S.solve_to(u, w, make_hook([&](int h) {
#pragma unroll
                for (int g = 0; g < P; ++g) {
                    const int s = g * 8 / P;
                    if (h == s) store_pair(g);
                    if (h == 8 + s / 2) load_pair(g);
                }
            }));
        } else {
            S.solve_to(u, w, make_hook([&](int h) {
#pragma unroll
                for (int g = 0; g < P; ++g) {
                    const int s = g * 8 / P;
                    if (h == s + (s > 0) + (s > 3)) store_pair(g);
                }
                if (h == 10) touch = *vt;
            }));
            S.solve_to(w, w, make_hook([&](int h) {
#pragma unroll
                for (int g = 0; g < P; ++g) {
                    const int s = g * 8 / P;
                    if (h == s + (s > 0) + (s > 3)) load_pair(g);
                }
            }));
            for (int s = 2; s < c; ++s) S.solve(w);
        }
        asm volatile("" ::"v"(touch));  // the touched value, consumed long after it landed
        const int j0 = t * C;
#pragma unroll
        for (int k = 0; k < C; ++k) u[k] = (j0 + k < M) ? w[k] + u[k] : 0.0;
    }
    store_chunk<NT, C, true>(z + (size_t)(N - 1) * ld, t, M, u);
}

// The slice loop is unrolled by two with two prefetch buffers (v_{n+2} is
// loaded while slices n and n+1 are computed) and the prefetch index is
// clamped instead of guarded, so the loaded registers are consumed where
// they land.
template <int NT, int C, int SCHEME, bool TR, bool PS>
__device__ __forceinline__ void sweep1d_f64_line(const LineTab<double> &tb, const double *v, double *z, int N,
                                                 int M, long ld, int c, double *lds)
{
    // A second prefetch buffer does not fit in the registers at 16 points per
    // thread (with the solver's four per-point tables the compiler parks the
    // buffers in AGPRs, and its copies then wait on loads just issued), nor
    // at 1024 threads (128 registers per lane).
    constexpr bool kTwoBuffers = C <= 8 && NT * C <= 4096;
    // The interleaved implicit-Euler path for one constant operator (with a
    // table per slice the reloads keep more values live and it spilled), in
    // the register form, at 8 or 16 points per lane and two or more waves:
    // there it measured faster than both prefetch forms at one and at two
    // solves per slice (512x8 and 1024x8 lines 15-50% faster, the 4096-point
    // line 18%).  At 4 points or one wave it was slower at one solve per slice.
    if constexpr (!PS && !line_compact(NT, C) && C >= 8 && NT >= 128 && SCHEME == SCHEME_IE && TR) {
        if (c == 1) sweep1d_ie_spread<NT, C, true>(tb, v, z, N, M, ld, c, lds);
        else sweep1d_ie_spread<NT, C, false>(tb, v, z, N, M, ld, c, lds);
        return;
    }
    const int t = threadIdx.x;
    LineSolver<double, NT, C> S;
    S.load(PS ? line_tab_slice(tb, 0) : tb, lds);
    // PS (an operator per slice): step n uses G_{n-1}, whose tables are
    // loaded before the step (after a barrier, since the previous step's
    // solves read the LDS slots that the load rewrites).  n is uniform.  A
    // separate instantiation, so the constant operator's kernel keeps its
    // registers.
    auto tables_for = [&](int n) {
        if constexpr (PS) {
            if (n < 2) return;
            if constexpr (LineSolver<double, NT, C>::W > 1) __syncthreads();
            S.load(line_tab_slice(tb, n - 1), lds);
        }
    };
    if constexpr (line_compact(NT, C)) {
        // 16 FP64 points per lane at 1024 threads leave no registers for a
        // prefetch buffer.  Instead, while step n-1 runs, every thread touches
        // one element of v_n at offset t*C (16 points = one 128-byte line per
        // thread in either layout), so the loads after the c solves of step n
        // hit L2.
        double u[C];
        load_chunk<NT, C, TR>(v, t, M, u);
        zero_pads<C>(t, M, u);
        store_chunk<NT, C, TR>(z, t, M, u);
        const long tofs = min(t * C, TR ? NT * C - 1 : M - 1);
        for (int n = 1; n < N; ++n) {
            const double touch = v[(size_t)n * ld + tofs];
            tables_for(n);
            for (int s = 0; s < c; ++s) {
                if constexpr (SCHEME == SCHEME_IE) {
                    S.solve(u);
                } else {
                    double w[C];
#pragma unroll
                    for (int k = 0; k < C; ++k) w[k] = u[k];
                    S.solve(w);
#pragma unroll
                    for (int k = 0; k < C; ++k) u[k] = fma(2.0, w[k], -u[k]);
                }
            }
            asm volatile("" ::"v"(touch));  // the touched value is consumed here, long after it landed
            double vn[C];
            load_chunk<NT, C, TR>(v + (size_t)n * ld, t, M, vn);
            const int j0 = t * C;
#pragma unroll
            for (int k = 0; k < C; ++k) u[k] = (j0 + k < M) ? u[k] + vn[k] : 0.0;
            store_chunk<NT, C, TR>(z + (size_t)n * ld, t, M, u);
        }
        return;
    }
    // Where a second prefetch buffer does not fit (see above), one is enough:
    // v_{n+1} is loaded at the end of step n and needed only after the c
    // solves of step n+1, and a touch of v_{n+2} (one element per 128-byte
    // line, as above) a step earlier makes that load an L2 hit.  (Implicit
    // Euler in the chunked layout takes the interleaved path instead.)
    double u[C], va[C];
    load_chunk<NT, C, TR>(v, t, M, u);
    zero_pads<C>(t, M, u);
    load_chunk<NT, C, TR>(v + (size_t)min(1, N - 1) * ld, t, M, va);
    store_chunk<NT, C, TR>(z, t, M, u);
    if constexpr (!kTwoBuffers) {
        const long tofs = min(t * C, TR ? NT * C - 1 : M - 1);
        for (int n = 1; n < N; ++n) {
            const double touch = v[(size_t)min(n + 2, N - 1) * ld + tofs];
            tables_for(n);
            coarse_step<NT, C, SCHEME>(S, u, va, c, t, M);
            asm volatile("" ::"v"(touch));  // consumed a whole step after it was issued
            load_chunk<NT, C, TR>(v + (size_t)min(n + 1, N - 1) * ld, t, M, va);
            store_chunk<NT, C, TR>(z + (size_t)n * ld, t, M, u);
        }
        return;
    }
    double vb[C];
    load_chunk<NT, C, TR>(v + (size_t)min(2, N - 1) * ld, t, M, vb);
    for (int n = 1; n < N; n += 2) {
        tables_for(n);
        coarse_step<NT, C, SCHEME>(S, u, va, c, t, M);
        load_chunk<NT, C, TR>(v + (size_t)min(n + 2, N - 1) * ld, t, M, va);
        store_chunk<NT, C, TR>(z + (size_t)n * ld, t, M, u);
        if (n + 1 >= N) break;
        tables_for(n + 1);
        coarse_step<NT, C, SCHEME>(S, u, vb, c, t, M);
        load_chunk<NT, C, TR>(v + (size_t)min(n + 3, N - 1) * ld, t, M, vb);
        store_chunk<NT, C, TR>(z + (size_t)(n + 1) * ld, t, M, u);
    }
}

template <int NT, int C, int SCHEME, bool TR, bool PS>
__global__ __launch_bounds__(NT) void k_sweep1d_f64(LineTab<double> tb, const double *v, double *z,
                                                    int N, int M, long ld, int c)
{
    __shared__ double lds[LineSolver<double, NT, C>::kLds];
    poison_lds(lds, LineSolver<double, NT, C>::kLds);
    sweep1d_f64_line<NT, C, SCHEME, TR, PS>(tb, v, z, N, M, ld, c, lds);
}

// ---------------------------------------------------------------------------
// Multi-instance launches: one launch runs the fine apply (or the coarse
// sweep) of every listed instance of one line shape; block b belongs to the
// listed instance k with first[k] <= b < first[k+1].  Block vectors are in the
// chunked layout.
// ---------------------------------------------------------------------------
template <int NT, int C, int SCHEME>
__global__ __launch_bounds__(NT) void k_fine1d_f64_multi(Group g)
{
    __shared__ double lds[LineSolver<double, NT, C>::kLds];
    poison_lds(lds, LineSolver<double, NT, C>::kLds);
    const int k = group_find(g.first, g.count, blockIdx.x);
    const int vin = g.aux[2 * k], vout = g.aux[2 * k + 1];
    const Inst1d &d = g.inst[g.list[k]];
    const long nv = (long)d.N * d.ld;
    fine1d_f64_slice<NT, C, SCHEME, true>(d.tf, d.vec + vin * nv, d.vec + vout * nv, d.M, d.ld, d.m, 0,
                                          blockIdx.x - g.first[k], lds);
}

template <int NT, int C>
__global__ __launch_bounds__(NT) void k_fine1d_f32_multi(Group g)
{
    __shared__ float lds[LineSolver<float, NT, C>::kLds];
    poison_lds(lds, LineSolver<float, NT, C>::kLds);
    const int k = group_find(g.first, g.count, blockIdx.x);
    const int vin = g.aux[2 * k], vout = g.aux[2 * k + 1];
    const Inst1d &d = g.inst[g.list[k]];
    const long nv = (long)d.N * d.ld;
    fine1d_f32_slice<NT, C, true>(d.tf32, d.vec + vin * nv, d.vec + vout * nv, d.M, d.ld, d.m, d.pd, d.pa, d.pr,
                                  d.periodic, 0, blockIdx.x - g.first[k], lds);
}

template <int NT, int C, int SCHEME, bool PS>
__global__ __launch_bounds__(NT) void k_sweep1d_f64_multi(Group g)
{
    __shared__ double lds[LineSolver<double, NT, C>::kLds];
    poison_lds(lds, LineSolver<double, NT, C>::kLds);
    const Inst1d &d = g.inst[g.list[blockIdx.x]];
    const int vin = g.aux[2 * blockIdx.x], vout = g.aux[2 * blockIdx.x + 1];
    const long nv = (long)d.N * d.ld;
    sweep1d_f64_line<NT, C, SCHEME, true, PS>(d.tc, d.vec + vin * nv, d.vec + vout * nv, d.N, d.M, d.ld, d.c,
                                              lds);
}

#define PIT_LINE_SHAPES(X)                                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(128, 8) X(256, 4) X(256, 8) X(256, 16) X(512, 4)     \
    X(512, 8) X(512, 16) X(1024, 4) X(1024, 8) X(1024, 16)

hipError_t launch_fine1d_f64(LineShape sh, const LineTab<double> &tb, const double *lam, double *y,
                             int N, int M, int m, int scheme, int raw, int last_only, bool chunked,
                             hipStream_t st)
{
    const int n0 = last_only ? N - 1 : 0;
    const int grid = last_only ? 1 : N;
    if (last_only) raw = 1;
#define LAUNCH(nt, c, SCH, TR)                                                                       \
    hipLaunchKernelGGL((k_fine1d_f64<nt, c, SCH, TR>), dim3(grid), dim3(nt), 0, st, tb, lam, y, N, M, \
                       (long)(TR ? nt * c : M), m, raw, n0)
#define X(nt, c)                                                       \
    if (sh.NT == nt && sh.C == c) {                                    \
        if (scheme == SCHEME_IE) {                                     \
            if (chunked) LAUNCH(nt, c, SCHEME_IE, true);               \
            else LAUNCH(nt, c, SCHEME_IE, false);                      \
        } else {                                                       \
            if (chunked) LAUNCH(nt, c, SCHEME_CN, true);               \
            else LAUNCH(nt, c, SCHEME_CN, false);                      \
        }                                                              \
        return hipGetLastError();                                      \
    }
    PIT_LINE_SHAPES(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_fine1d_f32(LineShape sh, const LineTab<float> &tb, const double *lam, double *y, int N,
                             int M, int m, float pd, float pa, float pr, int periodic, int raw, int last_only,
                             bool chunked, hipStream_t st)
{
    const int n0 = last_only ? N - 1 : 0;
    const int grid = last_only ? 1 : N;
    if (last_only) raw = 1;
#define LAUNCH(nt, c, TR)                                                                         \
    hipLaunchKernelGGL((k_fine1d_f32<nt, c, TR>), dim3(grid), dim3(nt), 0, st, tb, lam, y, N, M,   \
                       (long)(TR ? nt * c : M), m, pd, pa, pr, periodic, raw, n0)
#define X(nt, c)                                  \
    if (sh.NT == nt && sh.C == c) {               \
        if (chunked) LAUNCH(nt, c, true);         \
        else LAUNCH(nt, c, false);                \
        return hipGetLastError();                 \
    }
    PIT_LINE_SHAPES(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_sweep1d_f64(LineShape sh, const LineTab<double> &tb, const double *v, double *z,
                              int N, int M, int c, int scheme, bool chunked, hipStream_t st)
{
#define LAUNCH(nt, cc, SCH, TR, PS)                                                                    \
    hipLaunchKernelGGL((k_sweep1d_f64<nt, cc, SCH, TR, PS>), dim3(1), dim3(nt), 0, st, tb, v, z, N, M, \
                       (long)(TR ? nt * cc : M), c)
    // an operator per slice runs in the chunked layout only (pit_solve, the
    // batch engine and pit_coarse_sweep all sweep there)
    if (tb.sstride && !chunked) return hipErrorInvalidValue;
#define X(nt, cc)                                                      \
    if (sh.NT == nt && sh.C == cc) {                                   \
        if (scheme == SCHEME_IE) {                                     \
            if (tb.sstride) LAUNCH(nt, cc, SCHEME_IE, true, true);     \
            else if (chunked) LAUNCH(nt, cc, SCHEME_IE, true, false);  \
            else LAUNCH(nt, cc, SCHEME_IE, false, false);              \
        } else {                                                       \
            if (tb.sstride) LAUNCH(nt, cc, SCHEME_CN, true, true);     \
            else if (chunked) LAUNCH(nt, cc, SCHEME_CN, true, false);  \
            else LAUNCH(nt, cc, SCHEME_CN, false, false);              \
        }                                                              \
        return hipGetLastError();                                      \
    }
    PIT_LINE_SHAPES(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

// grid: g.first[g.count] blocks (the listed instances' slice counts)
hipError_t launch_fine1d_multi(LineShape sh, int fine32, int scheme, const Group &g, int nblocks, hipStream_t st)
{
#define X(nt, c)                                                                                             \
    if (sh.NT == nt && sh.C == c) {                                                                          \
        if (fine32)                                                                                          \
            hipLaunchKernelGGL((k_fine1d_f32_multi<nt, c>), dim3(nblocks), dim3(nt), 0, st, g);              \
        else if (scheme == SCHEME_IE)                                                                        \
            hipLaunchKernelGGL((k_fine1d_f64_multi<nt, c, SCHEME_IE>), dim3(nblocks), dim3(nt), 0, st, g);   \
        else                                                                                                 \
            hipLaunchKernelGGL((k_fine1d_f64_multi<nt, c, SCHEME_CN>), dim3(nblocks), dim3(nt), 0, st, g);   \
        return hipGetLastError();                                                                            \
    }
    PIT_LINE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

// grid: one block per listed instance
hipError_t launch_sweep1d_multi(LineShape sh, int scheme, bool per_slice, const Group &g, hipStream_t st)
{
#define L(nt, c, SCH, PS) hipLaunchKernelGGL((k_sweep1d_f64_multi<nt, c, SCH, PS>), dim3(g.count), dim3(nt), 0, st, g)
#define X(nt, c)                                                                      \
    if (sh.NT == nt && sh.C == c) {                                                   \
        if (scheme == SCHEME_IE) {                                                    \
            if (per_slice) L(nt, c, SCHEME_IE, true);                                 \
            else L(nt, c, SCHEME_IE, false);                                          \
        } else {                                                                      \
            if (per_slice) L(nt, c, SCHEME_CN, true);                                 \
            else L(nt, c, SCHEME_CN, false);                                          \
        }                                                                             \
        return hipGetLastError();                                                     \
    }
    PIT_LINE_SHAPES(X)
#undef X
#undef L
    return hipErrorInvalidValue;
}

}  // namespace pit
