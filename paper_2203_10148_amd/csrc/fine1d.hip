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

template <int NT, int C>
__global__ __launch_bounds__(NT) void k_fine1d_f64(LineTab<double> tb, const double *__restrict__ lam,
                                                   double *__restrict__ y, int N, int M, int m,
                                                   int scheme, int raw, int n0)
{
    constexpr int W = NT / kWave;
    __shared__ double lds[4 * W];
    const int n = n0 + blockIdx.x;
    const int t = threadIdx.x;
    if (!raw && n == 0) {  // y_0 = lam_0
        for (int j = t; j < M; j += NT) y[j] = lam[j];
        return;
    }
    LineSolver<double, NT, C> S;
    S.load(tb, lds);
    const double *src = lam + (size_t)(raw ? n : n - 1) * M;
    double u[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = t * C + k;
        u[k] = (j < M) ? src[j] : 0.0;
    }
    if (scheme == SCHEME_IE) {
        for (int s = 0; s < m; ++s) S.solve(u);
    } else {
        for (int s = 0; s < m; ++s) {
            double w[C];
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = u[k];
            S.solve(w);
#pragma unroll
            for (int k = 0; k < C; ++k) u[k] = fma(2.0, w[k], -u[k]);
        }
    }
    double *dst = y + (size_t)n * M;
    const double *own = lam + (size_t)n * M;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = t * C + k;
        if (j < M) dst[j] = raw ? u[k] : own[j] - u[k];
    }
}

template <int NT, int C>
__global__ __launch_bounds__(NT) void k_sweep1d_f64(LineTab<double> tb, const double *v, double *z,
                                                    int N, int M, int c, int scheme)
{
    constexpr int W = NT / kWave;
    __shared__ double lds[4 * W];
    const int t = threadIdx.x;
    LineSolver<double, NT, C> S;
    S.load(tb, lds);
    double u[C], nxt[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = t * C + k;
        u[k] = (j < M) ? v[j] : 0.0;
        nxt[k] = (j < M && N > 1) ? v[(size_t)M + j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = t * C + k;
        if (j < M) z[j] = u[k];
    }
    for (int n = 1; n < N; ++n) {
        if (scheme == SCHEME_IE) {
            for (int s = 0; s < c; ++s) S.solve(u);
        } else {
            for (int s = 0; s < c; ++s) {
                double w[C];
#pragma unroll
                for (int k = 0; k < C; ++k) w[k] = u[k];
                S.solve(w);
#pragma unroll
                for (int k = 0; k < C; ++k) u[k] = fma(2.0, w[k], -u[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < C; ++k) u[k] += nxt[k];
        if (n + 1 < N) {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int j = t * C + k;
                nxt[k] = (j < M) ? v[(size_t)(n + 1) * M + j] : 0.0;
            }
        }
        double *dst = z + (size_t)n * M;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int j = t * C + k;
            if (j < M) dst[j] = u[k];
        }
    }
}

#define PIT_LINE_SHAPES(X) \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(128, 8) X(256, 8) X(256, 16) X(512, 8) X(512, 16) \
    X(1024, 8) X(1024, 16)

hipError_t launch_fine1d_f64(LineShape sh, const LineTab<double> &tb, const double *lam, double *y,
                             int N, int M, int m, int scheme, int raw, int last_only, hipStream_t st)
{
    const int n0 = last_only ? N - 1 : 0;
    const int grid = last_only ? 1 : N;
    if (last_only) raw = 1;
#define X(nt, c)                                                                                \
    if (sh.NT == nt && sh.C == c) {                                                             \
        hipLaunchKernelGGL((k_fine1d_f64<nt, c>), dim3(grid), dim3(nt), 0, st, tb, lam, y, N, M, \
                           m, scheme, raw, n0);                                                 \
        return hipGetLastError();                                                               \
    }
    PIT_LINE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_sweep1d_f64(LineShape sh, const LineTab<double> &tb, const double *v, double *z,
                              int N, int M, int c, int scheme, hipStream_t st)
{
#define X(nt, cc)                                                                              \
    if (sh.NT == nt && sh.C == cc) {                                                           \
        hipLaunchKernelGGL((k_sweep1d_f64<nt, cc>), dim3(1), dim3(nt), 0, st, tb, v, z, N, M, c, \
                           scheme);                                                            \
        return hipGetLastError();                                                              \
    }
    PIT_LINE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace pit
