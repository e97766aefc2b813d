// Block-vector kernels of Algorithm 1: segmented FP64 inner products with a
// deterministic two-level reduction, and the BiCGStab vector updates.
//
// The block inner product is <U,V> = sum_n <u_n, v_n>_{L2(Omega)} (Sec. 3),
// with the L2 product approximated by h^d * sum_j; the stopping norm is the
// maximum over slices of the discrete L2 norm.  Both come out of one pass that
// produces per-slice sums.
#include <algorithm>
#include "check.hpp"
#include "pit_internal.hpp"
#include "ctx.hpp"

namespace pit {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_down(v, d, kWave);
    return v;
}

// A thread's strided share of a slice, elements i0, i0 + stride, ...: each
// accumulator takes them in that order, one fma each, as a one-element loop
// would, with the loads of U elements issued before their fmas (a loop that
// waited for each element's loads kept two loads in flight per thread).
template <int NQ>
__device__ __forceinline__ void dots_accumulate(const DotPairs &pr, size_t base, long i0, long stride, long npts,
                                                double (&acc)[4])
{
    constexpr int U = 4;
    long i = i0;
    for (; i + (U - 1) * stride < npts; i += U * stride) {
        double av[NQ][U], bv[NQ][U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                av[q][u] = pr.a[q][base + i + u * stride];
                bv[q][u] = pr.b[q][base + i + u * stride];
            }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[q] = fma(av[q][u], bv[q][u], acc[q]);
    }
    for (; i < npts; i += stride)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = fma(pr.a[q][base + i], pr.b[q][base + i], acc[q]);
}

// The same when every operand is one of two vectors x = a[0], y = b[0] (as in
// <K,S>, <K,K>, <S,S> and <R,R~>, <R,R>): each element of x and y is loaded
// once; bit 2q of sel picks y for a[q], bit 2q+1 for b[q].
template <int NQ>
__device__ __forceinline__ void dots_accumulate_xy(const double *__restrict__ x, const double *__restrict__ y,
                                                   unsigned sel, long i0, long stride, long npts, double (&acc)[4])
{
    constexpr int U = 4;
    long i = i0;
    auto add = [&](double xv, double yv) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double av = (sel >> (2 * q)) & 1 ? yv : xv, bv = (sel >> (2 * q + 1)) & 1 ? yv : xv;
            acc[q] = fma(av, bv, acc[q]);
        }
    };
    for (; i + (U - 1) * stride < npts; i += U * stride) {
        double xv[U], yv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xv[u] = x[i + u * stride];
            yv[u] = y[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) add(xv[u], yv[u]);
    }
    for (; i < npts; i += stride) add(x[i], y[i]);
}

// Block b of slice s sums a strided part of the slice for nq pairs (shared
// by the single- and multi-instance kernels).
__device__ __forceinline__ void seg_dots_block(const DotPairs &pr, int nq, int N, long npts, int bps,
                                               double *__restrict__ part, int b, int s)
{
    __shared__ double sh[4][kRedThreads / kWave];
    poison_lds(&sh[0][0], 4 * (kRedThreads / kWave));
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const size_t base = (size_t)s * npts;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long i0 = (long)b * kRedThreads + t, stride = (long)bps * kRedThreads;
    // operands drawn from the two vectors a[0], b[0] only? (uniform)
    const double *x = pr.a[0], *y = pr.b[0];
    bool two = nq >= 2 && x != y;
    unsigned sel = 0;
    for (int q = 0; q < 4 && q < nq; ++q) {
        const double *ops[2] = {pr.a[q], pr.b[q]};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (ops[k] == y) sel |= 1u << (2 * q + k);
            else if (ops[k] != x) two = false;
        }
    }
    if (two) {
        if (nq == 2) dots_accumulate_xy<2>(x + base, y + base, sel, i0, stride, npts, acc);
        else if (nq == 3) dots_accumulate_xy<3>(x + base, y + base, sel, i0, stride, npts, acc);
        else dots_accumulate_xy<4>(x + base, y + base, sel, i0, stride, npts, acc);
    } else {
        switch (nq) {  // uniform
        case 0: break;
        case 1: dots_accumulate<1>(pr, base, i0, stride, npts, acc); break;
        case 2: dots_accumulate<2>(pr, base, i0, stride, npts, acc); break;
        case 3: dots_accumulate<3>(pr, base, i0, stride, npts, acc); break;
        default: dots_accumulate<4>(pr, base, i0, stride, npts, acc); break;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < nq) {
            double v = wave_sum(acc[q]);
            if (lane == 0) sh[q][w] = v;
        }
    }
    __syncthreads();
    if (t < nq) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < kRedThreads / kWave; ++i) v += sh[t][i];
        part[((size_t)t * bps + b) * N + s] = v;  // [q][b][s]: the finalize reads each b across slices
    }
}

// grid (bps, N)
__global__ __launch_bounds__(kRedThreads) void k_seg_dots(DotPairs pr, int nq, int N, long npts,
                                                          int bps, double *__restrict__ part)
{
    seg_dots_block(pr, nq, N, npts, bps, part, blockIdx.x, blockIdx.y);
}

// One block: per-slice sums in block order, then totals and maxima over
// slices in a fixed order.
__device__ __forceinline__ void seg_finalize_block(const double *__restrict__ part, int nq, int N, int bps,
                                                   double w, RedOut *out)
{
    __shared__ double sd[kRedThreads];
    __shared__ double sm[kRedThreads];
    poison_lds(sd, kRedThreads);
    poison_lds(sm, kRedThreads);
    const int t = threadIdx.x;
    for (int q = 0; q < nq; ++q) {
        double tot = 0.0, mx = 0.0;
        for (int s = t; s < N; s += kRedThreads) {
            // the slice's partials in block order; consecutive threads read
            // consecutive slices, and eight loads go out before their adds
            const double *p = part + (size_t)q * bps * N + s;
            double ss = 0.0;
            int b = 0;
            for (; b + 8 <= bps; b += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(b + u) * N];
#pragma unroll
                for (int u = 0; u < 8; ++u) ss += v[u];
            }
            for (; b < bps; ++b) ss += p[(size_t)b * N];
            tot += ss;
            double nrm = sqrt(w * ss);
            mx = (nrm > mx || nrm != nrm) ? nrm : mx;  // NaN propagates
        }
        sd[t] = tot;
        sm[t] = mx;
        __syncthreads();
        for (int d = kRedThreads / 2; d >= 1; d >>= 1) {
            if (t < d) {
                sd[t] += sd[t + d];
                const double o = sm[t + d];
                sm[t] = (o > sm[t] || o != o) ? o : sm[t];
            }
            __syncthreads();
        }
        if (t == 0) {
            out->dot[q] = w * sd[0];
            out->nmax[q] = sm[0];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedThreads) void k_seg_finalize(const double *__restrict__ part, int nq,
                                                              int N, int bps, double w, RedOut *out)
{
    seg_finalize_block(part, nq, N, bps, w, out);
}

// Multi-instance dots: the blocks of listed instance k are its (b, s) pairs
// in the order b + bps*s.
__global__ __launch_bounds__(kRedThreads) void k_seg_dots_multi(Group g)
{
    const int k = group_find(g.first, g.count, blockIdx.x);
    const Inst1d &d = g.inst[g.list[k]];
    const long nv = (long)d.N * d.ld;
    const int *q9 = g.aux + kDotsAux * k;
    const int nq = q9[0];
    DotPairs pr{};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        pr.a[q] = d.vec + q9[1 + q] * nv;
        pr.b[q] = d.vec + q9[5 + q] * nv;
    }
    const int local = blockIdx.x - g.first[k];
    seg_dots_block(pr, nq, d.N, d.ld, d.bps, d.part, local % d.bps, local / d.bps);
}

__global__ __launch_bounds__(kRedThreads) void k_seg_finalize_multi(Group g)
{
    const Inst1d &d = g.inst[g.list[blockIdx.x]];
    seg_finalize_block(d.part, g.aux[kDotsAux * blockIdx.x], d.N, d.bps, d.w, g.red + blockIdx.x);
}

hipError_t launch_dots_multi(const Group &g, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_seg_dots_multi, dim3(nblocks), dim3(kRedThreads), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_finalize_multi, dim3(g.count), dim3(kRedThreads), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_seg_dots(const DotPairs &pr, int nq, int N, long npts, int bps, double *part,
                           double w, RedOut *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_seg_dots, dim3(bps, N), dim3(kRedThreads), 0, st, pr, nq, N, npts, bps, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_finalize, dim3(1), dim3(kRedThreads), 0, st, part, nq, N, bps, w, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise updates (grid-stride)
// ---------------------------------------------------------------------------
constexpr int kVecThreads = 256;

static inline dim3 vec_grid(long n)
{
    long b = (n + kVecThreads - 1) / kVecThreads;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// The update formulas, shared by the single- and multi-instance kernels.
__device__ __forceinline__ double axpby_elem(double a, double x, double b, double y) { return fma(a, x, b * y); }
__device__ __forceinline__ void update_xr_elem(double &X, double &R, double P, double S, double K, double alpha,
                                               double omega)
{
    X = fma(omega, S, fma(alpha, P, X));
    R = fma(-omega, K, S);
}
__device__ __forceinline__ double update_p_elem(double P, double R, double D, double beta, double omega)
{
    return fma(beta, fma(-omega, D, P), R);
}

__global__ void k_axpby(double *__restrict__ out, const double *__restrict__ x, double a,
                        const double *__restrict__ y, double b, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = axpby_elem(a, x[i], b, y[i]);
}

__global__ void k_update_xr(double *__restrict__ X, double *__restrict__ R, const double *__restrict__ P,
                            const double *__restrict__ S, const double *__restrict__ K, double alpha,
                            double omega, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double x = X[i], r;
        update_xr_elem(x, r, P[i], S[i], K[i], alpha, omega);
        X[i] = x;
        R[i] = r;
    }
}

__global__ void k_update_p(double *__restrict__ P, const double *__restrict__ R,
                           const double *__restrict__ D, double beta, double omega, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        P[i] = update_p_elem(P[i], R[i], D[i], beta, omega);
}

// Multi-instance updates: listed instance k owns blocks first[k]..first[k+1)-1,
// each covering kVecMultiSpan consecutive doubles of its block vectors.
__global__ __launch_bounds__(kVecThreads) void k_vec_multi(Group g)
{
    const int k = group_find(g.first, g.count, blockIdx.x);
    const int op = g.aux[k];
    const Inst1d &d = g.inst[g.list[k]];
    const long nv = (long)d.N * d.ld;
    const double alpha = g.scal[4 * k], omega = g.scal[4 * k + 1], beta = g.scal[4 * k + 2];
    double *R = d.vec + VEC_R * nv, *P = d.vec + VEC_P * nv, *D = d.vec + VEC_D * nv, *S = d.vec + VEC_S * nv;
    double *K = d.vec + VEC_K * nv, *X = d.vec + VEC_X * nv;
    const long i0 = (long)(blockIdx.x - g.first[k]) * kVecMultiSpan;
    const long i1 = min(i0 + kVecMultiSpan, nv);
    for (long i = i0 + threadIdx.x; i < i1; i += kVecThreads) {
        if (op == VOP_S_AXPY) {
            S[i] = axpby_elem(1.0, R[i], -alpha, D[i]);
        } else if (op == VOP_UPDATE_XR) {
            double x = X[i], r;
            update_xr_elem(x, r, P[i], S[i], K[i], alpha, omega);
            X[i] = x;
            R[i] = r;
        } else {
            P[i] = update_p_elem(P[i], R[i], D[i], beta, omega);
        }
    }
}

hipError_t launch_vec_multi(const Group &g, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_vec_multi, dim3(nblocks), dim3(kVecThreads), 0, st, g);
    return hipGetLastError();
}

__global__ void k_b_minus(double *__restrict__ out, const double *__restrict__ in,
                          const double *__restrict__ u0, long npts, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = (i < npts ? u0[i] : 0.0) - in[i];
}

__global__ void k_copy(double *__restrict__ dst, const double *__restrict__ src, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Streaming copy for bandwidth reference: 16-byte accesses, four in flight
// per thread (the loads of a group are issued before its stores), a
// grid-stride loop over groups of 4 * blockDim 16-byte units.
using U4 = __attribute__((ext_vector_type(4))) unsigned;
__global__ __launch_bounds__(256) void k_stream_copy(U4 *__restrict__ dst, const U4 *__restrict__ src, long n16)
{
    constexpr int K = 4;
    const long step = (long)gridDim.x * blockDim.x * K;
    for (long base = (long)blockIdx.x * blockDim.x * K + threadIdx.x; base < n16; base += step) {
        U4 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const long i = base + (long)k * blockDim.x;
            if (i < n16) v[k] = src[i];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const long i = base + (long)k * blockDim.x;
            if (i < n16) dst[i] = v[k];
        }
    }
}

__global__ void k_fill0(double *__restrict__ dst, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = 0.0;
}

// natural [N][M] <-> chunked [N][NT*C]: point j = t*C + k sits at
// chunk_pos(NT, C, t, k) (pairs of points, see pit_internal.hpp).
__global__ void k_to_chunked(const double *__restrict__ nat, double *__restrict__ chk, int N, int M, int NT,
                             int C)
{
    const long S = (long)NT * C, tot = (long)N * S, P = chunk_width(C);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long n = i / S, r = i % S;
        const long g = r / (P * NT), q = r % (P * NT);
        const long t = q / P, k = g * P + q % P, j = t * C + k;
        chk[i] = (j < M) ? nat[n * M + j] : 0.0;
    }
}

__global__ void k_from_chunked(const double *__restrict__ chk, double *__restrict__ nat, int N, int M, int NT,
                               int C)
{
    const long S = (long)NT * C, tot = (long)N * M;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long n = i / M, j = i % M;
        nat[i] = chk[n * S + chunk_pos(NT, C, j / C, j % C)];
    }
}

hipError_t launch_to_chunked(const double *nat, double *chk, int N, int M, int NT, int C, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_chunked, vec_grid((long)N * NT * C), dim3(kVecThreads), 0, st, nat, chk, N, M, NT, C);
    return hipGetLastError();
}

hipError_t launch_from_chunked(const double *chk, double *nat, int N, int M, int NT, int C, hipStream_t st)
{
    hipLaunchKernelGGL(k_from_chunked, vec_grid((long)N * M), dim3(kVecThreads), 0, st, chk, nat, N, M, NT, C);
    return hipGetLastError();
}

hipError_t launch_axpby(double *out, const double *x, double a, const double *y, double b, long n,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_axpby, vec_grid(n), dim3(kVecThreads), 0, st, out, x, a, y, b, n);
    return hipGetLastError();
}

hipError_t launch_update_xr(double *X, double *R, const double *P, const double *S, const double *K,
                            double alpha, double omega, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_update_xr, vec_grid(n), dim3(kVecThreads), 0, st, X, R, P, S, K, alpha, omega, n);
    return hipGetLastError();
}

hipError_t launch_update_p(double *P, const double *R, const double *D, double beta, double omega,
                           long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_update_p, vec_grid(n), dim3(kVecThreads), 0, st, P, R, D, beta, omega, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The same three updates with Algorithm 1's scalars taken from reduction
// outputs in device memory, so that an iteration needs no host round trip
// between its reductions.  Every thread forms the scalars with the host's
// operations and in its order (alpha = rho / dr, omega = ks / kk,
// beta = (alpha / omega) * (rho_new / rho)), so the results are the bits of
// the host-scalar kernels.  A step that meets one of the algorithm's special
// cases (dr, kk or omega exactly 0) changes nothing in X, R, P: the host
// reads the outputs afterwards and takes that branch itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool dev_scalars(const DevScalars &s, double &alpha, double &omega)
{
    const double dr = s.A->dot[0];
    if (dr == 0.0) return false;
    alpha = s.rho->dot[s.rho_idx] / dr;
    const double kk = s.B->dot[1];
    if (kk == 0.0) return false;
    omega = s.B->dot[0] / kk;
    return omega != 0.0;
}

// `one` is 1.0, passed at run time as k_axpby's coefficient is: with a
// literal 1 the compiler folds fma(1, R, b D) into R + b D and may then
// contract that into one fma, which rounds b D differently.
//
// V = 2 (every vector 16-byte aligned): two elements per access, the odd
// last element, if any, on its own; the same operations per element, so the
// same bits as V = 1.
using Dv2 = __attribute__((ext_vector_type(2))) double;
template <int V>
__global__ void k_axpby_dev(double *__restrict__ S, const double *__restrict__ R, const double *__restrict__ D,
                            DevScalars s, double one, long n)
{
    const double dr = s.A->dot[0];
    const double alpha = s.rho->dot[s.rho_idx] / dr;  // dr == 0: S is not used
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x, st = (long)gridDim.x * blockDim.x;
    if constexpr (V == 2) {
        for (long i = t0; i < n / 2; i += st) {
            const Dv2 r = reinterpret_cast<const Dv2 *>(R)[i], d = reinterpret_cast<const Dv2 *>(D)[i];
            reinterpret_cast<Dv2 *>(S)[i] = Dv2{axpby_elem(one, r.x, -alpha, d.x), axpby_elem(one, r.y, -alpha, d.y)};
        }
        if ((n & 1) && t0 == 0) S[n - 1] = axpby_elem(one, R[n - 1], -alpha, D[n - 1]);
    } else {
        for (long i = t0; i < n; i += st) S[i] = axpby_elem(one, R[i], -alpha, D[i]);
    }
}

template <int V>
__global__ void k_update_xr_dev(double *__restrict__ X, double *__restrict__ R, const double *__restrict__ P,
                                const double *__restrict__ S, const double *__restrict__ K, DevScalars s, long n)
{
    double alpha, omega;
    if (!dev_scalars(s, alpha, omega)) return;
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x, st = (long)gridDim.x * blockDim.x;
    if constexpr (V == 2) {
        for (long i = t0; i < n / 2; i += st) {
            const Dv2 x = reinterpret_cast<const Dv2 *>(X)[i], p = reinterpret_cast<const Dv2 *>(P)[i];
            const Dv2 sv = reinterpret_cast<const Dv2 *>(S)[i], k = reinterpret_cast<const Dv2 *>(K)[i];
            double x0 = x.x, x1 = x.y, r0, r1;
            update_xr_elem(x0, r0, p.x, sv.x, k.x, alpha, omega);
            update_xr_elem(x1, r1, p.y, sv.y, k.y, alpha, omega);
            reinterpret_cast<Dv2 *>(X)[i] = Dv2{x0, x1};
            reinterpret_cast<Dv2 *>(R)[i] = Dv2{r0, r1};
        }
        if ((n & 1) && t0 == 0) {
            double x = X[n - 1], r;
            update_xr_elem(x, r, P[n - 1], S[n - 1], K[n - 1], alpha, omega);
            X[n - 1] = x;
            R[n - 1] = r;
        }
    } else {
        for (long i = t0; i < n; i += st) {
            double x = X[i], r;
            update_xr_elem(x, r, P[i], S[i], K[i], alpha, omega);
            X[i] = x;
            R[i] = r;
        }
    }
}

template <int V>
__global__ void k_update_p_dev(double *__restrict__ P, const double *__restrict__ R, const double *__restrict__ D,
                               DevScalars s, long n)
{
    double alpha, omega;
    if (!dev_scalars(s, alpha, omega)) return;
    const double beta = (alpha / omega) * (s.C->dot[0] / s.rho->dot[s.rho_idx]);
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x, st = (long)gridDim.x * blockDim.x;
    if constexpr (V == 2) {
        for (long i = t0; i < n / 2; i += st) {
            const Dv2 p = reinterpret_cast<const Dv2 *>(P)[i], r = reinterpret_cast<const Dv2 *>(R)[i];
            const Dv2 d = reinterpret_cast<const Dv2 *>(D)[i];
            reinterpret_cast<Dv2 *>(P)[i] =
                Dv2{update_p_elem(p.x, r.x, d.x, beta, omega), update_p_elem(p.y, r.y, d.y, beta, omega)};
        }
        if ((n & 1) && t0 == 0) P[n - 1] = update_p_elem(P[n - 1], R[n - 1], D[n - 1], beta, omega);
    } else {
        for (long i = t0; i < n; i += st) P[i] = update_p_elem(P[i], R[i], D[i], beta, omega);
    }
}

static inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipError_t launch_axpby_dev(double *S, const double *R, const double *D, const DevScalars &s, long n,
                            hipStream_t st)
{
    if (aligned16(S) && aligned16(R) && aligned16(D))
        hipLaunchKernelGGL(k_axpby_dev<2>, vec_grid(n / 2), dim3(kVecThreads), 0, st, S, R, D, s, 1.0, n);
    else
        hipLaunchKernelGGL(k_axpby_dev<1>, vec_grid(n), dim3(kVecThreads), 0, st, S, R, D, s, 1.0, n);
    return hipGetLastError();
}

hipError_t launch_update_xr_dev(double *X, double *R, const double *P, const double *S, const double *K,
                                const DevScalars &s, long n, hipStream_t st)
{
    if (aligned16(X) && aligned16(R) && aligned16(P) && aligned16(S) && aligned16(K))
        hipLaunchKernelGGL(k_update_xr_dev<2>, vec_grid(n / 2), dim3(kVecThreads), 0, st, X, R, P, S, K, s, n);
    else
        hipLaunchKernelGGL(k_update_xr_dev<1>, vec_grid(n), dim3(kVecThreads), 0, st, X, R, P, S, K, s, n);
    return hipGetLastError();
}

hipError_t launch_update_p_dev(double *P, const double *R, const double *D, const DevScalars &s, long n,
                               hipStream_t st)
{
    if (aligned16(P) && aligned16(R) && aligned16(D))
        hipLaunchKernelGGL(k_update_p_dev<2>, vec_grid(n / 2), dim3(kVecThreads), 0, st, P, R, D, s, n);
    else
        hipLaunchKernelGGL(k_update_p_dev<1>, vec_grid(n), dim3(kVecThreads), 0, st, P, R, D, s, n);
    return hipGetLastError();
}

hipError_t launch_b_minus(double *out, const double *in, const double *u0, long npts, long n,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_b_minus, vec_grid(n), dim3(kVecThreads), 0, st, out, in, u0, npts, n);
    return hipGetLastError();
}

// dst[i] = src[i % len] (add = 0) or dst[i] += src[i % len] (add = 1), i < len*count:
// one slice repeated over `count` slices.
__global__ void k_repeat(double *__restrict__ dst, const double *__restrict__ src, long len, long n, int add)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = src[i % len];
        dst[i] = add ? dst[i] + v : v;
    }
}

hipError_t launch_repeat(double *dst, const double *src, long len, long count, int add, hipStream_t st)
{
    const long n = len * count;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_repeat, vec_grid(n), dim3(kVecThreads), 0, st, dst, src, len, n, add);
    return hipGetLastError();
}

// X_s += w[s * wstride] c for slices s < N of len points (grid.y = slice).
__global__ void k_slice_axpy(double *__restrict__ X, const double *__restrict__ c, const double *__restrict__ w,
                             long wstride, long len)
{
    const double a = w[(long)blockIdx.y * wstride];
    double *x = X + (long)blockIdx.y * len;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
        x[i] += a * c[i];
}

hipError_t launch_slice_axpy(double *X, const double *c, const double *w, long wstride, long len, int N,
                             hipStream_t st)
{
    if (len <= 0 || N <= 0) return hipSuccess;
    const long blocks = std::min<long>((len + kVecThreads - 1) / kVecThreads, 1024);
    hipLaunchKernelGGL(k_slice_axpy, dim3((unsigned)blocks, (unsigned)N), dim3(kVecThreads), 0, st, X, c, w,
                       wstride, len);
    return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy, vec_grid(n), dim3(kVecThreads), 0, st, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_fill0(double *dst, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill0, vec_grid(n), dim3(kVecThreads), 0, st, dst, n);
    return hipGetLastError();
}

}  // namespace pit

// 256 CUs x 8 workgroups of 256 threads: every SIMD holds 8 waves.
extern "C" int pit_stream_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
        return PIT_EINVAL;
    const long n16 = (long)(bytes / 16);
    if (n16 == 0) return PIT_OK;
    const long blocks = std::min<long>(2048, (n16 + 1023) / 1024);
    hipLaunchKernelGGL(pit::k_stream_copy, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<pit::U4 *>(dst), static_cast<const pit::U4 *>(src), n16);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pit::set_last_hip((int)e);
        return PIT_EHIP;
    }
    return PIT_OK;
}
