// Internal declarations shared by the host code and the HIP kernels of
// libpitsbicg.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pit {

constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kScanConsts = 7; // per-thread multipliers of one in-wave scan
constexpr int kMaxWaves = 16;  // 1024 threads per line at most
constexpr int kMaxLine = 16384;
constexpr int kCompactAbove = 8192;  // longer lines use the compact solver tables

constexpr bool line_compact(int NT, int C) { return NT * C > kCompactAbove; }

// ---------------------------------------------------------------------------
// 1D line solver tables.
//
// A line of M points is split over NT threads, C consecutive points per
// thread (point j = t*C + k).  The matrix is A = I - theta*L (tridiagonal,
// constant stencil, optionally cyclic).  For a cyclic A the solver works on
// B = A without its corners and with the first/last diagonal entries shifted
// (Sherman-Morrison), B = L_B U_B without pivoting:
//     forward   y_j = d_j + lm_j * y_{j-1}          (lm_j = -l_j)
//     backward  x_j = iu_j * y_j + cm_j * x_{j+1}   (iu_j = 1/u_j, cm_j = -c/u_j)
//     cyclic    x  -= phi * z,  phi = (x_0 + bg * x_{M-1}) * inv_den
// Both recurrences are first-order linear with constant multipliers, so the
// carries between threads are a scan whose multiplier products are constants
// precomputed here:
//     pf_t = prod_k lm_{tC+k},   pb_t = prod_k cm_{tC+k}
//   in-wave scan, lanes in rows of 16 (r = row of t, l = lane in row):
//     wf[i]_t   = prod_{q=t-s+1..t} pf_q, s = 2^i, i < 4   (0 if l < s)
//     wf[4+r']_t = prod_{q=16(r'+1)..t} pf_q, r' < 3      (0 if r <= r')
//     wb[i]_t   = prod_{q=t..t+s-1} pb_q, s = 2^i, i < 4   (0 if l + s > 15)
//     wb[3+r']_t = prod_{q=t..16r'-1} pb_q, r' = 1..3     (0 if r >= r')
//   (lane indices inside the wave), and across waves
//     qf_t = prod_{q=wavestart..t-1} pf_q,  qb_t = prod_{q=t+1..waveend} pb_q
//     pwf_w, pwb_w = products of pf / pb over wave w.
//   late right-hand-side terms at the first point P_w of wave w (increment form):
//     rf_t  = prod_{i=P_w+1..tC-1} lm_i  (0 for lane 0),
//     rfw_w = prod_{i=P_w+1..Q_w} lm_i   (Q_w = last point of wave w).
// Padding points j >= M carry lm = 1, iu = 0, cm = 0, z = 0 so that the
// forward total equals y_{M-1} and the pads solve to 0.
//
// Compact form (FP64 lines longer than kCompactAbove points): the off-diagonals of
// B are the constants a and c, so lm_j = -a iu_{j-1} and cm_j = -c iu_j, and
// the solver keeps only iu per point and forms the multipliers as it goes:
//     forward   y_j = d_j - a (iu_{j-1} y_{j-1})
//     backward  x_j = iu_j (y_j - c x_{j+1})
// which leaves room in the registers for 16 FP64 points per thread at 1024
// threads.  The scan constants are then built from these effective
// multipliers (lm_0 = 0, the first pad has lm = -a iu_{M-1}, later pads 0), so
// the forward total is not y_{M-1}: the owner of point M-1 hands it over in
// the backward LDS round instead, and the cyclic vector z lives in LDS.  The
// FP32 tables of such a line keep the register form.
//
// Device layout (element type T, one contiguous blob):
//   lm[C][NT] iu[C][NT] cm[C][NT] z[C][NT] wf[7][NT] wb[7][NT] qf[NT] qb[NT]
//   pwf[16] pwb[16] rfw[16] rf[NT]
// ---------------------------------------------------------------------------
template <typename T>
struct LineTab {
    const T *lm, *iu, *cm, *z, *wf, *wb, *qf, *qb, *pwf, *pwb, *rfw, *rf;
    T inv_den;  // 1 / (1 + v.z)
    T bg;       // beta_corner / gamma
    T iu_last;  // iu_{M-1}
    T na, nc;   // -a, -c: the negated off-diagonals (used by the compact form)
    int cyclic;
    int M;
    // A time-dependent operator (constant on each slice): slice n's tables
    // sit sstride elements after slice n-1's, and its scalars (inv_den, bg,
    // iu_last, na, nc and the FP32 step's diffusion coefficient) at
    // sscal[kSliceScalars * n ..].  sstride 0: one table for every slice.
    long sstride;
    const T *sscal;
};
constexpr int kSliceScalars = 6;

inline size_t line_tab_elems(int NT, int C) { return (size_t)(4 * C + 2 * kScanConsts + 3) * NT + 3 * kMaxWaves; }

template <typename T>
inline LineTab<T> line_tab_view(const T *base, int NT, int C)
{
    LineTab<T> tb{};
    size_t o = 0;
    const size_t pc = (size_t)C * NT;
    tb.lm = base + o; o += pc;
    tb.iu = base + o; o += pc;
    tb.cm = base + o; o += pc;
    tb.z = base + o; o += pc;
    tb.wf = base + o; o += (size_t)kScanConsts * NT;
    tb.wb = base + o; o += (size_t)kScanConsts * NT;
    tb.qf = base + o; o += NT;
    tb.qb = base + o; o += NT;
    tb.pwf = base + o; o += kMaxWaves;
    tb.pwb = base + o; o += kMaxWaves;
    tb.rfw = base + o; o += kMaxWaves;
    tb.rf = base + o;
    return tb;
}

// Supported (threads per line, points per thread) shapes of the 1D solver.
struct LineShape {
    int NT, C;
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
enum { SCHEME_IE = 0, SCHEME_CN = 1, SCHEME_ADI = 2 };

// Slice layouts of the 1D kernels: natural (point j at j, stride M) or
// chunked (stride NT*C, zero padding), see fine1d.hip.  In the chunked layout
// thread t's points t*C .. t*C+C-1 are stored in groups of P = chunk_width(C)
// consecutive points, group g of every thread side by side:
//   point t*C + k  at  (k / P) * P * NT + P * t + k % P.
// With P = 2 every access moves 16 bytes per lane and a wavefront's accesses
// are contiguous.
constexpr int chunk_width(int C) { return C % 2 == 0 ? 2 : 1; }
constexpr long chunk_pos(int NT, int C, long t, long k)
{
    return (k / chunk_width(C)) * chunk_width(C) * NT + chunk_width(C) * t + k % chunk_width(C);
}
//
// Fine apply, 1D, FP64 state.  y_0 = lam_0, y_n = lam_n - F(lam_{n-1}); raw: y_n = F(lam_n);
// last_only: y_{N-1} = F(lam_{N-1}) only.
hipError_t launch_fine1d_f64(LineShape sh, const LineTab<double> &tb, const double *lam, double *y,
                             int N, int M, int m, int scheme, int raw, int last_only, bool chunked,
                             hipStream_t st);

// Fine apply, 1D, FP32 state and arithmetic in increment form (see line1d.hpp);
// lam and y stay FP64.  pd, pa, pr: dt L u = pd (u_{j-1} - 2u_j + u_{j+1}) + pa (u_{j-1} - u_{j+1}) - pr u_j.
hipError_t launch_fine1d_f32(LineShape sh, const LineTab<float> &tb, const double *lam, double *y, int N,
                             int M, int m, float pd, float pa, float pr, int periodic, int raw, int last_only,
                             bool chunked, hipStream_t st);

// Coarse sweep, 1D, FP64: z_0 = v_0, z_n = v_n + G(z_{n-1}).
hipError_t launch_sweep1d_f64(LineShape sh, const LineTab<double> &tb, const double *v, double *z,
                              int N, int M, int c, int scheme, bool chunked, hipStream_t st);

// Layout conversions between natural [N][M] and chunked [N][NT*C] slices.
hipError_t launch_to_chunked(const double *nat, double *chk, int N, int M, int NT, int C, hipStream_t st);
hipError_t launch_from_chunked(const double *chk, double *nat, int N, int M, int NT, int C, hipStream_t st);

// ---------------------------------------------------------------------------
// 2D PR-ADI half steps (adi2d.hip)
// ---------------------------------------------------------------------------
// Row-constant tables of the y-direction solver for NS segments of CY rows
// (pads: lm = 1, iu = 0, cm = 0) and the per-segment products of lm and cm.
// Blob layout: lm[NR] iu[NR] cm[NR] pwf[32] pwb[32].
constexpr int kMaxSegs = 32;
struct ColTab {
    const double *lm, *iu, *cm, *pwf, *pwb;
};
inline size_t col_tab_elems(int nr) { return 3 * (size_t)nr + 2 * kMaxSegs; }
inline ColTab col_tab_view(const double *base, int nr)
{
    return ColTab{base, base + nr, base + 2 * (size_t)nr, base + 3 * (size_t)nr, base + 3 * (size_t)nr + kMaxSegs};
}
// x: a row on XW wavefronts, cx points per thread (64*XW*cx >= Mx); y: WY
// waves, each with SEG row segments of CY rows (64/SEG columns per
// workgroup).
struct AdiShape {
    int cx, wy, cy, seg, xw;
};
// A field buffer of either precision.
struct AdiBuf {
    float *f;
    double *d;
    bool f32;
};
// pre: each solved row is stored as the y half step's
// right-hand side (I + theta Lx) u* (ex2, ed2: that step's explicit
// coefficients) instead of u*; the y launch then takes pre as well.
hipError_t launch_adi_x(const AdiShape &sh, const LineTab<double> &tb, AdiBuf in, long in_off, AdiBuf out,
                        long out_off, int nslices, int Mx, int My, int R, double ex, double ed, hipStream_t st,
                        bool pre = false, double ex2 = 0.0, double ed2 = 0.0);
// FP64 y half step with one column per wavefront (columns of at most 512
// rows, 64*cy >= My; tb: the line tables of a column, shape {64, cy}), for
// the single-slice steps of the coarse sweep; cw (1, 2 or 4) columns per block.
// pre: `in` holds the right-hand side (I + theta Lx) u*, as launch_adi_x_pre
// stores it (no neighbour columns are read).
hipError_t launch_adi_yc(int cw, int cy, const LineTab<double> &tb, const double *in, long in_off, double *out,
                         long out_off, const double *base, long base_off, double sign, int nslices, int Mx, int My,
                         double ex, double ed, hipStream_t st, bool pre = false);
// FP64 x half step of one slice (rows of at most 512 points, one wave per
// row) that stores the next y half step's right-hand side (I + theta Lx) u*
// (coefficients ex2, ed2) instead of u*.
hipError_t launch_adi_x_pre(const AdiShape &sh, const LineTab<double> &tb, const double *in, long in_off,
                            double *out, int Mx, int My, double ex, double ed, double ex2, double ed2,
                            hipStream_t st);
// pre: `in` holds the right-hand side stored by a pre launch of the x half
// step, so no neighbour column is read.
hipError_t launch_adi_y(const AdiShape &sh, const ColTab &tb, AdiBuf in, long in_off, AdiBuf out, long out_off,
                        const double *base, long base_off, double sign, int nslices, int Mx, int My, double ex,
                        double ed, hipStream_t st, bool pre = false);

// Krylov block-vector kernels (krylov.hip).  n = total number of doubles.
// Segmented dot products: for each slice s and pair q < nq,
//   part[(q*N + s)*bps + b] = partial sum of a_q[s,:] . b_q[s,:] over block b.
struct DotPairs {
    const double *a[4];
    const double *b[4];
};
struct RedOut {
    double dot[4];   // w * sum over slices (fixed order)
    double nmax[4];  // max over slices of sqrt(w * slice sum)
};
// A context's reduction outputs: slot 0 for reductions read back one by one,
// slots 1..4 for pit_solve's one-sync iteration (dr; ks, kk, |S|; rho_new and
// |R| in two alternating slots), slot 5 for a rho set by the host.
constexpr int kRedSlots = 6;
hipError_t launch_seg_dots(const DotPairs &pr, int nq, int N, long npts, int bps, double *part,
                           double w, RedOut *out, hipStream_t st);
// S = R - alpha*D
hipError_t launch_axpby(double *out, const double *x, double a, const double *y, double b, long n,
                        hipStream_t st);
// X += alpha*P + omega*S; R = S - omega*K
hipError_t launch_update_xr(double *X, double *R, const double *P, const double *S, const double *K,
                            double alpha, double omega, long n, hipStream_t st);
// P = R + beta*(P - omega*D)
hipError_t launch_update_p(double *P, const double *R, const double *D, double beta, double omega,
                           long n, hipStream_t st);
// The same updates with the scalars read on the device from reduction outputs:
// rho = rho->dot[rho_idx], dr = A->dot[0], ks = B->dot[0], kk = B->dot[1],
// rho_new = C->dot[0].  update_xr / update_p change nothing when dr, kk or
// omega is exactly 0 (the host takes those branches).
struct DevScalars {
    const RedOut *rho;
    int rho_idx;
    const RedOut *A, *B, *C;
};
hipError_t launch_axpby_dev(double *S, const double *R, const double *D, const DevScalars &s, long n,
                            hipStream_t st);
hipError_t launch_update_xr_dev(double *X, double *R, const double *P, const double *S, const double *K,
                                const DevScalars &s, long n, hipStream_t st);
hipError_t launch_update_p_dev(double *P, const double *R, const double *D, const DevScalars &s, long n,
                               hipStream_t st);
// out = B - in, B = (u0, 0, ..); first slice uses u0
hipError_t launch_b_minus(double *out, const double *in, const double *u0, long npts, long n,
                          hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, long n, hipStream_t st);
hipError_t launch_fill0(double *dst, long n, hipStream_t st);

// ---------------------------------------------------------------------------
// Multi-instance launches (batched solves, batch.cpp).
//
// Every 1D instance of a batch keeps a device descriptor; a launch covers the
// instances listed in a Group.  Block b of a launch belongs to the listed
// instance k with first[k] <= b < first[k+1] (found by binary search over the
// count+1 prefix), so instances of different sizes share one launch.  The
// per-element and per-slice arithmetic is the single-instance kernels' own
// (shared device functions), so an instance's result does not depend on the
// other instances of the launch.
// ---------------------------------------------------------------------------
// Block vectors of a batched instance, in the chunked layout, vector q at
// vec + q*N*ld.
enum { VEC_R = 0, VEC_RT = 1, VEC_P = 2, VEC_D = 3, VEC_S = 4, VEC_K = 5, VEC_TM = 6, VEC_X = 7, VEC_COUNT = 8 };

struct Inst1d {
    LineTab<double> tf;   // fine step tables, FP64 form
    LineTab<float> tf32;  // fine step tables, FP32 increment form
    LineTab<double> tc;   // coarse step tables
    double *vec;          // VEC_COUNT block vectors
    double *part;         // partial sums of the segmented dots (4*N*bps)
    long ld;              // slice stride (NT*C of the fine line shape)
    int N, M, m, c, bps;
    double w;             // h^d, the weight of the discrete L2 product
    float pd, pa, pr;     // FP32 fine step: dt nu/h^2, dt a/(2h), dt r
    int periodic;
};

struct Group {
    const Inst1d *inst;   // descriptors of all instances (device)
    const int *list;      // descriptor index of each listed instance
    const int *first;     // block prefix, count+1 entries
    const int *aux;       // per listed instance: fine/sweep {vin, vout}; dots {nq, a[4], b[4]}; vec {op}
    const double *scal;   // 4 scalars per listed instance: alpha, omega, beta, spare
    RedOut *red;          // reduction result per listed instance
    int count;
};
constexpr int kDotsAux = 9;

__device__ __forceinline__ int group_find(const int *first, int count, int b)
{
    int lo = 0, hi = count;  // first[lo] <= b < first[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Fine apply y = (lam_n - F(lam_{n-1}))_n of vector aux[2k] into vector
// aux[2k+1] for the listed instances (all of line shape sh); nblocks = the sum
// of their N.
hipError_t launch_fine1d_multi(LineShape sh, int fine32, int scheme, const Group &g, int nblocks, hipStream_t st);
// Coarse sweep of vector aux[2k] into aux[2k+1], one block per listed instance.
hipError_t launch_sweep1d_multi(LineShape sh, int scheme, bool per_slice, const Group &g, hipStream_t st);
// Segmented dots of aux[9k] vector pairs (aux[9k+1+q], aux[9k+5+q]) per
// listed instance; g.first is the prefix of bps*N; results into g.red[k].
hipError_t launch_dots_multi(const Group &g, int nblocks, hipStream_t st);
// Element-wise updates per listed instance; g.first is the prefix of the
// blocks given to each instance (kVecMultiSpan doubles per block).
constexpr int kVecMultiSpan = 256 * 8;
enum { VOP_S_AXPY = 0, VOP_UPDATE_XR = 1, VOP_UPDATE_P = 2 };
// (op = aux[k])
hipError_t launch_vec_multi(const Group &g, int nblocks, hipStream_t st);

}  // namespace pit
