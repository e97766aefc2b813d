// Private host-side declarations of libpitsbicg: the context and what the
// solver drivers (pitsbicg.cpp, batch.cpp) share.  Not part of the ABI.
#pragma once

#include "../../include/pitsbicg.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "pit_internal.hpp"
#include "vel2d.hpp"

namespace pit {

// Records a HIP error code for pit_last_hip_error (per calling thread).
void set_last_hip(int code);

#define PIT_HIP(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) {               \
            ::pit::set_last_hip((int)e_);     \
            return PIT_EHIP;                  \
        }                                     \
    } while (0)

// One slice of `len` values written (add = 0) or added (add = 1) into `count`
// consecutive slices (krylov.hip).
hipError_t launch_repeat(double *dst, const double *src, long len, long count, int add, hipStream_t st);
// X_s += w[s * wstride] c for the N slices (len points each) of X.
hipError_t launch_slice_axpy(double *X, const double *c, const double *w, long wstride, long len, int N,
                             hipStream_t st);

constexpr size_t kAlign = 256;
constexpr int kSolveVectors = 8;  // R, shadow R, P, D, S, K, temporary, iterate
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Host-side description of one line operator A = I - theta*L.
struct LineHost {
    LineShape sh{0, 0};
    int M = 0;
    int cyclic = 0;
    double inv_den = 0.0, bg = 0.0, iu_last = 0.0;
    double a = 0.0, c = 0.0;  // off-diagonals of the line matrix
    std::vector<double> blob;  // layout of line_tab_view
    std::vector<float> blob32; // the same tables rounded to FP32
};

}  // namespace pit

using namespace pit;  // pit_ctx below is in the global namespace (the ABI type)

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct pit_ctx {
    pit_problem pb;
    int N = 0, m = 0;
    pit_stepper fine{}, coarse{};
    int npts = 0;
    double hx = 0, hy = 0, w = 0, DT = 0;
    // 1D line operators
    LineHost lf;  // fine step matrix
    LineHost lc;  // coarse step matrix
    // workspace layout (byte offsets)
    size_t off_tf = 0, off_tf32 = 0, off_tc = 0, off_vec = 0, off_part = 0, off_red = 0, total = 0;
    // increment-form stencil of the FP32 fine propagator, each part rounded on its own:
    // dt L u = pd (u_{j-1} - 2u_j + u_{j+1}) + pa (u_{j-1} - u_{j+1}) - pr u_j
    float pd = 0.f, pa = 0.f, pr = 0.f;
    int bps = 1;
    // bound workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;

    // 2D PR-ADI: x tables (64 lanes x cx points per row) and y row tables,
    // fine (theta = dt/2) and coarse (theta = DT/(2c)); explicit-part
    // coefficients: the x half step applies (I + theta Ly), the y half step
    // (I + theta Lx), each as ed*u + ex*(sum of the two neighbours).
    AdiShape ash{0, 0, 0, 0, 1};
    LineHost axf, axc;
    std::vector<double> ayf, ayc;
    double fx_ex = 0, fx_ed = 0, fy_ex = 0, fy_ed = 0, cx_ex = 0, cx_ed = 0, cy_ex = 0, cy_ed = 0;
    size_t off_axf = 0, off_axc = 0, off_ayf = 0, off_ayc = 0, off_ubuf = 0, off_sbuf = 0, off_ctmp = 0;
    int adi_R = 32;  // rows per wavefront in the fine x half step
    // coarse step, columns of at most 512 rows: line tables of one column
    // (shape {64, ycc}) for the one-column-per-wave y half step of the sweep
    LineHost aycl;
    int ycc = 0;  // 0: not built (taller columns, or PIT_ADI_YC=0)
    int ycw = 4;  // columns per workgroup of that kernel
    bool ypre = false;  // its right-hand side formed by the x half step
    bool fpre = false;  // the same in the fine apply
    size_t off_aycl = 0;
    // Source constant in time (host copy; empty: none) and, in the workspace,
    // the source (natural layout) and the forced response b = F(0) of one
    // slice in the working layout (1D chunked) and in the natural layout.
    std::vector<double> src;
    size_t off_src = 0, off_bf = 0, off_bfn = 0;
    bool has_src() const { return !src.empty(); }
    double *srcdev() const { return reinterpret_cast<double *>(ws + off_src); }
    double *bf() const { return reinterpret_cast<double *>(ws + off_bf); }
    double *bfn() const { return reinterpret_cast<double *>(ws + off_bfn); }
    // Separable source g(t) h(x) (src holds h): g at the fine step times
    // (N m + 1 values; empty: f constant in time) and, behind the base
    // workspace (base_total bytes), the forced responses b_n of all N slices
    // (natural layout) and the per-step source weights (N m values).
    std::vector<double> gt;
    size_t base_total = 0, off_bft = 0, off_gw = 0;
    bool src_t() const { return has_src() && !gt.empty(); }
    double *bft() const { return reinterpret_cast<double *>(ws + off_bft); }
    double *gw() const { return reinterpret_cast<double *>(ws + off_gw); }
    // Time-dependent operator, constant on each slice (1D): the diffusion
    // coefficient of slice n is nu * nus[n].  Per-slice fine, coarse and FP32
    // fine tables (slice n at n times the stride) and per-slice scalars
    // (kSliceScalars each) sit behind the rest of the workspace.
    std::vector<double> nus;
    bool nu_t() const { return !nus.empty(); }
    std::vector<double> tft, tct, scf, scc;
    std::vector<float> tf32t, scf32;
    long str_f = 0, str_c = 0;
    size_t off_tft = 0, off_tct = 0, off_tf32t = 0, off_scf = 0, off_scc = 0, off_scf32 = 0;
    // 2D with a velocity field: per-line tables of the fine and coarse PR-ADI
    // steps (layout of vel_tab_view), the y half-step's forward values for
    // all slices (wbuf) and for one slice (vwk).
    bool vel = false;
    std::vector<double> vtf, vtc;
    double vf_xdi = 0, vf_ydi = 0, vc_xdi = 0, vc_ydi = 0;
    size_t off_vtf = 0, off_vtc = 0, off_wbuf = 0, off_vwk = 0;
    VelTab vtab(bool fine_step) const
    {
        const double *b = reinterpret_cast<const double *>(ws + (fine_step ? off_vtf : off_vtc));
        return vel_tab_view(b, pb.M[0], pb.M[1], fine_step ? vf_xdi : vc_xdi, fine_step ? vf_ydi : vc_ydi,
                            (fine_step ? fine.scheme : coarse.scheme) == PIT_ADI_PR);
    }
    double *wbuf() const { return reinterpret_cast<double *>(ws + off_wbuf); }
    double *vwk() const { return reinterpret_cast<double *>(ws + off_vwk); }
    // 2D: the launch sequences of the fine apply (2m launches) and of the
    // coarse sweep (2(N-1)c launches) captured as HIP graphs, one per
    // (operation, input, output), replayed on the caller's stream
    struct Graph {
        int op;
        const void *in;
        void *out;
        int raw, last;
        hipGraphExec_t exec;
    };
    mutable std::vector<Graph> graphs;
    mutable hipStream_t capture = nullptr;
    // pinned host copy of the reduction results read by pit_solve and
    // pit_parareal (allocated at the first solve)
    RedOut *red_pin = nullptr;
    void drop_graphs() const;
    ~pit_ctx();
    bool dim2() const { return pb.dim == 2; }
    AdiBuf fbuf(size_t off) const
    {
        AdiBuf b{nullptr, nullptr, fine32()};
        if (b.f32) b.f = reinterpret_cast<float *>(ws + off);
        else b.d = reinterpret_cast<double *>(ws + off);
        return b;
    }
    double *ctmp(int i) const { return reinterpret_cast<double *>(ws + off_ctmp) + (size_t)i * npts; }

    long ld = 0;  // slice stride of the block vectors inside pit_solve (1D: chunked NT*C, 2D: npts)
    long nt() const { return (long)N * npts; }
    long ntc() const { return (long)N * ld; }
    double *vec(int i) const { return reinterpret_cast<double *>(ws + off_vec) + (size_t)i * ntc(); }
    double *part() const { return reinterpret_cast<double *>(ws + off_part); }
    RedOut *red(int slot = 0) const { return reinterpret_cast<RedOut *>(ws + off_red) + slot; }
    LineTab<float> tab32(const LineHost &L, size_t off) const
    {
        if (nu_t()) {  // per-slice tables: slice 0's view with the stride
            LineTab<float> t = line_tab_view<float>(reinterpret_cast<const float *>(ws + off_tf32t), L.sh.NT, L.sh.C);
            t.cyclic = L.cyclic;
            t.M = L.M;
            t.sstride = str_f;
            t.sscal = reinterpret_cast<const float *>(ws + off_scf32);
            return t;
        }
        LineTab<float> t = line_tab_view<float>(reinterpret_cast<const float *>(ws + off), L.sh.NT, L.sh.C);
        t.inv_den = (float)L.inv_den;
        t.bg = (float)L.bg;
        t.iu_last = (float)L.iu_last;
        t.na = (float)-L.a;
        t.nc = (float)-L.c;
        t.cyclic = L.cyclic;
        t.M = L.M;
        return t;
    }
    bool fine32() const { return fine.prec == PIT_F32; }
    LineTab<double> tab(const LineHost &L, size_t off) const
    {
        if (nu_t()) {  // per-slice tables: slice 0's view with the stride
            const bool fine_tab = &L == &lf;
            LineTab<double> t = line_tab_view<double>(
                reinterpret_cast<const double *>(ws + (fine_tab ? off_tft : off_tct)), L.sh.NT, L.sh.C);
            t.cyclic = L.cyclic;
            t.M = L.M;
            t.sstride = fine_tab ? str_f : str_c;
            t.sscal = reinterpret_cast<const double *>(ws + (fine_tab ? off_scf : off_scc));
            return t;
        }
        LineTab<double> t = line_tab_view<double>(reinterpret_cast<const double *>(ws + off), L.sh.NT, L.sh.C);
        t.inv_den = L.inv_den;
        t.bg = L.bg;
        t.iu_last = L.iu_last;
        t.na = -L.a;
        t.nc = -L.c;
        t.cyclic = L.cyclic;
        t.M = L.M;
        return t;
    }
};

namespace pit {

// The operators on block vectors of stride ld (chunked inside the solvers in 1D).
hipError_t op_apply(const pit_ctx *c, const double *lam, double *y, int raw, int last, bool internal, hipStream_t st);
hipError_t op_sweep(const pit_ctx *c, const double *v, double *z, bool internal, hipStream_t st);
// pit_coarse_sweep on natural-layout vectors, launched directly (no graph),
// with every temporary taken from `stage` (sweep_staging_bytes(c) bytes,
// 8-byte aligned): 1D the chunked copies of v and z, 2D one-slice fields.
hipError_t sweep_staged(const pit_ctx *c, const double *v, double *z, double *stage, hipStream_t st);
size_t sweep_staging_bytes(const pit_ctx *c);
// With a source: slices 1..N-1 of B (working layout) become b.  No-op without one.
hipError_t fill_forced(const pit_ctx *c, double *B, hipStream_t st);

}  // namespace pit
