// 2D Peaceman-Rachford ADI half steps (Dirichlet-0, constant coefficients).
//
// One PR-ADI step with theta = dt/2 (Lx, Ly: nu*D2 - r/2 along each axis):
//   x half step:  (I - theta Lx) u* = (I + theta Ly) u     solved along rows
//   y half step:  (I - theta Ly) u' = (I + theta Lx) u*    solved along columns
// Every slice of a block vector is independent, so each launch covers all the
// slices it is given.  What passes between the half steps is stored in S
// (float for the FP32 fine propagator, double otherwise); the arithmetic is
// FP64.  In the fine apply and the coarse sweep the x half step stores the y
// half step's right-hand side (I + theta Lx) u* rather than u* (PRE).
//
// x half step: one wavefront per strip of R rows (rows of more than 512
// points: a wavefront pair), lane l owns the x-points l*C .. l*C+C-1 of the
// row, the row solve is the register-resident in-wave line solver (no LDS, no
// barrier on one wave).  The y stencil uses a rolling window of three rows
// held in rotating registers (no copies, so the row loaded ahead stays in
// flight while the current row is solved).
//
// y half step: a workgroup owns 64/SEG columns of one slice; each wave holds
// SEG row segments of CY rows, one column per lane.  Each lane's tridiagonal
// recurrence along y runs locally with one LDS exchange of the per-lane
// carries per direction (two barriers per half step); the row constants are
// the same for every column and are read from LDS.  The coarse sweep's
// single slice uses a one-column-per-wavefront form (k_adi_yc).
#include "line1d.hpp"

namespace pit {

template <typename S>
__device__ __forceinline__ double to_d(S v)
{
    return (double)v;
}

// Buffer addressing: a scalar descriptor per slice, the row offset in a
// scalar register and only the lane's column offset in a vector register.
// Descriptor word 3 (0x00020000) selects raw 32-bit element access on CDNA.
// The range check covers the vector offset only (the scalar offset is added
// unchecked): a lane whose vector offset is at or past the descriptor's byte
// count reads 0 and its store is dropped, so callers keep the scalar offset
// inside the buffer and mark a lane or row out of range through the vector
// offset.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc make_rsrc(const void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(Rsrc r, int voff, int soff);
template <>
__device__ __forceinline__ float bload<float>(Rsrc r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(Rsrc r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, Rsrc r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, Rsrc r, int voff, int soff)
{
    using U2 = __attribute__((ext_vector_type(2))) unsigned;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, voff, soff, 0);
}

// ---------------------------------------------------------------------------
// x half step
// ---------------------------------------------------------------------------
// Lane l's C consecutive values of row j (clamped into the slice).  When
// every lane's chunk is inside the row and 16-byte aligned (vec), the chunk
// is read with 16-byte loads: the address unit handles a 64-lane instruction
// in a fixed number of cycles, so wide accesses move 4x the bytes per cycle.
template <int C, typename SIN>
__device__ __forceinline__ void load_row(const SIN *__restrict__ slice, int j, int My, int Mx, int lane, bool vec,
                                         SIN (&r)[C])
{
    const SIN *row = slice + (size_t)min(max(j, 0), My - 1) * Mx;
    constexpr int V = 16 / sizeof(SIN);
    if constexpr (C % V == 0) {
        if (vec) {
            using VT = __attribute__((ext_vector_type(V))) SIN;
            const VT *p = reinterpret_cast<const VT *>(row + lane * C);
#pragma unroll
            for (int q = 0; q < C / V; ++q) {
                const VT x = p[q];
#pragma unroll
                for (int i = 0; i < V; ++i) r[q * V + i] = x[i];
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) r[k] = row[min(lane * C + k, Mx - 1)];
}

// PRE: the row is stored as the next y half step's right-hand side
// (I + theta Lx) u* (ex2, ed2) instead of u*, formed from the solved row with
// the same operations, in the same order, as the y kernel would form it from
// the stored u* (left + right neighbour, zero outside the row).  With FP64
// fields the result is the same to the bit; with FP32 fields this value is
// the one rounded to FP32 in place of u*.  A row on two wavefronts
// (NT = 128) swaps the points beside the wave edge through xch (two LDS
// slots) and one barrier.
template <int NT, int C, typename SIN, typename SOUT, bool PRE = false>
__device__ __forceinline__ void x_row(LineSolver<double, NT, C, false> &LS, const SIN (&pv)[C], const SIN (&cu)[C],
                                      const SIN (&nx)[C], int j, int My, int Mx, int lane, bool vec, double ex,
                                      double ed, SOUT *__restrict__ oslice, double ex2 = 0.0, double ed2 = 0.0,
                                      double *xch = nullptr)
{
    const double fp = (j > 0) ? 1.0 : 0.0, fn = (j + 1 < My) ? 1.0 : 0.0;
    double d[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double v = fma(ed, to_d(cu[k]), ex * fma(fp, to_d(pv[k]), fn * to_d(nx[k])));
        d[k] = (lane * C + k < Mx) ? v : 0.0;
    }
    LS.solve(d);
    if constexpr (PRE) {
        static_assert(NT == kWave || NT == 2 * kWave, "one or two waves per row");
        double dl = dpp<0x138>(d[C - 1]);  // lane-1's last point (lane 0 reads 0: the boundary)
        double dr = dpp<0x130>(d[0]);      // lane+1's first point (lane 63 reads 0)
        if constexpr (NT == 2 * kWave) {
            // wave 0's last point and wave 1's first cross through LDS; the
            // previous row's reads finished before this row's solve passed
            // its barriers
            if (lane == kWave - 1) xch[0] = d[C - 1];
            if (lane == kWave) xch[1] = d[0];
            __syncthreads();
            if (lane == kWave) dl = xch[0];
            if (lane == kWave - 1) dr = xch[1];
        }
        double rr[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const double left = (k == 0) ? dl : d[k - 1];
            const double right = (lane * C + k + 1 < Mx) ? ((k == C - 1) ? dr : d[k + 1]) : 0.0;
            rr[k] = fma(ed2, d[k], ex2 * (left + right));
        }
#pragma unroll
        for (int k = 0; k < C; ++k) d[k] = rr[k];
    }
    SOUT *row = oslice + (size_t)j * Mx;
    constexpr int V = 16 / sizeof(SOUT);
    if constexpr (C % V == 0) {
        if (vec) {
            using VT = __attribute__((ext_vector_type(V))) SOUT;
            VT *p = reinterpret_cast<VT *>(row + lane * C);
#pragma unroll
            for (int q = 0; q < C / V; ++q) {
                VT x;
#pragma unroll
                for (int i = 0; i < V; ++i) x[i] = (SOUT)d[q * V + i];
                p[q] = x;
            }
            return;
        }
    }
    if (lane * C + C <= Mx) {
#pragma unroll
        for (int k = 0; k < C; ++k) row[lane * C + k] = (SOUT)d[k];
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k)
            if (lane * C + k < Mx) row[lane * C + k] = (SOUT)d[k];
    }
}

// Workgroups are dealt to the 8 XCDs round-robin by block id, and each XCD
// has its own L2.  Renumbering the blocks so that XCD x runs one contiguous
// range of logical blocks keeps neighbouring strips (which share halo rows or
// columns) on one L2, so a halo line is fetched from HBM once.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + k;
}

// A row of Mx points is solved by XW wavefronts (NT = 64*XW threads, C points
// each).  XW = 1: blocks of 4 independent waves, wave g handles strip g of
// all nslices*strips strips (strip: R consecutive rows of one slice).  XW = 2
// (rows wider than 512 points): blocks of one wave pair, block g handles strip
// g, and the pair's line solves exchange their carries through LDS.  in/out
// slice s sits at in + (s + in_off)*npts.
// XW = 1 launches carry WPB independent waves per block: 4 over many
// slices, 1 for a single slice, where 4 would leave half the CUs without a
// row (512 rows: 128 blocks of 4 waves; 512 blocks of one measured 9% faster
// per coarse step).
template <int XW, int C, typename SIN, typename SOUT, int WPB = 4, bool PRE = false>
__global__ __launch_bounds__(XW == 1 ? 64 * WPB : 128) void k_adi_x(LineTab<double> tb, const SIN *__restrict__ in,
                                                                    long in_off, SOUT *__restrict__ out,
                                                                    long out_off, int nslices, int Mx, int My, int R,
                                                                    double ex, double ed, double ex2, double ed2)
{
    constexpr int NT = kWave * XW;
    __shared__ double lds[XW == 1 ? 1 : LineSolver<double, NT, C, false>::kLds];
    __shared__ double xch[XW == 2 && PRE ? 2 : 1];  // the wave-edge points of a pre-formed row
    poison_lds(lds, (int)(sizeof(lds) / sizeof(double)));
    const int lane = threadIdx.x & (NT - 1);  // thread of the row group
    const int strips = (My + R - 1) / R;
    // group-uniform indices in scalar registers, so row addresses stay scalar
    const int g = XW == 1 ? __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * WPB + threadIdx.x / kWave)
                          : xcd_block(blockIdx.x, gridDim.x);
    if (g >= nslices * strips) return;  // the whole group exits (a block for XW = 2); no barriers skipped
    const int s = g / strips, j0 = (g % strips) * R, j1 = min(j0 + R, My);
    const long npts = (long)Mx * My;
    const SIN *islice = in + (size_t)(s + in_off) * npts;
    SOUT *oslice = out + (size_t)(s + out_off) * npts;
    // 16-byte accesses when the row length keeps every thread's chunk aligned
    const bool vec = (Mx == NT * C) && (Mx * sizeof(SIN)) % 16 == 0 && (Mx * sizeof(SOUT)) % 16 == 0;
    LineSolver<double, NT, C, false> LS;
    LS.load(tb, XW == 1 ? nullptr : lds);
    // Five rotating row buffers: row r uses the buffers of rows r-1, r, r+1
    // while rows r+2 .. r+4 are in flight.  Rows past the strip's last halo
    // row jl are not read: a buffer that would hold one is only ever the
    // neighbour below the slice's last row, which enters with weight 0, so
    // it starts as zeros (a strip of one row reads three rows, not five).
    // Every thread of a group runs the same rows, so the solver's barriers
    // (XW = 2) match.
    SIN B[5][C];
    const int jl = min(j1, My - 1);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (j0 - 1 + q <= jl) {
            load_row<C>(islice, j0 - 1 + q, My, Mx, lane, vec, B[q]);
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) B[q][k] = SIN(0);
        }
    }
    for (int j = j0; j < j1; j += 5) {
#define PIT_XSTEP(u)                                                                                           \
    {                                                                                                          \
        const int r = j + (u);                                                                                 \
        if (r >= j1) break;                                                                                    \
        x_row<NT, C, SIN, SOUT, PRE>(LS, B[(u) % 5], B[((u) + 1) % 5], B[((u) + 2) % 5], r, My, Mx, lane, vec, \
                                     ex, ed, oslice, ex2, ed2, xch);                                            \
        if (r + 4 <= jl) load_row<C>(islice, r + 4, My, Mx, lane, vec, B[(u) % 5]);                            \
    }
        PIT_XSTEP(0) PIT_XSTEP(1) PIT_XSTEP(2) PIT_XSTEP(3) PIT_XSTEP(4)
#undef PIT_XSTEP
    }
}

// ---------------------------------------------------------------------------
// y half step
// ---------------------------------------------------------------------------
// grid: nslices * ceil(Mx/CW) blocks of WY waves, CW = 64/SEG columns per
// block.  A wave holds SEG row segments of CY rows: lane l works on column
// col0 + l % CW, segment g = SEG*w + l / CW (rows g*CY .. g*CY+CY-1), so
// WY*SEG*CY rows in all.  Epilogue EPI: 0 stores u', 1 stores base +
// sign*u' (FP64) -- the all-at-once apply's lam_n - F(...) and the coarse
// sweep's v_n + G(...).  PRE: `in` already holds the right-hand side
// (I + theta Lx) u* (formed by the x half step), so no halo column is read.
template <int WY, int CY, int SEG, typename SIN, typename SOUT, int EPI, bool PRE = false>
__global__ __launch_bounds__(WY * 64) void k_adi_y(ColTab tb, const SIN *__restrict__ in, long in_off,
                                                   SOUT *__restrict__ out, long out_off,
                                                   const double *__restrict__ base, long base_off, double sign,
                                                   int nslices, int Mx, int My, double ex, double ed)
{
    constexpr int CW = kWave / SEG, NS = WY * SEG, NR = NS * CY;
    static_assert(SEG == 1 || SEG == 2, "one or two segments per wave");
    static_assert(2 * CY <= kWave, "halo lanes");
    __shared__ double s_lm[NR], s_iu[NR], s_cm[NR];
    __shared__ double s_pf[NS], s_pb[NS];
    __shared__ double s_agg[2][NS][CW];
    poison_lds(s_lm, NR);
    poison_lds(s_iu, NR);
    poison_lds(s_cm, NR);
    poison_lds(s_pf, NS);
    poison_lds(s_pb, NS);
    poison_lds(&s_agg[0][0][0], 2 * NS * CW);
    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);  // wave-uniform (scalar)
    const int cl = lane % CW, sg = lane / CW;
    const int g = w * SEG + sg;  // this lane's row segment
    const int bx = (Mx + CW - 1) / CW;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk / bx, col0 = (blk % bx) * CW;
    for (int i = t; i < NR; i += WY * kWave) {
        s_lm[i] = tb.lm[i];
        s_iu[i] = tb.iu[i];
        s_cm[i] = tb.cm[i];
    }
    if (t < NS) {
        s_pf[t] = tb.pwf[t];
        s_pb[t] = tb.pwb[t];
    }
    __syncthreads();
    if (s >= nslices) return;  // uniform per block
    const long npts = (long)Mx * My;
    const int col = col0 + cl;
    const bool live = col < Mx;
    const Rsrc rin = make_rsrc(in + (size_t)(s + in_off) * npts, (unsigned)(npts * sizeof(SIN)));
    const int r0 = g * CY;
    constexpr int zi = sizeof(SIN), zo = sizeof(SOUT);
    // Out-of-range buffer reads return 0, which supplies the zeros the
    // stencil needs in lanes past the last column and for the Dirichlet
    // boundary values left and right of the slice.
    constexpr int kOut = 0x40000000;
    // With one segment per wave the row offset is wave-uniform (scalar) and
    // rows past the last one re-read the last row; with two the segment's
    // first row goes into the lane's offset and rows past the last one are
    // marked out of range there (read as 0, stores dropped).  Either way the
    // pad rows' table entries (lm 1, iu 0, cm 0) keep them out of the real
    // rows.
    const int vlane = live ? (col + (SEG == 1 ? 0 : r0 * Mx)) * zi : kOut;
    auto row_off = [&](int r, int v, int z) {  // (vector, scalar) offsets of row r0 + r
        if constexpr (SEG == 1) return int2{v, min(r0 + r, My - 1) * Mx * z};
        else return int2{(r0 + r < My) ? v : kOut, r * Mx * z};
    };
    auto in_row = [&](int r) {
        const int2 o = row_off(r, vlane, zi);
        return bload<SIN>(rin, o.x, o.y);
    };
    // The halo columns of the strip for this wave's SEG*CY rows: lane i <
    // SEG*CY of hv reads column col0-1 of the wave's i-th row, hv2 (or the
    // upper lanes of hv when SEG*CY <= 32) column col0+CW; row r's halo
    // values are then taken with readlane.  They are loaded after the strip's
    // rows: each halo load touches one cache line per row, and issued first
    // they held the row loads back in the wave's memory queue (the 512^2 fine
    // apply took 6.64 ms that way, 6.27 ms this way; 1024^2: 34.9, 33.6 ms).
    constexpr int HR = SEG * CY;  // halo rows per wave
    SIN hv, hv2;
    auto load_halos = [&] {
        const int wr0 = w * HR;
        const int i = lane % HR;
        const bool split = 2 * HR <= kWave;
        const int hc = (split && lane >= HR) ? col0 + CW : col0 - 1;
        hv = bload<SIN>(rin, (hc >= 0 && hc < Mx && wr0 + i < My) ? ((wr0 + i) * Mx + hc) * zi : kOut, 0);
        hv2 = hv;
        if constexpr (2 * HR > kWave) {
            const int hc2 = col0 + CW;
            hv2 = bload<SIN>(rin, (hc2 < Mx && wr0 + lane < My) ? ((wr0 + lane) * Mx + hc2) * zi : kOut, 0);
        }
    };

    // Right-hand side (I + theta Lx) u* for this lane's column segment; the
    // x-neighbours inside the strip come from DPP lane shifts of the stored
    // values.  Every lane runs the cross-lane reads (DPP and readlane are not
    // speculatable, so inside a conditional they would become a divergent
    // branch); the strip-edge lanes then select the halo values.
    auto rhs = [&](SIN v, int r) {
        if constexpr (PRE) return to_d(v);
        SIN hl, hr;
        if constexpr (SEG == 1) {
            hl = readlane(hv, r);
            hr = (2 * HR > kWave) ? readlane(hv2, r) : readlane(hv, HR + (r % (kWave - HR + 1)));
        } else {
            // segment sg's row r is the wave's row sg*CY + r; its left halo sits
            // in that lane of hv, its right halo in the same lane of hv2 or, when
            // both fit one load, HR lanes further up in hv
            constexpr bool split = 2 * HR <= kWave;
            const SIN l0 = readlane(hv, r), l1 = readlane(hv, CY + r);
            const SIN r0v = split ? readlane(hv, HR + r) : readlane(hv2, r);
            const SIN r1v = split ? readlane(hv, HR + CY + r) : readlane(hv2, CY + r);
            hl = sg ? l1 : l0;
            hr = sg ? r1v : r0v;
        }
        const SIN sl = dpp<0x138>(v), sr = dpp<0x130>(v);
        const SIN vl = (cl == 0) ? hl : sl;
        const SIN vr = (cl == CW - 1) ? hr : sr;
        return fma(ed, to_d(v), ex * (to_d(vl) + to_d(vr)));
    };
    double d[CY];
    if constexpr (sizeof(SIN) == sizeof(double)) {
        // FP64 input: load straight into d and form the right-hand side in
        // place (a separate copy of the rows would not fit in registers)
#pragma unroll
        for (int r = 0; r < CY; ++r) d[r] = in_row(r);
        if constexpr (!PRE) load_halos();
#pragma unroll
        for (int r = 0; r < CY; ++r) d[r] = rhs(d[r], r);
    } else {
        SIN raw[CY];
#pragma unroll
        for (int r = 0; r < CY; ++r) raw[r] = in_row(r);
        if constexpr (!PRE) load_halos();
#pragma unroll
        for (int r = 0; r < CY; ++r) d[r] = rhs(raw[r], r);
    }
    // forward elimination along y
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < CY; ++r) e = fma(s_lm[r0 + r], e, d[r]);
    s_agg[0][g][cl] = e;
    __syncthreads();
    double cw = 0.0;
    for (int q = 0; q < w * SEG + SEG - 1; ++q) {  // segments before g (predicated: g differs by half-wave)
        const double n = fma(s_pf[q], cw, s_agg[0][q][cl]);
        cw = (q < g) ? n : cw;
    }
    // FP32 fields: d[r] then holds y_r / u_r, the term both backward passes
    // add, formed once (the same product, so the same bits).  With FP64 fields
    // the extra live products cost the 8-wave block its second slot on a CU.
    constexpr bool PS = sizeof(SIN) == sizeof(float);
    double y = cw;
#pragma unroll
    for (int r = 0; r < CY; ++r) {
        y = fma(s_lm[r0 + r], y, d[r]);
        d[r] = PS ? s_iu[r0 + r] * y : y;
    }
    // back substitution along y
    const Rsrc rout = make_rsrc(out + (size_t)(s + out_off) * npts, (unsigned)(npts * zo));
    const Rsrc rbase = make_rsrc(EPI ? base + (size_t)(s + base_off) * npts : base, EPI ? (unsigned)(npts * 8) : 0u);
    const int vout = live ? (col + (SEG == 1 ? 0 : r0 * Mx)) * zo : kOut;
    const int vbase = live ? (col + (SEG == 1 ? 0 : r0 * Mx)) * 8 : kOut;
    // The epilogue's base rows are read PB rows ahead of the second backward
    // pass (the first PB before the backward exchange), so their latency is
    // hidden behind the recurrence instead of stalling every row.
    constexpr int PB = EPI ? (CY < 8 ? CY : ((SEG == 2 && WY == 16 && sizeof(SIN) == 8) ? 4 : 8)) : 1;
    auto base_row = [&](int r) {
        const int2 o = row_off(r, vbase, 8);
        return bload<double>(rbase, o.x, o.y);
    };
    double bq[PB];
    if constexpr (EPI) {
#pragma unroll
        for (int q = 0; q < PB; ++q) bq[q] = base_row(CY - 1 - q);
    }
    double bsum = 0.0;
#pragma unroll
    for (int r = CY - 1; r >= 0; --r) bsum = fma(s_cm[r0 + r], bsum, PS ? d[r] : s_iu[r0 + r] * d[r]);
    s_agg[1][g][cl] = bsum;
    __syncthreads();
    double cb = 0.0;
    for (int q = NS - 1; q > w * SEG; --q) {  // segments after g
        const double n = fma(s_pb[q], cb, s_agg[1][q][cl]);
        cb = (q > g) ? n : cb;
    }
    // second backward pass: each solution value is stored as it is produced
    double x = cb;
#pragma unroll
    for (int r = CY - 1; r >= 0; --r) {
        x = fma(s_cm[r0 + r], x, PS ? d[r] : s_iu[r0 + r] * d[r]);
        double o = x;
        if constexpr (EPI) {
            const int q = (CY - 1 - r) % PB;
            o = fma(sign, x, bq[q]);
            if (r - PB >= 0) bq[q] = base_row(r - PB);
        }
        if constexpr (SEG == 1) {
            if (r0 + r < My) bstore((SOUT)o, rout, vout, (r0 + r) * Mx * zo);  // wave-uniform branch
        } else {
            const int2 of = row_off(r, vout, zo);
            bstore((SOUT)o, rout, of.x, of.y);
        }
    }
}

// ---------------------------------------------------------------------------
// y half step, one column per wavefront (few slices: the coarse sweep)
// ---------------------------------------------------------------------------
// grid: nslices * ceil(Mx/CW) blocks of CW waves, for columns of at most 512
// rows.  With one slice the column-strip kernel above has only Mx/32
// workgroups; here a block owns CW columns.  It stages columns col0-1 ..
// col0+CW of its slice in LDS (row by row, so the loads are contiguous per
// row), wave w then forms the right-hand side of column col0+w from its two
// neighbours and solves it with the register-resident line solver (lane l
// holds rows l*C .. l*C+C-1; one wave per line, so no barrier inside the
// solve), and the solution goes back through LDS so that the stores and the
// epilogue's base reads are row-wise again.  In LDS a column keeps row r at
// (r % C)*64 + r / C: the 64 lanes of one access read consecutive slots.
// PRE: `in` already holds the right-hand side (I + theta Lx) u* (formed by
// the x half step), so only the block's own CW columns are staged and no
// neighbour column is read.
template <int CW, int C, typename SIN, typename SOUT, int EPI, bool PRE = false>
__global__ __launch_bounds__(CW * 64) void k_adi_yc(LineTab<double> tb, const SIN *__restrict__ in, long in_off,
                                                    SOUT *__restrict__ out, long out_off,
                                                    const double *__restrict__ base, long base_off, double sign,
                                                    int nslices, int Mx, int My, double ex, double ed)
{
    constexpr int H = PRE ? 0 : 1;  // halo columns on each side
    constexpr int L = kWave * C, TW = CW + 2 * H, NTH = CW * kWave;
    __shared__ double tile[TW * L];
    poison_lds(tile, TW * L);
    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);
    const int bx = (Mx + CW - 1) / CW;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk / bx, col0 = (blk % bx) * CW;
    if (s >= nslices) return;  // uniform per block, before any barrier
    const long npts = (long)Mx * My;
    const SIN *islice = in + (size_t)(s + in_off) * npts;
    auto slot = [](int r) { return (r % C) * kWave + r / C; };
    // stage the CW (+ 2 halo) columns (zeros left and right of the slice and
    // below its last row: the Dirichlet values and the solver's pad rows)
    // FP64 columns of an even-width slice (PAIR2, an even CW): a row's CW
    // values are CW/2 aligned pairs, each moved with one 16-byte access, for
    // the staging, the epilogue's base values and the stores.
    constexpr bool PAIR2 = TW == CW && CW % 2 == 0 && sizeof(SIN) == 8 && sizeof(SOUT) == 8;
    constexpr int NP = CW / 2 > 0 ? CW / 2 : 1;  // pairs per row
    const bool pair = PAIR2 && (Mx % 2) == 0;
    using D2 = __attribute__((ext_vector_type(2))) double;
    constexpr int kRow = (L * NP + NTH - 1) / NTH;  // pairs per thread in the pair form
    SOUT *oslice = out + (size_t)(s + out_off) * npts;
    const double *bslice = EPI ? base + (size_t)(s + base_off) * npts : nullptr;
    constexpr int kIn = (TW * L + NTH - 1) / NTH;
    constexpr int kOut = (CW * L + NTH - 1) / NTH;
    double bq[EPI ? (kOut > 2 * kRow ? kOut : 2 * kRow) : 1];
    if (PAIR2 && pair) {
        D2 v2[kRow];
#pragma unroll
        for (int q = 0; q < kRow; ++q) {
            const int i = q * NTH + t, r = i / NP, c = 2 * (i % NP);
            // with Mx even a pair is inside the row or wholly past it
            v2[q] = (r < L && r < My && col0 + c < Mx)
                        ? *reinterpret_cast<const D2 *>(islice + (size_t)r * Mx + col0 + c)
                        : D2{0.0, 0.0};
        }
#pragma unroll
        for (int q = 0; q < kRow; ++q) {
            const int i = q * NTH + t, r = i / NP, c = 2 * (i % NP);
            if (r < L) {
                tile[c * L + slot(r)] = v2[q].x;
                tile[(c + 1) * L + slot(r)] = v2[q].y;
            }
        }
        if constexpr (EPI) {
#pragma unroll
            for (int q = 0; q < kRow; ++q) {
                const int i = q * NTH + t, r = i / NP, c = 2 * (i % NP);
                const D2 b2 = (r < My && col0 + c < Mx)
                                  ? *reinterpret_cast<const D2 *>(bslice + (size_t)r * Mx + col0 + c)
                                  : D2{0.0, 0.0};
                bq[2 * q] = b2.x;
                bq[2 * q + 1] = b2.y;
            }
        }
    } else {
        double v[kIn];
#pragma unroll
        for (int q = 0; q < kIn; ++q) {
            const int i = q * NTH + t, r = i / TW, col = col0 - H + i % TW;
            v[q] = (i < TW * L && r < My && col >= 0 && col < Mx) ? to_d(islice[(size_t)r * Mx + col]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kIn; ++q) {
            const int i = q * NTH + t;
            if (i < TW * L) tile[(i % TW) * L + slot(i / TW)] = v[q];
        }
        // the epilogue's base values, read now so that their latency hides
        // behind the staging and the solve
        if constexpr (EPI) {
#pragma unroll
            for (int q = 0; q < kOut; ++q) {
                const int i = q * NTH + t, r = i / CW, col = col0 + i % CW;
                bq[q] = (r < My && col < Mx) ? bslice[(size_t)r * Mx + col] : 0.0;
            }
        }
    }
    LineSolver<double, kWave, C, false> LS;
    LS.load(tb, nullptr);
    __syncthreads();
    // right-hand side (I + theta Lx) u* of column col0 + w, then the solve
    double d[C];
    const int cc = w + H;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int q = k * kWave + lane;  // slot of row lane*C + k
        double u;
        if constexpr (PRE) u = tile[cc * L + q];
        else u = fma(ed, tile[cc * L + q], ex * (tile[(cc - 1) * L + q] + tile[(cc + 1) * L + q]));
        d[k] = (lane * C + k < My) ? u : 0.0;
    }
    LS.solve(d);
    __syncthreads();  // every wave has read its neighbours' columns
#pragma unroll
    for (int k = 0; k < C; ++k) tile[cc * L + k * kWave + lane] = d[k];
    __syncthreads();
    if (PAIR2 && pair) {
#pragma unroll
        for (int q = 0; q < kRow; ++q) {
            const int i = q * NTH + t, r = i / NP, c = 2 * (i % NP);
            if (r < My && col0 + c < Mx) {
                double x0 = tile[c * L + slot(r)], x1 = tile[(c + 1) * L + slot(r)];
                if constexpr (EPI) {
                    x0 = fma(sign, x0, bq[2 * q]);
                    x1 = fma(sign, x1, bq[2 * q + 1]);
                }
                *reinterpret_cast<D2 *>(oslice + (size_t)r * Mx + col0 + c) = D2{x0, x1};
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int i = q * NTH + t, r = i / CW, c = i % CW, col = col0 + c;
        if (r < My && col < Mx) {
            double x = tile[(c + H) * L + slot(r)];
            if constexpr (EPI) x = fma(sign, x, bq[q]);
            oslice[(size_t)r * Mx + col] = (SOUT)x;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define PIT_ADI_XC(X) X(1, 1) X(1, 2) X(1, 4) X(1, 8) X(2, 8)
#define PIT_ADI_YSHAPES(X) X(8, 16, 1) X(8, 32, 1) X(16, 32, 1) X(8, 32, 2) X(16, 32, 2) X(8, 16, 2) X(16, 16, 2)

template <typename SIN, typename SOUT>
static hipError_t adi_x_t(const AdiShape &sh, const LineTab<double> &tb, const SIN *in, long in_off, SOUT *out,
                          long out_off, int nslices, int Mx, int My, int R, double ex, double ed, bool pre,
                          double ex2, double ed2, hipStream_t st)
{
    const int strips = (My + R - 1) / R;
    const bool one = nslices == 1;  // one wave per block over a single slice
    const int blocks = sh.xw == 1 ? (one ? strips : (nslices * strips + 3) / 4) : nslices * strips;
#define X(XW_, C_)                                                                                              \
    if (sh.xw == XW_ && sh.cx == C_) {                                                                          \
        if (pre) {                                                                                              \
            if (XW_ == 1 && one)                                                                                \
                hipLaunchKernelGGL((k_adi_x<XW_, C_, SIN, SOUT, 1, true>), dim3(blocks), dim3(64), 0, st, tb,   \
                                   in, in_off, out, out_off, nslices, Mx, My, R, ex, ed, ex2, ed2);             \
            else                                                                                                \
                hipLaunchKernelGGL((k_adi_x<XW_, C_, SIN, SOUT, 4, true>), dim3(blocks),                        \
                                   dim3(XW_ == 1 ? 256 : 128), 0, st, tb, in, in_off, out, out_off, nslices, Mx, \
                                   My, R, ex, ed, ex2, ed2);                                                     \
            return hipGetLastError();                                                                           \
        }                                                                                                       \
        if (XW_ == 1 && one)                                                                                    \
            hipLaunchKernelGGL((k_adi_x<XW_, C_, SIN, SOUT, 1>), dim3(blocks), dim3(64), 0, st, tb, in, in_off,  \
                               out, out_off, nslices, Mx, My, R, ex, ed, 0.0, 0.0);                             \
        else                                                                                                    \
            hipLaunchKernelGGL((k_adi_x<XW_, C_, SIN, SOUT>), dim3(blocks), dim3(XW_ == 1 ? 256 : 128), 0, st,   \
                               tb, in, in_off, out, out_off, nslices, Mx, My, R, ex, ed, 0.0, 0.0);             \
        return hipGetLastError();                                                                               \
    }
    PIT_ADI_XC(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename SIN, typename SOUT, int EPI, bool PRE>
static hipError_t adi_y_t(const AdiShape &sh, const ColTab &tb, const SIN *in, long in_off, SOUT *out,
                          long out_off, const double *base, long base_off, double sign, int nslices, int Mx, int My,
                          double ex, double ed, hipStream_t st)
{
    const int cw = kWave / sh.seg;
    const int blocks = nslices * ((Mx + cw - 1) / cw);
#define X(WY_, CY_, SG_)                                                                                         \
    if (sh.wy == WY_ && sh.cy == CY_ && sh.seg == SG_) {                                                        \
        hipLaunchKernelGGL((k_adi_y<WY_, CY_, SG_, SIN, SOUT, EPI, PRE>), dim3(blocks), dim3(WY_ * 64), 0, st,  \
                           tb, in, in_off, out, out_off, base, base_off, sign, nslices, Mx, My, ex, ed);          \
        return hipGetLastError();                                                                                \
    }
    PIT_ADI_YSHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

template <int CW, typename SIN, typename SOUT, int EPI, bool PRE>
static hipError_t adi_yc_t(int cy, const LineTab<double> &tb, const SIN *in, long in_off, SOUT *out, long out_off,
                           const double *base, long base_off, double sign, int nslices, int Mx, int My, double ex,
                           double ed, hipStream_t st)
{
    const int blocks = nslices * ((Mx + CW - 1) / CW);
#define X(C_)                                                                                                  \
    if (cy == C_) {                                                                                            \
        hipLaunchKernelGGL((k_adi_yc<CW, C_, SIN, SOUT, EPI, PRE>), dim3(blocks), dim3(CW * 64), 0, st, tb, in, \
                           in_off, out, out_off, base, base_off, sign, nslices, Mx, My, ex, ed);               \
        return hipGetLastError();                                                                              \
    }
    X(1) X(2) X(4) X(8)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adi_yc(int cw, int cy, const LineTab<double> &tb, const double *in, long in_off, double *out,
                         long out_off, const double *base, long base_off, double sign, int nslices, int Mx, int My,
                         double ex, double ed, hipStream_t st, bool pre)
{
    if (64 * cy < My) return hipErrorInvalidValue;
#define Y(CW_, PRE_)                                                                                           \
    if (cw == CW_ && pre == PRE_) {                                                                            \
        if (base)                                                                                              \
            return adi_yc_t<CW_, double, double, 1, PRE_>(cy, tb, in, in_off, out, out_off, base, base_off,     \
                                                          sign, nslices, Mx, My, ex, ed, st);                  \
        return adi_yc_t<CW_, double, double, 0, PRE_>(cy, tb, in, in_off, out, out_off, nullptr, 0, 0.0,        \
                                                      nslices, Mx, My, ex, ed, st);                            \
    }
    Y(1, false) Y(2, false) Y(4, false) Y(1, true) Y(2, true) Y(4, true)
#undef Y
    return hipErrorInvalidValue;
}

hipError_t launch_adi_x_pre(const AdiShape &sh, const LineTab<double> &tb, const double *in, long in_off,
                            double *out, int Mx, int My, double ex, double ed, double ex2, double ed2,
                            hipStream_t st)
{
    if (sh.xw != 1) return hipErrorInvalidValue;
#define X(XW_, C_)                                                                                              \
    if (XW_ == 1 && sh.cx == C_) {                                                                              \
        hipLaunchKernelGGL((k_adi_x<1, C_, double, double, 1, true>), dim3(My), dim3(64), 0, st, tb, in, in_off, \
                           out, 0, 1, Mx, My, 1, ex, ed, ex2, ed2);                                             \
        return hipGetLastError();                                                                               \
    }
    PIT_ADI_XC(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adi_x(const AdiShape &sh, const LineTab<double> &tb, AdiBuf in, long in_off, AdiBuf out,
                        long out_off, int nslices, int Mx, int My, int R, double ex, double ed, hipStream_t st,
                        bool pre, double ex2, double ed2)
{
    if (in.f32 && out.f32)
        return adi_x_t<float, float>(sh, tb, in.f, in_off, out.f, out_off, nslices, Mx, My, R, ex, ed, pre, ex2, ed2,
                                     st);
    if (!in.f32 && out.f32)
        return adi_x_t<double, float>(sh, tb, in.d, in_off, out.f, out_off, nslices, Mx, My, R, ex, ed, pre, ex2,
                                      ed2, st);
    if (!in.f32 && !out.f32)
        return adi_x_t<double, double>(sh, tb, in.d, in_off, out.d, out_off, nslices, Mx, My, R, ex, ed, pre, ex2,
                                       ed2, st);
    return hipErrorInvalidValue;
}

template <typename SIN, typename SOUT, int EPI>
static hipError_t adi_y_pre(bool pre, const AdiShape &sh, const ColTab &tb, const SIN *in, long in_off, SOUT *out,
                            long out_off, const double *base, long base_off, double sign, int nslices, int Mx,
                            int My, double ex, double ed, hipStream_t st)
{
    if (pre)
        return adi_y_t<SIN, SOUT, EPI, true>(sh, tb, in, in_off, out, out_off, base, base_off, sign, nslices, Mx,
                                             My, ex, ed, st);
    return adi_y_t<SIN, SOUT, EPI, false>(sh, tb, in, in_off, out, out_off, base, base_off, sign, nslices, Mx, My,
                                          ex, ed, st);
}

hipError_t launch_adi_y(const AdiShape &sh, const ColTab &tb, AdiBuf in, long in_off, AdiBuf out, long out_off,
                        const double *base, long base_off, double sign, int nslices, int Mx, int My, double ex,
                        double ed, hipStream_t st, bool pre)
{
    const bool epi = base != nullptr;
    if (in.f32 && out.f32 && !epi)
        return adi_y_pre<float, float, 0>(pre, sh, tb, in.f, in_off, out.f, out_off, nullptr, 0, 0.0, nslices, Mx,
                                          My, ex, ed, st);
    if (in.f32 && !out.f32 && epi)
        return adi_y_pre<float, double, 1>(pre, sh, tb, in.f, in_off, out.d, out_off, base, base_off, sign,
                                           nslices, Mx, My, ex, ed, st);
    if (in.f32 && !out.f32 && !epi)
        return adi_y_pre<float, double, 0>(pre, sh, tb, in.f, in_off, out.d, out_off, nullptr, 0, 0.0, nslices,
                                           Mx, My, ex, ed, st);
    if (!in.f32 && !out.f32 && epi)
        return adi_y_pre<double, double, 1>(pre, sh, tb, in.d, in_off, out.d, out_off, base, base_off, sign,
                                            nslices, Mx, My, ex, ed, st);
    if (!in.f32 && !out.f32 && !epi)
        return adi_y_pre<double, double, 0>(pre, sh, tb, in.d, in_off, out.d, out_off, nullptr, 0, 0.0, nslices,
                                            Mx, My, ex, ed, st);
    return hipErrorInvalidValue;
}

}  // namespace pit
