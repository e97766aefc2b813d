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
