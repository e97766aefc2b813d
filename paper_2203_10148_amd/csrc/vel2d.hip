// 2D PR-ADI half-steps with per-line operators (velocity field), FP64.
//
// One thread per line (row for the x half-step, column for the y half-step,
// grid.y = slice) runs the Thomas recurrences of its line with the
// precomputed pivots.  Column threads of a wavefront touch consecutive
// addresses at every point of their walk; row threads touch one point of 64
// rows per step and reuse each fetched 128-byte line over the next 15 steps
// from L1.
#include "vel2d.hpp"

namespace pit {

constexpr int kVelThreads = 64;

__global__ __launch_bounds__(kVelThreads) void k_vel_x(VelTab t, const double *__restrict__ in, long in_off,
                                                        double *__restrict__ out, long out_off, int Mx, int My,
                                                        int expl)
{
    const int j = blockIdx.x * kVelThreads + threadIdx.x;
    if (j >= My) return;
    const long np = (long)Mx * My;
    const double *u = in + (in_off + blockIdx.y) * np;
    double *o = out + (out_off + blockIdx.y) * np;
    const long row = (long)j * Mx;
    const double a = t.xa[j];
    double d = 0.0;
    for (int i = 0; i < Mx; ++i) {
        const long q = row + i;
        double r = u[q];
        if (expl) {
            const double cm = (j > 0) ? u[q - Mx] : 0.0;
            const double cq = (j < My - 1) ? u[q + Mx] : 0.0;
            r = r + t.ylo[i] * cm + t.ydi * r + t.yup[i] * cq;
        }
        d = (r - a * d) * t.xw[q];
        o[q] = d;
    }
    double x = d;
    for (int i = Mx - 2; i >= 0; --i) {
        const long q = row + i;
        x = o[q] - t.xc[q] * x;
        o[q] = x;
    }
}

__global__ __launch_bounds__(kVelThreads) void k_vel_y(VelTab t, const double *__restrict__ in, long in_off,
                                                        double *out, long out_off, const double *base,
                                                        long base_off, double sign, double *__restrict__ wk,
                                                        int Mx, int My, int expl)
{
    const int i = blockIdx.x * kVelThreads + threadIdx.x;
    if (i >= Mx) return;
    const long np = (long)Mx * My;
    const double *u = in + (in_off + blockIdx.y) * np;
    double *o = out + (out_off + blockIdx.y) * np;
    double *w = wk + (long)blockIdx.y * np;
    const double *b = base ? base + (base_off + blockIdx.y) * np : nullptr;
    const double a = t.ya[i];
    double d = 0.0;
    for (int j = 0; j < My; ++j) {
        const long q = (long)j * Mx + i;
        double r = u[q];
        if (expl) {
            const double cm = (i > 0) ? u[q - 1] : 0.0;
            const double cq = (i < Mx - 1) ? u[q + 1] : 0.0;
            r = r + t.xlo[j] * cm + t.xdi * r + t.xup[j] * cq;
        }
        d = (r - a * d) * t.yw[q];
        w[q] = d;
    }
    double x = d;
    {
        const long q = (long)(My - 1) * Mx + i;
        o[q] = b ? b[q] + sign * x : x;
    }
    for (int j = My - 2; j >= 0; --j) {
        const long q = (long)j * Mx + i;
        x = w[q] - t.yc[q] * x;
        o[q] = b ? b[q] + sign * x : x;
    }
}

hipError_t launch_vel_x(const VelTab &t, const double *in, long in_off, double *out, long out_off, int ns,
                        int Mx, int My, int expl, hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const dim3 grid((My + kVelThreads - 1) / kVelThreads, ns);
    hipLaunchKernelGGL(k_vel_x, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, Mx, My, expl);
    return hipGetLastError();
}

hipError_t launch_vel_y(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                        const double *base, long base_off, double sign, double *wk, int ns, int Mx, int My,
                        int expl, hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    const dim3 grid((Mx + kVelThreads - 1) / kVelThreads, ns);
    hipLaunchKernelGGL(k_vel_y, grid, dim3(kVelThreads), 0, st, t, in, in_off, out, out_off, base, base_off, sign,
                       wk, Mx, My, expl);
    return hipGetLastError();
}

}  // namespace pit
