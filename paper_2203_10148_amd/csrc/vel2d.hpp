// 2D PR-ADI with a velocity field (constant plus a rigid rotation about the
// domain centre): every row has its own x-operator and every column its own
// y-operator (the advection-diffusion-reaction test of Sec. 4 with
// u = [-y, x]).  Private to libpitsbicg.
#pragma once

#include <hip/hip_runtime.h>

namespace pit {

// Tables of one propagator (fine or coarse) with theta = dt/2 folded in.
// Row j's x-solve (I - th Lx_j) x = r is a constant-stencil tridiagonal
// system (sub xa[j], diagonal, super): the Thomas forward pass is
//   d_0 = r_0 xw_0,  d_i = (r_i - xa[j] d_{i-1}) xw_i,
// and the backward pass x_{M-1} = d_{M-1}, x_i = d_i - xc_i x_{i+1}, where
// xw = 1/pivot and xc = super/pivot are stored per point [My][Mx]; column
// i's y-solve likewise with ya[i], yw, yc.  The explicit parts:
//   x half-step: (I + th Ly_i) u = u + ylo[i] u(j-1) + ydi u + yup[i] u(j+1)
//   y half-step: (I + th Lx_j) u = u + xlo[j] u(i-1) + xdi u + xup[j] u(i+1)
// (Dirichlet 0 outside).
struct VelTab {
    const double *xw, *xc, *yw, *yc;      // [My][Mx]
    const double *xa, *xlo, *xup;         // [My]
    const double *ya, *ylo, *yup;         // [Mx]
    double xdi, ydi;
    int expl;  // 1: the PR-ADI explicit halves; 0: identity (backward-Euler splitting)
};

// Doubles of one VelTab in the workspace, and its view.
inline size_t vel_tab_elems(int Mx, int My) { return 4 * (size_t)Mx * My + 3 * (size_t)My + 3 * (size_t)Mx; }
inline VelTab vel_tab_view(const double *b, int Mx, int My, double xdi, double ydi, int expl)
{
    const size_t np = (size_t)Mx * My;
    VelTab t{};
    t.xw = b;
    t.xc = b + np;
    t.yw = b + 2 * np;
    t.yc = b + 3 * np;
    const double *r = b + 4 * np;
    t.xa = r;
    t.xlo = r + My;
    t.xup = r + 2 * My;
    const double *c = r + 3 * My;
    t.ya = c;
    t.ylo = c + Mx;
    t.yup = c + 2 * Mx;
    t.xdi = xdi;
    t.ydi = ydi;
    t.expl = expl;
    return t;
}

// x half-step on `ns` slices: out_{s+out_off} = X^{-1} E u,  u = in_{s+in_off},
// E = (I + th Ly) (expl != 0) or I.  in and out must not overlap.
hipError_t launch_vel_x(const VelTab &t, const double *in, long in_off, double *out, long out_off, int ns,
                        int Mx, int My, int expl, hipStream_t st);
// y half-step: x = Y^{-1} E u (E = (I + th Lx) or I), then
// out = base + sign x (base != NULL) or x; wk (ns slices) holds the forward
// values, so base may be out itself.  in must not overlap out or wk.
hipError_t launch_vel_y(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                        const double *base, long base_off, double sign, double *wk, int ns, int Mx, int My,
                        int expl, hipStream_t st);

// Slices small enough for LDS run whole on chip: the apply with one
// workgroup per slice for all m steps, the sweep with one workgroup marching
// the slices.  Same arithmetic, in the same order, as the half-step kernels.
// vel_lds_mode: 2 when three FP64 fields and the tables fit in kVelLdsMax
// bytes, 1 when the fields alone fit (tables read from global memory), 0
// otherwise (or more than 512 lines on an axis).
constexpr size_t kVelLdsMax = 160 * 1024;
size_t vel_lds_bytes(int Mx, int My, bool tab);
int vel_lds_mode(int Mx, int My);
// out_{s+out_off} = base_{s+out_off} + sign F(in_{s+in_off}) (base NULL: F(in)),
// s < ns, F = m steps; in must not overlap out.
hipError_t launch_vel_apply_lds(const VelTab &t, const double *in, long in_off, double *out, long out_off,
                                const double *base, long base_off, double sign, int ns, int m, int Mx, int My,
                                hipStream_t st);
// z_0 = v_0, z_n = v_n + G(z_{n-1}), G = c steps; v == z allowed.
hipError_t launch_vel_sweep_lds(const VelTab &t, const double *v, double *z, int N, int c, int Mx, int My,
                                hipStream_t st);

}  // namespace pit
