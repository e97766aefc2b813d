// libpitsbicg host side: context, coefficient tables, workspace binding, the
// operator entry points and the Algorithm 1 driver.
//
// The driver keeps Algorithm 1's control flow on the host: after each
// reduction it reads a few FP64 scalars back (one small copy and one stream
// synchronisation), decides as the algorithm does, and launches the next
// kernels with the scalars as arguments.  All block-vector work runs in the
// HIP kernels.
#include "../../include/pitsbicg.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.hpp"
#include "pit_internal.hpp"

using namespace pit;

namespace {

thread_local int t_last_hip = 0;

}  // namespace

void pit::set_last_hip(int code) { t_last_hip = code; }

namespace {

constexpr int kMaxAdi = 1024;  // points per axis of the 2D half-step kernels

const LineShape kShapes[] = {{64, 1},  {64, 2},  {64, 4},  {64, 8},    {128, 8},  {256, 4},  {256, 8},
                             {256, 16}, {512, 4}, {512, 8}, {512, 16}, {1024, 4}, {1024, 8}, {1024, 16}};

bool shape_supported(LineShape s)
{
    for (const auto &k : kShapes)
        if (k.NT == s.NT && k.C == s.C) return true;
    return false;
}

// Default shape: eight points per thread once the line is long enough, the
// thread count growing with M; sixteen per thread above 4096 points (with
// 1024 threads a lane has only 128 registers, too few for 8 FP64 points of
// state, prefetch and tables).
LineShape default_shape(int M)
{
    if (M <= 64) return {64, 1};
    if (M <= 128) return {64, 2};
    if (M <= 256) return {64, 4};
    if (M <= 512) return {64, 8};
    if (M <= 1024) return {128, 8};
    if (M <= 2048) return {256, 8};
    if (M <= 4096) return {256, 16};
    if (M <= 8192) return {512, 16};
    return {1024, 16};
}

// Shapes chosen by pit_autotune, per line-length class and stepper kinds.
struct TuneKey {
    int mclass, bc, fine_scheme, fine_prec, coarse_scheme, c;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(mclass, bc, fine_scheme, fine_prec, coarse_scheme, c) <
               std::tie(o.mclass, o.bc, o.fine_scheme, o.fine_prec, o.coarse_scheme, o.c);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, LineShape> g_tuned;

int length_class(int M)
{
    int k = 64;
    while (k < M) k *= 2;
    return k;
}

TuneKey tune_key(const pit_problem &p, const pit_stepper &f, const pit_stepper &g)
{
    return TuneKey{length_class(p.M[0]), p.bc, f.scheme, f.prec, g.scheme, g.substeps};
}

bool tuned_shape(const TuneKey &k, int M, LineShape &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(k);
    if (it == g_tuned.end() || it->second.NT * it->second.C < M) return false;
    out = it->second;
    return true;
}

// 2D launch shapes: rows per wavefront of the fine x half step, the y
// half step's (waves, rows per segment, segments per wave), and the columns
// per workgroup of the coarse sweep's one-column y kernel (0: not used).
struct AdiTune {
    int R, wy, cy, seg, ycw;
};
// Shapes chosen by pit_autotune for 2D problems, per size class of each axis
// and stepper kinds.
struct TuneKey2 {
    int mx, my, fine_scheme, fine_prec, coarse_scheme, c, vel;
    bool operator<(const TuneKey2 &o) const
    {
        return std::tie(mx, my, fine_scheme, fine_prec, coarse_scheme, c, vel) <
               std::tie(o.mx, o.my, o.fine_scheme, o.fine_prec, o.coarse_scheme, o.c, o.vel);
    }
};
std::map<TuneKey2, AdiTune> g_tuned2;

TuneKey2 tune_key2(const pit_problem &p, const pit_stepper &f, const pit_stepper &g)
{
    const int vel = p.adv[0] != 0.0 || p.adv[1] != 0.0 || p.rot != 0.0;
    return TuneKey2{length_class(p.M[0]), length_class(p.M[1]), f.scheme, f.prec, g.scheme, g.substeps, vel};
}

bool tuned_adi(const TuneKey2 &k, AdiTune &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned2.find(k);
    if (it == g_tuned2.end()) return false;
    out = it->second;
    return true;
}

LineShape shape_from_env(const char *name, int M)
{
    const char *s = std::getenv(name);
    if (s) {
        LineShape sh{0, 0};
        if (std::sscanf(s, "%d,%d", &sh.NT, &sh.C) == 2 && shape_supported(sh) && sh.NT * sh.C >= M)
            return sh;
    }
    return default_shape(M);
}


// Build the tables of the line solver for the tridiagonal matrix with
// sub-diagonal a (coefficient of x_{j-1}), diagonal b and super-diagonal c
// (coefficient of x_{j+1}); periodic adds the corners A[0][M-1] = a and
// A[M-1][0] = c.  Returns false if the factorisation is not finite.
bool build_line(int M, bool periodic, double a, double b, double c, LineShape sh, LineHost &L)
{
    const int NT = sh.NT, C = sh.C, P = NT * C, W = NT / kWave;
    std::vector<double> lm(P, 1.0), iu(P, 0.0), cm(P, 0.0), zz(P, 0.0);
    std::vector<double> bd(M, b), u(M), l(M);
    double gam = 0.0;
    if (periodic) {  // Sherman-Morrison split A = B + (gam,0..,c)(1,0..,a/gam)^T
        gam = -b;
        bd[0] = b - gam;
        bd[M - 1] = b - c * a / gam;
    }
    u[0] = bd[0];
    l[0] = 0.0;
    for (int j = 1; j < M; ++j) {
        l[j] = a / u[j - 1];
        u[j] = bd[j] - l[j] * c;
    }
    for (int j = 0; j < M; ++j) {
        lm[j] = -l[j];
        iu[j] = 1.0 / u[j];
        cm[j] = (j < M - 1) ? -c / u[j] : 0.0;
    }
    L.cyclic = periodic ? 1 : 0;
    L.inv_den = 0.0;
    L.bg = 0.0;
    if (periodic) {  // z = B^{-1} (gam, 0, .., 0, c)
        std::vector<double> y(M), z(M);
        for (int j = 0; j < M; ++j) {
            const double rhs = (j == 0) ? gam : (j == M - 1 ? c : 0.0);
            y[j] = rhs + (j > 0 ? lm[j] * y[j - 1] : 0.0);
        }
        for (int j = M - 1; j >= 0; --j) z[j] = iu[j] * y[j] + (j < M - 1 ? cm[j] * z[j + 1] : 0.0);
        for (int j = 0; j < M; ++j) zz[j] = z[j];
        L.bg = a / gam;
        L.inv_den = 1.0 / (1.0 + z[0] + L.bg * z[M - 1]);
    }
    L.iu_last = iu[M - 1];
    L.a = a;
    L.c = c;
    // Scan constants and device layout for the multipliers lm, cm.
    auto fill = [&](const std::vector<double> &lm, const std::vector<double> &cm, std::vector<double> &blob) {
        std::vector<double> pf(NT, 1.0), pb(NT, 1.0);
        for (int t = 0; t < NT; ++t)
            for (int k = 0; k < C; ++k) {
                pf[t] *= lm[t * C + k];
                pb[t] *= cm[t * C + k];
            }
        blob.assign(line_tab_elems(NT, C), 0.0);
        double *base = blob.data();
        LineTab<double> v = line_tab_view<double>(base, NT, C);
        auto W_ = [&](const double *p) { return const_cast<double *>(p); };
        for (int t = 0; t < NT; ++t) {
            for (int k = 0; k < C; ++k) {
                W_(v.lm)[k * NT + t] = lm[t * C + k];
                W_(v.iu)[k * NT + t] = iu[t * C + k];
                W_(v.cm)[k * NT + t] = cm[t * C + k];
                W_(v.z)[k * NT + t] = zz[t * C + k];
            }
            const int lane = t % kWave, ws = t - lane, we = ws + kWave - 1;
            const int row = lane / 16, l16 = lane % 16;
            auto prodf = [&](int a, int b) {  // prod pf over wave lanes a..b
                double f = 1.0;
                for (int q = a; q <= b; ++q) f *= pf[ws + q];
                return f;
            };
            auto prodb = [&](int a, int b) {
                double g = 1.0;
                for (int q = a; q <= b; ++q) g *= pb[ws + q];
                return g;
            };
            for (int i = 0; i < 4; ++i) {
                const int s = 1 << i;
                W_(v.wf)[i * NT + t] = (l16 >= s) ? prodf(lane - s + 1, lane) : 0.0;
                W_(v.wb)[i * NT + t] = (l16 + s <= 15) ? prodb(lane, lane + s - 1) : 0.0;
            }
            for (int r = 0; r < 3; ++r)  // lower row totals (rows 0..2) into row `row`
                W_(v.wf)[(4 + r) * NT + t] = (row > r) ? prodf(16 * (r + 1), lane) : 0.0;
            for (int r = 1; r <= 3; ++r)  // upper row totals (rows 1..3) into row `row`
                W_(v.wb)[(3 + r) * NT + t] = (row < r) ? prodb(lane, 16 * r - 1) : 0.0;
            double qf = 1.0, qb = 1.0;
            for (int q = ws; q < t; ++q) qf *= pf[q];
            for (int q = t + 1; q <= we; ++q) qb *= pb[q];
            W_(v.qf)[t] = qf;
            W_(v.qb)[t] = qb;
        }
        for (int w = 0; w < W; ++w) {
            double f = 1.0, g = 1.0;
            for (int q = w * kWave; q < (w + 1) * kWave; ++q) {
                f *= pf[q];
                g *= pb[q];
            }
            W_(v.pwf)[w] = f;
            W_(v.pwb)[w] = g;
            // late terms at the first point of the wave: products of lm after it
            const int Pw = w * kWave * C, Qw = Pw + kWave * C - 1;
            double r = 1.0;
            for (int i = Pw + 1; i <= Qw; ++i) r *= lm[i];
            W_(v.rfw)[w] = r;
            for (int lane = 0; lane < kWave; ++lane) {
                const int t = w * kWave + lane;
                double rt = 0.0;
                if (lane > 0) {
                    rt = 1.0;
                    for (int i = Pw + 1; i <= t * C - 1; ++i) rt *= lm[i];
                }
                W_(v.rf)[t] = rt;
            }
        }
    };
    L.sh = sh;
    L.M = M;
    fill(lm, cm, L.blob);
    // FP32 tables keep the register form: forming an FP32 multiplier from
    // rounded a and iu would add two roundings to every step of the
    // recurrences, which a stiff line amplifies.
    L.blob32.assign(L.blob.begin(), L.blob.end());
    if (line_compact(NT, C)) {  // FP64: the multipliers the compact solver forms from iu
        std::vector<double> lme(P), cme(P);
        for (int j = 0; j < P; ++j) {
            lme[j] = (j == 0) ? 0.0 : -a * iu[j - 1];
            cme[j] = -c * iu[j];
        }
        fill(lme, cme, L.blob);
    }
    for (double x : L.blob)
        if (!std::isfinite(x)) return false;
    for (float x : L.blob32)
        if (!std::isfinite(x)) return false;
    return std::isfinite(L.inv_den) && std::isfinite(L.bg) && std::isfinite(L.iu_last);
}

}  // namespace


namespace {

// theta*(L stencil) for the 1D operator nu*D2 - a*D1c - r:
//   (L u)_j = lo*u_{j-1} + di*u_j + up*u_{j+1}
void stencil1d(const pit_problem &p, double h, double *lo, double *di, double *up)
{
    *lo = p.nu / (h * h) + p.adv[0] / (2.0 * h);
    *di = -2.0 * p.nu / (h * h) - p.react;
    *up = p.nu / (h * h) - p.adv[0] / (2.0 * h);
}

// Row tables of the y-direction solver: the LU factors of the My x My
// tridiagonal (sub a, diagonal b, super c), padded to ns*cy rows, and the
// products of lm and cm over each segment's rows.
bool build_col(int My, double a, double b, double c, int ns, int cy, std::vector<double> &blob)
{
    const int nr = ns * cy;
    std::vector<double> lm(nr, 1.0), iu(nr, 0.0), cm(nr, 0.0);
    double u = b;
    for (int j = 0; j < My; ++j) {
        if (j > 0) {
            const double l = a / u;
            u = b - l * c;
            lm[j] = -l;
        } else {
            lm[j] = 0.0;
        }
        iu[j] = 1.0 / u;
        cm[j] = (j < My - 1) ? -c / u : 0.0;
    }
    blob.assign(col_tab_elems(nr), 0.0);
    for (int j = 0; j < nr; ++j) {
        blob[j] = lm[j];
        blob[nr + j] = iu[j];
        blob[2 * (size_t)nr + j] = cm[j];
    }
    for (int w = 0; w < ns; ++w) {
        double f = 1.0, g = 1.0;
        for (int j = w * cy; j < (w + 1) * cy; ++j) {
            f *= lm[j];
            g *= cm[j];
        }
        blob[3 * (size_t)nr + w] = f;
        blob[3 * (size_t)nr + kMaxSegs + w] = g;
    }
    for (double x : blob)
        if (!std::isfinite(x)) return false;
    return true;
}

// Tables for A = I - theta*L with theta = dt (IE) or dt/2 (CN).
bool make_line(const pit_problem &pb, double h, int scheme, double dt, LineShape sh, LineHost &out)
{
    double lo, di, up;
    stencil1d(pb, h, &lo, &di, &up);
    const double th = (scheme == PIT_IE) ? dt : 0.5 * dt;
    return build_line(pb.M[0], pb.bc == PIT_PERIODIC, -th * lo, 1.0 - th * di, -th * up, sh, out);
}
bool make_line(const pit_ctx &c, int scheme, double dt, LineShape sh, LineHost &out)
{
    return make_line(c.pb, c.hx, scheme, dt, sh, out);
}

// Per-slice tables of a time-dependent operator (1D): slice n's fine and
// coarse step matrices with nu * s[n], in the layout of line_tab_view, each
// slice's block `stride` elements after the previous one, and its scalars.
bool build_slice_tables(pit_ctx &c, const double *s)
{
    const int N = c.N;
    c.tft.clear();
    c.tct.clear();
    c.tf32t.clear();
    c.scf.assign((size_t)kSliceScalars * N, 0.0);
    c.scc.assign((size_t)kSliceScalars * N, 0.0);
    c.scf32.assign((size_t)kSliceScalars * N, 0.0f);
    for (int n = 0; n < N; ++n) {
        pit_problem pb = c.pb;
        pb.nu = c.pb.nu * s[n];
        LineHost f, g;
        if (!make_line(pb, c.hx, c.fine.scheme, c.DT / c.m, c.lf.sh, f) ||
            !make_line(pb, c.hx, c.coarse.scheme, c.DT / c.coarse.substeps, c.lc.sh, g))
            return false;
        if (n == 0) {
            c.str_f = (long)f.blob.size();
            c.str_c = (long)g.blob.size();
        }
        c.tft.insert(c.tft.end(), f.blob.begin(), f.blob.end());
        c.tct.insert(c.tct.end(), g.blob.begin(), g.blob.end());
        if (c.fine32()) c.tf32t.insert(c.tf32t.end(), f.blob32.begin(), f.blob32.end());
        const double pd = (c.DT / c.m) * (pb.nu / (c.hx * c.hx));
        const double vf[kSliceScalars] = {f.inv_den, f.bg, f.iu_last, -f.a, -f.c, pd};
        const double vc[kSliceScalars] = {g.inv_den, g.bg, g.iu_last, -g.a, -g.c, 0.0};
        for (int q = 0; q < kSliceScalars; ++q) {
            c.scf[(size_t)kSliceScalars * n + q] = vf[q];
            c.scc[(size_t)kSliceScalars * n + q] = vc[q];
            c.scf32[(size_t)kSliceScalars * n + q] = (float)vf[q];
        }
    }
    return true;
}

// theta of the fine or coarse 2D step: dt/2 (PR-ADI) or dt (backward-Euler
// splitting).
double adi_theta(const pit_ctx &c, bool fine_step)
{
    const pit_stepper &s = fine_step ? c.fine : c.coarse;
    const double dt = c.DT / (fine_step ? c.m : c.coarse.substeps);
    return s.scheme == PIT_ADI_PR ? 0.5 * dt : dt;
}

// 2D setup: shapes, x and y tables and explicit coefficients for the fine
// and coarse steps: theta = dt/2 with the explicit halves (I + theta L) for
// PR-ADI, theta = dt with identity explicit parts for the backward-Euler
// splitting.
// The y shapes the kernels in adi2d.hip are instantiated for, smallest
// first (two segments of 32 rows beat one segment up to 512 rows: 32-column
// blocks, twice as many workgroups and two resident per CU).
const AdiShape kYMenu[] = {{0, 8, 16, 1, 0}, {0, 8, 32, 1, 0}, {0, 8, 32, 2, 0}, {0, 16, 32, 2, 0},
                           {0, 16, 32, 1, 0}, {0, 8, 16, 2, 0}, {0, 16, 16, 2, 0}};
int yshape_rows(const AdiShape &a) { return a.wy * a.cy * a.seg; }
bool yshape_known(int wy, int cy, int seg)
{
    for (const auto &a : kYMenu)
        if (a.wy == wy && a.cy == cy && a.seg == seg) return true;
    return false;
}

bool setup_2d(pit_ctx &c, const AdiTune *force)
{
    const int Mx = c.pb.M[0], My = c.pb.M[1];
    // rows up to 512 points on one wavefront (up to 8 points per lane), wider
    // rows on two (128 threads x 8 points)
    const int xw = Mx > 512 ? 2 : 1;
    int cx = 1;
    while (64 * xw * cx < Mx) cx *= 2;
    // y shape: the smallest of the menu that covers the column; then the
    // autotuned choice for this size class, the PIT_ADI_YSHAPE override
    // "wy,cy,seg", and an autotuning candidate, each if it covers the column
    AdiShape sh{cx, 0, 0, 0, xw};
    for (const auto &a : kYMenu)
        if (yshape_rows(a) >= My) {
            sh = a;
            sh.cx = cx;
            sh.xw = xw;
            break;
        }
    if (!sh.wy || cx > 8) return false;
    AdiTune tuned{};
    const bool have_tuned = tuned_adi(tune_key2(c.pb, c.fine, c.coarse), tuned);
    auto take = [&](int wy, int cy, int seg) {
        const AdiShape o{cx, wy, cy, seg, xw};
        if (yshape_known(wy, cy, seg) && yshape_rows(o) >= My) sh = o;
    };
    if (have_tuned) take(tuned.wy, tuned.cy, tuned.seg);
    if (const char *e = std::getenv("PIT_ADI_YSHAPE")) {
        int wy = 0, cy = 0, seg = 0;
        if (std::sscanf(e, "%d,%d,%d", &wy, &cy, &seg) == 3) take(wy, cy, seg);
    }
    if (force) take(force->wy, force->cy, force->seg);
    c.ash = sh;
    // rows per wavefront of the fine x half step
    if (have_tuned && tuned.R > 0) c.adi_R = tuned.R;
    if (const char *e = std::getenv("PIT_ADI_ROWS")) c.adi_R = std::max(1, std::atoi(e));
    if (force && force->R > 0) c.adi_R = force->R;
    const double nu = c.pb.nu, r = c.pb.react;
    const double kx = nu / (c.hx * c.hx), ky = nu / (c.hy * c.hy);
    auto tables = [&](double th, bool pr, LineHost &ax, std::vector<double> &ay, double &xex, double &xed,
                      double &yex, double &yed) {
        xex = pr ? th * ky : 0.0;  // x half step: (I + th Ly), or I
        xed = pr ? 1.0 - 2.0 * th * ky - 0.5 * th * r : 1.0;
        yex = pr ? th * kx : 0.0;  // y half step: (I + th Lx), or I
        yed = pr ? 1.0 - 2.0 * th * kx - 0.5 * th * r : 1.0;
        const bool okx = build_line(Mx, false, -th * kx, 1.0 + 2.0 * th * kx + 0.5 * th * r, -th * kx,
                                    LineShape{64 * xw, cx}, ax);
        const bool oky = build_col(My, -th * ky, 1.0 + 2.0 * th * ky + 0.5 * th * r, -th * ky, sh.wy * sh.seg, sh.cy, ay);
        return okx && oky;
    };
    const bool prf = c.fine.scheme == PIT_ADI_PR, prc = c.coarse.scheme == PIT_ADI_PR;
    if (!tables(adi_theta(c, true), prf, c.axf, c.ayf, c.fx_ex, c.fx_ed, c.fy_ex, c.fy_ed) ||
        !tables(adi_theta(c, false), prc, c.axc, c.ayc, c.cx_ex, c.cx_ed, c.cy_ex, c.cy_ed))
        return false;
    // the coarse sweep's single-slice y half steps: one column per wavefront
    // (PIT_ADI_YC=0 keeps the column-strip kernel; 1, 2, 4: columns per
    // workgroup, as is the autotuned value)
    const char *yc = std::getenv("PIT_ADI_YC");
    int ycw = 2;  // columns per workgroup: 2 measured fastest at 512 x 512
    if (have_tuned) ycw = tuned.ycw;
    if (yc && (yc[0] == '0' || yc[0] == '1' || yc[0] == '2' || yc[0] == '4')) ycw = yc[0] - '0';
    if (force) ycw = force->ycw;
    if (My <= 512 && ycw > 0) {
        int cyc = 1;
        while (64 * cyc < My) cyc *= 2;
        const double th = adi_theta(c, false);
        if (!build_line(My, false, -th * ky, 1.0 + 2.0 * th * ky + 0.5 * th * r, -th * ky, LineShape{64, cyc},
                        c.aycl))
            return false;
        c.ycc = cyc;
        c.ycw = ycw;
        // the x half step hands it the right-hand side (PIT_ADI_PRE=0: the
        // y kernel forms it from u* and its neighbour columns)
        const char *pe = std::getenv("PIT_ADI_PRE");
        c.ypre = !(pe && pe[0] == '0');
    }
    // the same hand-over in the fine apply (PIT_ADI_FPRE=0: the y kernel
    // forms its right-hand side from u* and two halo columns)
    const char *fe = std::getenv("PIT_ADI_FPRE");
    c.fpre = !(fe && fe[0] == '0');
    return true;
}

// Per-line tables of one 2D step with a velocity field (theta = th; pr:
// the PR-ADI explicit halves, else identity explicit parts):
// row j's x-operator Lx_j = nu D2x - ux(y_j) D1x - r/2, column i's
// Ly_i = nu D2y - uy(x_i) D1y - r/2, with ux = adv0 - rot (y - Ly/2) and
// uy = adv1 + rot (x - Lx/2) (a rigid rotation about the domain centre);
// Thomas pivots of I - th L per line, layout of vel_tab_view.
bool vel_tables(const pit_ctx &c, double th, bool pr, std::vector<double> &v, double &xdi, double &ydi)
{
    const int Mx = c.pb.M[0], My = c.pb.M[1];
    const double nu = c.pb.nu, r = c.pb.react, hx = c.hx, hy = c.hy;
    const size_t np = (size_t)Mx * My;
    v.assign(vel_tab_elems(Mx, My), 0.0);
    double *xw = v.data(), *xc = xw + np, *yw = xw + 2 * np, *yc = xw + 3 * np;
    double *xa = xw + 4 * np, *xlo = xa + My, *xup = xa + 2 * My;
    double *ya = xa + 3 * My, *ylo = ya + Mx, *yup = ya + 2 * Mx;
    const double dix = -2.0 * nu / (hx * hx) - 0.5 * r, diy = -2.0 * nu / (hy * hy) - 0.5 * r;
    xdi = pr ? th * dix : 0.0;
    ydi = pr ? th * diy : 0.0;
    for (int j = 0; j < My; ++j) {
        const double ux = c.pb.adv[0] - c.pb.rot * ((j + 1) * hy - 0.5 * c.pb.length[1]);
        const double lo = nu / (hx * hx) + ux / (2.0 * hx), up = nu / (hx * hx) - ux / (2.0 * hx);
        xlo[j] = pr ? th * lo : 0.0;
        xup[j] = pr ? th * up : 0.0;
        xa[j] = -th * lo;
        const double b = 1.0 - th * dix, cc = -th * up;
        double cp = 0.0;
        for (int i = 0; i < Mx; ++i) {
            const double piv = b - (i > 0 ? xa[j] * cp : 0.0);
            const size_t q = (size_t)j * Mx + i;
            xw[q] = 1.0 / piv;
            cp = xc[q] = cc / piv;
        }
    }
    for (int i = 0; i < Mx; ++i) {
        const double uy = c.pb.adv[1] + c.pb.rot * ((i + 1) * hx - 0.5 * c.pb.length[0]);
        const double lo = nu / (hy * hy) + uy / (2.0 * hy), up = nu / (hy * hy) - uy / (2.0 * hy);
        ylo[i] = pr ? th * lo : 0.0;
        yup[i] = pr ? th * up : 0.0;
        ya[i] = -th * lo;
        const double b = 1.0 - th * diy, cc = -th * up;
        double cp = 0.0;
        for (int j = 0; j < My; ++j) {
            const double piv = b - (j > 0 ? ya[i] * cp : 0.0);
            const size_t q = (size_t)j * Mx + i;
            yw[q] = 1.0 / piv;
            cp = yc[q] = cc / piv;
        }
    }
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

int validate(const pit_problem *p, int N, int m, const pit_stepper &f, const pit_stepper &g)
{
    if (!p || N < 1 || m < 1) return PIT_EINVAL;
    if (p->dim != 1 && p->dim != 2) return PIT_EINVAL;
    if (!(p->length[0] > 0.0) || !(p->T > 0.0) || !(p->nu >= 0.0)) return PIT_EINVAL;
    if (!std::isfinite(p->adv[0]) || !std::isfinite(p->adv[1]) || !std::isfinite(p->react) ||
        !std::isfinite(p->rot))
        return PIT_EINVAL;
    if (p->dim == 2) {
        if (p->M[0] < 3 || p->M[1] < 3 || p->M[0] > kMaxAdi || p->M[1] > kMaxAdi) return PIT_EINVAL;
        if (p->bc != PIT_DIRICHLET0) return PIT_EINVAL;
        // a velocity field runs the per-line FP64 half-steps
        if ((p->adv[0] != 0.0 || p->adv[1] != 0.0 || p->rot != 0.0) && f.prec != PIT_F64) return PIT_EINVAL;
        if (!(p->length[1] > 0.0)) return PIT_EINVAL;
        if ((f.scheme != PIT_ADI_PR && f.scheme != PIT_ADI_IE) || (g.scheme != PIT_ADI_PR && g.scheme != PIT_ADI_IE))
            return PIT_EINVAL;
    } else {
        if (p->M[0] < 3 || p->M[0] > kMaxLine || p->rot != 0.0) return PIT_EINVAL;
        if (p->bc != PIT_DIRICHLET0 && p->bc != PIT_PERIODIC) return PIT_EINVAL;
        if (f.scheme != PIT_IE && f.scheme != PIT_CN) return PIT_EINVAL;
        if (g.scheme != PIT_IE && g.scheme != PIT_CN) return PIT_EINVAL;
    }
    if (f.substeps != 0 && f.substeps != m) return PIT_EINVAL;
    if (g.substeps < 1) return PIT_EINVAL;
    if ((f.prec != PIT_F64 && f.prec != PIT_F32) || g.prec != PIT_F64) return PIT_EINVAL;
    if (f.reserved != 0 || g.reserved != 0) return PIT_EINVAL;
    return PIT_OK;
}

}  // namespace

namespace {

// The fine apply in the precision the context was created with.
hipError_t fine_launch(const pit_ctx *c, const double *lam, double *y, int raw, int last, bool chunked,
                       hipStream_t st)
{
    if (c->fine32())
        return launch_fine1d_f32(c->lf.sh, c->tab32(c->lf, c->off_tf32), lam, y, c->N, c->npts, c->m, c->pd,
                                 c->pa, c->pr, c->pb.bc == PIT_PERIODIC ? 1 : 0, raw, last, chunked, st);
    return launch_fine1d_f64(c->lf.sh, c->tab(c->lf, c->off_tf), lam, y, c->N, c->npts, c->m, c->fine.scheme,
                             raw, last, chunked, st);
}

// 2D all-at-once apply: m PR-ADI steps on every slice, two launches per step.
// Work slice s reads lam_{s+in_off} and writes y_{s+out_off}.
hipError_t apply_2d(const pit_ctx *c, const double *lam, double *y, int raw, int last, hipStream_t st)
{
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    const long np = c->npts;
    if (last) raw = 1;
    const int ns = last ? 1 : (raw ? c->N : c->N - 1);
    const long in_off = last ? c->N - 1 : 0;
    const long out_off = last ? c->N - 1 : (raw ? 0 : 1);
    hipError_t e;
    if (!raw && (e = launch_copy(y, lam, np, st)) != hipSuccess) return e;  // y_0 = lam_0
    if (ns == 0) return hipSuccess;
    const LineTab<double> tx = [&] {
        LineTab<double> t = line_tab_view<double>(reinterpret_cast<const double *>(c->ws + c->off_axf), 64 * c->ash.xw, c->ash.cx);
        t.cyclic = 0;
        t.M = Mx;
        return t;
    }();
    const ColTab ty = col_tab_view(reinterpret_cast<const double *>(c->ws + c->off_ayf), c->ash.wy * c->ash.cy * c->ash.seg);
    const AdiBuf lamb{nullptr, const_cast<double *>(lam), false}, yb{nullptr, y, false};
    const AdiBuf ub = c->fbuf(c->off_ubuf), sb = c->fbuf(c->off_sbuf);
    // the x half step stores the y half step's right-hand side, so the y
    // kernel reads no halo columns
    const bool pre = c->fpre;
    for (int step = 0; step < c->m; ++step) {
        const bool first = step == 0, fin = step == c->m - 1;
        if ((e = launch_adi_x(c->ash, tx, first ? lamb : ub, first ? in_off : 0, sb, 0, ns, Mx, My, c->adi_R,
                              c->fx_ex, c->fx_ed, st, pre, c->fy_ex, c->fy_ed)) != hipSuccess)
            return e;
        if (fin)
            e = launch_adi_y(c->ash, ty, sb, 0, yb, out_off, raw ? nullptr : lam, out_off, -1.0, ns, Mx, My,
                             c->fy_ex, c->fy_ed, st, pre);
        else
            e = launch_adi_y(c->ash, ty, sb, 0, ub, 0, nullptr, 0, 0.0, ns, Mx, My, c->fy_ex, c->fy_ed, st, pre);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Whole slices in LDS when they fit (PIT_VEL_LDS=0 keeps the half-step kernels).
bool vel_lds(const pit_ctx *c)
{
    const char *e = std::getenv("PIT_VEL_LDS");
    return !(e && e[0] == '0') && vel_lds_mode(c->pb.M[0], c->pb.M[1]) > 0;
}

// 2D all-at-once apply with a velocity field: the per-line half-steps.
hipError_t apply_2dv(const pit_ctx *c, const double *lam, double *y, int raw, int last, hipStream_t st)
{
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    const long np = c->npts;
    if (last) raw = 1;
    const int ns = last ? 1 : (raw ? c->N : c->N - 1);
    const long in_off = last ? c->N - 1 : 0;
    const long out_off = last ? c->N - 1 : (raw ? 0 : 1);
    hipError_t e;
    if (!raw && (e = launch_copy(y, lam, np, st)) != hipSuccess) return e;  // y_0 = lam_0
    if (ns == 0) return hipSuccess;
    const VelTab t = c->vtab(true);
    if (vel_lds(c))
        return launch_vel_apply_lds(t, lam, in_off, y, out_off, raw ? nullptr : lam, out_off, -1.0, ns, c->m, Mx, My,
                                    st);
    double *ub = reinterpret_cast<double *>(c->ws + c->off_ubuf), *sb = reinterpret_cast<double *>(c->ws + c->off_sbuf);
    for (int step = 0; step < c->m; ++step) {
        const bool first = step == 0, fin = step == c->m - 1;
        if ((e = launch_vel_x(t, first ? lam : ub, first ? in_off : 0, sb, 0, ns, Mx, My, t.expl, st)) != hipSuccess)
            return e;
        if (fin)
            e = launch_vel_y(t, sb, 0, y, out_off, raw ? nullptr : lam, out_off, -1.0, c->wbuf(), ns, Mx, My, t.expl,
                             st);
        else
            e = launch_vel_y(t, sb, 0, ub, 0, nullptr, 0, 0.0, c->wbuf(), ns, Mx, My, t.expl, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// 2D coarse sweep with a velocity field, one slice at a time.  ta, tb: two
// one-slice FP64 temporaries; wk: one slice of the y half-step's forward
// values (none of them used by the whole-slice LDS kernel).
hipError_t sweep_2dv(const pit_ctx *c, const double *v, double *z, double *ta, double *tb, double *wk,
                     hipStream_t st)
{
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    const long np = c->npts;
    hipError_t e;
    const VelTab t = c->vtab(false);
    if (vel_lds(c)) return launch_vel_sweep_lds(t, v, z, c->N, c->coarse.substeps, Mx, My, st);
    if (z != v && (e = launch_copy(z, v, np, st)) != hipSuccess) return e;
    const int cs = c->coarse.substeps;
    for (int n = 1; n < c->N; ++n) {
        for (int s = 0; s < cs; ++s) {
            if ((e = launch_vel_x(t, s == 0 ? z : tb, s == 0 ? n - 1 : 0, ta, 0, 1, Mx, My, t.expl, st)) != hipSuccess)
                return e;
            if (s == cs - 1)
                e = launch_vel_y(t, ta, 0, z, n, v, n, 1.0, wk, 1, Mx, My, t.expl, st);
            else
                e = launch_vel_y(t, ta, 0, tb, 0, nullptr, 0, 0.0, wk, 1, Mx, My, t.expl, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// 2D coarse sweep: z_0 = v_0, z_n = v_n + G(z_{n-1}), G = c PR-ADI steps of
// DT/c, FP64, one slice at a time (one row per wavefront for latency).  ta,
// tb: two one-slice FP64 temporaries.
hipError_t sweep_2d(const pit_ctx *c, const double *v, double *z, double *tmpa, double *tmpb, hipStream_t st)
{
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    const long np = c->npts;
    hipError_t e;
    if (z != v && (e = launch_copy(z, v, np, st)) != hipSuccess) return e;
    LineTab<double> tx = line_tab_view<double>(reinterpret_cast<const double *>(c->ws + c->off_axc), 64 * c->ash.xw, c->ash.cx);
    tx.cyclic = 0;
    tx.M = Mx;
    const ColTab ty = col_tab_view(reinterpret_cast<const double *>(c->ws + c->off_ayc), c->ash.wy * c->ash.cy * c->ash.seg);
    LineTab<double> tyc{};
    if (c->ycc) {
        tyc = line_tab_view<double>(reinterpret_cast<const double *>(c->ws + c->off_aycl), 64, c->ycc);
        tyc.cyclic = 0;
        tyc.M = My;
    }
    const AdiBuf zb{nullptr, z, false};
    const AdiBuf ta{nullptr, tmpa, false}, tb{nullptr, tmpb, false};
    const int cs = c->coarse.substeps;
    // With the one-column y kernel and rows that fit one wave, the x half
    // step stores the y half step's right-hand side (I + theta Lx) u* itself
    // (bitwise what the y kernel would form), so the y kernel stages only
    // its own columns.
    const bool pre = c->ycc && c->ypre && c->ash.xw == 1;
    // y half step of slice n: one column per wavefront where the tables exist
    auto yhalf = [&](const AdiBuf &out, long out_off, const double *base, long base_off, double sign) {
        if (c->ycc)
            return launch_adi_yc(c->ycw, c->ycc, tyc, tmpa, 0, out.d, out_off, base, base_off, sign, 1, Mx, My,
                                 c->cy_ex, c->cy_ed, st, pre);
        return launch_adi_y(c->ash, ty, ta, 0, out, out_off, base, base_off, sign, 1, Mx, My, c->cy_ex, c->cy_ed, st);
    };
    for (int n = 1; n < c->N; ++n) {
        for (int s = 0; s < cs; ++s) {
            if (pre)
                e = launch_adi_x_pre(c->ash, tx, s == 0 ? z : tmpb, s == 0 ? n - 1 : 0, tmpa, Mx, My, c->cx_ex,
                                     c->cx_ed, c->cy_ex, c->cy_ed, st);
            else
                e = launch_adi_x(c->ash, tx, s == 0 ? zb : tb, s == 0 ? n - 1 : 0, ta, 0, 1, Mx, My, 1, c->cx_ex,
                                 c->cx_ed, st);
            if (e != hipSuccess) return e;
            e = (s == cs - 1) ? yhalf(zb, n, v, n, 1.0) : yhalf(tb, 0, nullptr, 0, 0.0);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Workspace of the source term: the source and the forced response (working
// and natural layouts); reserved for every context, a few slices at most.
size_t source_slots(pit_ctx &c, size_t o)
{
    c.off_src = o;
    o = align_up(o + (size_t)c.npts * sizeof(double));
    c.off_bf = o;
    o = align_up(o + (size_t)std::max<long>(c.ld, c.npts) * sizeof(double));
    c.off_bfn = o;
    return align_up(o + (size_t)c.npts * sizeof(double));
}

// The workspace with or without the slots of a time-dependent source: the
// forced responses of all N slices and the N m per-step weights, behind the
// base workspace.
void size_source_t(pit_ctx *c)
{
    size_t o = align_up(c->base_total);
    if (!c->gt.empty()) {
        c->off_bft = o;
        o = align_up(o + (size_t)c->N * c->npts * sizeof(double));
        c->off_gw = o;
        o = align_up(o + (size_t)c->N * c->m * sizeof(double));
    }
    if (c->nu_t()) {  // per-slice tables of a time-dependent operator
        c->off_tft = o;
        o = align_up(o + c->tft.size() * sizeof(double));
        c->off_tct = o;
        o = align_up(o + c->tct.size() * sizeof(double));
        c->off_tf32t = o;
        o = align_up(o + c->tf32t.size() * sizeof(float));
        c->off_scf = o;
        o = align_up(o + c->scf.size() * sizeof(double));
        c->off_scc = o;
        o = align_up(o + c->scc.size() * sizeof(double));
        c->off_scf32 = o;
        o = align_up(o + c->scf32.size() * sizeof(float));
    }
    c->total = o;
}

// Upload the per-slice tables (synchronous, null stream).
int upload_slice_tables(pit_ctx *c)
{
    if (!c->nu_t()) return PIT_OK;
    auto up = [&](size_t off, const void *p, size_t bytes) {
        return bytes ? hipMemcpy(c->ws + off, p, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    PIT_HIP(up(c->off_tft, c->tft.data(), c->tft.size() * sizeof(double)));
    PIT_HIP(up(c->off_tct, c->tct.data(), c->tct.size() * sizeof(double)));
    PIT_HIP(up(c->off_tf32t, c->tf32t.data(), c->tf32t.size() * sizeof(float)));
    PIT_HIP(up(c->off_scf, c->scf.data(), c->scf.size() * sizeof(double)));
    PIT_HIP(up(c->off_scc, c->scc.data(), c->scc.size() * sizeof(double)));
    PIT_HIP(up(c->off_scf32, c->scf32.data(), c->scf32.size() * sizeof(float)));
    return PIT_OK;
}

// One fine step of every slice: out_n = S in_n, n < N (natural layout,
// FP64; tmp is a block vector for the 2D half-steps).
hipError_t step_all(pit_ctx *c, const double *in, double *out, double *tmp, hipStream_t st)
{
    const int N = c->N;
    if (!c->dim2())
        return launch_fine1d_f64(c->lf.sh, c->tab(c->lf, c->off_tf), in, out, N, c->npts, 1, c->fine.scheme, 1, 0,
                                 false, st);
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    hipError_t e;
    if (c->vel) {
        const VelTab vt = c->vtab(true);
        if (vel_lds(c)) return launch_vel_apply_lds(vt, in, 0, out, 0, nullptr, 0, 0.0, N, 1, Mx, My, st);
        if ((e = launch_vel_x(vt, in, 0, tmp, 0, N, Mx, My, vt.expl, st)) != hipSuccess) return e;
        return launch_vel_y(vt, tmp, 0, out, 0, nullptr, 0, 0.0, c->wbuf(), N, Mx, My, vt.expl, st);
    }
    LineTab<double> tx =
        line_tab_view<double>(reinterpret_cast<const double *>(c->ws + c->off_axf), 64 * c->ash.xw, c->ash.cx);
    tx.cyclic = 0;
    tx.M = Mx;
    const ColTab ty =
        col_tab_view(reinterpret_cast<const double *>(c->ws + c->off_ayf), c->ash.wy * c->ash.cy * c->ash.seg);
    auto B = [](const double *p) { return AdiBuf{nullptr, const_cast<double *>(p), false}; };
    if ((e = launch_adi_x(c->ash, tx, B(in), 0, B(tmp), 0, N, Mx, My, c->adi_R, c->fx_ex, c->fx_ed, st)) !=
        hipSuccess)
        return e;
    return launch_adi_y(c->ash, ty, B(tmp), 0, B(out), 0, nullptr, 0, 0.0, N, Mx, My, c->fy_ex, c->fy_ed, st);
}

// Time-dependent source: the forced responses of all N slices at once into
// bft(): from 0, u_{j+1} = S u_j + w_j c over the m steps of each slice, c
// the response of one step to the profile h, w_j the profile's weight in
// global step j (g(t_{j+1}) under IE, the mean of g(t_j) and g(t_{j+1})
// under CN and PR-ADI).  One fine step of every slice per launch, then one
// per-slice axpy.
hipError_t forced_t(pit_ctx *c, const double *cc, hipStream_t st)
{
    const long np = c->npts;
    const int N = c->N, m = c->m;
    std::vector<double> w((size_t)N * m);
    const bool ie = c->dim2() ? c->fine.scheme == PIT_ADI_IE : c->fine.scheme == SCHEME_IE;
    for (size_t j = 0; j < w.size(); ++j) w[j] = ie ? c->gt[j + 1] : 0.5 * (c->gt[j] + c->gt[j + 1]);
    hipError_t e;
    if ((e = hipMemcpy(c->gw(), w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    double *X = c->vec(4), *Y = c->vec(5), *T = c->vec(6);
    if ((e = launch_fill0(X, (long)N * np, st)) != hipSuccess) return e;
    if ((e = launch_slice_axpy(X, cc, c->gw(), m, np, N, st)) != hipSuccess) return e;
    for (int k = 1; k < m; ++k) {
        if ((e = step_all(c, X, Y, T, st)) != hipSuccess) return e;
        if ((e = launch_slice_axpy(Y, cc, c->gw() + k, m, np, N, st)) != hipSuccess) return e;
        std::swap(X, Y);
    }
    return launch_copy(c->bft(), X, (long)N * np, st);
}

// The forced response b = F(0) of one slice for the source f (constant in
// time), into bfn() (natural) and bf() (working layout), FP64.  F is affine,
// F(u) = S^m u + b with S one fine step, and b = sum_{i<m} S^i c where c is
// the response of one step from 0:
//   IE and CN: c = A^{-1} (dt f)  (A = I - theta dt L, the step's matrix);
//   PR-ADI:    c = dt Y^{-1} X^{-1} f  (X, Y the half-step matrices: the
//              source's dt/2 f enters both half-steps, and (I + th Lx) X^{-1}
//              = 2 X^{-1} - I).
// 1D sums by doubling, b(2k) = b(k) + S^k b(k), b(k+1) = S b(k) + c, with
// S^k one fine launch of k steps; 2D sums step by step.  Uses the context's
// block vectors as scratch (at bind, no solve runs).
hipError_t compute_forced(pit_ctx *c, hipStream_t st)
{
    const long np = c->npts;
    const double dt = c->DT / c->m;
    double *h = c->vec(0), *t = c->vec(1), *cc = c->vec(2), *g = c->vec(3);
    hipError_t e;
#define FH(x)                              \
    if ((e = (x)) != hipSuccess) return e
    FH(hipMemcpyAsync(c->srcdev(), c->src.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
    if (!c->dim2()) {
        const LineTab<double> tb = c->tab(c->lf, c->off_tf);
        auto steps = [&](const double *in, double *out, int k, int scheme) {
            return launch_fine1d_f64(c->lf.sh, tb, in, out, 1, c->npts, k, scheme, 1, 0, false, st);
        };
        FH(launch_axpby(g, c->srcdev(), dt, c->srcdev(), 0.0, np, st));
        FH(steps(g, cc, 1, SCHEME_IE));  // one solve with A: A^{-1} (dt f)
        if (c->src_t()) return forced_t(c, cc, st);
        FH(launch_copy(h, cc, np, st));
        int top = 0;
        while ((c->m >> (top + 1)) != 0) ++top;
        int count = 1;
        for (int bit = top - 1; bit >= 0; --bit) {
            FH(steps(h, t, count, c->fine.scheme));
            FH(launch_axpby(h, t, 1.0, h, 1.0, np, st));
            count *= 2;
            if ((c->m >> bit) & 1) {
                FH(steps(h, t, 1, c->fine.scheme));
                FH(launch_axpby(h, t, 1.0, cc, 1.0, np, st));
                count += 1;
            }
        }
        FH(launch_copy(c->bfn(), h, np, st));
        FH(launch_to_chunked(h, c->bf(), 1, c->npts, c->lf.sh.NT, c->lf.sh.C, st));
        return hipSuccess;
    }
    const int Mx = c->pb.M[0], My = c->pb.M[1];
    if (c->vel) {  // per-line half-steps
        const VelTab vt = c->vtab(true);
        FH(launch_vel_x(vt, c->srcdev(), 0, t, 0, 1, Mx, My, 0, st));             // X^{-1} f
        FH(launch_vel_y(vt, t, 0, g, 0, nullptr, 0, 0.0, c->vwk(), 1, Mx, My, 0, st));  // Y^{-1} X^{-1} f
        FH(launch_axpby(cc, g, dt, g, 0.0, np, st));
        if (c->src_t()) return forced_t(c, cc, st);
        FH(launch_copy(h, cc, np, st));
        for (int k = 1; k < c->m; ++k) {
            FH(launch_vel_x(vt, h, 0, t, 0, 1, Mx, My, vt.expl, st));
            FH(launch_vel_y(vt, t, 0, g, 0, nullptr, 0, 0.0, c->vwk(), 1, Mx, My, vt.expl, st));
            FH(launch_axpby(h, g, 1.0, cc, 1.0, np, st));
        }
        FH(launch_copy(c->bfn(), h, np, st));
        FH(launch_copy(c->bf(), h, np, st));
        return hipSuccess;
    }
    LineTab<double> tx = line_tab_view<double>(reinterpret_cast<const double *>(c->ws + c->off_axf), 64 * c->ash.xw, c->ash.cx);
    tx.cyclic = 0;
    tx.M = Mx;
    const ColTab ty = col_tab_view(reinterpret_cast<const double *>(c->ws + c->off_ayf), c->ash.wy * c->ash.cy * c->ash.seg);
    auto B = [](double *p) { return AdiBuf{nullptr, p, false}; };
    auto half_x = [&](const double *in, double *out, double ex, double ed) {
        return launch_adi_x(c->ash, tx, B(const_cast<double *>(in)), 0, B(out), 0, 1, Mx, My, 1, ex, ed, st);
    };
    auto half_y = [&](const double *in, double *out, double ex, double ed) {
        return launch_adi_y(c->ash, ty, B(const_cast<double *>(in)), 0, B(out), 0, nullptr, 0, 0.0, 1, Mx, My, ex,
                            ed, st);
    };
    FH(half_x(c->srcdev(), t, 0.0, 1.0));  // X^{-1} f (explicit part off)
    FH(half_y(t, g, 0.0, 1.0));            // Y^{-1} X^{-1} f
    FH(launch_axpby(cc, g, dt, g, 0.0, np, st));
    if (c->src_t()) return forced_t(c, cc, st);
    FH(launch_copy(h, cc, np, st));
    for (int k = 1; k < c->m; ++k) {
        FH(half_x(h, t, c->fx_ex, c->fx_ed));
        FH(half_y(t, g, c->fy_ex, c->fy_ed));
        FH(launch_axpby(h, g, 1.0, cc, 1.0, np, st));
    }
    FH(launch_copy(c->bfn(), h, np, st));
    FH(launch_copy(c->bf(), h, np, st));
#undef FH
    return hipSuccess;
}

// With a source: upload it and compute the forced response (synchronous, on
// the null stream, like the table uploads of pit_bind_workspace).
int bind_source(pit_ctx *ctx)
{
    if (!ctx->has_src()) return PIT_OK;
    PIT_HIP(compute_forced(ctx, nullptr));
    PIT_HIP(hipStreamSynchronize(nullptr));
    return PIT_OK;
}

}  // namespace

hipError_t pit::fill_forced(const pit_ctx *c, double *B, hipStream_t st)
{
    if (!c->has_src() || c->N < 2) return hipSuccess;
    if (c->src_t()) {  // b_0 .. b_{N-2} into slices 1 .. N-1
        if (c->dim2()) return launch_copy(B + c->npts, c->bft(), (long)(c->N - 1) * c->npts, st);
        return launch_to_chunked(c->bft(), B + c->ld, c->N - 1, c->npts, c->lf.sh.NT, c->lf.sh.C, st);
    }
    const long len = c->dim2() ? c->npts : c->ld;
    return launch_repeat(B + len, c->bf(), len, c->N - 1, 0, st);
}

void pit_ctx::drop_graphs() const
{
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

pit_ctx::~pit_ctx()
{
    drop_graphs();
    if (capture) (void)hipStreamDestroy(capture);
    if (red_pin) (void)hipHostFree(red_pin);
}

namespace {

// Graph replay is on unless PIT_GRAPHS=0 (eager launches, for comparison).
bool graphs_enabled()
{
    const char *e = std::getenv("PIT_GRAPHS");
    return !(e && e[0] == '0');
}

// pit_solve's one-sync iteration is on unless PIT_DEV_SCALARS=0 (a host round
// trip after every reduction, for comparison).
bool dev_scalars_enabled()
{
    const char *e = std::getenv("PIT_DEV_SCALARS");
    return !(e && e[0] == '0');
}

// Run the launch sequence `launches` as a HIP graph: captured once per
// (op, in, out, flags) on the context's own capture stream (a capture cannot
// run on the legacy null stream), then replayed on `st`.  The sequences hold
// kernels only.
template <class F>
hipError_t replay(const pit_ctx *c, int op, const void *in, void *out, int raw, int last, hipStream_t st,
                  F &&launches)
{
    // graphs pay off for the many launches of the half-step kernels; the
    // whole-slice LDS kernels are one launch (two for an apply) anyway
    if (!graphs_enabled() || (c->vel && vel_lds(c))) return launches(st);
    for (const auto &g : c->graphs)
        if (g.op == op && g.in == in && g.out == out && g.raw == raw && g.last == last)
            return hipGraphLaunch(g.exec, st);
    if (c->graphs.size() >= 8) c->drop_graphs();  // bounded: callers cycle through few buffers
    hipError_t e;
    if (!c->capture && (e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t el = launches(c->capture);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(c->capture, &gr);
    if (el != hipSuccess || e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return el != hipSuccess ? el : e;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return e;
    c->graphs.push_back(pit_ctx::Graph{op, in, out, raw, last, ex});
    return hipGraphLaunch(ex, st);
}

}  // namespace

hipError_t pit::op_apply(const pit_ctx *c, const double *lam, double *y, int raw, int last, bool internal,
                         hipStream_t st)
{
    if (c->dim2())
        return replay(c, 0, lam, y, raw, last, st, [&](hipStream_t s) {
            return c->vel ? apply_2dv(c, lam, y, raw, last, s) : apply_2d(c, lam, y, raw, last, s);
        });
    return fine_launch(c, lam, y, raw, last, internal, st);
}

hipError_t pit::op_sweep(const pit_ctx *c, const double *v, double *z, bool internal, hipStream_t st)
{
    if (c->dim2())
        return replay(c, 1, v, z, 0, 0, st, [&](hipStream_t s) {
            return c->vel ? sweep_2dv(c, v, z, c->ctmp(0), c->ctmp(1), c->vwk(), s)
                          : sweep_2d(c, v, z, c->ctmp(0), c->ctmp(1), s);
        });
    return launch_sweep1d_f64(c->lc.sh, c->tab(c->lc, c->off_tc), v, z, c->N, c->npts, c->coarse.substeps,
                              c->coarse.scheme, internal, st);
}

size_t pit::sweep_staging_bytes(const pit_ctx *c)
{
    if (!c->dim2()) return 2 * (size_t)c->ntc() * sizeof(double);
    if (c->vel && vel_lds(c)) return 0;
    return (c->vel ? 3 : 2) * (size_t)c->npts * sizeof(double);
}

hipError_t pit::sweep_staged(const pit_ctx *c, const double *v, double *z, double *stage, hipStream_t st)
{
    if (c->dim2()) {
        const size_t np = (size_t)c->npts;
        return c->vel ? sweep_2dv(c, v, z, stage, stage + np, stage + 2 * np, st)
                      : sweep_2d(c, v, z, stage, stage + np, st);
    }
    // 1D: through the chunked layout, where every load and store of the
    // sequential sweep is coalesced (the layout passes cost far less than the
    // strided accesses they replace)
    const int NT = c->lc.sh.NT, C = c->lc.sh.C;
    double *a = stage, *b = stage + c->ntc();
    hipError_t e;
    if ((e = launch_to_chunked(v, a, c->N, c->npts, NT, C, st)) != hipSuccess) return e;
    if ((e = op_sweep(c, a, b, true, st)) != hipSuccess) return e;
    return launch_from_chunked(b, z, c->N, c->npts, NT, C, st);
}

extern "C" {

const char *pit_strerror(int code)
{
    switch (code) {
    case PIT_OK: return "ok";
    case PIT_EINVAL: return "invalid argument or unsupported combination";
    case PIT_ENOMEM: return "workspace or fixed scratch too small, or over the memory budget";
    case PIT_EHIP: return "HIP runtime error";
    case PIT_ENOCONV: return "not converged (max_iter or stagnation)";
    case PIT_EBREAKDOWN: return "breakdown (non-finite residual)";
    case PIT_EAGAIN: return "not finished yet";
    default: return "unknown status";
    }
}

int pit_last_hip_error(void) { return t_last_hip; }

}  // extern "C"

namespace {

// pit_create with the 1D line shape forced (autotuning) or chosen: an
// environment override, else the tuned table, else the default.
int create_ctx(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
               const LineShape *force, pit_ctx **out, const AdiTune *force2 = nullptr)
{
    if (!out) return PIT_EINVAL;
    *out = nullptr;
    int rc = validate(problem, N, m, fine, coarse);
    if (rc != PIT_OK) return rc;
    pit_ctx *c = new (std::nothrow) pit_ctx();
    if (!c) return PIT_ENOMEM;
    c->pb = *problem;
    c->N = N;
    c->m = m;
    c->fine = fine;
    c->fine.substeps = m;
    c->coarse = coarse;
    const int M = problem->M[0];
    c->DT = problem->T / N;
    if (problem->dim == 2) {
        c->npts = problem->M[0] * problem->M[1];
        c->hx = problem->length[0] / (problem->M[0] + 1);
        c->hy = problem->length[1] / (problem->M[1] + 1);
        c->w = c->hx * c->hy;
        if (!setup_2d(*c, force2)) {
            delete c;
            return PIT_EINVAL;
        }
        // Per-line tables: with a velocity field, and also without one for FP64
        // slices small enough for LDS, where the whole-slice kernels beat two
        // launches per step (PIT_VEL_LDS=0 keeps the shared-table kernels).
        const bool velocity = problem->adv[0] != 0.0 || problem->adv[1] != 0.0 || problem->rot != 0.0;
        const char *lds_env = std::getenv("PIT_VEL_LDS");
        const bool lds_small = !c->fine32() && !(lds_env && lds_env[0] == '0') &&
                               vel_lds_mode(problem->M[0], problem->M[1]) > 0;
        c->vel = velocity || lds_small;
        if (c->vel && (!vel_tables(*c, adi_theta(*c, true), fine.scheme == PIT_ADI_PR, c->vtf, c->vf_xdi, c->vf_ydi) ||
                       !vel_tables(*c, adi_theta(*c, false), coarse.scheme == PIT_ADI_PR, c->vtc, c->vc_xdi,
                                   c->vc_ydi))) {
            delete c;
            return PIT_EINVAL;
        }
        c->ld = c->npts;
        c->bps = (int)std::min<long>(64, std::max<long>(1, (c->ld + 4095) / 4096));
        const size_t fs = c->fine32() ? sizeof(float) : sizeof(double);
        size_t o = 0;
        c->off_axf = o;
        o = align_up(o + c->axf.blob.size() * sizeof(double));
        c->off_axc = o;
        o = align_up(o + c->axc.blob.size() * sizeof(double));
        c->off_ayf = o;
        o = align_up(o + c->ayf.size() * sizeof(double));
        c->off_ayc = o;
        o = align_up(o + c->ayc.size() * sizeof(double));
        c->off_aycl = o;
        o = align_up(o + c->aycl.blob.size() * sizeof(double));
        c->off_ubuf = o;
        o = align_up(o + (size_t)N * c->npts * fs);
        c->off_sbuf = o;
        o = align_up(o + (size_t)N * c->npts * fs);
        c->off_ctmp = o;
        o = align_up(o + 2 * (size_t)c->npts * sizeof(double));
        c->off_vec = o;
        o = align_up(o + kSolveVectors * (size_t)c->ntc() * sizeof(double));
        c->off_part = o;
        o = align_up(o + 4 * (size_t)N * c->bps * sizeof(double));
        c->off_red = o;
        o = align_up(o + kRedSlots * sizeof(RedOut));
        o = source_slots(*c, o);
        if (c->vel) {
            c->off_vtf = o;
            o = align_up(o + c->vtf.size() * sizeof(double));
            c->off_vtc = o;
            o = align_up(o + c->vtc.size() * sizeof(double));
            c->off_wbuf = o;
            o = align_up(o + (size_t)N * c->npts * sizeof(double));
            c->off_vwk = o;
            o = align_up(o + (size_t)c->npts * sizeof(double));
        }
        c->total = c->base_total = o;
        *out = c;
        return PIT_OK;
    }
    c->npts = M;
    c->hx = (problem->bc == PIT_PERIODIC) ? problem->length[0] / M : problem->length[0] / (M + 1);
    c->hy = 1.0;
    c->w = c->hx;
    // One shape for both line operators: pit_solve keeps its block vectors in
    // the chunked layout of that shape, shared by the fine and coarse kernels.
    LineShape sh = shape_from_env("PIT_LINE_SHAPE", M);
    if (force) {
        sh = *force;
    } else if (!std::getenv("PIT_LINE_SHAPE")) {
        LineShape t{0, 0};
        if (tuned_shape(tune_key(*problem, fine, coarse), M, t)) sh = t;
    }
    if (!make_line(*c, fine.scheme, c->DT / m, sh, c->lf) ||
        !make_line(*c, coarse.scheme, c->DT / coarse.substeps, sh, c->lc)) {
        delete c;
        return PIT_EINVAL;
    }
    {
        // the FP32 step's stencil: diffusion, advection and reaction parts,
        // each rounded once (their sums lo, up would carry the small
        // advection part with the rounding error of the large diffusion part)
        const double dt = c->DT / m, h = c->hx;
        c->pd = (float)(dt * (problem->nu / (h * h)));
        c->pa = (float)(dt * (problem->adv[0] / (2.0 * h)));
        c->pr = (float)(dt * problem->react);
    }
    c->ld = (long)sh.NT * sh.C;
    c->bps = (int)std::min<long>(64, std::max<long>(1, (c->ld + 2047) / 2048));
    size_t o = 0;
    c->off_tf = o;
    o = align_up(o + c->lf.blob.size() * sizeof(double));
    c->off_tf32 = o;
    o = align_up(o + (c->fine32() ? c->lf.blob32.size() * sizeof(float) : 0));
    c->off_tc = o;
    o = align_up(o + c->lc.blob.size() * sizeof(double));
    c->off_vec = o;
    o = align_up(o + kSolveVectors * (size_t)c->ntc() * sizeof(double));
    c->off_part = o;
    o = align_up(o + 4 * (size_t)N * c->bps * sizeof(double));
    c->off_red = o;
    o = align_up(o + kRedSlots * sizeof(RedOut));
    o = source_slots(*c, o);
    c->total = c->base_total = o;
    *out = c;
    return PIT_OK;
}

}  // namespace

extern "C" {

int pit_create(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
               pit_ctx **out)
{
    return create_ctx(problem, N, m, fine, coarse, nullptr, out);
}

int pit_destroy(pit_ctx *ctx)
{
    delete ctx;
    return PIT_OK;
}

size_t pit_workspace_bytes(const pit_ctx *ctx) { return ctx ? ctx->total : 0; }

int pit_kernel_shape(const pit_ctx *ctx, int32_t out[4])
{
    if (!ctx || !out) return PIT_EINVAL;
    if (ctx->dim2() && ctx->vel) {  // one thread per line; where a slice lives
        out[0] = 1;
        out[1] = 0;
        out[2] = vel_lds(ctx) ? vel_lds_mode(ctx->pb.M[0], ctx->pb.M[1]) : 0;
        out[3] = 0;
        return PIT_OK;
    }
    if (ctx->dim2()) {  // 2D: 64 lanes x cx points per row; wy waves x cy rows per column
        out[0] = 64 * ctx->ash.xw;
        out[1] = ctx->ash.cx;
        out[2] = 64 * ctx->ash.wy;
        out[3] = ctx->ash.cy * ctx->ash.seg;
        return PIT_OK;
    }
    out[0] = ctx->lf.sh.NT;
    out[1] = ctx->lf.sh.C;
    out[2] = ctx->lc.sh.NT;
    out[3] = ctx->lc.sh.C;
    return PIT_OK;
}

int pit_bind_workspace(pit_ctx *ctx, void *dev_ptr, size_t bytes)
{
    if (!ctx || !dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) != 0) return PIT_EINVAL;
    if (bytes < ctx->total) return PIT_ENOMEM;
    ctx->ws = static_cast<char *>(dev_ptr);
    ctx->ws_bytes = bytes;
    ctx->drop_graphs();  // captured launches point into the old workspace
    if (ctx->dim2()) {
        PIT_HIP(hipMemcpy(ctx->ws + ctx->off_axf, ctx->axf.blob.data(), ctx->axf.blob.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        PIT_HIP(hipMemcpy(ctx->ws + ctx->off_axc, ctx->axc.blob.data(), ctx->axc.blob.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        PIT_HIP(hipMemcpy(ctx->ws + ctx->off_ayf, ctx->ayf.data(), ctx->ayf.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        PIT_HIP(hipMemcpy(ctx->ws + ctx->off_ayc, ctx->ayc.data(), ctx->ayc.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        if (ctx->ycc)
            PIT_HIP(hipMemcpy(ctx->ws + ctx->off_aycl, ctx->aycl.blob.data(), ctx->aycl.blob.size() * sizeof(double),
                              hipMemcpyHostToDevice));
        if (ctx->vel) {
            PIT_HIP(hipMemcpy(ctx->ws + ctx->off_vtf, ctx->vtf.data(), ctx->vtf.size() * sizeof(double),
                              hipMemcpyHostToDevice));
            PIT_HIP(hipMemcpy(ctx->ws + ctx->off_vtc, ctx->vtc.data(), ctx->vtc.size() * sizeof(double),
                              hipMemcpyHostToDevice));
        }
        return bind_source(ctx);
    }
    PIT_HIP(hipMemcpy(ctx->ws + ctx->off_tf, ctx->lf.blob.data(), ctx->lf.blob.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    PIT_HIP(hipMemcpy(ctx->ws + ctx->off_tc, ctx->lc.blob.data(), ctx->lc.blob.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    if (ctx->fine32())
        PIT_HIP(hipMemcpy(ctx->ws + ctx->off_tf32, ctx->lf.blob32.data(), ctx->lf.blob32.size() * sizeof(float),
                          hipMemcpyHostToDevice));
    if (int rc = upload_slice_tables(ctx)) return rc;
    return bind_source(ctx);
}

int pit_set_source(pit_ctx *ctx, const double *f)
{
    if (!ctx) return PIT_EINVAL;
    if (f && ctx->nu_t()) return PIT_EINVAL;  // not with a time-dependent operator
    if (f)
        for (int j = 0; j < ctx->npts; ++j)
            if (!std::isfinite(f[j])) return PIT_EINVAL;
    ctx->gt.clear();
    size_source_t(ctx);
    if (!f) {
        ctx->src.clear();
        return PIT_OK;
    }
    ctx->src.assign(f, f + ctx->npts);
    return ctx->ws ? bind_source(ctx) : PIT_OK;
}

int pit_set_source_t(pit_ctx *ctx, const double *h, const double *g)
{
    if (!ctx) return PIT_EINVAL;
    if (h && ctx->nu_t()) return PIT_EINVAL;  // not with a time-dependent operator
    if (!h || !g) return pit_set_source(ctx, h);
    const size_t ng = (size_t)ctx->N * ctx->m + 1;
    for (int j = 0; j < ctx->npts; ++j)
        if (!std::isfinite(h[j])) return PIT_EINVAL;
    for (size_t j = 0; j < ng; ++j)
        if (!std::isfinite(g[j])) return PIT_EINVAL;
    ctx->gt.assign(g, g + ng);
    ctx->src.assign(h, h + ctx->npts);
    size_source_t(ctx);
    if (ctx->ws && ctx->ws_bytes < ctx->total) {  // the bound workspace is too small: unbind
        ctx->drop_graphs();
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        return PIT_ENOMEM;
    }
    return ctx->ws ? bind_source(ctx) : PIT_OK;
}

int pit_set_nu_t(pit_ctx *ctx, const double *s)
{
    if (!ctx) return PIT_EINVAL;
    if (!s) {
        ctx->nus.clear();
        size_source_t(ctx);
        return PIT_OK;
    }
    if (ctx->dim2() || ctx->has_src()) return PIT_EINVAL;
    for (int n = 0; n < ctx->N; ++n)
        if (!(s[n] > 0.0) || !std::isfinite(s[n])) return PIT_EINVAL;
    if (!build_slice_tables(*ctx, s)) return PIT_EINVAL;  // a factorisation that is not finite
    ctx->nus.assign(s, s + ctx->N);
    size_source_t(ctx);
    if (ctx->ws && ctx->ws_bytes < ctx->total) {  // the bound workspace is too small: unbind
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        return PIT_ENOMEM;
    }
    return ctx->ws ? upload_slice_tables(ctx) : PIT_OK;
}

int pit_apply_F(pit_ctx *ctx, const double *lam, double *y, int32_t flags, void *stream)
{
    if (!ctx || !ctx->ws || !lam || !y || (flags & ~(PIT_APPLY_RAW | PIT_APPLY_LAST))) return PIT_EINVAL;
    if (lam == y) return PIT_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int raw = (flags & PIT_APPLY_RAW) ? 1 : 0, last = (flags & PIT_APPLY_LAST) ? 1 : 0;
    const int NT = ctx->lf.sh.NT, C = ctx->lf.sh.C;
    if (!ctx->dim2() && line_compact(NT, C)) {
        // Lines above 8192 points: the natural-layout kernels of that shape
        // spill, so convert through two of the context's block vectors and
        // run the chunked kernels (as pit_solve does).
        double *a = ctx->vec(0), *b = ctx->vec(1);
        const long n1 = (long)(ctx->N - 1);
        PIT_HIP(launch_to_chunked(lam, a, ctx->N, ctx->npts, NT, C, st));
        PIT_HIP(op_apply(ctx, a, b, raw, last, true, st));
        if (last) PIT_HIP(launch_from_chunked(b + n1 * ctx->ld, y + n1 * ctx->npts, 1, ctx->npts, NT, C, st));
        else PIT_HIP(launch_from_chunked(b, y, ctx->N, ctx->npts, NT, C, st));
    } else {
        PIT_HIP(op_apply(ctx, lam, y, raw, last, false, st));
    }
    // with a source F is affine: F_n(lam_n) = F0(lam_n) + b_n
    if (ctx->has_src() && (raw || last)) {
        const long np = ctx->npts, l0 = (long)(ctx->N - 1) * np;
        if (ctx->src_t()) {
            if (last) PIT_HIP(launch_axpby(y + l0, ctx->bft() + l0, 1.0, y + l0, 1.0, np, st));
            else PIT_HIP(launch_axpby(y, ctx->bft(), 1.0, y, 1.0, (long)ctx->N * np, st));
        } else if (last) {
            PIT_HIP(launch_repeat(y + l0, ctx->bfn(), np, 1, 1, st));
        } else {
            PIT_HIP(launch_repeat(y, ctx->bfn(), np, ctx->N, 1, st));
        }
    }
    return PIT_OK;
}

int pit_coarse_sweep(pit_ctx *ctx, const double *v, double *z, void *stream)
{
    if (!ctx || !ctx->ws || !v || !z) return PIT_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->dim2()) {
        PIT_HIP(op_sweep(ctx, v, z, false, st));  // captured once, replayed as a graph
        return PIT_OK;
    }
    // 1D: staged through two of the context's block vectors (contiguous)
    PIT_HIP(sweep_staged(ctx, v, z, ctx->vec(0), st));
    return PIT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Algorithm 1 driver
// ---------------------------------------------------------------------------
namespace {

struct EventPair {
    hipEvent_t a, b;
};

struct Solver {
    pit_ctx *c;
    hipStream_t st;
    double *R, *Rt, *P, *D, *S, *K, *Tm, *Xc;
    long n;
    int matvecs = 0;
    int n_fine = 0, n_coarse = 0;
    int timing = 0;  // > 0: time the first launch of each kind and every timing-th after it
    std::vector<EventPair> ev_fine, ev_coarse, ev_kry;
    bool kry_timed = false;  // the current iteration's Krylov launches are timed
    int n_kry_timed = 0;

    ~Solver()
    {
        for (auto &e : ev_fine) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        for (auto &e : ev_coarse) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        for (auto &e : ev_kry) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    }

    // iteration k's Krylov launches are timed when timing > 0 and k is a
    // multiple of the stride
    void time_iteration(int k)
    {
        kry_timed = timing > 0 && k % timing == 0;
        if (kry_timed) ++n_kry_timed;
    }
    // brackets around a group of Krylov launches of a timed iteration
    int kopen() { return kry_timed ? begin(ev_kry) : PIT_OK; }
    int kclose()
    {
        if (kry_timed) PIT_HIP(hipEventRecord(ev_kry.back().b, st));
        return PIT_OK;
    }

    int begin(std::vector<EventPair> &v)
    {
        EventPair e{};
        PIT_HIP(hipEventCreate(&e.a));
        PIT_HIP(hipEventCreate(&e.b));
        v.push_back(e);
        PIT_HIP(hipEventRecord(e.a, st));
        return PIT_OK;
    }

    // fine apply and coarse sweep on chunked-layout block vectors
    int apply(const double *in, double *out)
    {
        int rc;
        const bool timed = timing > 0 && n_fine % timing == 0;
        if (timed && (rc = begin(ev_fine))) return rc;
        PIT_HIP(op_apply(c, in, out, 0, 0, true, st));
        if (timed) PIT_HIP(hipEventRecord(ev_fine.back().b, st));
        ++n_fine;
        return PIT_OK;
    }

    int sweep(const double *in, double *out)
    {
        int rc;
        const bool timed = timing > 0 && n_coarse % timing == 0;
        if (timed && (rc = begin(ev_coarse))) return rc;
        PIT_HIP(op_sweep(c, in, out, true, st));
        if (timed) PIT_HIP(hipEventRecord(ev_coarse.back().b, st));
        ++n_coarse;
        return PIT_OK;
    }

    static float total_ms(const std::vector<EventPair> &v)
    {
        float t = 0.0f;
        for (const auto &e : v) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) t += ms;
        }
        return t;
    }

    // out = G^{-1} F in  (one preconditioned matrix-by-vector product)
    int matvec(const double *in, double *out)
    {
        int rc = apply(in, Tm);
        if (rc) return rc;
        rc = sweep(Tm, out);
        if (rc) return rc;
        ++matvecs;
        return PIT_OK;
    }

    // nq inner products of (a[q], b[q]); fills dots and the N,inf norms of the pairs
    int reduce(int nq, const double *const *a, const double *const *b, RedOut &h)
    {
        DotPairs pr{};
        for (int q = 0; q < nq; ++q) {
            pr.a[q] = a[q];
            pr.b[q] = b[q];
        }
        if (int e = kopen()) return e;
        PIT_HIP(launch_seg_dots(pr, nq, c->N, c->ld, c->bps, c->part(), c->w, c->red(), st));
        if (int e = kclose()) return e;
        if (int e = pin()) return e;
        PIT_HIP(hipMemcpyAsync(c->red_pin, c->red(), sizeof(RedOut), hipMemcpyDeviceToHost, st));
        PIT_HIP(hipStreamSynchronize(st));
        h = *c->red_pin;
        return PIT_OK;
    }

    int pin()
    {
        if (!c->red_pin)
            PIT_HIP(hipHostMalloc(reinterpret_cast<void **>(&c->red_pin), kRedSlots * sizeof(RedOut),
                                  hipHostMallocDefault));
        return PIT_OK;
    }

    // nq inner products into `out` on the device, not read back
    int dots(int nq, const double *const *a, const double *const *b, RedOut *out)
    {
        DotPairs pr{};
        for (int q = 0; q < nq; ++q) {
            pr.a[q] = a[q];
            pr.b[q] = b[q];
        }
        PIT_HIP(launch_seg_dots(pr, nq, c->N, c->ld, c->bps, c->part(), c->w, out, st));
        return PIT_OK;
    }

    // slots 1..4 to the host, after everything queued so far
    int fetch(RedOut (&h)[kRedSlots])
    {
        if (int e = pin()) return e;
        PIT_HIP(hipMemcpyAsync(c->red_pin + 1, c->red(1), 4 * sizeof(RedOut), hipMemcpyDeviceToHost, st));
        PIT_HIP(hipStreamSynchronize(st));
        for (int i = 1; i <= 4; ++i) h[i] = c->red_pin[i];
        return PIT_OK;
    }

    // rho as the host holds it, into slot 5 (the device-scalar kernels read it there)
    int set_rho(double rho)
    {
        if (int e = pin()) return e;
        c->red_pin[5].dot[0] = rho;
        PIT_HIP(hipMemcpyAsync(c->red(5), c->red_pin + 5, sizeof(double), hipMemcpyHostToDevice, st));
        PIT_HIP(hipStreamSynchronize(st));
        return PIT_OK;
    }
};

}  // namespace

extern "C" int pit_solve(pit_ctx *ctx, const double *u0, double *X, const pit_solve_opts *opts,
                         pit_solve_info *info, void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !ctx->ws || !u0 || !X) return PIT_EINVAL;
    pit_solve_opts o{};
    o.tol = 1e-10;
    o.restart_tol = 1e-30;
    o.max_iter = 0;
    o.norm_mode = PIT_ABS;
    o.x0_mode = PIT_X0_ZERO;
    if (opts) o = *opts;
    if (o.max_iter <= 0) o.max_iter = 2 * ctx->N;
    if (o.x0_mode < PIT_X0_ZERO || o.x0_mode > PIT_X0_COARSE || !(o.tol >= 0.0)) return PIT_EINVAL;

    Solver s{};
    s.c = ctx;
    s.st = static_cast<hipStream_t>(stream);
    s.R = ctx->vec(0);
    s.Rt = ctx->vec(1);
    s.P = ctx->vec(2);
    s.D = ctx->vec(3);
    s.S = ctx->vec(4);
    s.K = ctx->vec(5);
    s.Tm = ctx->vec(6);
    s.Xc = ctx->vec(7);
    s.n = ctx->ntc();
    if (o.timing < 0) return PIT_EINVAL;
    s.timing = o.timing;
    const long n = s.n;
    const int NT = ctx->lf.sh.NT, C = ctx->lf.sh.C;
    hipStream_t st = s.st;
    double *const Xu = X;  // the caller's iterate (natural layout)
    X = s.Xc;              // the working iterate (chunked layout)
    int rc;
    RedOut h{};

    // initial residual R^0 = G^{-1}(B - F X^0), B = (u0, b, .., b) (b = 0 without a source)
    PIT_HIP(launch_fill0(s.S, n, st));
    if (ctx->dim2()) PIT_HIP(launch_copy(s.S, u0, ctx->npts, st));  // S holds B for now
    else PIT_HIP(launch_to_chunked(u0, s.S, 1, ctx->npts, NT, C, st));
    PIT_HIP(fill_forced(ctx, s.S, st));
    if (o.x0_mode == PIT_X0_ZERO) {
        PIT_HIP(launch_fill0(X, n, st));
        if ((rc = s.sweep(s.S, s.R))) return rc;
    } else {
        if (o.x0_mode == PIT_X0_COARSE) {
            if ((rc = s.sweep(s.S, X))) return rc;
        } else {
            if (ctx->dim2()) PIT_HIP(launch_copy(X, Xu, n, st));
            else PIT_HIP(launch_to_chunked(Xu, X, ctx->N, ctx->npts, NT, C, st));
        }
        if ((rc = s.apply(X, s.D))) return rc;
        PIT_HIP(launch_axpby(s.Tm, s.S, 1.0, s.D, -1.0, n, st));
        if ((rc = s.sweep(s.Tm, s.R))) return rc;
        s.matvecs++;
    }
    // shadow residual, first direction, rho
    PIT_HIP(launch_copy(s.Rt, s.R, n, st));
    PIT_HIP(launch_copy(s.P, s.R, n, st));
    {
        const double *a[2] = {s.R, s.R}, *b[2] = {s.Rt, s.R};
        if ((rc = s.reduce(2, a, b, h))) return rc;
    }
    double rho = h.dot[0];
    double nrm = h.nmax[1];
    const double scale = (o.norm_mode == PIT_REL && h.nmax[1] > 0.0) ? h.nmax[1] : 1.0;
    double best = nrm;
    int best_at = 0, k = 0, restarts = 0, status = PIT_ENOCONV, hl = 0;
    // One host round trip per iteration: the update kernels read alpha, omega
    // and beta from the reductions' device outputs, and the host reads all of
    // them once, at the end (see launch_update_xr_dev).  rho_src[rho_idx]
    // holds the host's rho bit for bit: the previous iteration's slot 3 or 4,
    // or slot 5 after the host changed rho itself.
    const bool one_sync = !o.half_step_check && dev_scalars_enabled();
    const RedOut *rho_src = nullptr;
    int rho_idx = 0;
    double rho_dev = 0.0;

    for (;;) {
        bool dr_zero = false;  // the one-sync iteration found <D, R~> = 0 for the current P
        if (info && info->history && hl < info->history_cap) info->history[hl++] = nrm;
        if (!std::isfinite(nrm)) {
            status = PIT_EBREAKDOWN;
            break;
        }
        if (!(nrm > o.tol * scale)) {  // stopping test
            status = PIT_OK;
            break;
        }
        if (k >= o.max_iter) {
            status = PIT_ENOCONV;
            break;
        }
        if (o.stall_window > 0) {
            if (nrm <= 0.5 * best) {
                best = nrm;
                best_at = k;
            } else if (k - best_at >= o.stall_window) {
                status = PIT_ENOCONV;
                break;
            }
        }
        s.time_iteration(k);
        if (one_sync) {
            if (!rho_src || std::memcmp(&rho, &rho_dev, sizeof(double)) != 0) {
                if ((rc = s.set_rho(rho))) return rc;
                rho_src = ctx->red(5);
                rho_idx = 0;
                rho_dev = rho;
            }
            RedOut *const A = ctx->red(1), *const Bq = ctx->red(2);
            RedOut *const Cn = ctx->red(rho_src == ctx->red(3) ? 4 : 3);
            const DevScalars ds{rho_src, rho_idx, A, Bq, Cn};
            if ((rc = s.matvec(s.P, s.D))) return rc;
            if ((rc = s.kopen())) return rc;
            {
                const double *a[1] = {s.D}, *b[1] = {s.Rt};
                if ((rc = s.dots(1, a, b, A))) return rc;
            }
            PIT_HIP(launch_axpby_dev(s.S, s.R, s.D, ds, n, st));  // S = R - alpha D
            if ((rc = s.kclose())) return rc;
            if ((rc = s.matvec(s.S, s.K))) return rc;
            if ((rc = s.kopen())) return rc;
            {
                const double *a[3] = {s.K, s.K, s.S}, *b[3] = {s.S, s.K, s.S};
                if ((rc = s.dots(3, a, b, Bq))) return rc;
            }
            PIT_HIP(launch_update_xr_dev(X, s.R, s.P, s.S, s.K, ds, n, st));
            {
                const double *a[2] = {s.R, s.R}, *b[2] = {s.Rt, s.R};
                if ((rc = s.dots(2, a, b, Cn))) return rc;
            }
            PIT_HIP(launch_update_p_dev(s.P, s.R, s.D, ds, n, st));
            if ((rc = s.kclose())) return rc;
            RedOut hs[kRedSlots];
            if ((rc = s.fetch(hs))) return rc;
            const double dr = hs[1].dot[0];
            // dr == 0: the update kernels left X, R and P unchanged; the
            // iteration is redone below from the restart (the products of D
            // and K queued before the breakdown was known are spent)
            dr_zero = dr == 0.0;
            if (!dr_zero) {
                const double alpha = rho / dr;
                const double ks = hs[2].dot[0], kk = hs[2].dot[1], snorm = hs[2].nmax[2];
                if (kk == 0.0) {  // S = 0: the half step solved the system
                    PIT_HIP(launch_axpby(X, X, 1.0, s.P, alpha, n, st));
                    PIT_HIP(launch_copy(s.R, s.S, n, st));
                    nrm = snorm;
                    k++;
                    continue;
                }
                const double omega = ks / kk;
                if (omega == 0.0) {
                    PIT_HIP(launch_axpby(X, X, 1.0, s.P, alpha, n, st));
                    PIT_HIP(launch_copy(s.R, s.S, n, st));
                    PIT_HIP(launch_copy(s.Rt, s.R, n, st));
                    PIT_HIP(launch_copy(s.P, s.R, n, st));
                    const double *a[1] = {s.R}, *b[1] = {s.R};
                    if ((rc = s.reduce(1, a, b, h))) return rc;
                    rho = h.dot[0];
                    nrm = h.nmax[0];
                    restarts++;
                    k++;
                    continue;
                }
                const RedOut &hc = hs[Cn == ctx->red(3) ? 3 : 4];
                double rho_new = hc.dot[0];
                nrm = hc.nmax[1];
                rho_src = Cn;
                rho_idx = 0;
                if (std::fabs(rho_new) <= o.restart_tol) {  // restart test with epsilon_0
                    PIT_HIP(launch_copy(s.Rt, s.R, n, st));
                    PIT_HIP(launch_copy(s.P, s.R, n, st));
                    rho_new = hc.dot[1];
                    rho_idx = 1;
                    restarts++;
                }
                rho = rho_dev = rho_new;
                k++;
                continue;
            }
        }
        // D = G^{-1} F P (known already when the one-sync iteration broke down)
        double dr = 0.0;
        if (!dr_zero) {
            if ((rc = s.matvec(s.P, s.D))) return rc;
            const double *a[1] = {s.D}, *b[1] = {s.Rt};
            if ((rc = s.reduce(1, a, b, h))) return rc;
            dr = h.dot[0];
        }
        if (dr == 0.0) {  // restart with the current residual, redo D = G^{-1} F P
            PIT_HIP(launch_copy(s.Rt, s.R, n, st));
            PIT_HIP(launch_copy(s.P, s.R, n, st));
            const double *a[1] = {s.R}, *b[1] = {s.R};
            if ((rc = s.reduce(1, a, b, h))) return rc;
            rho = h.dot[0];
            restarts++;
            if ((rc = s.matvec(s.P, s.D))) return rc;
            const double *a2[1] = {s.D}, *b2[1] = {s.Rt};
            if ((rc = s.reduce(1, a2, b2, h))) return rc;
            dr = h.dot[0];
            if (dr == 0.0) {
                status = PIT_EBREAKDOWN;
                break;
            }
        }
        const double alpha = rho / dr;
        if ((rc = s.kopen())) return rc;
        PIT_HIP(launch_axpby(s.S, s.R, 1.0, s.D, -alpha, n, st));  // S = R - alpha D
        if ((rc = s.kclose())) return rc;
        if (o.half_step_check) {
            const double *a[1] = {s.S}, *b[1] = {s.S};
            if ((rc = s.reduce(1, a, b, h))) return rc;
            if (!(h.nmax[0] > o.tol * scale)) {
                PIT_HIP(launch_axpby(X, X, 1.0, s.P, alpha, n, st));
                PIT_HIP(launch_copy(s.R, s.S, n, st));
                nrm = h.nmax[0];
                k++;
                continue;
            }
        }
        // K = G^{-1} F S
        if ((rc = s.matvec(s.S, s.K))) return rc;
        {
            const double *a[3] = {s.K, s.K, s.S}, *b[3] = {s.S, s.K, s.S};
            if ((rc = s.reduce(3, a, b, h))) return rc;
        }
        const double ks = h.dot[0], kk = h.dot[1], snorm = h.nmax[2];
        if (kk == 0.0) {  // S = 0: the half step solved the system
            PIT_HIP(launch_axpby(X, X, 1.0, s.P, alpha, n, st));
            PIT_HIP(launch_copy(s.R, s.S, n, st));
            nrm = snorm;
            k++;
            continue;
        }
        const double omega = ks / kk;
        if (omega == 0.0) {
            PIT_HIP(launch_axpby(X, X, 1.0, s.P, alpha, n, st));
            PIT_HIP(launch_copy(s.R, s.S, n, st));
            PIT_HIP(launch_copy(s.Rt, s.R, n, st));
            PIT_HIP(launch_copy(s.P, s.R, n, st));
            const double *a[1] = {s.R}, *b[1] = {s.R};
            if ((rc = s.reduce(1, a, b, h))) return rc;
            rho = h.dot[0];
            nrm = h.nmax[0];
            restarts++;
            k++;
            continue;
        }
        // X and R updates
        if ((rc = s.kopen())) return rc;
        PIT_HIP(launch_update_xr(X, s.R, s.P, s.S, s.K, alpha, omega, n, st));
        if ((rc = s.kclose())) return rc;
        // beta (and the norm for the next stopping test)
        {
            const double *a[2] = {s.R, s.R}, *b[2] = {s.Rt, s.R};
            if ((rc = s.reduce(2, a, b, h))) return rc;
        }
        double rho_new = h.dot[0];
        nrm = h.nmax[1];
        const double beta = (alpha / omega) * (rho_new / rho);
        // new direction P
        if ((rc = s.kopen())) return rc;
        PIT_HIP(launch_update_p(s.P, s.R, s.D, beta, omega, n, st));
        if ((rc = s.kclose())) return rc;
        // restart test with epsilon_0
        if (std::fabs(rho_new) <= o.restart_tol) {
            PIT_HIP(launch_copy(s.Rt, s.R, n, st));
            PIT_HIP(launch_copy(s.P, s.R, n, st));
            rho_new = h.dot[1];
            restarts++;
        }
        rho = rho_new;
        k++;
    }
    if (ctx->dim2()) PIT_HIP(launch_copy(Xu, X, n, st));
    else PIT_HIP(launch_from_chunked(X, Xu, ctx->N, ctx->npts, NT, C, st));
    PIT_HIP(hipStreamSynchronize(st));
    if (info) {
        info->status = status;
        info->iters = k;
        info->matvecs = s.matvecs;
        info->restarts = restarts;
        info->res_norm = nrm;
        info->history_len = hl;
        info->n_fine = s.n_fine;
        info->n_coarse = s.n_coarse;
        info->ms_fine = Solver::total_ms(s.ev_fine);
        info->ms_coarse = Solver::total_ms(s.ev_coarse);
        info->n_fine_timed = (int)s.ev_fine.size();
        info->n_coarse_timed = (int)s.ev_coarse.size();
        info->ms_krylov = Solver::total_ms(s.ev_kry);
        info->n_krylov_timed = s.n_kry_timed;
        info->ms_total =
            std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

// ---------------------------------------------------------------------------
// Line-shape autotuner: times one preconditioned product (fine apply plus
// coarse sweep, in the layout pit_solve uses) for every supported shape that
// covers the line, and records the fastest for pit_create.
// ---------------------------------------------------------------------------
namespace {

// 2D candidates: x strip heights x the y shapes that cover the column
// (at most four times its length), and the coarse columns per workgroup
// (columns up to 512 rows; otherwise the column-strip kernel, 0).  The
// first candidate carries the first value of every axis, so the apply is
// timed once per (R, y shape) and the sweep once per column count.
std::vector<AdiTune> adi_candidates(const pit_problem &p)
{
    const int My = p.M[1];
    std::vector<AdiTune> v;
    std::vector<int> ycws = My <= 512 ? std::vector<int>{2, 1, 4} : std::vector<int>{0};
    bool first = true;
    for (int R : {32, 8, 16, 64})
        for (const auto &a : kYMenu) {
            if (yshape_rows(a) < My || yshape_rows(a) > std::max(4 * My, 256)) continue;
            if (first) {
                for (int w : ycws) v.push_back(AdiTune{R, a.wy, a.cy, a.seg, w});
                first = false;
            } else {
                v.push_back(AdiTune{R, a.wy, a.cy, a.seg, ycws.front()});
            }
        }
    return v;
}

std::vector<LineShape> tune_candidates(int M)
{
    std::vector<LineShape> v;
    for (const auto &k : kShapes)
        if (k.NT * k.C >= M && k.NT * k.C <= std::max(4 * M, 64)) v.push_back(k);
    if (v.empty()) v.push_back(default_shape(M));
    return v;
}

struct EventGuard {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventGuard()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct CtxGuard {
    pit_ctx *c = nullptr;
    ~CtxGuard() { delete c; }
};

}  // namespace

extern "C" {

size_t pit_autotune_scratch_bytes(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine,
                                  pit_stepper coarse)
{
    if (validate(problem, N, m, fine, coarse) != PIT_OK) return 0;
    size_t mx = 0;
    if (problem->dim == 2) {
        for (const AdiTune &a : adi_candidates(*problem)) {
            CtxGuard g;
            if (create_ctx(problem, N, m, fine, coarse, nullptr, &g.c, &a) == PIT_OK && !g.c->vel)
                mx = std::max(mx, g.c->total);
        }
        return mx;
    }
    for (LineShape sh : tune_candidates(problem->M[0])) {
        CtxGuard g;
        if (create_ctx(problem, N, m, fine, coarse, &sh, &g.c) == PIT_OK) mx = std::max(mx, g.c->total);
    }
    return mx;
}

int pit_autotune_adi(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
                     void *scratch, size_t bytes, int32_t out[5], float out_ms[2], void *stream)
{
    if (!problem || !out || !scratch || (reinterpret_cast<uintptr_t>(scratch) % kAlign) != 0) return PIT_EINVAL;
    int rc = validate(problem, N, m, fine, coarse);
    if (rc != PIT_OK) return rc;
    if (problem->dim != 2) return PIT_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    EventGuard ev;
    PIT_HIP(hipEventCreate(&ev.a));
    PIT_HIP(hipEventCreate(&ev.b));
    // best apply shape (R, y shape) and best sweep shape (coarse columns per
    // workgroup), each timed on its own operation
    float best_apply = -1.0f, best_sweep = -1.0f;
    AdiTune win{0, 0, 0, 0, 0};
    bool shared_tables = false;
    const std::vector<AdiTune> cands = adi_candidates(*problem);
    if (cands.empty()) return PIT_EINVAL;
    const AdiTune f0 = cands.front();
    for (const AdiTune &a : cands) {
        CtxGuard g;
        if (create_ctx(problem, N, m, fine, coarse, nullptr, &g.c, &a) != PIT_OK) continue;
        if (g.c->vel) {  // per-line or whole-slice kernels: no shape to choose
            shared_tables = true;
            break;
        }
        if (g.c->total > bytes) continue;
        if ((rc = pit_bind_workspace(g.c, scratch, bytes)) != PIT_OK) return rc;
        pit_ctx *c = g.c;
        PIT_HIP(launch_fill0(c->vec(0), kSolveVectors * c->ntc(), st));
        for (int op = 0; op < 2; ++op) {
            // the apply depends on (R, y shape) only, the sweep on the coarse
            // columns only: time each where the candidate varies it
            const bool first_y = a.ycw == f0.ycw;
            const bool first_ry = a.R == f0.R && a.wy == f0.wy && a.cy == f0.cy && a.seg == f0.seg;
            if ((op == 0 && !first_y) || (op == 1 && !first_ry)) continue;
            float t = 0.0f;
            for (int rep = 0; rep < 3; ++rep) {  // the first is a warm-up (and the graph capture)
                PIT_HIP(hipEventRecord(ev.a, st));
                if (op == 0) PIT_HIP(op_apply(c, c->vec(2), c->vec(6), 0, 0, true, st));
                else PIT_HIP(op_sweep(c, c->vec(6), c->vec(3), true, st));
                PIT_HIP(hipEventRecord(ev.b, st));
                PIT_HIP(hipEventSynchronize(ev.b));
                float ms = 0.0f;
                PIT_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                if (rep == 1 || (rep > 1 && ms < t)) t = ms;
            }
            if (op == 0 && (best_apply < 0.0f || t < best_apply)) {
                best_apply = t;
                win.R = c->adi_R;
                win.wy = c->ash.wy;
                win.cy = c->ash.cy;
                win.seg = c->ash.seg;
            }
            if (op == 1 && (best_sweep < 0.0f || t < best_sweep)) {
                best_sweep = t;
                win.ycw = c->ycc ? c->ycw : 0;
            }
        }
    }
    if (shared_tables) return PIT_EINVAL;
    if (best_apply < 0.0f || best_sweep < 0.0f) return PIT_ENOMEM;  // nothing fitted the scratch memory
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned2[tune_key2(*problem, fine, coarse)] = win;
    }
    out[0] = win.R;
    out[1] = win.wy;
    out[2] = win.cy;
    out[3] = win.seg;
    out[4] = win.ycw;
    if (out_ms) {
        out_ms[0] = best_apply;
        out_ms[1] = best_sweep;
    }
    return PIT_OK;
}

int pit_autotune(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
                 void *scratch, size_t bytes, int32_t out[2], float *out_ms, void *stream)
{
    if (!problem || !out || !scratch || (reinterpret_cast<uintptr_t>(scratch) % kAlign) != 0) return PIT_EINVAL;
    int rc = validate(problem, N, m, fine, coarse);
    if (rc != PIT_OK) return rc;
    if (problem->dim != 1) return PIT_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    EventGuard ev;
    PIT_HIP(hipEventCreate(&ev.a));
    PIT_HIP(hipEventCreate(&ev.b));
    float best = 0.0f;
    LineShape bs{0, 0};
    for (LineShape sh : tune_candidates(problem->M[0])) {
        CtxGuard g;
        if (create_ctx(problem, N, m, fine, coarse, &sh, &g.c) != PIT_OK || g.c->total > bytes) continue;
        if ((rc = pit_bind_workspace(g.c, scratch, bytes)) != PIT_OK) return rc;
        pit_ctx *c = g.c;
        PIT_HIP(launch_fill0(c->vec(0), kSolveVectors * c->ntc(), st));
        float t = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {  // the first is a warm-up
            PIT_HIP(hipEventRecord(ev.a, st));
            PIT_HIP(op_apply(c, c->vec(2), c->vec(6), 0, 0, true, st));
            PIT_HIP(op_sweep(c, c->vec(6), c->vec(3), true, st));
            PIT_HIP(hipEventRecord(ev.b, st));
            PIT_HIP(hipEventSynchronize(ev.b));
            float ms = 0.0f;
            PIT_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            if (rep == 1 || (rep > 1 && ms < t)) t = ms;
        }
        if (bs.NT == 0 || t < best) {
            best = t;
            bs = sh;
        }
    }
    if (bs.NT == 0) return PIT_ENOMEM;  // no candidate fitted the scratch memory
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(*problem, fine, coarse)] = bs;
    }
    out[0] = bs.NT;
    out[1] = bs.C;
    if (out_ms) *out_ms = best;
    return PIT_OK;
}

int pit_autotune_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_tuned2.clear();
    return PIT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Parareal as preconditioned Richardson (Sec. 2, eq. (pararealAlgebraic)):
//   X^{k+1} = X^k + G^{-1}(B - F X^k),
// one preconditioned product per iteration on the same apply and sweep as
// Algorithm 1; exact after N iterations (the iteration matrix I - G^{-1}F is
// nilpotent).
// ---------------------------------------------------------------------------
extern "C" int pit_parareal(pit_ctx *ctx, const double *u0, double *X, const pit_solve_opts *opts,
                            pit_solve_info *info, void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !ctx->ws || !u0 || !X) return PIT_EINVAL;
    pit_solve_opts o{};
    o.tol = 0.0;
    o.max_iter = 0;
    o.norm_mode = PIT_ABS;
    o.x0_mode = PIT_X0_ZERO;
    if (opts) o = *opts;
    // X^N is exact; the (N+1)-th update (zero up to rounding) is what shows it
    if (o.max_iter <= 0) o.max_iter = ctx->N + 1;
    if (o.x0_mode < PIT_X0_ZERO || o.x0_mode > PIT_X0_COARSE || !(o.tol >= 0.0)) return PIT_EINVAL;
    Solver s{};
    s.c = ctx;
    s.st = static_cast<hipStream_t>(stream);
    if (o.timing < 0) return PIT_EINVAL;
    s.timing = o.timing;
    const long n = ctx->ntc();
    const int NT = ctx->lf.sh.NT, C = ctx->lf.sh.C;
    hipStream_t st = s.st;
    double *const Xu = X;
    double *const Xc = ctx->vec(7), *const R = ctx->vec(0), *const U0 = ctx->vec(1);
    // B in the working layout: u0 in slice 0, b (or 0) in the others
    PIT_HIP(launch_fill0(U0, n, st));
    if (ctx->dim2()) PIT_HIP(launch_copy(U0, u0, ctx->npts, st));
    else PIT_HIP(launch_to_chunked(u0, U0, 1, ctx->npts, NT, C, st));
    PIT_HIP(fill_forced(ctx, U0, st));
    int rc;
    if (o.x0_mode == PIT_X0_ZERO) {
        PIT_HIP(launch_fill0(Xc, n, st));
    } else if (o.x0_mode == PIT_X0_COARSE) {
        if ((rc = s.sweep(U0, Xc))) return rc;
    } else if (ctx->dim2()) {
        PIT_HIP(launch_copy(Xc, Xu, n, st));
    } else {
        PIT_HIP(launch_to_chunked(Xu, Xc, ctx->N, ctx->npts, NT, C, st));
    }
    RedOut h{};
    double nrm = 0.0, scale = 1.0;
    int k = 0, hl = 0, status = PIT_ENOCONV;
    for (; k < o.max_iter; ++k) {
        // R = G^{-1}(B - F X)
        if ((rc = s.apply(Xc, R))) return rc;
        if (ctx->has_src()) PIT_HIP(launch_axpby(R, U0, 1.0, R, -1.0, n, st));
        else PIT_HIP(launch_b_minus(R, R, U0, ctx->ld, n, st));
        if ((rc = s.sweep(R, R))) return rc;
        s.matvecs++;
        {
            const double *a[1] = {R}, *b[1] = {R};
            if ((rc = s.reduce(1, a, b, h))) return rc;
        }
        nrm = h.nmax[0];
        if (k == 0 && o.norm_mode == PIT_REL && nrm > 0.0) scale = nrm;
        if (info && info->history && hl < info->history_cap) info->history[hl++] = nrm;
        PIT_HIP(launch_axpby(Xc, Xc, 1.0, R, 1.0, n, st));  // X^{k+1} = X^k + R^k
        if (!std::isfinite(nrm)) {
            status = PIT_EBREAKDOWN;
            ++k;
            break;
        }
        if (!(nrm > o.tol * scale)) {
            status = PIT_OK;
            ++k;
            break;
        }
    }
    if (status == PIT_ENOCONV && o.tol == 0.0) status = PIT_OK;  // a fixed number of iterations asked for
    if (ctx->dim2()) PIT_HIP(launch_copy(Xu, Xc, n, st));
    else PIT_HIP(launch_from_chunked(Xc, Xu, ctx->N, ctx->npts, NT, C, st));
    PIT_HIP(hipStreamSynchronize(st));
    if (info) {
        info->status = status;
        info->iters = k;
        info->matvecs = s.matvecs;
        info->restarts = 0;
        info->res_norm = nrm;
        info->history_len = hl;
        info->n_fine = s.n_fine;
        info->n_coarse = s.n_coarse;
        info->ms_fine = Solver::total_ms(s.ev_fine);
        info->ms_coarse = Solver::total_ms(s.ev_coarse);
        info->n_fine_timed = (int)s.ev_fine.size();
        info->n_coarse_timed = (int)s.ev_coarse.size();
        info->ms_krylov = Solver::total_ms(s.ev_kry);
        info->n_krylov_timed = s.n_kry_timed;
        info->ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}
