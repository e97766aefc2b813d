/*
 * pit_oracle.c -- plain, slow, obviously correct CPU reference for PiTSBiCG
 * (Riahi, "PiTSBiCG: Parallel in Time Stable Bi-Conjugate Gradient Algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.  Everything is IEEE FP64, built without fast-math and without FMA
 * contraction.
 *
 * What it computes, in the paper's terms:
 *   - slice propagators: the fine solver F and the coarse solver G over one
 *     slice of length DT = T/N (Sec. 2, eq. (Cauchyn) and the continuity
 *     condition eq. (continuity)); here F = m implicit steps, G = c steps;
 *   - the all-at-once operator  (F Lambda)_0 = lambda_0,
 *     (F Lambda)_n = lambda_n - F(lambda_{n-1})  (Sec. 2, eq. (algebraiclinearsystem));
 *   - the coarse preconditioner solve z = G^{-1} v by forward substitution
 *     (Sec. 3, eq. (eqinverse) and the paragraph after Algorithm 1);
 *   - the block inner product <U,V> = sum_n <u_n,v_n>_{L2(Omega)} (Sec. 3);
 *   - Algorithm 1 (PiTSBiCG): left-preconditioned BiCGStab with the
 *     shadow-residual restart (Sec. 3, Algorithm 1);
 *   - parareal, both as the preconditioned Richardson iteration
 *     (Sec. 2, eq. (pararealAlgebraic)) and as the predictor-corrector
 *     recursion (Sec. 2, eq. (pararealscheme), read with the standard
 *     superscripts);
 *   - the serial fine trajectory lambda_{n+1} = F(lambda_n), the exact
 *     solution of the all-at-once system (Sec. 2, eq. (continuity)).
 *
 * Discretisation (synthetic finite-difference stand-ins for the paper's FEM
 * experiments): 1D Dirichlet-0 or periodic, 2D Dirichlet-0 on a rectangle,
 * second-order central differences.
 *   L u = nu*D2 u - a*D1c u - r*u                       (1D)
 *   IE:  (I - dt L) u' = u + dt f
 *   CN:  (I - dt/2 L) u' = (I + dt/2 L) u + dt f
 *   PR-ADI (2D): (I - dt/2 Lx) u* = (I + dt/2 Ly) u + dt/2 f,
 *                (I - dt/2 Ly) u' = (I + dt/2 Lx) u* + dt/2 f,
 *       with Lx = nu*D2x - ux(y)*D1x - r/2 and Ly = nu*D2y - uy(x)*D1y - r/2;
 *   backward-Euler splitting (2D): (I - dt Lx) u* = u + dt f,
 *                                  (I - dt Ly) u' = u*  (same Lx, Ly);
 *       the velocity is a constant (ax, ay) plus a rigid rotation of rate rot
 *       about the centre (xc, yc) of the domain:
 *           ux = ax - rot*(y - yc),  uy = ay + rot*(x - xc)
 *       (rot = 1 with the centre at the origin is the u = [-y, x] of the
 *       advection-diffusion-reaction test of Sec. 4).  ux is constant along a
 *       row and uy along a column, so every line is a constant-stencil
 *       tridiagonal system, one per row or column.
 * The operator may depend on time, constant on each slice: nu s_n on slice
 * n (s_n > 0 given, orc_set_nu_t); F_n and G_n then differ from slice to
 * slice, and the all-at-once operator carries F_{n-1} below the diagonal in
 * row n and the preconditioner G_{n-1}.
 * f is an optional source (the source term of Sec. 2, eq. (Cauchy)); without
 * it f = 0.  It is either constant in time or separable, f(t, x) = g(t) h(x),
 * with g given at the fine step times t_j = j dt, j = 0..N m.  Fine step j
 * (from t_j to t_{j+1}) takes f(t_{j+1}) under IE and the backward-Euler
 * splitting, the trapezoidal mean
 * (f(t_j) + f(t_{j+1}))/2 under CN, and the midpoint value, read as that same
 * mean, in both PR-ADI half-steps.  With a source the propagator of slice n
 * is affine, F_n(u) = F0(u) + b_n with b_n = F_n(0), the forced response of
 * slice n (one b for all slices when f is constant).  The all-at-once system
 * keeps its linear operator (F0 below the diagonal) and gets
 * B = (u0, b_0, .., b_{N-2}) (eq. (Cauchyn): slice n carries f restricted to
 * [T_n, T_{n+1}]): its solution is again the serial trajectory
 * lambda_{n+1} = F_n(lambda_n) (the middle entries of B in Sec. 2, eq.
 * (algebraiclinearsystem)).  The preconditioner uses the linear coarse
 * propagator G0.
 * Tridiagonal systems: Thomas algorithm without pivoting.  Periodic (cyclic)
 * systems: Sherman-Morrison rank-one correction.
 *
 * Layout: a block vector is N slices, each slice npts contiguous doubles;
 * 2D slices are row-major u[j*Mx + i] with x (index i) fastest.  Dirichlet
 * vectors hold interior points only; periodic vectors hold j = 0..M-1.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_DIRICHLET = 0, ORC_PERIODIC = 1 };
enum { ORC_IE = 0, ORC_CN = 1, ORC_ADI = 2, ORC_ADI_IE = 3 };
enum { ORC_ABS = 0, ORC_REL = 1 };
enum { ORC_X0_ZERO = 0, ORC_X0_GIVEN = 1, ORC_X0_COARSE = 2 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOCONV = -4, ORC_EBREAKDOWN = -5 };

typedef struct {
    int dim, Mx, My, bc;
    double Lx, Ly, nu, ax, ay, react, T, rot;
    int N, m, fine_scheme, c, coarse_scheme;
    /* derived */
    int npts;      /* points per slice */
    double hx, hy; /* grid spacing */
    double w;      /* L2 quadrature weight h^d */
    double DT;     /* slice length T/N */
    double *src;   /* source f, or its profile h (npts values, owned), or NULL */
    double *gt;    /* g(t_j), j = 0..N m (owned), or NULL: f constant in time */
    int fine_f32;  /* 1: the fine propagator is the FP32-fine form (emulated) */
    double *nus;   /* per-slice diffusion factors s_n (N values, owned): nu on
                      slice n is nu * s_n; NULL: nu constant in time */
} orc_ctx;

static int g_threads = 1;

void orc_set_threads(int n)
{
    g_threads = n > 0 ? n : 1;
#ifdef _OPENMP
    omp_set_num_threads(g_threads);
#endif
}
int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------- */
/* Tridiagonal solves                                                         */
/* ------------------------------------------------------------------------- */

/* Solve the n x n tridiagonal system with sub-diagonal a[1..n-1], diagonal
 * b[0..n-1], super-diagonal c[0..n-2] and right-hand side d; result in x.
 * Thomas algorithm, no pivoting.  cp and dp are work arrays of length n. */
static void thomas(int n, const double *a, const double *b, const double *c,
                   const double *d, double *x, double *cp, double *dp)
{
    cp[0] = (n > 1) ? c[0] / b[0] : 0.0;
    dp[0] = d[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / den : 0.0;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* Solve the cyclic tridiagonal system whose row i has a[i] on column i-1,
 * b[i] on column i and c[i] on column i+1, columns taken modulo n (a[0] sits
 * on column n-1, c[n-1] on column 0).  Sherman-Morrison: A = B + u v^T with
 * u = (gam, 0, .., 0, c[n-1]), v = (1, 0, .., 0, a[0]/gam), gam = -b[0], so
 * B is A without the corners and with its first and last diagonal entries
 * shifted.  x = y - (v.y)/(1 + v.z) z where B y = d and B z = u.
 * work: 6n doubles.  Requires n >= 3. */
static void cyclic(int n, const double *a, const double *b, const double *c,
                   const double *d, double *x, double *work)
{
    double *bb = work, *y = work + n, *z = work + 2 * n, *cp = work + 3 * n,
           *dp = work + 4 * n, *u = work + 5 * n;
    double gam = -b[0];
    double alpha = c[n - 1]; /* A[n-1][0] */
    double beta = a[0];      /* A[0][n-1] */
    for (int i = 0; i < n; ++i) {
        bb[i] = b[i];
        u[i] = 0.0;
    }
    bb[0] = b[0] - gam;
    bb[n - 1] = b[n - 1] - alpha * beta / gam;
    u[0] = gam;
    u[n - 1] = alpha;
    thomas(n, a, bb, c, d, y, cp, dp);
    thomas(n, a, bb, c, u, z, cp, dp);
    double vy = y[0] + beta / gam * y[n - 1];
    double vz = z[0] + beta / gam * z[n - 1];
    double fac = vy / (1.0 + vz);
    for (int i = 0; i < n; ++i) x[i] = y[i] - fac * z[i];
}

/* Exported for the brute-force pins against dense Gaussian elimination. */
void orc_tridiag_solve(int n, const double *a, const double *b, const double *c,
                       const double *d, double *x)
{
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    thomas(n, a, b, c, d, x, w, w + n);
    free(w);
}

void orc_cyclic_solve(int n, const double *a, const double *b, const double *c,
                      const double *d, double *x)
{
    double *w = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    cyclic(n, a, b, c, d, x, w);
    free(w);
}

/* ------------------------------------------------------------------------- */
/* One implicit step of the 1D and 2D schemes                                 */
/* ------------------------------------------------------------------------- */

/* Stencil of the 1D operator L along one axis:
 *   (L u)_j = lo*u_{j-1} + di*u_j + up*u_{j+1}. */
static void op1d(double nu, double a, double r, double h, double *lo, double *di, double *up)
{
    *lo = nu / (h * h) + a / (2.0 * h);
    *di = -2.0 * nu / (h * h) - r;
    *up = nu / (h * h) - a / (2.0 * h);
}

/* Solve (I - th*L) x = d along one line of n points, L given by (lo,di,up),
 * Dirichlet-0 or periodic.  work: >= 9n doubles. */
static void implicit_line(int n, int bc, double th, double lo, double di, double up,
                          const double *d, double *x, double *work)
{
    double *a = work, *b = work + n, *c = work + 2 * n, *w = work + 3 * n;
    for (int i = 0; i < n; ++i) {
        a[i] = -th * lo;
        b[i] = 1.0 - th * di;
        c[i] = -th * up;
    }
    if (bc == ORC_PERIODIC)
        cyclic(n, a, b, c, d, x, w);
    else
        thomas(n, a, b, c, d, x, w, w + n);
}

/* 2D velocity: x-component on row j (constant along the row), y-component on
 * column i; interior points x_i = (i+1) hx, y_j = (j+1) hy. */
static double ux_at(const orc_ctx *C, int j)
{
    return C->ax - C->rot * ((j + 1) * C->hy - 0.5 * C->Ly);
}
static double uy_at(const orc_ctx *C, int i)
{
    return C->ay + C->rot * ((i + 1) * C->hx - 0.5 * C->Lx);
}

/* True when a 2D step should share its lines among the threads: called
 * outside a parallel region (slices already running in parallel keep one
 * thread each) on a slice large enough to pay for it. */
static int lines_in_parallel(const orc_ctx *C)
{
#ifdef _OPENMP
    return g_threads > 1 && !omp_in_parallel() && C->npts >= 4096;
#else
    (void)C;
    return 0;
#endif
}

/* Work size in doubles needed by one_step. */
static size_t step_work(const orc_ctx *C)
{
    int nmax = C->Mx > C->My ? C->Mx : C->My;
    return (size_t)C->npts + 12 * (size_t)nmax;
}

/* Value stored by a 2D half step: rounded to float when `rnd` says so (the
 * FP32-fine form's field storage). */
static double stored(double v, int rnd) { return rnd ? (double)(float)v : v; }

/* out = one step of `scheme` with time step dt applied to u (no aliasing);
 * the source of the step is wf * f (f NULL: none).  2D only: rnd bit 1 rounds
 * to float what the first half step hands to the second (PR-ADI: the second
 * half's right-hand side; the backward-Euler splitting: the intermediate
 * field), bit 2 the output. */
static void one_step(const orc_ctx *C, int scheme, double dt, const double *u, double *out,
                     double *work, const double *f, double wf, int rnd)
{
    if (C->dim == 1) {
        int n = C->Mx;
        double lo, di, up;
        op1d(C->nu, C->ax, C->react, C->hx, &lo, &di, &up);
        double *rhs = work, *lw = work + n;
        if (scheme == ORC_IE) {
            if (f) { /* rhs = u + dt f */
                for (int j = 0; j < n; ++j) rhs[j] = u[j] + dt * (wf * f[j]);
                implicit_line(n, C->bc, dt, lo, di, up, rhs, out, lw);
            } else {
                implicit_line(n, C->bc, dt, lo, di, up, u, out, lw);
            }
        } else { /* CN: rhs = (I + dt/2 L) u + dt f */
            double th = 0.5 * dt;
            for (int j = 0; j < n; ++j) {
                double um, uq;
                if (C->bc == ORC_PERIODIC) {
                    um = u[(j - 1 + n) % n];
                    uq = u[(j + 1) % n];
                } else {
                    um = (j > 0) ? u[j - 1] : 0.0;
                    uq = (j < n - 1) ? u[j + 1] : 0.0;
                }
                rhs[j] = u[j] + th * (lo * um + di * u[j] + up * uq);
                if (f) rhs[j] += dt * (wf * f[j]);
            }
            implicit_line(n, C->bc, th, lo, di, up, rhs, out, lw);
        }
        return;
    }
    /* 2D Peaceman-Rachford ADI, Dirichlet-0.  Row j: x-operator with velocity
     * ux(y_j); column i: y-operator with velocity uy(x_i).  The lines of a
     * half step are independent; outside a parallel region (one slice at a
     * time, as in the serial trajectory) they are shared among the threads,
     * each line computed exactly as by one thread. */
    int nx = C->Mx, ny = C->My;
    int nmax = nx > ny ? nx : ny;
    double *star = work; /* npts */
    int par = lines_in_parallel(C);
    if (scheme == ORC_ADI_IE) {
        /* (I - dt*Lx) u* = u + dt*f row by row, then (I - dt*Ly) u' = u* column by column */
#pragma omp parallel num_threads(g_threads) if (par)
        {
            double *line = (double *)malloc(sizeof(double) * 11 * (size_t)nmax);
            double *sol = line + nmax, *lw = sol + nmax;
            double xlo, xdi, xup, ylo, ydi, yup;
#pragma omp for schedule(static)
            for (int j = 0; j < ny; ++j) {
                for (int i = 0; i < nx; ++i) {
                    line[i] = u[j * nx + i];
                    if (f) line[i] += dt * (wf * f[j * nx + i]);
                }
                op1d(C->nu, ux_at(C, j), 0.5 * C->react, C->hx, &xlo, &xdi, &xup);
                implicit_line(nx, ORC_DIRICHLET, dt, xlo, xdi, xup, line, sol, lw);
                for (int i = 0; i < nx; ++i) star[j * nx + i] = stored(sol[i], rnd & 1);
            }
#pragma omp for schedule(static)
            for (int i = 0; i < nx; ++i) {
                for (int j = 0; j < ny; ++j) line[j] = star[j * nx + i];
                op1d(C->nu, uy_at(C, i), 0.5 * C->react, C->hy, &ylo, &ydi, &yup);
                implicit_line(ny, ORC_DIRICHLET, dt, ylo, ydi, yup, line, sol, lw);
                for (int j = 0; j < ny; ++j) out[j * nx + i] = stored(sol[j], rnd & 2);
            }
            free(line);
        }
        return;
    }
    double th = 0.5 * dt;
#pragma omp parallel num_threads(g_threads) if (par)
    {
        double *line = (double *)malloc(sizeof(double) * 11 * (size_t)nmax);
        double *sol = line + nmax, *lw = sol + nmax;
        double xlo, xdi, xup, ylo, ydi, yup;
        /* half-step 1: rhs = (I + th*Ly) u + th*f, then (I - th*Lx) u* = rhs row by row */
#pragma omp for schedule(static)
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                op1d(C->nu, uy_at(C, i), 0.5 * C->react, C->hy, &ylo, &ydi, &yup);
                double c0 = u[j * nx + i];
                double cm = (j > 0) ? u[(j - 1) * nx + i] : 0.0;
                double cq = (j < ny - 1) ? u[(j + 1) * nx + i] : 0.0;
                line[i] = c0 + th * (ylo * cm + ydi * c0 + yup * cq);
                if (f) line[i] += th * (wf * f[j * nx + i]);
            }
            op1d(C->nu, ux_at(C, j), 0.5 * C->react, C->hx, &xlo, &xdi, &xup);
            implicit_line(nx, ORC_DIRICHLET, th, xlo, xdi, xup, line, sol, lw);
            for (int i = 0; i < nx; ++i) star[j * nx + i] = sol[i];
        }
        /* half-step 2: rhs = (I + th*Lx) u* + th*f, then (I - th*Ly) u' = rhs column by column
         * (the implicit barrier of the loop above orders the two halves).  What the
         * first half hands to the second is this right-hand side: in the FP32-fine
         * form (rnd bit 1) it is the value stored in FP32. */
#pragma omp for schedule(static)
        for (int i = 0; i < nx; ++i) {
            for (int j = 0; j < ny; ++j) {
                op1d(C->nu, ux_at(C, j), 0.5 * C->react, C->hx, &xlo, &xdi, &xup);
                double c0 = star[j * nx + i];
                double cm = (i > 0) ? star[j * nx + i - 1] : 0.0;
                double cq = (i < nx - 1) ? star[j * nx + i + 1] : 0.0;
                line[j] = c0 + th * (xlo * cm + xdi * c0 + xup * cq);
                if (f) line[j] += th * (wf * f[j * nx + i]);
                line[j] = stored(line[j], rnd & 1);
            }
            op1d(C->nu, uy_at(C, i), 0.5 * C->react, C->hy, &ylo, &ydi, &yup);
            implicit_line(ny, ORC_DIRICHLET, th, ylo, ydi, yup, line, sol, lw);
            for (int j = 0; j < ny; ++j) out[j * nx + i] = stored(sol[j], rnd & 2);
        }
        free(line);
    }
}

/* Weight of the source profile in global fine step j (from t_j to t_{j+1}),
 * 1 when the source is constant in time or j < 0. */
static double src_weight(const orc_ctx *C, int scheme, int j)
{
    if (!C->gt || j < 0) return 1.0;
    return (scheme == ORC_IE || scheme == ORC_ADI_IE) ? C->gt[j + 1] : 0.5 * (C->gt[j] + C->gt[j + 1]);
}

static void propagate_f32_1d(const orc_ctx *C, int scheme, int nsteps, double span, const double *in,
                             double *out);

/* Apply `nsteps` steps of `scheme`, each of length span/nsteps, with source f
 * (NULL: none): out = step^nsteps(in).  j0 is the global index of the first
 * step (for the weights of a time-dependent source), -1 for none.  in and
 * out may alias. */
static void propagate(const orc_ctx *C, int scheme, int nsteps, double span, const double *in,
                      double *out, const double *f, int j0, int f32)
{
    if (f32 && C->dim == 1 && !f) {
        propagate_f32_1d(C, scheme, nsteps, span, in, out);
        return;
    }
    size_t np = (size_t)C->npts;
    double dt = span / nsteps;
    double *base = (double *)malloc(sizeof(double) * (2 * np + step_work(C)));
    double *a = base, *b = base + np, *work = base + 2 * np;
    memcpy(a, in, sizeof(double) * np);
    for (int s = 0; s < nsteps; ++s) {
        one_step(C, scheme, dt, a, b, work, f, src_weight(C, scheme, j0 < 0 ? -1 : j0 + s),
                 f32 ? 1 | (s < nsteps - 1 ? 2 : 0) : 0);
        double *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, sizeof(double) * np);
    free(base);
}

/* ------------------------------------------------------------------------- */
/* The FP32-fine form, emulated                                               */
/* ------------------------------------------------------------------------- */
/* The paper fixes no precision.  The FP32-fine form (a reading: the fine
 * propagator in FP32, everything else in FP64) is emulated here, so that the
 * accuracy it can reach is known on the CPU.
 *
 * 1D (IE, CN): FP32 state and step arithmetic, in increment form:
 *   u' = u + D,   (I - th L) D = dt L u   (th = dt for IE, dt/2 for CN),
 * equal to the standard form in exact arithmetic; a constant field gives
 * D = 0 exactly.  dt L u is evaluated from differences,
 *   pd (u_{j-1} - 2 u_j + u_{j+1}) + pa (u_{j-1} - u_{j+1}) - pr u_j,
 * with pd = dt nu/h^2, pa = dt a/(2h), pr = dt r each rounded once to float.
 * The Thomas factors of I - th L (and, periodic, the Sherman-Morrison vector)
 * are formed in FP64 and rounded to float; the solve runs in float.  The
 * state is an unevaluated float pair (u, e), u + e the value, updated with
 * Fast2Sum (Dekker 1971): y = D + e, s = u + y, e' = y - (s - u), u' = s.
 * The slice's input and output are FP64.
 * 2D (PR-ADI, backward-Euler splitting): FP64 arithmetic with the fields
 * between half steps stored in FP32: every half step's output is rounded to
 * float except the last one of the slice.
 * No source in either. */
typedef struct {
    int n, cyc;
    float *l, *ip, *cp, *z; /* multipliers, inverse pivots, c/pivot, SM vector */
    float bg, inv_den;      /* SM: beta/gam and 1/(1 + v.z) */
} f32_line;

/* Float factors of the n x n matrix with constant sub a, diagonal b, super c
 * (cyclic: the corners too), in the layout of thomas() and cyclic(). */
static void f32_line_build(int n, int cyc, double a, double b, double c, f32_line *F)
{
    double *bb = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *piv = bb + n, *y = bb + 2 * n;
    F->n = n;
    F->cyc = cyc;
    F->l = (float *)malloc(sizeof(float) * 4 * (size_t)n);
    F->ip = F->l + n;
    F->cp = F->l + 2 * n;
    F->z = F->l + 3 * n;
    double gam = -b;
    for (int i = 0; i < n; ++i) bb[i] = b;
    if (cyc) {
        bb[0] = b - gam;
        bb[n - 1] = b - c * a / gam;
    }
    piv[0] = bb[0];
    F->l[0] = 0.0f;
    for (int i = 1; i < n; ++i) {
        double l = a / piv[i - 1];
        piv[i] = bb[i] - l * c;
        F->l[i] = (float)l;
    }
    for (int i = 0; i < n; ++i) {
        F->ip[i] = (float)(1.0 / piv[i]);
        F->cp[i] = (float)((i < n - 1) ? c / piv[i] : 0.0);
        F->z[i] = 0.0f;
    }
    F->bg = 0.0f;
    F->inv_den = 0.0f;
    if (cyc) { /* z = B^{-1} (gam, 0, .., 0, c), in FP64 */
        for (int i = 0; i < n; ++i) y[i] = (i == 0) ? gam : (i == n - 1 ? c : 0.0);
        for (int i = 1; i < n; ++i) y[i] -= (a / piv[i - 1]) * y[i - 1];
        y[n - 1] = y[n - 1] / piv[n - 1];
        for (int i = n - 2; i >= 0; --i) y[i] = (y[i] - c * y[i + 1]) / piv[i];
        for (int i = 0; i < n; ++i) F->z[i] = (float)y[i];
        F->bg = (float)(a / gam);
        F->inv_den = (float)(1.0 / (1.0 + y[0] + (a / gam) * y[n - 1]));
    }
    free(bb);
}

/* d := A^{-1} d in float with the factors of F. */
static void f32_line_solve(const f32_line *F, float *d)
{
    int n = F->n;
    for (int i = 1; i < n; ++i) d[i] = d[i] - F->l[i] * d[i - 1];
    d[n - 1] = d[n - 1] * F->ip[n - 1];
    for (int i = n - 2; i >= 0; --i) d[i] = d[i] * F->ip[i] - F->cp[i] * d[i + 1];
    if (F->cyc) {
        float fac = (d[0] + F->bg * d[n - 1]) * F->inv_den;
        for (int i = 0; i < n; ++i) d[i] = d[i] - fac * F->z[i];
    }
}

/* out = nsteps FP32 increment-form steps of `scheme` (IE or CN) of length
 * span/nsteps applied to in (1D, no source); in and out may alias. */
static void propagate_f32_1d(const orc_ctx *C, int scheme, int nsteps, double span, const double *in,
                             double *out)
{
    int n = C->Mx, per = C->bc == ORC_PERIODIC;
    double dt = span / nsteps, th = (scheme == ORC_IE) ? dt : 0.5 * dt, h = C->hx;
    double lo, di, up;
    op1d(C->nu, C->ax, C->react, h, &lo, &di, &up);
    f32_line F;
    f32_line_build(n, per, -th * lo, 1.0 - th * di, -th * up, &F);
    float pd = (float)(dt * (C->nu / (h * h))), pa = (float)(dt * (C->ax / (2.0 * h)));
    float pr = (float)(dt * C->react);
    float *u = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    float *e = u + n, *d = u + 2 * n;
    for (int j = 0; j < n; ++j) {
        u[j] = (float)in[j];
        e[j] = (float)(in[j] - (double)u[j]);
    }
    for (int s = 0; s < nsteps; ++s) {
        for (int j = 0; j < n; ++j) {
            float um, uq;
            if (per) {
                um = u[(j - 1 + n) % n];
                uq = u[(j + 1) % n];
            } else {
                um = (j > 0) ? u[j - 1] : 0.0f;
                uq = (j < n - 1) ? u[j + 1] : 0.0f;
            }
            d[j] = pd * ((um - u[j]) + (uq - u[j])) + pa * (um - uq) - pr * u[j];
        }
        f32_line_solve(&F, d);
        for (int j = 0; j < n; ++j) {
            float y = d[j] + e[j];
            float sum = u[j] + y;
            e[j] = y - (sum - u[j]);
            u[j] = sum;
        }
    }
    for (int j = 0; j < n; ++j) out[j] = (double)u[j] + (double)e[j];
    free(u);
    free(F.l);
}

/* ------------------------------------------------------------------------- */
/* Context                                                                    */
/* ------------------------------------------------------------------------- */

orc_ctx *orc_create(int dim, int Mx, int My, int bc, double Lx, double Ly, double nu, double ax,
                    double ay, double react, double T, int N, int m, int fine_scheme, int c,
                    int coarse_scheme, double rot)
{
    if (dim != 1 && dim != 2) return NULL;
    if (Mx < 3 || N < 1 || m < 1 || c < 1) return NULL;
    if (dim == 2 && (My < 3 || bc != ORC_DIRICHLET)) return NULL;
    if (dim == 1 && rot != 0.0) return NULL; /* rotation: 2D only */
    if (dim == 1 && (fine_scheme >= ORC_ADI || coarse_scheme >= ORC_ADI)) return NULL;
    if (dim == 2 && ((fine_scheme != ORC_ADI && fine_scheme != ORC_ADI_IE) ||
                     (coarse_scheme != ORC_ADI && coarse_scheme != ORC_ADI_IE)))
        return NULL;
    orc_ctx *C = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    C->dim = dim;
    C->Mx = Mx;
    C->My = (dim == 2) ? My : 1;
    C->bc = bc;
    C->Lx = Lx;
    C->Ly = Ly;
    C->nu = nu;
    C->ax = ax;
    C->ay = ay;
    C->react = react;
    C->T = T;
    C->rot = rot;
    C->N = N;
    C->m = m;
    C->fine_scheme = fine_scheme;
    C->c = c;
    C->coarse_scheme = coarse_scheme;
    C->npts = Mx * C->My;
    /* Dirichlet: interior points x_j = (j+1) h, h = L/(M+1); periodic: x_j = j h, h = L/M */
    C->hx = (bc == ORC_PERIODIC) ? Lx / Mx : Lx / (Mx + 1);
    C->hy = (dim == 2) ? Ly / (My + 1) : 1.0;
    C->w = (dim == 2) ? C->hx * C->hy : C->hx;
    C->DT = T / N;
    return C;
}

void orc_destroy(orc_ctx *C)
{
    if (C) {
        free(C->src);
        free(C->gt);
        free(C->nus);
    }
    free(C);
}

/* Set (a copy of) the source f, constant in time, npts values in slice
 * layout; NULL removes it.  A source switches the FP32-fine form off. */
void orc_set_source(orc_ctx *C, const double *f)
{
    if (f) C->fine_f32 = 0;
    free(C->src);
    free(C->gt);
    C->src = NULL;
    C->gt = NULL;
    if (f) {
        C->src = (double *)malloc(sizeof(double) * (size_t)C->npts);
        memcpy(C->src, f, sizeof(double) * (size_t)C->npts);
    }
}

/* Set the separable source f(t, x) = g(t) h(x): h npts values, g its values
 * at the fine step times t_j = j dt, j = 0..N m (N m + 1 values). */
void orc_set_source_t(orc_ctx *C, const double *h, const double *g)
{
    orc_set_source(C, h);
    size_t ng = (size_t)C->N * (size_t)C->m + 1;
    C->gt = (double *)malloc(sizeof(double) * ng);
    memcpy(C->gt, g, sizeof(double) * ng);
}

/* Switch the fine propagator to the emulated FP32-fine form (on = 1) or
 * back to FP64 (on = 0).  Returns -1 (and changes nothing) with a source
 * set, which the FP32 form does not take. */
int orc_set_fine_f32(orc_ctx *C, int on)
{
    if (on && C->src) return ORC_EINVAL;
    C->fine_f32 = on ? 1 : 0;
    return ORC_OK;
}

/* A time-dependent operator, constant on each slice: L(t) = nu s_n D2 - a D1
 * - r on [T_n, T_{n+1}) (the operator of the Cauchy problem restricted to
 * slice n, Sec. 2, eq. (Cauchyn)).  Set (a copy of) the N factors s_n, or
 * NULL for nu constant in time.  Returns -1 unless every s_n is finite and
 * positive. */
int orc_set_nu_t(orc_ctx *C, const double *s)
{
    if (s)
        for (int n = 0; n < C->N; ++n)
            if (!(s[n] > 0.0) || !isfinite(s[n])) return ORC_EINVAL;
    free(C->nus);
    C->nus = NULL;
    if (s) {
        C->nus = (double *)malloc(sizeof(double) * (size_t)C->N);
        memcpy(C->nus, s, sizeof(double) * (size_t)C->N);
    }
    return ORC_OK;
}

/* The context of slice n: C itself, or a copy with nu * s_n. */
static const orc_ctx *on_slice(const orc_ctx *C, int n, orc_ctx *tmp)
{
    if (!C->nus) return C;
    *tmp = *C;
    tmp->nu = C->nu * C->nus[n];
    return tmp;
}

/* The linear part F0 of the fine propagator of slice n (no source). */
static void F_lin(const orc_ctx *C, int n, const double *in, double *out)
{
    orc_ctx t;
    const orc_ctx *S = on_slice(C, n, &t);
    propagate(S, C->fine_scheme, C->m, C->DT, in, out, NULL, -1, C->fine_f32);
}

/* b_n = F_n(0): the forced response of slice n (0 without a source). */
void orc_forced_slice(const orc_ctx *C, int n, double *b)
{
    orc_ctx t;
    const orc_ctx *S = on_slice(C, n, &t);
    memset(b, 0, sizeof(double) * (size_t)C->npts);
    if (C->src) propagate(S, C->fine_scheme, C->m, C->DT, b, b, C->src, n * C->m, 0);
}

/* The forced response of slice 0 (of every slice when f is constant). */
void orc_forced(const orc_ctx *C, double *b) { orc_forced_slice(C, 0, b); }

/* B = (u0, b_0, .., b_{N-2}) (Sec. 2, eq. (algebraiclinearsystem)). */
static void build_B(const orc_ctx *C, const double *u0, double *B)
{
    size_t np = (size_t)C->npts;
    memcpy(B, u0, sizeof(double) * np);
    if (C->N > 1) {
        orc_forced_slice(C, 0, B + np);
        for (int n = 2; n < C->N; ++n) {
            if (C->gt || C->nus) orc_forced_slice(C, n - 1, B + (size_t)n * np);
            else memcpy(B + (size_t)n * np, B + np, sizeof(double) * np);
        }
    }
}
int orc_npts(const orc_ctx *C) { return C->npts; }
double orc_weight(const orc_ctx *C) { return C->w; }

/* Fine propagator over slice n: m steps of dt = DT/m (Sec. 2), with the
 * source if one is set (affine). */
void orc_F_slice(const orc_ctx *C, int n, const double *in, double *out)
{
    orc_ctx t;
    const orc_ctx *S = on_slice(C, n, &t);
    propagate(S, C->fine_scheme, C->m, C->DT, in, out, C->src, n * C->m, C->fine_f32);
}

/* The fine propagator of slice 0 (of every slice when f is constant). */
void orc_F(const orc_ctx *C, const double *in, double *out) { orc_F_slice(C, 0, in, out); }

/* Coarse propagator over slice n: c steps of DT/c, linear (the
 * preconditioner's G; a source cancels from the parareal corrections), with
 * the slice's operator. */
void orc_G_slice(const orc_ctx *C, int n, const double *in, double *out)
{
    orc_ctx t;
    const orc_ctx *S = on_slice(C, n, &t);
    propagate(S, C->coarse_scheme, C->c, C->DT, in, out, NULL, -1, 0);
}

/* The coarse propagator of slice 0 (of every slice when nu is constant). */
void orc_G(const orc_ctx *C, const double *in, double *out) { orc_G_slice(C, 0, in, out); }

/* One step of `scheme` with step dt and the source if set (exported for the
 * closed-form pins). */
void orc_step(const orc_ctx *C, int scheme, double dt, const double *in, double *out)
{
    double *work = (double *)malloc(sizeof(double) * step_work(C));
    one_step(C, scheme, dt, in, out, work, C->src, 1.0, 0);
    free(work);
}

/* ------------------------------------------------------------------------- */
/* Block operators (Sec. 2 eq. (algebraiclinearsystem), Sec. 3 eq. (eqinverse)) */
/* ------------------------------------------------------------------------- */

/* y_0 = lam_0,  y_n = lam_n - F0(lam_{n-1}),  n = 1..N-1 (the linear
 * all-at-once operator).  y must not alias lam. */
void orc_apply(const orc_ctx *C, const double *lam, double *y)
{
    size_t np = (size_t)C->npts;
    memcpy(y, lam, sizeof(double) * np);
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int n = 1; n < C->N; ++n) {
        double *f = (double *)malloc(sizeof(double) * np);
        F_lin(C, n - 1, lam + (size_t)(n - 1) * np, f);
        for (size_t j = 0; j < np; ++j) y[(size_t)n * np + j] = lam[(size_t)n * np + j] - f[j];
        free(f);
    }
}

/* y_n = F_n(lam_n) for n = 0..N-1, the source included (the last row gives
 * u(T) = F_{N-1}(lam_{N-1})). */
void orc_apply_raw(const orc_ctx *C, const double *lam, double *y)
{
    size_t np = (size_t)C->npts;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int n = 0; n < C->N; ++n) orc_F_slice(C, n, lam + (size_t)n * np, y + (size_t)n * np);
}

/* z = G^{-1} v by forward substitution: z_0 = v_0, z_n = v_n + G(z_{n-1}).
 * In-place (v == z) is allowed. */
void orc_sweep(const orc_ctx *C, const double *v, double *z)
{
    size_t np = (size_t)C->npts;
    double *g = (double *)malloc(sizeof(double) * np);
    if (z != v) memcpy(z, v, sizeof(double) * np);
    for (int n = 1; n < C->N; ++n) {
        orc_G_slice(C, n - 1, z + (size_t)(n - 1) * np, g);
        for (size_t j = 0; j < np; ++j) z[(size_t)n * np + j] = v[(size_t)n * np + j] + g[j];
    }
    free(g);
}

/* Serial fine trajectory: lam_0 = u0, lam_{n+1} = F_n(lam_n); uT = F_{N-1}(lam_{N-1}) if non-NULL. */
void orc_serial(const orc_ctx *C, const double *u0, double *lam, double *uT)
{
    size_t np = (size_t)C->npts;
    memcpy(lam, u0, sizeof(double) * np);
    for (int n = 1; n < C->N; ++n) orc_F_slice(C, n - 1, lam + (size_t)(n - 1) * np, lam + (size_t)n * np);
    if (uT) orc_F_slice(C, C->N - 1, lam + (size_t)(C->N - 1) * np, uT);
}

/* Block inner product <U,V> = sum_n h^d sum_j u_{n,j} v_{n,j}, summed per
 * slice in index order and then over slices in order (Sec. 3). */
double orc_dot(const orc_ctx *C, const double *U, const double *V)
{
    size_t np = (size_t)C->npts;
    double tot = 0.0;
    for (int n = 0; n < C->N; ++n) {
        double s = 0.0;
        for (size_t j = 0; j < np; ++j) s += U[(size_t)n * np + j] * V[(size_t)n * np + j];
        tot += C->w * s;
    }
    return tot;
}

/* ||U||_{N,inf} = max_n ( h^d sum_j u_{n,j}^2 )^{1/2}: the maximum over slices
 * of the discrete L2(Omega) norm (the paper leaves this norm undefined). */
double orc_norm(const orc_ctx *C, const double *U)
{
    size_t np = (size_t)C->npts;
    double mx = 0.0;
    for (int n = 0; n < C->N; ++n) {
        double s = 0.0;
        for (size_t j = 0; j < np; ++j) s += U[(size_t)n * np + j] * U[(size_t)n * np + j];
        s = sqrt(C->w * s);
        if (!(s <= mx)) mx = s; /* NaN propagates */
    }
    return mx;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1: PiTSBiCG                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int status, iters, matvecs, restarts;
    double res_norm;
} orc_info;

/* out = G^{-1} F in  (one "matrix-by-vector product" of the preconditioned system) */
static void precond_apply(const orc_ctx *C, const double *in, double *out)
{
    orc_apply(C, in, out);
    orc_sweep(C, out, out);
}

/*
 * Solve G^{-1} F X = G^{-1} B with B = (u0, b, .., b) by Algorithm 1.
 * X: initial guess on entry when x0_mode == ORC_X0_GIVEN, solution on exit.
 * history (optional, capacity hist_cap): ||R^k|| for k = 0.. (the value tested
 * at the head of the loop).  Returns the status; fills *info.
 *
 * Readings where the algorithm is silent:
 *  - stopping test ||R^k||_{N,inf} > tol, absolute (norm_mode ORC_ABS) or
 *    relative to ||R^0|| (ORC_REL);
 *  - the restart (test with epsilon_0) replaces both the shadow residual and the *new*
 *    direction P^{k+1} by R^{k+1}; rho is then <R^{k+1}, R^{k+1}>;
 *  - <D,Rt> == 0: restart with the current R and redo the direction;
 *    <K,K> == 0 (then S = 0): X += alpha P, R = S, stop;
 *    omega == 0 with K != 0: X += alpha P, R = S, then restart;
 *    a NaN/Inf norm stops with ORC_EBREAKDOWN;
 *  - half_step_check != 0 stops after S = R - alpha D when ||S|| <= tol;
 *  - stall_window > 0: stop with ORC_ENOCONV when ||R|| has not halved over
 *    the last stall_window iterations (used for reduced-precision fine solvers).
 */
int orc_pitsbicg(const orc_ctx *C, const double *u0, double *X, double tol, double eps0,
                 int max_iter, int norm_mode, int x0_mode, int half_step_check, int stall_window,
                 orc_info *info, double *history, int hist_cap, int *hist_len)
{
    size_t np = (size_t)C->npts, nt = (size_t)C->N * np;
    double *B = (double *)calloc(nt, sizeof(double));
    double *R = (double *)malloc(sizeof(double) * nt);
    double *Rt = (double *)malloc(sizeof(double) * nt);
    double *P = (double *)malloc(sizeof(double) * nt);
    double *D = (double *)malloc(sizeof(double) * nt);
    double *S = (double *)malloc(sizeof(double) * nt);
    double *K = (double *)malloc(sizeof(double) * nt);
    double *Tm = (double *)malloc(sizeof(double) * nt);
    int status = ORC_ENOCONV, k = 0, matvecs = 0, restarts = 0, hl = 0;
    double nrm = 0.0;

    build_B(C, u0, B); /* B = (lambda_0, b_0, ..., b_{N-2}), b = 0 without a source */

    /* initial residual R^0 = G^{-1}(B - F X^0) */
    if (x0_mode == ORC_X0_ZERO) {
        memset(X, 0, sizeof(double) * nt);
        orc_sweep(C, B, R);
    } else {
        if (x0_mode == ORC_X0_COARSE) orc_sweep(C, B, X);
        orc_apply(C, X, Tm);
        for (size_t i = 0; i < nt; ++i) Tm[i] = B[i] - Tm[i];
        orc_sweep(C, Tm, R);
        matvecs++;
    }
    /* shadow residual, first direction, rho */
    memcpy(Rt, R, sizeof(double) * nt);
    memcpy(P, R, sizeof(double) * nt);
    double rho = orc_dot(C, R, Rt);
    double nrm0 = orc_norm(C, R);
    double scale = (norm_mode == ORC_REL && nrm0 > 0.0) ? nrm0 : 1.0;
    double best = nrm0, best_at = 0;

    for (;;) {
        nrm = orc_norm(C, R);
        if (history && hl < hist_cap) history[hl++] = nrm;
        if (!isfinite(nrm)) {
            status = ORC_EBREAKDOWN;
            break;
        }
        /* stopping test */
        if (!(nrm > tol * scale)) {
            status = ORC_OK;
            break;
        }
        if (k >= max_iter) {
            status = ORC_ENOCONV;
            break;
        }
        if (stall_window > 0) {
            if (nrm <= 0.5 * best) {
                best = nrm;
                best_at = k;
            } else if (k - best_at >= stall_window) {
                status = ORC_ENOCONV;
                break;
            }
        }
        /* D = G^{-1} F P */
        precond_apply(C, P, D);
        matvecs++;
        double dr = orc_dot(C, D, Rt);
        if (dr == 0.0) { /* breakdown of the shadow product: restart with R */
            memcpy(Rt, R, sizeof(double) * nt);
            memcpy(P, R, sizeof(double) * nt);
            rho = orc_dot(C, R, R);
            restarts++;
            precond_apply(C, P, D);
            matvecs++;
            dr = orc_dot(C, D, Rt);
            if (dr == 0.0) {
                status = ORC_EBREAKDOWN;
                break;
            }
        }
        /* alpha */
        double alpha = rho / dr;
        /* S = R - alpha D */
        for (size_t i = 0; i < nt; ++i) S[i] = R[i] - alpha * D[i];
        if (half_step_check && !(orc_norm(C, S) > tol * scale)) {
            for (size_t i = 0; i < nt; ++i) X[i] += alpha * P[i];
            memcpy(R, S, sizeof(double) * nt);
            k++;
            continue; /* the head of the loop tests ||R|| = ||S|| and stops */
        }
        /* K = G^{-1} F S */
        precond_apply(C, S, K);
        matvecs++;
        double ks = orc_dot(C, K, S);
        double kk = orc_dot(C, K, K);
        if (kk == 0.0) { /* S = 0: the half step solved the system */
            for (size_t i = 0; i < nt; ++i) X[i] += alpha * P[i];
            memcpy(R, S, sizeof(double) * nt);
            k++;
            continue;
        }
        /* omega */
        double omega = ks / kk;
        if (omega == 0.0) {
            for (size_t i = 0; i < nt; ++i) X[i] += alpha * P[i];
            memcpy(R, S, sizeof(double) * nt);
            memcpy(Rt, R, sizeof(double) * nt);
            memcpy(P, R, sizeof(double) * nt);
            rho = orc_dot(C, R, R);
            restarts++;
            k++;
            continue;
        }
        /* X and R updates */
        for (size_t i = 0; i < nt; ++i) {
            X[i] = X[i] + alpha * P[i] + omega * S[i];
            R[i] = S[i] - omega * K[i];
        }
        /* beta */
        double rho_new = orc_dot(C, R, Rt);
        double beta = (alpha / omega) * (rho_new / rho);
        /* new direction P */
        for (size_t i = 0; i < nt; ++i) P[i] = R[i] + beta * (P[i] - omega * D[i]);
        /* restart test with epsilon_0 */
        if (fabs(rho_new) <= eps0) {
            memcpy(Rt, R, sizeof(double) * nt);
            memcpy(P, R, sizeof(double) * nt);
            rho_new = orc_dot(C, R, R);
            restarts++;
        }
        rho = rho_new;
        /* next iteration */
        k++;
    }
    if (info) {
        info->status = status;
        info->iters = k;
        info->matvecs = matvecs;
        info->restarts = restarts;
        info->res_norm = nrm;
    }
    if (hist_len) *hist_len = hl;
    free(B);
    free(R);
    free(Rt);
    free(P);
    free(D);
    free(S);
    free(K);
    free(Tm);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Parareal                                                                    */
/* ------------------------------------------------------------------------- */

/* Preconditioned Richardson X^{k+1} = X^k + G^{-1}(B - F X^k), `iters` steps
 * from the X given on entry (Sec. 2, eq. (pararealAlgebraic)).
 * history[k] = ||G^{-1}(B - F X^k)||_{N,inf}, k = 0..iters-1 (if non-NULL). */
void orc_parareal_richardson(const orc_ctx *C, const double *u0, double *X, int iters,
                             double *history)
{
    size_t np = (size_t)C->npts, nt = (size_t)C->N * np;
    double *Tm = (double *)malloc(sizeof(double) * nt);
    double *B = (double *)malloc(sizeof(double) * nt);
    build_B(C, u0, B);
    for (int k = 0; k < iters; ++k) {
        orc_apply(C, X, Tm);
        for (size_t i = 0; i < nt; ++i) Tm[i] = B[i] - Tm[i];
        orc_sweep(C, Tm, Tm);
        if (history) history[k] = orc_norm(C, Tm);
        for (size_t i = 0; i < nt; ++i) X[i] += Tm[i];
    }
    free(Tm);
    free(B);
}

/* Predictor-corrector recursion (Sec. 2, eq. (pararealscheme)), read as
 *   lambda_0^{k+1} = u0,
 *   lambda_{n+1}^{k+1} = G(lambda_n^{k+1}) + F(lambda_n^k) - G(lambda_n^k).
 * Lam holds lambda^k on entry (N slices) and lambda^{k+iters} on exit. */
void orc_parareal_pc(const orc_ctx *C, const double *u0, double *Lam, int iters)
{
    size_t np = (size_t)C->npts, nt = (size_t)C->N * np;
    double *old = (double *)malloc(sizeof(double) * nt);
    double *f = (double *)malloc(sizeof(double) * nt);
    double *g = (double *)malloc(sizeof(double) * np);
    for (int k = 0; k < iters; ++k) {
        memcpy(old, Lam, sizeof(double) * nt);
        /* fine and old-coarse corrections of all slices (the parallel part) */
        for (int n = 0; n + 1 < C->N; ++n) {
            orc_F_slice(C, n, old + (size_t)n * np, f + (size_t)n * np);
            orc_G_slice(C, n, old + (size_t)n * np, g);
            for (size_t j = 0; j < np; ++j) f[(size_t)n * np + j] -= g[j];
        }
        /* sequential coarse prediction */
        memcpy(Lam, u0, sizeof(double) * np);
        for (int n = 0; n + 1 < C->N; ++n) {
            orc_G_slice(C, n, Lam + (size_t)n * np, g);
            for (size_t j = 0; j < np; ++j)
                Lam[(size_t)(n + 1) * np + j] = g[j] + f[(size_t)n * np + j];
        }
    }
    free(old);
    free(f);
    free(g);
}
