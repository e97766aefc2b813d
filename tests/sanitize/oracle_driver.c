/* Exercises every entry point of the CPU oracle once or more, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Exit 0 when every call returned; the sanitizers abort on a fault. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_ctx orc_ctx;
typedef struct {
    int status, iters, matvecs, restarts;
    double res_norm;
} orc_info;

orc_ctx *orc_create(int dim, int Mx, int My, int bc, double Lx, double Ly, double nu, double ax, double ay,
                    double react, double T, int N, int m, int fine_scheme, int c, int coarse_scheme, double rot);
void orc_destroy(orc_ctx *C);
void orc_set_threads(int n);
void orc_set_source(orc_ctx *C, const double *f);
void orc_set_source_t(orc_ctx *C, const double *h, const double *g);
int orc_set_fine_f32(orc_ctx *C, int on);
int orc_set_nu_t(orc_ctx *C, const double *s);
int orc_npts(const orc_ctx *C);
void orc_F_slice(const orc_ctx *C, int n, const double *in, double *out);
void orc_G_slice(const orc_ctx *C, int n, const double *in, double *out);
void orc_forced_slice(const orc_ctx *C, int n, double *b);
void orc_apply(const orc_ctx *C, const double *lam, double *y);
void orc_apply_raw(const orc_ctx *C, const double *lam, double *y);
void orc_sweep(const orc_ctx *C, const double *v, double *z);
void orc_serial(const orc_ctx *C, const double *u0, double *lam, double *uT);
double orc_dot(const orc_ctx *C, const double *U, const double *V);
double orc_norm(const orc_ctx *C, const double *U);
int orc_pitsbicg(const orc_ctx *C, const double *u0, double *X, double tol, double eps0, int max_iter,
                 int norm_mode, int x0_mode, int half_step_check, int stall_window, orc_info *info, double *hist,
                 int hist_cap, int *hist_len);
void orc_parareal_richardson(const orc_ctx *C, const double *u0, double *X, int iters, double *hist);
void orc_parareal_pc(const orc_ctx *C, const double *u0, double *Lam, int iters);
void orc_tridiag_solve(int n, const double *a, const double *b, const double *c, const double *d, double *x);
void orc_cyclic_solve(int n, const double *a, const double *b, const double *c, const double *d, double *x);

static double *vec(size_t n, unsigned seed)
{
    double *v = (double *)malloc(sizeof(double) * n);
    for (size_t i = 0; i < n; ++i) v[i] = sin(0.37 * (double)(i + 1) * (seed + 1)) + 0.1 * cos(1.3 * (double)i);
    return v;
}

/* one context through every operation */
static int exercise(orc_ctx *C, int N, int m, int f32, int nu_t, int src)
{
    const size_t np = (size_t)orc_npts(C), nt = (size_t)N * np;
    double *lam = vec(nt, 1), *y = vec(nt, 2), *z = vec(nt, 3), *u0 = vec(np, 4), *X = vec(nt, 5), *uT = vec(np, 6);
    double *hist = (double *)calloc(64, sizeof(double));
    if (src) {
        double *h = vec(np, 7), *g = vec((size_t)N * m + 1, 8);
        orc_set_source_t(C, h, g);
        free(h);
        free(g);
    }
    if (nu_t) {
        double *s = (double *)malloc(sizeof(double) * (size_t)N);
        for (int n = 0; n < N; ++n) s[n] = 0.5 + 0.25 * n;
        if (orc_set_nu_t(C, s) != 0) return 1;
        free(s);
    }
    if (f32 && orc_set_fine_f32(C, 1) != 0) return 2;
    orc_F_slice(C, N - 1, u0, uT);
    orc_G_slice(C, N - 1, u0, uT);
    orc_forced_slice(C, N - 1, uT);
    orc_apply(C, lam, y);
    orc_apply_raw(C, lam, y);
    orc_sweep(C, lam, z);
    orc_sweep(C, z, z); /* in place */
    orc_serial(C, u0, lam, uT);
    (void)orc_dot(C, lam, z);
    (void)orc_norm(C, lam);
    orc_info info;
    int hl = 0;
    for (int mode = 0; mode < 3; ++mode) /* X0 zero, given, coarse */
        orc_pitsbicg(C, u0, X, 1e-10, mode == 1 ? 1e30 : 1e-30, 2 * N, mode == 2, mode, mode == 1, 3, &info, hist,
                     64, &hl);
    orc_parareal_richardson(C, u0, X, N, hist);
    orc_parareal_pc(C, u0, lam, 2);
    free(lam), free(y), free(z), free(u0), free(X), free(uT), free(hist);
    return 0;
}

int main(void)
{
    orc_set_threads(4);
    struct {
        int dim, Mx, My, bc;
        double nu, ax, ay, r, rot;
        int N, m, fs, c, cs;
    } cases[] = {
        {1, 17, 1, 0, 0.1, 0.0, 0.0, 0.0, 0.0, 5, 4, 0, 1, 0},     /* IE Dirichlet */
        {1, 19, 1, 1, 0.02, 1.0, 0.0, 0.3, 0.0, 6, 5, 1, 2, 0},    /* CN periodic */
        {2, 9, 7, 0, 0.05, 0.0, 0.0, 0.2, 0.0, 4, 3, 2, 1, 2},     /* PR-ADI */
        {2, 8, 9, 0, 0.05, 0.0, 0.0, 0.5, 0.0, 4, 2, 3, 1, 3},     /* backward-Euler splitting */
        {2, 9, 8, 0, 0.02, 0.3, -0.2, 0.5, 1.0, 4, 3, 2, 2, 2},    /* rotating velocity */
    };
    int rc = 0;
    for (size_t k = 0; k < sizeof cases / sizeof cases[0]; ++k)
        for (int variant = 0; variant < 4; ++variant) {
            /* 0 plain, 1 FP32 fine, 2 time-dependent operator, 3 separable source */
            if (variant == 1 && cases[k].dim == 2 && cases[k].rot != 0.0) continue;
            orc_ctx *C = orc_create(cases[k].dim, cases[k].Mx, cases[k].My, cases[k].bc, 1.0, 1.1, cases[k].nu,
                                    cases[k].ax, cases[k].ay, cases[k].r, 0.5, cases[k].N, cases[k].m, cases[k].fs,
                                    cases[k].c, cases[k].cs, cases[k].rot);
            if (!C) return 10;
            rc |= exercise(C, cases[k].N, cases[k].m, variant == 1, variant == 2, variant == 3);
            orc_destroy(C);
        }
    /* invalid descriptions are refused, not crashed on */
    if (orc_create(1, 2, 1, 0, 1, 1, 0.1, 0, 0, 0, 1, 4, 4, 0, 1, 0, 0.0)) return 11;
    if (orc_create(3, 8, 8, 0, 1, 1, 0.1, 0, 0, 0, 1, 4, 4, 0, 1, 0, 0.0)) return 12;
    /* the brute-force helpers */
    double a[6] = {0, -1, -1, -1, -1, -1}, b[6] = {4, 4, 4, 4, 4, 4}, c[6] = {-1, -1, -1, -1, -1, 0};
    double d[6] = {1, 2, 3, 4, 5, 6}, x[6];
    orc_tridiag_solve(6, a, b, c, d, x);
    orc_cyclic_solve(6, a, b, c, d, x);
    printf("oracle driver: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
