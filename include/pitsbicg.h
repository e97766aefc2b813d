/*
 * pitsbicg.h -- C ABI of libpitsbicg, an MI355X (gfx950) implementation of the
 * data-parallel hot path of PiTSBiCG (Riahi, "PiTSBiCG: Parallel in Time Stable
 * Bi-Conjugate Gradient Algorithm").
 *
 * The method (Sec. 2-3 of the paper): split [0,T] into N slices of length
 * DT = T/N; the slice initial values Lambda = (lambda_0, .., lambda_{N-1})
 * satisfy the all-at-once block system  F Lambda = B  (Sec. 2,
 * eq. (algebraiclinearsystem)), with identity blocks on the diagonal, -F on
 * the first sub-diagonal and B = (u0, 0, .., 0), where F is the fine
 * propagator over one slice.  It is solved by Algorithm 1 (left-preconditioned
 * BiCGStab) with the preconditioner G^{-1} (Sec. 3, eq. (eqinverse)), G built
 * from a cheap coarse propagator and applied by sequential forward
 * substitution.
 *
 * Conventions for every entry point:
 *  - All block vectors are FP64, contiguous, slice-major: [N][M] in 1D,
 *    [N][My][Mx] (x fastest) in 2D.  Dirichlet vectors hold interior points
 *    only; periodic vectors hold the points j = 0..M-1.  u0 is one slice.
 *  - Device pointers are HIP device (or managed) memory of the current device,
 *    8-byte aligned.  Host pointers are marked "host".
 *  - The caller owns every buffer it passes (u0, X, lam, y, v, z, the
 *    workspace).  The library owns only its context and server structs and
 *    allocates no device memory: it works inside the caller's workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Return codes: PIT_OK (0); negative values are errors (below); positive
 *    values are "not yet" (PIT_EAGAIN).  No exception crosses the ABI.
 *  - A context may be used from one thread at a time; different contexts are
 *    independent.
 */
#ifndef PITSBICG_H
#define PITSBICG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PIT_OK 0
#define PIT_EINVAL (-1)      /* bad argument / unsupported combination      */
#define PIT_ENOMEM (-2)      /* workspace too small / over the memory budget */
#define PIT_EHIP (-3)        /* a HIP runtime call failed (see pit_last_hip_error) */
#define PIT_ENOCONV (-4)     /* max_iter or stagnation: X holds the last iterate */
#define PIT_EBREAKDOWN (-5)  /* NaN/Inf residual or unrecoverable breakdown   */
#define PIT_EAGAIN 1         /* served request not finished yet               */

/* ---- enumerations ------------------------------------------------------ */
#define PIT_DIRICHLET0 0 /* homogeneous Dirichlet on the whole boundary */
#define PIT_PERIODIC 1   /* periodic (1D only)                          */

#define PIT_IE 0     /* implicit Euler: (I - dt L) u' = u                        */
#define PIT_CN 1     /* Crank-Nicolson: (I - dt/2 L) u' = (I + dt/2 L) u         */
#define PIT_ADI_PR 2 /* Peaceman-Rachford ADI (2D): x-implicit then y-implicit  */
#define PIT_ADI_IE 3 /* backward-Euler splitting (2D): (I - dt Lx) u* = u,       */
                     /* (I - dt Ly) u' = u*, the reaction split r/2 per factor;  */
                     /* a source enters the first factor (u + dt f)              */

#define PIT_F64 0 /* FP64 state and arithmetic                                 */
#define PIT_F32 1 /* fine propagator only: FP32 state (see pit_stepper.prec)    */

#define PIT_ABS 0 /* stop when ||R||_{N,inf} <= tol                            */
#define PIT_REL 1 /* stop when ||R||_{N,inf} <= tol * ||R^0||_{N,inf}          */

#define PIT_X0_ZERO 0   /* X^0 = 0                                          */
#define PIT_X0_GIVEN 1  /* X^0 = the X passed in                            */
#define PIT_X0_COARSE 2 /* X^0 = G^{-1} B (the coarse trajectory)           */

#define PIT_APPLY_RAW 1  /* pit_apply_F flag: y_n = F(lam_n) for all n            */
#define PIT_APPLY_LAST 2 /* pit_apply_F flag: only y_{N-1} = F(lam_{N-1}) = u(T) */

/* ---- problem description ----------------------------------------------- */
/* The evolution problem dy/dt - A y = 0 (Sec. 2, eq. (Cauchy), source f = 0)
 * with the constant-coefficient operator
 *     A y = nu * Laplace(y) - adv . grad(y) - react * y
 * discretised by second-order central differences on a uniform grid:
 *   1D: M[0] points; Dirichlet h = length[0]/(M[0]+1), periodic h = length[0]/M[0];
 *   2D: M[0] x M[1] interior points, h = length[i]/(M[i]+1); Dirichlet only,
 *       adv must be 0 (the ADI factors are per axis: Lx = nu*D2x - react/2,
 *       Ly = nu*D2y - react/2). */
typedef struct {
    int32_t dim;       /* 1 or 2                                       */
    int32_t M[2];      /* points per axis (M[1] ignored in 1D), >= 3    */
    int32_t bc;        /* PIT_DIRICHLET0 or PIT_PERIODIC               */
    double length[2];  /* domain length per axis (> 0)                 */
    double nu;         /* diffusion coefficient (>= 0)                 */
    double adv[2];     /* advection velocity (1D uses adv[0])          */
    double react;      /* reaction coefficient                         */
    double T;          /* final time (> 0)                             */
    double rot;        /* 2D: rate of a rigid rotation about the domain
                          centre added to adv, 0 in 1D (the u = [-y, x]
                          of the advection test of Sec. 4)             */
} pit_problem;

/* A time stepper over one slice: `substeps` steps of length DT/substeps.
 * For the fine propagator F (Sec. 2, the "accurate but expensive" solver)
 * substeps must equal the m passed to pit_create (or be 0 = m).  For the
 * coarse propagator G (the "cheap" solver of the preconditioner) substeps is
 * c >= 1.  prec applies to the fine propagator only: PIT_F32 keeps the fine
 * state in FP32 (1D: FP32 arithmetic in increment form; 2D: FP32 state between
 * the ADI half steps, FP64 arithmetic); the coarse sweep, the dot products and
 * the BiCGStab scalars are always FP64. */
typedef struct {
    int32_t scheme;   /* PIT_IE, PIT_CN (1D); PIT_ADI_PR, PIT_ADI_IE (2D) */
    int32_t substeps; /* m (fine) or c (coarse)                */
    int32_t prec;     /* PIT_F64 or PIT_F32                     */
    int32_t reserved; /* must be 0                              */
} pit_stepper;

/* Options of Algorithm 1 (Sec. 3): tolerance epsilon, restart tolerance
 * epsilon_0, initial guess X^0. */
typedef struct {
    double tol;              /* epsilon of the stopping test                        */
    double restart_tol;      /* epsilon_0 of the restart test                       */
    int32_t max_iter;        /* <= 0 means 2*N                                      */
    int32_t norm_mode;       /* PIT_ABS (the test as written) or PIT_REL            */
    int32_t x0_mode;         /* PIT_X0_ZERO, PIT_X0_GIVEN, PIT_X0_COARSE            */
    int32_t half_step_check; /* !=0: also stop after S = R - alpha D if ||S|| <= tol */
    int32_t stall_window;    /* >0: PIT_ENOCONV when ||R|| has not halved in this
                                many iterations (for FP32 fine propagators)         */
    int32_t timing;          /* >0: time launches with HIP events on `stream`: the
                                first fine apply and coarse sweep and then every
                                timing-th one of each (1: every launch), and the
                                vector updates and inner products of the first
                                and every timing-th iteration.  Fills ms_fine /
                                ms_coarse / ms_krylov and n_fine_timed /
                                n_coarse_timed / n_krylov_timed.  Each timed
                                launch or group adds two event records, and with
                                them a gap, to the stream.
                                <0 is PIT_EINVAL.                                   */
} pit_solve_opts;

/* Result of pit_solve.  history (host, optional, capacity history_cap)
 * receives ||R^k||_{N,inf} for k = 0.. as tested at the head of the loop. */
typedef struct {
    int32_t status;   /* same value pit_solve returns                         */
    int32_t iters;    /* completed passes of the loop                         */
    int32_t matvecs;  /* applications of G^{-1} F (2 per iteration, +1 for X^0) */
    int32_t restarts; /* shadow-residual restarts (restart test and breakdowns) */
    double res_norm;  /* last ||R||_{N,inf}                                    */
    double *history;  /* host, may be NULL                                     */
    int32_t history_cap;
    int32_t history_len;
    float ms_total;   /* wall time of the call, milliseconds                  */
    float ms_fine;    /* summed duration of the timed fine-apply launches     */
    float ms_coarse;  /* summed duration of the timed coarse-sweep launches   */
    int32_t n_fine;   /* fine-apply launches in the call                      */
    int32_t n_coarse; /* coarse-sweep launches in the call                    */
    int32_t n_fine_timed;   /* of those, timed (opts->timing); 0 in batches   */
    int32_t n_coarse_timed;
    float ms_krylov;  /* summed duration of the vector updates and inner
                         products of the timed iterations (the first and
                         every timing-th; pit_solve only)                     */
    int32_t n_krylov_timed; /* iterations whose Krylov launches were timed    */
} pit_solve_info;

typedef struct pit_ctx pit_ctx;

/* ---- context ------------------------------------------------------------ */

/* Create a context for `problem` split into N >= 1 slices with m >= 1 fine
 * steps per slice.  Validates the combination, chooses kernel shapes and
 * precomputes (on the host, FP64) the factorisations of the fine and coarse
 * step matrices.  Does not touch the GPU.
 * Errors: PIT_EINVAL for N < 1, m < 1, M < 3, dim not 1/2, 2D periodic or
 * advective, IE/CN in 2D, ADI in 1D, M above the largest supported line
 * (16384 points), a factorisation that is not finite.  *out is set to NULL on
 * error. */
int pit_create(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine,
               pit_stepper coarse, pit_ctx **out);

/* Destroy a context (host memory only; the workspace stays the caller's). */
int pit_destroy(pit_ctx *ctx);

/* Device bytes the context needs: coefficient tables, the BiCGStab block
 * vectors (R, shadow R, P, D, S, K and one temporary, N*npts FP64 each),
 * intermediate ADI fields and reduction scratch. */
size_t pit_workspace_bytes(const pit_ctx *ctx);

/* Bind `bytes` of device memory at dev_ptr (256-byte aligned) as the
 * context's workspace and upload the tables (a synchronous copy on the null
 * stream).  The memory must stay valid until the context is destroyed or
 * rebound.  Errors: PIT_EINVAL (NULL / misaligned), PIT_ENOMEM (too small),
 * PIT_EHIP. */
int pit_bind_workspace(pit_ctx *ctx, void *dev_ptr, size_t bytes);

/* Source term constant in time: the problem becomes u_t = L u + f(x) (the
 * source f of the Cauchy problem, Sec. 2, eq. (Cauchy)).  Each step adds it:
 * IE  (I - dt L) u' = u + dt f;  CN  (I - dt/2 L) u' = (I + dt/2 L) u + dt f;
 * PR-ADI  dt/2 f in each half-step.  The slice propagator is then affine,
 * F(u) = F0(u) + b with b = F(0) the forced response of one slice, and the
 * all-at-once system of Sec. 2, eq. (algebraiclinearsystem) keeps its linear
 * operator with B = (u0, b, .., b), whose solution is again the serial
 * trajectory.  f: host array of npts values in slice layout, copied; NULL
 * removes the source.  If the workspace is bound, f is uploaded and b computed
 * at once (synchronous, null stream, with the context's block vectors as
 * scratch: no other call on the context may be in flight), otherwise at
 * pit_bind_workspace.
 * Effects: pit_solve and pit_parareal (and batched solves of the context) use
 * B = (u0, b, .., b); pit_apply_F with PIT_APPLY_RAW or PIT_APPLY_LAST returns
 * the affine F(lam_n); the plain pit_apply_F (the system operator) and
 * pit_coarse_sweep (the preconditioner, linear G) are unchanged.  Requests to
 * a server carry no source.  Errors: PIT_EINVAL (NULL ctx, non-finite value),
 * PIT_EHIP. */
int pit_set_source(pit_ctx *ctx, const double *f);

/* Source term separable in time, f(t, x) = g(t) h(x): slice n carries f on
 * [T_n, T_{n+1}] (Sec. 2, eq. (Cauchyn)).  Fine step j, from t_j = j dt to
 * t_{j+1}, adds the source as in pit_set_source with f = w_j h, where w_j =
 * g(t_{j+1}) under IE and (g(t_j) + g(t_{j+1}))/2 under CN and in both PR-ADI
 * half-steps (the midpoint value, read as the mean of the two ends).  The
 * propagator of slice n is affine, F_n(u) = F0(u) + b_n with b_n = F_n(0),
 * and the all-at-once system keeps its linear operator with
 * B = (u0, b_0, .., b_{N-2}).
 * h: npts values in slice layout; g: the profile at the N m + 1 fine step
 * times t_0 .. t_{N m}; both copied.  NULL g sets the constant source h
 * (pit_set_source), NULL h removes the source.
 * Workspace: the context then needs N slices and N m values more, behind
 * the rest: pit_workspace_bytes reports the size for the source set.  If a
 * workspace is bound and smaller, the source is set, the context is left
 * unbound and the call returns PIT_ENOMEM: bind a workspace of
 * pit_workspace_bytes.  b_0 .. b_{N-1} are computed for all slices at once
 * (m fine steps of every slice, synchronous, null stream, the context's
 * block vectors as scratch) as soon as both the workspace and the source
 * are set.
 * Effects as pit_set_source, with b_n in place of b: pit_solve and
 * pit_parareal use B = (u0, b_0, .., b_{N-2}), and pit_apply_F with
 * PIT_APPLY_RAW or PIT_APPLY_LAST returns F_n(lam_n).  pit_set_source
 * replaces a separable source.  Errors: PIT_EINVAL (NULL ctx, non-finite
 * value), PIT_ENOMEM, PIT_EHIP. */
int pit_set_source_t(pit_ctx *ctx, const double *h, const double *g);

/* A time-dependent operator, constant on each slice (1D): the Cauchy problem
 * of Sec. 2, eq. (Cauchy), with its operator depending on time, restricted
 * to slice n as in eq. (Cauchyn).  The diffusion coefficient on slice n is
 * nu * s[n] (s: host, N positive finite values, copied; NULL: nu constant in
 * time again), advection and reaction unchanged.  Slice n's fine propagator
 * F_n and coarse propagator G_n then use that coefficient: row n of the
 * all-at-once operator carries F_{n-1} (pit_apply_F: y_n = lam_n -
 * F_{n-1}(lam_{n-1}); with PIT_APPLY_RAW y_n = F_n(lam_n)), the sweep
 * z_n = v_n + G_{n-1}(z_{n-1}), and pit_solve, pit_parareal and batched
 * solves follow.  Every slice gets its own step tables (N times the fine and
 * coarse line tables, placed behind the rest of the workspace: call
 * pit_workspace_bytes after this).  If the workspace is bound they are
 * uploaded at once (synchronous, null stream); a bound workspace that is now
 * too small is unbound and PIT_ENOMEM returned.  Errors: PIT_EINVAL (NULL
 * ctx; s given for a 2D context, with a value not positive or not finite, or
 * while a source is set), PIT_ENOMEM, PIT_EHIP.  A source cannot be set
 * while s is. */
int pit_set_nu_t(pit_ctx *ctx, const double *s);

/* ---- operators ------------------------------------------------------------ */

/* All-at-once operator (Sec. 2, eq. (algebraiclinearsystem)):
 *     y_0 = lam_0,   y_n = lam_n - F(lam_{n-1}),  n = 1..N-1,
 * every slice's F (m fine steps) running concurrently.  With flags =
 * PIT_APPLY_RAW:  y_n = F(lam_n) for n = 0..N-1.  With PIT_APPLY_LAST: only
 * y_{N-1} = F(lam_{N-1}) is written (the state u(T) at the final time when
 * lam is the solution, by the continuity condition of Sec. 2).  lam and y are device [N][npts] FP64 and must not
 * overlap.  Asynchronous on `stream`.  For 1D lines above 8192 points two of
 * the context's block vectors serve as scratch, so the call must not overlap
 * another call on the same context.  Errors: PIT_EINVAL (NULL pointers,
 * unbound workspace, unknown flags), PIT_EHIP (launch failure). */
int pit_apply_F(pit_ctx *ctx, const double *lam, double *y, int32_t flags, void *stream);

/* Coarse preconditioner solve z = G^{-1} v by forward substitution (Sec. 3,
 * eq. (eqinverse) and the remark that it is solved sequentially):
 *     z_0 = v_0,   z_n = v_n + G(z_{n-1}),  n = 1..N-1,
 * in FP64.  v == z (in place) is allowed.  Asynchronous on `stream`.  In 1D
 * two of the context's block vectors serve as scratch, so the call must not
 * overlap another call on the same context.  Errors as pit_apply_F. */
int pit_coarse_sweep(pit_ctx *ctx, const double *v, double *z, void *stream);

/* Size of the library's fixed device scratch array (one per GPU, held from
 * the library's load until the process ends). */
#define PIT_NOALLOC_SCRATCH_BYTES (32u << 20)

/* pit_coarse_sweep for callers that cannot allocate device memory (code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same z = G^{-1} v with the same kernels and the same bits,
 * but every temporary lives in the library's fixed scratch array of
 * PIT_NOALLOC_SCRATCH_BYTES on the current device instead of the context's
 * workspace, and the launches are issued directly (never through a HIP
 * graph the library instantiates).  The call allocates nothing: no hipMalloc,
 * hipFree, graph instantiation or host allocation.
 * Scratch needed: 1D 16*N*L bytes, L = NT*C >= M the line shape that
 * pit_kernel_shape reports (the chunked copies of v and z); 2D 16*Mx*My
 * bytes (two one-slice fields), 24*Mx*My with a velocity field, none when
 * the whole-slice LDS kernels run.  The context's workspace must be bound on
 * the current device (it holds the coefficient tables) and `stream` must
 * belong to that device.  Every call on a GPU shares that GPU's scratch
 * array, so calls that overlap on one GPU (any context, any stream) race;
 * serialise them.  v == z is allowed.  Asynchronous on `stream`.
 * Errors: PIT_EINVAL (NULL pointers, unbound workspace), PIT_ENOMEM (the
 * problem needs more scratch than PIT_NOALLOC_SCRATCH_BYTES), PIT_EHIP. */
int pit_coarse_sweep_noalloc(pit_ctx *ctx, const double *v, double *z, void *stream);

/* ---- solver ---------------------------------------------------------------- */

/* Algorithm 1 (Sec. 3) on  G^{-1} F X = G^{-1} B,  B = (u0, 0, .., 0):
 * u0 (device, one slice), X (device, [N][npts]): the initial guess on entry
 * when opts->x0_mode == PIT_X0_GIVEN, the solution Lambda on exit (also on
 * PIT_ENOCONV, where it is the last iterate).  opts NULL = defaults
 * (tol 1e-10, restart_tol 1e-30, max_iter 2N, PIT_ABS, PIT_X0_ZERO).
 * info may be NULL.  Inner products are the block L2 product of Sec. 3; the
 * stopping norm is max over slices of the discrete L2 norm.  Host-synchronous
 * (the stopping test needs the norm): one read-back of the iteration's FP64
 * reduction outputs per iteration, with alpha, omega and beta formed on the
 * device by the host's operations in the host's order (without
 * half_step_check; the environment variable PIT_DEV_SCALARS=0 selects a
 * read-back after every reduction, which gives the same bits).  Returns
 * PIT_OK, PIT_ENOCONV, PIT_EBREAKDOWN, PIT_EINVAL or PIT_EHIP. */
int pit_solve(pit_ctx *ctx, const double *u0, double *X, const pit_solve_opts *opts,
              pit_solve_info *info, void *stream);

/* ---- line-shape autotuning (1D) --------------------------------------------- */

/* A 1D line of M points is solved by NT threads holding C points each
 * (NT*C >= M); the best (NT, C) depends on M, on the steppers and on the GPU.
 * pit_autotune times one preconditioned product (the fine apply and the coarse
 * sweep, as pit_solve runs them) of this problem for every supported shape
 * with M <= NT*C <= 4M, using `scratch` (device, 256-byte aligned, at least
 * pit_autotune_scratch_bytes) as the workspace, and records the fastest in a
 * process-wide table keyed by the line-length class (M rounded up to a power
 * of two), the boundary condition, both steppers' schemes, the fine precision
 * and the coarse substeps.  Later pit_create calls for matching problems use
 * the recorded shape (unless the PIT_LINE_SHAPE environment variable forces
 * one).  Host-synchronous on `stream`.  out = {NT, C}; *out_ms (may be NULL)
 * = the winner's time.  Errors: PIT_EINVAL (2D: see pit_autotune_adi; bad
 * arguments), PIT_ENOMEM (no shape fits the scratch), PIT_EHIP. */
size_t pit_autotune_scratch_bytes(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine,
                                  pit_stepper coarse);
int pit_autotune(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
                 void *scratch, size_t bytes, int32_t out[2], float *out_ms, void *stream);
/* The same for 2D problems without a velocity field (PR-ADI or the
 * backward-Euler splitting): the launch shapes of the half-step kernels.  It
 * times the fine apply for every x strip height R (rows per wavefront of the
 * x half step: 8, 16, 32, 64) and every y shape (waves, rows per segment,
 * segments per wave) of the kernel menu that covers the column, and the
 * coarse sweep for every number of columns per workgroup (1, 2, 4) of its
 * one-column-per-wavefront y kernel (columns up to 512 rows; 0 otherwise),
 * using `scratch` as the workspace (pit_autotune_scratch_bytes also answers
 * for 2D).  The winners are recorded per size class of each axis (rounded up
 * to a power of two), both steppers' schemes, the fine precision and the
 * coarse substeps; pit_create uses them for matching problems unless the
 * PIT_ADI_ROWS, PIT_ADI_YSHAPE or PIT_ADI_YC environment variables force a
 * choice.  Host-synchronous on `stream`.  out = {R, wy, cy, seg, columns};
 * out_ms (may be NULL) = {the apply's time, the sweep's time}.  Errors:
 * PIT_EINVAL (1D, a velocity field or a small FP64 slice that runs the
 * whole-slice kernels: nothing to choose; bad arguments), PIT_ENOMEM (no
 * candidate fits the scratch), PIT_EHIP. */
int pit_autotune_adi(const pit_problem *problem, int32_t N, int32_t m, pit_stepper fine, pit_stepper coarse,
                     void *scratch, size_t bytes, int32_t out[5], float out_ms[2], void *stream);
/* Forget every recorded shape (pit_create falls back to its defaults). */
int pit_autotune_reset(void);

/* ---- measurement ------------------------------------------------------------ */

/* Device-to-device copy of `bytes` (a multiple of 16; both pointers 16-byte
 * aligned) with 16-byte loads and stores, four in flight per thread, on
 * enough workgroups to fill every CU: the achievable-bandwidth reference the
 * HBM-bound half-step kernels are measured against (it reads and writes
 * `bytes` each).  Asynchronous on `stream`.  Errors: PIT_EINVAL (NULL or
 * misaligned), PIT_EHIP. */
int pit_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* ---- batched solves --------------------------------------------------------- */

/* Many independent PiTSBiCG solves advanced together (any mix of 1D problems
 * of different M, N, m and coefficients, and 2D problems).  Each instance
 * follows exactly the control flow of pit_solve; its result does not depend
 * on which other instances share the batch (the same kernels compute it with
 * the same operation order), so a solve alone and the same solve inside any
 * batch give identical bits.  1D instances of one line shape share each
 * launch: one fine-apply launch covers all their slices, one coarse-sweep
 * launch runs their sweeps concurrently (one workgroup each), and the
 * inner products and vector updates of all listed instances take one launch
 * each.  2D instances run their operators with their own launches.  Ready
 * instances are advanced on up to four HIP streams. */
typedef struct pit_batch pit_batch;

/* Create a batch engine for up to max_count instances at once (no GPU work;
 * creates its streams on the current device at bind). */
int pit_batch_create(int32_t max_count, pit_batch **out);
/* Device bytes the engine needs for its descriptors and argument buffers. */
size_t pit_batch_workspace_bytes(const pit_batch *b);
/* Bind device memory (256-byte aligned) as the engine's workspace; creates
 * its HIP streams and events on the current device.  Errors: PIT_EINVAL,
 * PIT_ENOMEM, PIT_EHIP. */
int pit_batch_bind_workspace(pit_batch *b, void *dev_ptr, size_t bytes);
int pit_batch_destroy(pit_batch *b);

/* Solve count <= max_count problems: ctxs[i] (bound contexts, all distinct),
 * u0[i] and X[i] as in pit_solve, opts NULL (defaults) or count entries,
 * infos NULL or count entries.  Supported options: tol, restart_tol,
 * max_iter, norm_mode, stall_window; x0_mode must be PIT_X0_ZERO and
 * half_step_check 0 (else PIT_EINVAL before any work).  The engine first
 * waits for `stream` and returns when every instance has finished
 * (host-synchronous).  Returns PIT_OK when every instance returned PIT_OK,
 * otherwise the first failing instance's status (each infos[i].status holds
 * its own). */
int pit_batch_solve(pit_batch *b, pit_ctx *const *ctxs, int32_t count, const double *const *u0,
                    double *const *X, const pit_solve_opts *opts, pit_solve_info *infos, void *stream);

/* ---- serving ------------------------------------------------------------------ */

/* A request loop with continuous batching: submitted solves queue in arrival
 * order and are admitted while a slot is free and their workspace fits in the
 * device arena (the HBM budget); admitted solves advance in the batch engine
 * above, so requests that arrive while others run join them on the GPU, and
 * leave as they finish, freeing their slot and memory for the queue.  The
 * caller provides the arena (device memory it owns); the server carves every
 * request's workspace and its own buffers out of it and allocates no device
 * memory.  A worker thread drives the GPU; pit_submit and pit_poll are
 * thread-safe. */
typedef struct pit_server pit_server;

typedef struct {
    void *arena;          /* device memory (256-byte aligned) = the HBM budget   */
    uint64_t arena_bytes;
    int32_t device;       /* HIP device of the arena                             */
    int32_t max_slots;    /* solves on the GPU at once (>= 1)                    */
    int32_t reserved[2];
} pit_server_cfg;

typedef struct {
    pit_problem problem;
    int32_t N, m;
    pit_stepper fine, coarse;
    const double *u0;     /* device, one slice; read after admission             */
    double *X;            /* device [N][npts]; written before the request is done */
    pit_solve_opts opts;  /* as pit_batch_solve                                  */
} pit_request;

typedef struct {
    int32_t status;       /* the solve's status (as pit_solve), or PIT_ENOMEM when
                             the request can never fit the arena                 */
    int32_t iters, matvecs, restarts;
    double res_norm;
    double t_submit_ms;   /* times since server creation (steady clock)          */
    double t_admit_ms;
    double t_done_ms;
    uint64_t workspace_bytes;
    int32_t hip_error;    /* hipError_t of a failing HIP call (status PIT_EHIP)  */
    int32_t reserved;
} pit_result;

/* Start a server (creates its worker thread).  Errors: PIT_EINVAL, PIT_ENOMEM
 * (arena too small for the server's own buffers), PIT_EHIP. */
int pit_server_create(const pit_server_cfg *cfg, pit_server **out);
/* Queue a solve; *ticket identifies it.  The problem is validated here
 * (PIT_EINVAL, nothing queued).  u0 and X must stay valid until pit_poll
 * reports the request done. */
int pit_submit(pit_server *s, const pit_request *req, uint64_t *ticket);
/* PIT_EAGAIN while the request is queued or running; PIT_OK once it is done,
 * with *res filled (then the ticket is retired); PIT_EINVAL for an unknown
 * ticket. */
int pit_poll(pit_server *s, uint64_t ticket, pit_result *res);
/* Number of requests queued and running, and the arena bytes in use. */
int pit_server_load(pit_server *s, int32_t *queued, int32_t *running, uint64_t *arena_used);
/* Finish every queued and running request, stop the worker, free host state. */
int pit_server_destroy(pit_server *s);

/* ---- parareal ------------------------------------------------------------- */

/* Parareal in its algebraic form (Sec. 2, eq. (pararealAlgebraic)): the
 * Richardson iteration on the preconditioned system,
 *     X^{k+1} = X^k + G^{-1}(B - F X^k),
 * one preconditioned product per iteration (Algorithm 1 uses two), on the
 * same fine apply and coarse sweep.  It is exact after N iterations.
 * history[k] receives ||G^{-1}(B - F X^k)||_{N,inf} (the norm of the update).
 * Stops after the update whose norm passes the test of opts->tol (absolute,
 * or relative to the first with PIT_REL), or after max_iter iterations
 * (default N + 1: X^N is exact and the next update, zero up to rounding,
 * shows it); tol 0 runs exactly max_iter iterations and returns PIT_OK.
 * opts->x0_mode as pit_solve; restart_tol, half_step_check and stall_window
 * are ignored.  Host-synchronous.  Returns PIT_OK, PIT_ENOCONV (max_iter
 * reached above tol), PIT_EBREAKDOWN, PIT_EINVAL or PIT_EHIP. */
int pit_parareal(pit_ctx *ctx, const double *u0, double *X, const pit_solve_opts *opts,
                 pit_solve_info *info, void *stream);

/* ---- diagnostics ----------------------------------------------------------- */

/* Static description of an error code. */
const char *pit_strerror(int code);

/* The hipError_t of the last failing HIP call in this thread (0 if none). */
int pit_last_hip_error(void);

/* Kernel shape the context chose (for reports).  1D: threads per line and
 * points per thread of the fine and coarse line solvers.  2D: lanes and
 * points per lane of the x half-step, lanes and rows per lane of the y
 * half-step.  2D on per-line tables (a velocity field, or FP64 slices small
 * enough for LDS): {1, 0, L, 0}, one thread per line, where L says where a
 * slice lives during its steps: 2 = its fields and tables in LDS, 1 = its
 * fields in LDS, 0 = HBM (one launch per half-step).
 * PIT_EINVAL on a NULL argument. */
int pit_kernel_shape(const pit_ctx *ctx, int32_t out[4]);

#ifdef __cplusplus
}
#endif

#endif /* PITSBICG_H */
