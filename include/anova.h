/*
 * anova.h -- C ABI of the ANOVA-kernel fast summation library (gfx950 / HIP).
 *
 * The library applies the shifted kernel matrix (K + beta I) of kernel ridge
 * regression, where K is the extended Gaussian ANOVA kernel
 *
 *     K_ij = sum_{l=1}^{P} eta_l exp(-||x_i^{W_l} - x_j^{W_l}||^2 / ell^2)
 *
 * (Sec. 3, eq. extended_Gaussian_ANOVA_kernel; Sec. 5, combined kernel
 * K = eta_1 K_1 + ... + eta_P K_P), each feature window W_l holding one, two
 * or three features (Sec. 4.1: every NFFT acts in dimension at most 3).  Each
 * window's product is computed by NFFT-based fast summation (Sec. 4.2, eq.
 * fastsum; K alpha ~ Phi D Phi^* alpha, Sec. 4.3): window-function spreading
 * onto an oversampled grid, a d_A-dimensional FFT, multiplication by the
 * regularised kernel's Fourier coefficients, an inverse FFT and gathering
 * back to the points.  The product runs inside conjugate gradients for the
 * system (K + beta I) alpha = y (Sec. 2, normal equation and CG).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Device pointers are plain HIP device addresses (hipMalloc'd or any
 *   allocator's, e.g. a torch CUDA tensor's data_ptr()).  Host pointers are
 *   marked "host".
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * - Vectors of several right-hand sides are column-major N x nrhs arrays
 *   with leading dimension ld >= N (element (i, c) at [c*ld + i]), float64.
 * - X is N x d row-major float64 with leading dimension ldx >= d
 *   (feature t of point i at [i*ldx + t]).
 * - Every call returns an anova_status; nothing aborts and no exception
 *   crosses the ABI.  On any status other than ANOVA_OK or
 *   ANOVA_E_NOT_CONVERGED the contents of output arrays are unspecified, and
 *   anova_last_error() returns a message (thread-local).
 * - A plan is used by one stream at a time; calls on one plan from several
 *   host threads or streams concurrently race.
 */
#ifndef ANOVA_H
#define ANOVA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct anova_plan_s *anova_plan_t;
typedef struct anova_cg_s *anova_cg_t;

typedef enum {
    ANOVA_OK = 0,
    ANOVA_E_INVALID = 1,        /* bad argument (see each call) */
    ANOVA_E_NOMEM = 2,          /* device or host allocation failed */
    ANOVA_E_HIP = 3,            /* a HIP runtime call failed */
    ANOVA_E_NOT_CONVERGED = 4,  /* CG reached maxit; the iterate is returned */
    ANOVA_E_BREAKDOWN = 5,      /* CG: p^T A p <= 0 or a non-finite value */
    ANOVA_E_ACCURACY = 6        /* fixed (M, m, n) cannot meet target_err */
} anova_status;

typedef enum {
    ANOVA_FP64 = 0,        /* spreading, FFT and gathering in float64 */
    ANOVA_FP32_NFFT = 1    /* spreading, FFT and gathering in float32;
                              output accumulation and CG stay float64 */
} anova_precision;

/* One feature window W_l (Sec. 3, eq. index_window): d_A in {1,2,3},
 * 0-based feature indices feat[0..d_A-1] (distinct, < d), weight eta_l
 * (Sec. 5; equal weights 1/P in the paper, any finite weights here). */
typedef struct {
    int32_t d_A;
    int32_t feat[3];
    double eta;
} anova_window;

/* Plan parameters.  Zero in M, m, n or h means "choose": the plan then picks
 * the cheapest (M, m, n) whose per-entry error estimate (images + truncation
 * + window aliasing + rounding, weighted by eta, summed) is at most
 * target_err; for float32 windows on the per-cell kernels it may raise h so
 * that the points fill whole tiles of grid cells (estimate still within
 * target_err) when that is modelled to run faster. */
typedef struct {
    double ell;          /* Gaussian width: exp(-||r||^2 / ell^2), ell > 0 */
    int32_t precision;   /* anova_precision */
    int32_t M;           /* bandwidth: frequencies -M/2..M/2-1 per dimension
                            (Sec. 4.1 index set), even, 4..256 */
    int32_t m;           /* window half-width in grid points, 2..8 */
    int32_t n;           /* oversampled FFT length per dimension: a power of
                            two, 8..256, n >= M */
    double h;            /* period of the regularised kernel (Sec. 4.2) */
    double target_err;   /* 0 -> 1e-4 (FP32_NFFT) or 1e-9 (FP64) */
    int32_t center;      /* 0: centre each window's bounding box before
                            scaling by 1/h; 1: scale only, x~ = x/h (Sec. 4.2) */
    int32_t residual;    /* anova_residual: how CG recomputes its residual
                            on a FP32_NFFT plan (ignored for FP64 plans) */
    int32_t tune;        /* 0: choose (M, m, n) by the cost model;
                            1: measured: build the cheapest candidates that
                            meet target_err (model cost within 8x, at most 4
                            per window) on these points and keep the one
                            whose product runs fastest on this device (the
                            plan then launches kernels and takes several
                            times longer) */
    int32_t reg_q;       /* 0: periodise the Gaussian, with h large enough
                            that its periodic images decay (or the given h);
                            1..12: regularise it instead (Sec. 4.2), in each
                            dimension: keep exp(-r^2/ell^2) for |r| <= L (L
                            the window's extent, so the kernel is exact for
                            every pair of points) and join it to its h-periodic
                            continuation on (L, h - L) by the polynomial
                            matching its derivatives of orders 0..reg_q at
                            both ends; h must exceed 2L (when 0 the cheapest
                            of 2.5L, 3L and 4L).  Serves kernels too wide
                            for the given h. */
} anova_params;

/* Residual product of CG on FP32_NFFT plans.  The float32 product's rounding
 * error grows with ||K|| (about N times the mean kernel value), so for large
 * N it exceeds tol * beta and CG's recursive residual stagnates or drifts
 * away from the true one.  With ANOVA_RESIDUAL_FP64 the plan also holds the
 * same windows in float64 (same M, n, m, h; about twice the plan memory and
 * planning time), every periodic residual recomputation y - (K~ + beta I) x
 * uses the float64 product, and a column counts as converged only on such a
 * recomputed residual. */
typedef enum {
    ANOVA_RESIDUAL_FP64 = 0,  /* default */
    ANOVA_RESIDUAL_SAME = 1   /* residuals with the plan's own float32 product */
} anova_residual;

/* What a plan chose for window l (host struct filled by anova_plan_query). */
typedef struct {
    int32_t d_A, M, n, m;
    double h;
    double center[3];       /* the point mapped to the torus origin */
    double extent;          /* largest coordinate range over the window's features */
    double err_images;      /* per-entry error estimates, already times eta_l */
    double err_trunc;
    double err_window;
    double err_round;
    double err_total;
    int64_t n_tiles;        /* grid tiles holding at least one point */
    int64_t n_subproblems;  /* work items of the spreading / gathering launches */
    int32_t per_cell;       /* 1: points are accumulated per grid cell in
                               registers (many points per cell); 0: per point */
    int32_t tile;           /* tile edge in grid points */
} anova_window_info;

typedef struct {
    int32_t iters;          /* CG iterations taken */
    int32_t converged;      /* 1 if ||r|| <= tol ||y|| */
    double relres;          /* recursive residual norm / ||y|| */
    double true_relres;     /* ||y - (K~ + beta I) alpha|| / ||y|| recomputed at exit */
} krr_cg_info;

/*
 * Build a plan for the points X (device, N x d row-major float64, ldx >= d)
 * and the windows win[0..P-1] (host).  The plan copies what it needs (sorted
 * grid coordinates, permutations, Fourier multipliers) and does not keep X.
 * It owns all its device memory until anova_plan_destroy.
 * Steps (Sec. 4.2): period h with h >= 2 * extent, scaled nodes x~ = (x-c)/h
 * on the torus [-1/2, 1/2)^d_A, Fourier coefficients of the periodised
 * kernel from the FFT of M equidistant samples per dimension, divided by the
 * squared window transform; points binned and sorted by grid tile.
 * Synchronises `stream`.
 * Errors: ANOVA_E_INVALID for out == NULL, X == NULL, N < 1, N > 2^31-1,
 * d < 1, ldx < d, P < 1, P > 64, d_A not in {1,2,3}, a feature index out of
 * range or repeated inside one window, a non-finite eta or X, ell <= 0,
 * odd M, n not a power of two or n < M, m out of range, residual not an anova_residual,
 * tune not 0 or 1, reg_q outside 0..12, and with reg_q > 0 an h not above
 * twice the extent.
 * ANOVA_E_ACCURACY when fixed parameters miss target_err.
 */
anova_status anova_fastsum_plan(anova_plan_t *out, const double *X, int64_t N, int32_t d,
                                int64_t ldx, const anova_window *win, int32_t P,
                                const anova_params *prm, void *stream);

/*
 * anova_fastsum_plan with X in host memory (N x d row-major float64, ldx >=
 * d): the same plan without a device copy of the points.  Safe to call from
 * several host threads at once and while other threads run solves; the
 * library's own device allocations and uploads are serialised with its graph
 * captures.  Errors as anova_fastsum_plan.
 */
anova_status anova_fastsum_plan_host(anova_plan_t *out, const double *X, int64_t N, int32_t d,
                                     int64_t ldx, const anova_window *win, int32_t P,
                                     const anova_params *prm);

/*
 * out = (K~ + beta I) alpha for nrhs columns (device arrays, column-major,
 * leading dimension ld >= N; alpha and out must not overlap).  K~ is the
 * fast-summation approximation of K (Sec. 4.3, K alpha ~ Phi D Phi^* alpha,
 * summed over windows with weights eta_l, Sec. 5); the shift beta alpha is
 * added exactly.  Asynchronous on `stream`.
 * Errors: ANOVA_E_INVALID for a NULL plan/pointer, nrhs < 1, ld < N.
 */
anova_status anova_matvec(anova_plan_t plan, const double *alpha, double *out, int32_t nrhs,
                          int64_t ld, double beta, void *stream);

/*
 * anova_matvec for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product and kernels, bit for bit, with the work space (grids,
 * spread regions, interpolated values) and launch tables in a static device
 * array of anova_matvec_noalloc_max_bytes() bytes (64 MiB) that each device
 * holds until the process ends.  The call allocates no device memory; it
 * synchronises `stream` (an earlier call may still read the array), copies
 * its launch tables with synchronous host-to-device copies, and then
 * launches on `stream` asynchronously.  Every call on a device shares that
 * device's array: calls that overlap on one device (other streams or host
 * threads) race.  About 4 bytes per point per window and column in float32
 * (8 in float64) plus the grids: a float32 product over three 3-D windows of
 * 1e6 points and one column needs about 14 MB.
 * Errors: as anova_matvec; ANOVA_E_INVALID also when the work space of this
 * plan and nrhs exceeds the maximum (nothing is launched then) or when the
 * current device is not the plan's.
 */
anova_status anova_matvec_noalloc(anova_plan_t plan, const double *alpha, double *out,
                                  int32_t nrhs, int64_t ld, double beta, void *stream);

/* Size in bytes of anova_matvec_noalloc's static work space. */
int64_t anova_matvec_noalloc_max_bytes(void);

/*
 * Plan for prediction at new points: the sum over training points
 * s(z_i) = sum_j alpha_j kappa(z_i, x_j) at targets z_i (Sec. 4.2, the fast
 * summation with target set Z and source set X; Sec. 4.3 evaluates the
 * trained model at test data this way).  Builds the plan anova_fastsum_plan
 * builds for the training points X, except that each window's period h and
 * centre are chosen for the points of X and Z together (every difference
 * z - x must lie in the periodised kernel's fundamental cell); anova_matvec,
 * krr_cg_solve and the other plan calls work on it unchanged.  The targets Z
 * (device, Nz x d row-major float64, ldz >= d, same features as X) are
 * binned and sorted on the same grids; the plan does not keep Z.
 * Synchronises `stream`.
 * Errors: as anova_fastsum_plan, and ANOVA_E_INVALID for Z == NULL, Nz < 1,
 * Nz > 2^31-1, ldz < d or a non-finite Z.
 */
anova_status anova_predict_plan(anova_plan_t *out, const double *X, int64_t N, const double *Z,
                                int64_t Nz, int32_t d, int64_t ldx, int64_t ldz,
                                const anova_window *win, int32_t P, const anova_params *prm,
                                void *stream);

/* anova_predict_plan with X and Z in host memory.  Errors as anova_predict_plan. */
anova_status anova_predict_plan_host(anova_plan_t *out, const double *X, int64_t N,
                                     const double *Z, int64_t Nz, int32_t d, int64_t ldx,
                                     int64_t ldz, const anova_window *win, int32_t P,
                                     const anova_params *prm);

/*
 * out = K~(Z, X) alpha for nrhs columns: out_i = s(z_i), the weighted window
 * sums of Sec. 5 evaluated by spreading alpha at the training points, the
 * windows' Fourier multiplications, and interpolation at the targets (in
 * matrix form Phi_Z D Phi_X^* alpha, Sec. 4.3).  No shift is added.
 * alpha: device, N x nrhs column-major, lda >= N; out: device, Nz x nrhs
 * column-major, ldo >= Nz; they must not overlap.  Arithmetic as anova_matvec
 * in the plan's precision.  Asynchronous on `stream`.
 * Errors: ANOVA_E_INVALID for a NULL plan/pointer, a plan built without
 * targets, nrhs < 1, lda < N, ldo < Nz.
 */
anova_status anova_predict(anova_plan_t plan, const double *alpha, double *out, int32_t nrhs,
                           int64_t lda, int64_t ldo, void *stream);

/*
 * Solve (K~ + beta I) alpha = y by conjugate gradients (Sec. 2), one
 * independent recurrence per column, no preconditioner.  x0 = 0; dot
 * products, vector updates and residual recomputations are float64.  Every
 * R = 50 iterations of a column its residual is recomputed as
 * y - (K~ + beta I) x (residual replacement); on FP32_NFFT plans the
 * recomputation uses the float64 product (ANOVA_RESIDUAL_FP64,
 * the default) and a column stops only when such a recomputed residual
 * satisfies ||r||_2 <= tol ||y||_2 (on FP64 plans, and with
 * ANOVA_RESIDUAL_SAME, any iteration's residual may stop it).  At exit the
 * true residual is recomputed the same way.
 * y, alpha: device, column-major N x nrhs, leading dimension ld.
 * info: host array of nrhs entries (may be NULL).  Synchronises `stream`.
 * Returns ANOVA_E_NOT_CONVERGED if some column reached maxit (alpha then
 * holds the last iterate), ANOVA_E_BREAKDOWN on p^T A p <= 0 or NaN.
 * Errors: ANOVA_E_INVALID for beta <= 0, tol < 0, maxit < 1, nrhs < 1, ld < N.
 */
anova_status krr_cg_solve(anova_plan_t plan, const double *y, double *alpha, int32_t nrhs,
                          int64_t ld, double beta, double tol, int32_t maxit,
                          krr_cg_info *info, void *stream);

/*
 * Solves that advance together.  krr_cg_start sets up one problem's CG
 * (x0 = 0, r = p = y) for nrhs columns on `stream` (asynchronous); alpha
 * receives the iterate and must stay valid until krr_cg_destroy.
 * krr_cg_iterate runs `iters` CG iterations of every listed solve (each
 * column stops at its own tolerance or maxit): one iteration is a batched
 * product over every (solve, window, column), one launch per stage and
 * kernel signature, plus five float64 vector kernels over all columns of
 * all solves; it is captured once per solve list into a hipGraph and
 * replayed (lists of up to 4 recently used combinations are cached).  At
 * each column's iterations R, 2R, ... (as in krr_cg_solve) its residual is
 * recomputed as y - A x, so a column iterates the same way alone and in any
 * list.  The solves of one list must share the precision and the residual
 * mode; a solve may appear in several lists over time (continuous
 * batching).  Asynchronous on `stream`.
 * krr_cg_poll reads the number of still-iterating columns and the current
 * per-column info (synchronises).  krr_cg_finish recomputes the true residual
 * of every column and returns ANOVA_OK, ANOVA_E_NOT_CONVERGED or
 * ANOVA_E_BREAKDOWN like krr_cg_solve (synchronises).  krr_cg_destroy frees
 * the solve (synchronises the device; NULL is a no-op).
 * Not thread-safe across threads sharing solves.
 */
anova_status krr_cg_start(anova_cg_t *out, anova_plan_t plan, const double *y, double *alpha,
                          int32_t nrhs, int64_t ld, double beta, double tol, int32_t maxit,
                          void *stream);
anova_status krr_cg_iterate(anova_cg_t *solves, int32_t count, int32_t iters, void *stream);
anova_status krr_cg_poll(anova_cg_t solve, int32_t *active, krr_cg_info *info, void *stream);
/*
 * Asynchronous poll of a list: enqueues on `stream`, after the work already
 * there, the count of still-iterating columns of every listed solve into
 * dev_counts (device, count int32) and a copy of it to host_counts (host,
 * count int32; pinned memory keeps the copy asynchronous; read it once the
 * stream has passed this point).  Nothing synchronises, so a caller can
 * launch the next iterations before reading the counts.
 * Errors: ANOVA_E_INVALID for an empty list, a NULL solve or array.
 */
anova_status krr_cg_active(anova_cg_t *solves, int32_t count, int32_t *dev_counts,
                           int32_t *host_counts, void *stream);
anova_status krr_cg_finish(anova_cg_t solve, krr_cg_info *info, void *stream);
anova_status krr_cg_destroy(anova_cg_t solve);

/*
 * Solve `count` independent problems together (krr_cg_start for each,
 * krr_cg_iterate over the list of unfinished ones until every column has
 * stopped, krr_cg_finish, krr_cg_destroy).  Arrays of `count` entries;
 * info receives sum(nrhs) entries, problem by problem.  Returns the worst
 * status over the problems.  Synchronises `stream`.
 */
anova_status krr_cg_solve_batched(int32_t count, const anova_plan_t *plans,
                                  const double *const *y, double *const *alpha,
                                  const int32_t *nrhs, const int64_t *ld, const double *beta,
                                  double tol, int32_t maxit, krr_cg_info *info, void *stream);

/*
 * Solve (K~ + lambda_s I) alpha_s = y for nshift regularisation parameters
 * lambda_s at once (the grid over the regularisation parameter in the
 * paper's grid search, Sec. 6; each system is the normal equation of
 * Sec. 2).  The systems share one Krylov space: CG runs on the system with
 * the smallest lambda, and every other system's residual stays a multiple
 * zeta_s of its residual (shifted CG), so one kernel product per iteration
 * serves all of them; each adds two float64 vector updates per iteration.
 * A system stops when zeta_s ||r|| <= tol ||y||.  Then each system's true
 * residual y - (K~ + lambda_s I) alpha_s is recomputed (float64 product;
 * on FP32_NFFT plans the plan's float64 residual windows when it has them),
 * and one that misses tol ||y|| is refined by krr_cg_solve on that
 * residual.  x0 = 0; no preconditioner.
 * y: device, N floats64.  alpha: device, N x nshift column-major, leading
 * dimension ld >= N, not overlapping y; column s solves for shifts[s].
 * shifts: host, nshift
 * values, finite and > 0 (any order, repeats allowed).  info: host array
 * of nshift entries (may be NULL): iters counts the shared iterations the
 * system took part in plus any refinement iterations; relres is the recursive (or refinement)
 * residual, true_relres the recomputed one, both / ||y||.
 * Synchronises `stream`.  Returns ANOVA_E_NOT_CONVERGED if some system
 * missed tol within maxit (alpha holds the last iterates),
 * ANOVA_E_BREAKDOWN on p^T A p <= 0 or NaN.
 * Errors: ANOVA_E_INVALID for a NULL plan/pointer, nshift < 1 or > 32, a
 * shift <= 0 or non-finite, ld < N, tol < 0, maxit < 1.
 */
anova_status krr_cg_solve_shifts(anova_plan_t plan, const double *y, double *alpha,
                                 int32_t nshift, const double *shifts, int64_t ld, double tol,
                                 int32_t maxit, krr_cg_info *info, void *stream);

/* Free every resource of the plan (synchronises the device).  NULL is a no-op. */
anova_status anova_plan_destroy(anova_plan_t plan);

/* Message for the last non-OK status on the calling thread ("" if none).
 * The pointer stays valid until the next call on this thread. */
const char *anova_last_error(void);

/* Parameters and error estimates chosen for window l (0 <= l < P).  Host. */
anova_status anova_plan_query(anova_plan_t plan, int32_t l, anova_window_info *info);

/*
 * Device memory, for admission by memory footprint (the solver's memory of
 * Sec. 2's CG around the Sec. 3 products).  plan_bytes: bytes the plan holds
 * now (its sorted nodes, permutations, tile lists, window polynomials,
 * multipliers, and the work space of anova_matvec once it has run).
 * solve_bytes: bytes that krr_cg_start with nrhs columns on this plan
 * allocates (three float64 N x nrhs vectors, reduction partials, scalars and
 * the product work space of its (window, column) instances); iterate and
 * finish add only launch tables of under 1 KB per window and column.
 * The caller's y and alpha are not counted.  Host outputs (may be NULL).
 * Errors: ANOVA_E_INVALID for a NULL plan or nrhs < 1.
 */
anova_status anova_plan_footprint(anova_plan_t plan, int32_t nrhs, int64_t *plan_bytes,
                                  int64_t *solve_bytes);

/* Number of points and windows of a plan (host outputs, may be NULL). */
anova_status anova_plan_shape(anova_plan_t plan, int64_t *N, int32_t *P, int32_t *precision);

/*
 * Stage entry points for window l (Sec. 4.1 and 4.2), exposing the three
 * steps of one window's fast summation separately.  The grid is the
 * oversampled n^d_A real grid of the window, float32 for ANOVA_FP32_NFFT
 * plans and float64 for ANOVA_FP64 plans, laid out with the first feature of
 * the window fastest: element (u_1, .., u_dA) at u_1 + n u_2 + n^2 u_3.  Grid
 * point u sits at torus position u/n - 1/2 per dimension.
 *
 * anova_stage_spread:   grid = sum_j alpha_j prod_t phi(n x~_j^t - u_t)
 *     (first step of the adjoint NFFT, eq. adjnfft), alpha a device float64
 *     vector of N entries in the caller's point order.  Overwrites grid.
 * anova_stage_convolve: grid <- inverse DFT of (b~_k * DFT(grid)_k) with
 *     b~_k = b_k / prod_t phihat(k_t/n)^2 for k in the index set, 0 outside
 *     (FFT + multiplication by the kernel coefficients + inverse FFT, eq.
 *     fastsum).  In place.  eta_l is not applied here.
 * anova_stage_gather:   out_i += eta_l sum_u grid_u prod_t phi(n x~_i^t - u_t)
 *     (last step of the NFFT, eq. nfft), out a device float64 vector of N
 *     entries in the caller's point order.
 * All three are asynchronous on `stream`.
 */
anova_status anova_stage_spread(anova_plan_t plan, int32_t l, const double *alpha, void *grid,
                                void *stream);
anova_status anova_stage_convolve(anova_plan_t plan, int32_t l, void *grid, void *stream);
anova_status anova_stage_gather(anova_plan_t plan, int32_t l, const void *grid, double *out,
                                void *stream);

/*
 * Per-stage device-time accounting, for benchmarks.  While enabled, every
 * anova_matvec and krr_cg_solve matvec records HIP events on the caller's
 * stream around each launch group of the seven stage kinds, in execution
 * order: 0 permute (coefficients into each window's sorted point order),
 * 1 spread (window-weighted sums into per-tile grid regions), 2 tile sum
 * (regions of one tile added, where a tile holds several), 3 fold (tile
 * regions added into the grid with periodic wrap), 4 convolve (FFT, multiply,
 * inverse FFT, one launch per axis; for n <= 32 in 2-D and 3-D the same filter
 * as a circular convolution, x and y in one launch, z in another), 5 gather
 * (interpolation at the points,
 * written in the caller's order), 6 combine (weighted sum over windows plus
 * the shift).  anova_plan_stage_times synchronises, writes the
 * accumulated milliseconds and launch counts per kind (host arrays of 7) and
 * resets the counters.  Enabling adds a few microseconds of
 * event overhead per launch; disabled by default.
 */
anova_status anova_plan_set_timing(anova_plan_t plan, int32_t enable);
anova_status anova_plan_stage_times(anova_plan_t plan, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* ANOVA_H */
