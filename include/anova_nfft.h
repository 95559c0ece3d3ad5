/*
 * anova_nfft.h — C ABI of the MI355X (gfx950) library for the ANOVA-kernel
 * matrix-vector product by NFFT fast summation and the interior point SVM
 * solver built on it (Wagner, Pearson, Stoll, arXiv 2312.00538).
 *
 * Conventions for every entry point
 *   - Return value: int status, ANOVA_OK (0) on success; nothing is thrown
 *     across the ABI. On failure anova_last_error() returns a message for the
 *     calling thread. Outputs are unspecified on error except where noted.
 *   - "device" pointers address GPU memory (e.g. a torch tensor's data_ptr()
 *     on the current device); "host" pointers address CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *     GPU work of a call is enqueued on that stream, in stream order.
 *   - The caller owns every buffer it passes in. The library never keeps a
 *     caller pointer after a call returns; it owns only the memory behind an
 *     anova_plan_t (transformed coordinates, window weights, grids, scratch),
 *     released by anova_plan_destroy.
 *   - A plan must not be used by two calls at the same time (its scratch
 *     buffers are shared); distinct plans are independent.
 */
#ifndef ANOVA_NFFT_H
#define ANOVA_NFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define ANOVA_OK              0
#define ANOVA_INVALID_ARG     1  /* bad size, index, parameter or label       */
#define ANOVA_OUT_OF_MEMORY   2  /* a device or host allocation failed        */
#define ANOVA_HIP_ERROR       3  /* a HIP runtime call or kernel launch failed */
#define ANOVA_NOT_CONVERGED   4  /* iteration cap reached; outputs hold the last iterate */
#define ANOVA_NUMERICAL       5  /* NaN/Inf, or a factorisation broke down     */

/* arithmetic of the NFFT stages (spreading, grid convolution, gathering) */
#define ANOVA_PREC_FP64   0  /* everything in FP64                                   */
#define ANOVA_PREC_MIXED  1  /* FP32 weights, grids and taps; FP64 window sums        */

/* preconditioner of the Krylov solve inside the IPM */
#define ANOVA_PRECOND_NONE     0  /* unpreconditioned MINRES                           */
#define ANOVA_PRECOND_PCHOL    1  /* greedy pivoted Cholesky, Algorithm 2 (Section 4)   */
#define ANOVA_PRECOND_NYSTROM  2  /* randomized Nystrom, Q = orth(K G) (Section 4)      */
#define ANOVA_PRECOND_RPCHOL   4  /* randomly pivoted Cholesky (Section 4 cites it as
                                     the random-pivot variant of Algorithm 2); pivot
                                     draws from anova_ipm_opts.seed                  */
#define ANOVA_PRECOND_RFF      5  /* random Fourier features (Section 4): rank split
                                     over the windows, draws from anova_ipm_opts.seed */
#define ANOVA_PRECOND_DIAG     3  /* the block-diagonal preconditioner of Section 5
                                     with no low-rank term: diag(Theta, y^T Theta^{-1} y),
                                     the barrier diagonal only (no approximation of K) */

/* Krylov method of the Newton solves inside the IPM (Section 5) */
#define ANOVA_KRYLOV_MINRES 0  /* MINRES with the SPD block-diagonal preconditioner
                                  diag(A_hat, y^T A_hat^{-1} y)                     */
#define ANOVA_KRYLOV_GMRES  1  /* GMRES preconditioned from the right with the
                                  block-triangular P = [[A_hat, 0], [-y^T, -1]];
                                  restarted every min(max_kry, 100) steps; its
                                  residual is the unpreconditioned 2-norm. With
                                  ANOVA_PRECOND_NONE, P = I. HIP graphs unused.   */

#define ANOVA_OPTS_VERSION 1
#define ANOVA_IPM_OPTS_VERSION 3

typedef struct anova_plan_s* anova_plan_t;

/* NFFT fast-summation options (Section 3: bandwidth N and window parameter m
 * of the NFFT; the oversampling factor and the periodic regularisation of the
 * Gaussian are those of the NFFT fast-summation literature the paper cites). */
typedef struct {
    int32_t version;     /* ANOVA_OPTS_VERSION                                     */
    int32_t n_bw;        /* bandwidth N: frequencies -N/2..N/2-1 per axis (even)   */
    int32_t oversample;  /* FFT length per axis = oversample * n_bw                */
    int32_t cutoff_m;    /* Kaiser-Bessel half-width m in grid cells (2..4)        */
    double  eps_b;       /* boundary width of the periodic regularisation, (0,1/2) */
    int32_t reg_p;       /* smoothness of the regularisation; <= 0 picks per axis  */
    int32_t precision;   /* ANOVA_PREC_FP64 or ANOVA_PREC_MIXED                    */
    int32_t seg_points;  /* points per spreading work item; <= 0 = default         */
    int32_t batch_min_rhs; /* cutoff_m = 4 only (either precision): anova_matvec
                            calls with R >= batch_min_rhs run the batched kernels
                            (16 right-hand sides per pass, matrix-core spreading
                            and gathering); 0 = default 2, < 0 = never        */
} anova_opts;

/* Fill `o` with the defaults: n_bw = 32, oversample = 2, cutoff_m = 4,
 * eps_b = 1/4, reg_p = 0 (automatic), precision = FP64, seg_points = 0,
 * batch_min_rhs = 0. */
int anova_opts_default(anova_opts* o);

/* Build a fast-summation plan for the ANOVA Gaussian kernel of Section 3:
 *     K = sum_{l=1..P} eta_l K_l,
 *     (K_l)_{ij} = exp(-||x_i^{W_l} - x_j^{W_l}||^2 / sigma_l^2),
 * each window W_l holding 1..3 features.
 *   X        device, N x d FP64, row i at X + i*ldx (ldx >= d). Read during the
 *            call only; the plan keeps transformed copies.
 *   windows  host, P x 3 int32 feature indices in [0, d), -1 marks an unused
 *            slot; every window has 1..3 distinct features.
 *   sigma    host, P FP64 kernel widths (> 0), one per window.
 *   eta      host, P FP64 window weights, or NULL for eta_l = 1.
 *   opts     host, NULL for the defaults.
 *   out      host, receives the plan handle.
 * Errors: ANOVA_INVALID_ARG (N < 1, d < 1, P < 1, bad window, sigma <= 0,
 * unsupported options), ANOVA_OUT_OF_MEMORY, ANOVA_HIP_ERROR. The call
 * synchronises `stream` (it reads back bin counts to lay out the work). */
int anova_plan_create(const double* X, int64_t N, int32_t d, int64_t ldx,
                      const int32_t* windows, int32_t P,
                      const double* sigma, const double* eta,
                      const anova_opts* opts, void* stream, anova_plan_t* out);

/* y = K x for R right-hand sides (Section 3, "(K_1 + ... + K_P) v"): every
 * window is evaluated by NFFT fast summation (spread with the Kaiser-Bessel
 * window, grid convolution with the kernel's Fourier coefficients, gather)
 * and the windows are summed in FP64 in a fixed order, so results are
 * bitwise reproducible for a given plan, input and R. Plans with
 * cutoff_m = 4 take R >= batch_min_rhs right-hand sides 16 at a time through
 * the batched kernels (same algorithm, spreading and gathering as matrix-core
 * contractions): FP64 plans on FP64 matrix cores, agreeing with the
 * one-at-a-time kernels to FP64 rounding (below 1e-11 relative); mixed plans
 * spread in FP32 and gather in split-bf16 (three bf16 products per FP32
 * product), agreeing with the one-at-a-time kernels to FP32 rounding. Neither
 * is bit for bit the one-vector result. The batched path allocates its
 * scratch (about 16x the single-vector scratch) on first use.
 *   x   device, N x R FP64, column r at x + r*ldx_ (ldx_ >= N).
 *   y   device, N x R FP64 output, column r at y + r*ldy (ldy >= N); must not
 *       overlap x.
 * Asynchronous on `stream`. Errors: ANOVA_INVALID_ARG (NULL plan/pointers,
 * R < 1, leading dimensions < N), ANOVA_HIP_ERROR. */
int anova_matvec(anova_plan_t plan, const double* x, int32_t R, int64_t ldx_,
                 double* y, int64_t ldy, void* stream);

/* Allocation-free form of anova_matvec, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. It computes what anova_matvec computes with R
 * one-vector passes (bit for bit the same result as anova_matvec for R = 1,
 * and for any R on plans that do not batch), through the same kernels, but
 * the passes' scratch arrays (permuted input, slabs, fold target, grids,
 * gathered values) live in one static array of the library instead of the
 * plan's buffers. That array holds ANOVA_NOALLOC_SCRATCH_BYTES (64 MiB) per
 * device; it is part of the loaded library and stays allocated on every
 * device the library runs on until the process ends. The call allocates no
 * device memory (no hipMalloc, hipFree or allocating library routine); its
 * first call on a device looks up that device's copy of the array.
 * All calls on one device share its array, which keeps the last call's
 * contents (every pass writes what it reads): calls that overlap in time on
 * one device, on different streams or threads, race and must be serialised
 * by the caller; calls in order on one stream are safe.
 *   plan, x, R, ldx_, y, ldy, stream: as for anova_matvec.
 * Errors: as for anova_matvec, and ANOVA_INVALID_ARG when the plan's
 * one-vector scratch exceeds ANOVA_NOALLOC_SCRATCH_BYTES (the message gives
 * the size it needs). */
#define ANOVA_NOALLOC_SCRATCH_BYTES (64ll << 20)
int anova_matvec_noalloc(anova_plan_t plan, const double* x, int32_t R, int64_t ldx_,
                         double* y, int64_t ldy, void* stream);

/* The Kaiser-Bessel window of the plans' NFFT (Section 3 names the window
 * parameter m; the window is the Kaiser-Bessel pair of the NFFT literature it
 * cites), for checking it outside a plan. Host only: no device work.
 *   opts     as for anova_plan_create (NULL: defaults); uses n_bw, oversample
 *            (FFT length n = oversample * n_bw) and cutoff_m.
 *   u, nu    host, nu offsets in grid cells, |u| <= cutoff_m.
 *   phi      host, nu outputs: phi(u) / phi(0) with
 *            phi(u) = sinh(b sqrt(m^2 - u^2)) / (pi sqrt(m^2 - u^2)),
 *            b = pi (2 - n_bw / n).
 *   phi_hat  host, n/2 + 1 outputs or NULL: for k = 0 .. n/2 the transform
 *            (1/n) I0(m sqrt(b^2 - (2 pi k / n)^2)) / phi(0) (J0 of the
 *            imaginary argument past b), i.e. the integral of
 *            phi(u) e^{-2 pi i k u / n} du divided by n phi(0).
 * Errors: ANOVA_INVALID_ARG (bad options, NULL pointers, |u| > m). */
int anova_kaiser_bessel(const anova_opts* opts, const double* u, int32_t nu, double* phi, double* phi_hat);

/* The one-axis coefficients a plan builds for a feature with data range
 * [lo, hi] and kernel width sigma (Section 3: the kernel replaced by a
 * trigonometric polynomial, evaluated by an adjoint and a forward NFFT), for
 * checking them outside a plan. Host only: no device work.
 *   opts   as for anova_plan_create (NULL: defaults).
 *   bk     host, n_bw outputs or NULL: b_k for k = -n_bw/2 .. n_bw/2 - 1 (index
 *          k + n_bw/2), the trigonometric interpolation coefficients of the
 *          1-periodic regularised Gaussian exp(-t^2 / sigma_a^2) in torus units.
 *   circ   host, n = oversample * n_bw outputs or NULL: first column of the real
 *          symmetric circulant that the grid step applies along this axis
 *          (forward FFT, times B_k = b_k / (n phi_hat(k))^2, inverse FFT; the
 *          unpaired frequency -n_bw/2 split evenly between +-n_bw/2).
 *   axis   host, 4 outputs or NULL: center and scale of the torus map
 *          u = (x - center) * scale, sigma_a = sigma * scale, and the largest
 *          |trigonometric interpolant - Gaussian| on the box |t| <= 1/2 - eps_b.
 *   reg_p  host or NULL: smoothness p of the regularisation chosen.
 * Errors: ANOVA_INVALID_ARG (bad options, lo > hi, sigma <= 0, NaN). */
int anova_axis_coefficients(double lo, double hi, double sigma, const anova_opts* opts, double* bk, double* circ,
                            double* axis, int32_t* reg_p);

/* Release a plan and all device memory it owns (synchronises the device).
 * NULL is accepted. */
int anova_plan_destroy(anova_plan_t plan);

/* Plan facts for diagnostics and tests (host struct filled by the call). */
typedef struct {
    int64_t n_points;
    int32_t n_windows;
    int32_t n_segments;      /* spreading/gathering work items                  */
    int32_t cutoff_m;
    int32_t precision;
    double  eps_b;
    double  max_kernel_err;  /* max over windows/axes of the 1D regularised-
                                kernel interpolation error (absolute)           */
    int64_t grid_cells;      /* occupied grid cells summed over windows          */
    int64_t device_bytes;    /* device memory owned by the plan                  */
} anova_plan_info_t;
int anova_plan_info(anova_plan_t plan, anova_plan_info_t* info);

/* Stage timing for measurement tools. Between anova_profile_begin and
 * anova_profile_end, every anova_matvec on the plan also records HIP events on
 * the caller's stream between its stages (no extra synchronisation):
 *   0 permute input, 1 spread, 2 fold slabs, 3 grid convolution (3 axis
 *   passes), 4 gather, 5 window sum.
 * anova_profile_end synchronises on the last event and writes, for each
 * stage s < nstage, the mean duration per pass in ms (stage_ms, host) and
 * the number of passes measured (*passes, host). A pass covers one
 * right-hand side, or up to 16 in the batched path.
 * Errors: ANOVA_INVALID_ARG, ANOVA_HIP_ERROR. */
#define ANOVA_NSTAGES 6
int anova_profile_begin(anova_plan_t plan);
int anova_profile_end(anova_plan_t plan, double* stage_ms, int32_t nstage, int32_t* passes);

/* ------------------------------------------------------------------ IPM
 * Interior point method of Algorithm 1 (Section 2) for the soft-margin SVM
 * dual (Section 1, eq. "kernelsvm"):
 *     max e^T a - 1/2 a^T Y K Y a  s.t. 0 <= a <= C, y^T a = 0,
 * with K the plan's ANOVA kernel. Each Newton system (Section 2, eq.
 * "Newton") is solved by MINRES preconditioned with the block-diagonal SPD
 * matrix diag(A_hat, y^T A_hat^{-1} y), A_hat = Theta + Y Z^T Z Y, applied
 * through the Sherman-Morrison-Woodbury identity (Section 5), with the
 * low-rank factor Z^T from Algorithm 2 or the Nystrom method (Section 4);
 * or (krylov = ANOVA_KRYLOV_GMRES) by GMRES with the block-triangular
 * preconditioner of Section 5 and the same A_hat. */
typedef struct {
    int32_t version;     /* ANOVA_IPM_OPTS_VERSION                               */
    int32_t max_ip;      /* IPM iteration cap (Table 1: 50)                      */
    int32_t max_kry;     /* Krylov iterations per Newton solve (Table 1: 100)    */
    int32_t precond;     /* ANOVA_PRECOND_*                                      */
    double  tol;         /* on mu, |y^T a|/|y^T a0| and the relative duality gap;
                            on FP64 plans the gap, measured with the plan's
                            fast-summation operator, must fall to tol / 2 (the
                            other half covers its difference from the exact
                            kernel's gap); mixed-precision plans stop at tol.
                            mu is never reduced below tol / 1000              */
    double  tol_inf;     /* on ||xi_lambda||/||xi_lambda^0|| (Table 1: 1e-1)    */
    double  tol_kry;     /* upper bound of the Krylov relative tolerance (1e-3)  */
    double  sigma_bar;   /* barrier reduction (Table 1: 0.6)                     */
    double  gamma0;      /* step-to-boundary factor (Algorithm 1: 0.99995)       */
    double  mu0;         /* initial barrier parameter (Algorithm 1: 1.0); <= 0:
                            the mean complementarity |1 - y_i (KYa)_i| min(a_i, C - a_i)
                            at the starting point, at least 1                    */
    int32_t rank;        /* low-rank factor rank k                               */
    int32_t mu_rule;     /* 0: sigma_it = 1 - (1 - sigma_bar) * (previous step);
                            1: constant sigma_bar (Section 2 allows either)      */
    double  err_tol;     /* pivoted-Cholesky trace tolerance (Table 1: 1e-5)     */
    uint64_t seed;       /* Gaussian test matrix of the Nystrom method           */
    int32_t graphs;      /* 1: each MINRES iteration is captured once as a HIP
                            graph and replayed (solves outside a server or grid);
                            0: launched kernel by kernel. Same arithmetic.       */
    int32_t krylov;      /* ANOVA_KRYLOV_MINRES (0) or ANOVA_KRYLOV_GMRES (1)    */
    int32_t factor_fp32; /* 1: the low-rank factor is built in FP64 and rounded
                            to FP32 values; Z^T u and Z t read an FP32 copy
                            (half the bytes) and the capacitance Gram matrix the
                            FP64 copy of the same values, all with FP64
                            multiplies and sums, so the preconditioner is
                            exactly that of the rounded factor and stays SPD
                            (FP32 arithmetic in the Woodbury form, whose two
                            terms cancel where theta is small, can make it
                            indefinite); 0: the unrounded FP64 factor. Only the
                            preconditioner changes, not the Newton systems.     */
} anova_ipm_opts;

typedef struct {
    int32_t ip_iters;
    int32_t kry_iters_total;
    int32_t kry_iters_max;
    int32_t rank_used;
    int32_t status;
    int32_t matvecs;
    double  mu;
    double  rel_gap;         /* (Pr - D)/(1 + |Pr|) with the plan's operator     */
    double  dual_obj;        /* D = e^T a - 1/2 a^T Y K Y a                      */
    double  primal_obj;      /* 1/2 a^T Y K Y a + C sum max(0, 1 - y_i f_i)      */
    double  xi_alpha_rel;
    double  xi_lambda_rel;
    double  t_setup_ms;      /* preconditioner build                             */
    double  t_solve_ms;      /* whole call                                       */
} anova_ipm_stats;

/* Fill `o` with the defaults: Table 1 values (max_ip = 50 raised to 100,
 * max_kry = 100, tol_kry = 1e-3, sigma_bar = 0.6, gamma0 = 0.99995,
 * mu0 = 1, err_tol = 1e-5), tol = 1e-6, tol_inf = 1e-1, precond = PCHOL,
 * rank = 200, mu_rule = 0 (step-scaled reduction), seed = 0, graphs = 1,
 * krylov = MINRES, factor_fp32 = 1. */
int anova_ipm_opts_default(anova_ipm_opts* o);

/* Train: alpha (device, N FP64 out), lambda (host, 1 FP64 out; the bias of
 * the decision function f(x) = sum_j alpha_j y_j k(x, x_j) - lambda).
 *   labels  device, N FP64 values in {-1, +1}, both classes present.
 *   C       box bound (> 0).
 *   opts    host or NULL (defaults); stats host or NULL.
 * Synchronises `stream` (host-driven iteration). Errors: ANOVA_INVALID_ARG,
 * ANOVA_OUT_OF_MEMORY, ANOVA_HIP_ERROR, ANOVA_NUMERICAL; ANOVA_NOT_CONVERGED
 * when max_ip is reached, with alpha/lambda/stats holding the last iterate. */
int svm_ipm_solve(anova_plan_t plan, const double* labels, double C,
                  const anova_ipm_opts* opts, double* alpha, double* lambda,
                  anova_ipm_stats* stats, void* stream);

/* Greedy pivoted Cholesky of the plan's kernel (Algorithm 2, Section 4),
 * column by column with exact kernel columns: K ~= L L^T.
 *   rank     maximum rank k; err_tol stops early when the remaining trace is
 *            <= err_tol * trace(K).
 *   L        device, N x rank FP64 output, column j at L + j*ldl (ldl >= N);
 *            columns >= *rank_used are unspecified.
 *   piv      host, rank int64 output, pivot indices in the order chosen.
 *   rank_used host output.
 * Synchronises `stream`. Errors: ANOVA_INVALID_ARG, ANOVA_HIP_ERROR. */
int anova_pivoted_cholesky(anova_plan_t plan, int32_t rank, double err_tol,
                           double* L, int64_t ldl, int64_t* piv, int32_t* rank_used,
                           void* stream);

/* Randomly pivoted Cholesky of the plan's kernel: Algorithm 2 with the pivot
 * of step j drawn with probability proportional to the residual diagonal.
 * With C_i = sum_{t <= i} max(d_t, 0) over the residual diagonal d, step j
 * takes the smallest i with C_i > uniforms[j] * C_{N-1}.
 *   uniforms host, rank FP64 values in [0, 1) (the draws, supplied by the
 *            caller so that results are reproducible and checkable).
 * Other arguments, outputs and errors as for anova_pivoted_cholesky. */
int anova_rp_cholesky(anova_plan_t plan, int32_t rank, double err_tol, const double* uniforms,
                      double* L, int64_t ldl, int64_t* piv, int32_t* rank_used, void* stream);

/* Random Fourier features of the plan's kernel (Section 4): K ~= Z Z^T with
 * rank k split over the windows (k_l = floor(k / P), the first k mod P windows
 * one more). Feature j of window l is
 *     sqrt(eta_l) sqrt(2 / k_l) cos(w_j^T x^{W_l} + b_j),
 * which for w_j ~ N(0, (2 / sigma_l^2) I) and b_j ~ U(0, 2 pi) has expectation
 * K_l (Bochner's theorem for the Gaussian).
 *   w   host, k x 3 FP64: row j holds w_j for the window's features in order
 *       (entries past the window's size are ignored).
 *   b   host, k FP64.
 *   Z   device, N x k FP64 output, column j at Z + j*ldz (ldz >= N).
 * Synchronises `stream`. Errors: ANOVA_INVALID_ARG, ANOVA_HIP_ERROR. */
int anova_rff_factor(anova_plan_t plan, int32_t k, const double* w, const double* b, double* Z, int64_t ldz,
                     void* stream);

/* Randomized Nystrom factor (Section 4): Q = orth(K G) and
 * K ~= (KQ)(Q^T K Q)^{-1}(KQ)^T = Z^T Z, with Q^T K Q = L D L^T and diagonal
 * entries of D below 1e-12 * max(diag(Q^T K Q)) raised to that value.
 *   G    device, N x k FP64 test matrix (column j at G + j*ldg); drawn by the
 *        caller so that the factor is reproducible.
 *   Zt   device, N x k FP64 output Z^T (column j at Zt + j*ldz).
 * Synchronises `stream`. Errors: ANOVA_INVALID_ARG (k < 1 or k > N),
 * ANOVA_NUMERICAL (orthonormalisation broke down), ANOVA_HIP_ERROR. */
int anova_nystrom(anova_plan_t plan, const double* G, int32_t k, int64_t ldg,
                  double* Zt, int64_t ldz, void* stream);

/* The low-rank-plus-diagonal preconditioner of Section 5 applied to one
 * vector: out = (Theta + Y Z Z^T Y)^{-1} r with Theta = diag(theta) and
 * Y = diag(y), through the Sherman-Morrison-Woodbury form of Section 5,
 *   Theta^{-1} r - Theta^{-1} Y Z (I + Z^T Theta^{-1} Z)^{-1} Z^T Y Theta^{-1} r,
 * by the kernels the interior point method uses every iteration (the
 * capacitance matrix on the matrix cores, its Cholesky factor, the two N x k
 * passes).
 *   N, k   sizes, N >= 1, 1 <= k <= 1024.
 *   Z      device, N x k FP64 factor, column j at Z + j*ldz (ldz >= N);
 *          copied, not modified.
 *   theta  device, N FP64 diagonal, every entry > 0.
 *   y      device, N FP64 signs (+-1), or NULL for Y = I.
 *   r      device, N FP64 input.   out  device, N FP64 output (not r).
 *   fp32_products  0: the N x k passes read the FP64 factor; 1: the factor is
 *          first rounded to FP32 values and the passes read an FP32 copy (the
 *          solver's anova_ipm_opts.factor_fp32 form; the result is that of the
 *          rounded factor).
 * Allocates its scratch per call and synchronises `stream`. Errors:
 * ANOVA_INVALID_ARG (sizes, NULL pointers, ldz < N), ANOVA_NUMERICAL (the
 * capacitance matrix is not numerically positive definite),
 * ANOVA_OUT_OF_MEMORY, ANOVA_HIP_ERROR. */
int anova_lowrank_apply(int64_t N, int32_t k, const double* Z, int64_t ldz,
                        const double* theta, const double* y, const double* r,
                        int32_t fp32_products, double* out, void* stream);

/* ------------------------------------------------------------------ serving
 * A request server that runs interior point solves (svm_ipm_solve semantics)
 * of different sizes on one GPU with continuous batching. Requests are
 * admitted, first fit in arrival order, while fewer than max_active solves are
 * resident and the estimated device footprint of the resident solves
 * (anova_request_footprint) stays within hbm_budget; a request that fits no
 * budget still runs when nothing else is resident. An admitted solve keeps its
 * plan, iterates and preconditioner on the device until it finishes and runs
 * on its own stream and host thread, so the work of resident solves overlaps
 * on the GPU, and admission continues as slots and memory free up. With
 * share_launches, the one-vector matvecs of the resident solves are collected
 * and run together: every matvec stage is one kernel launch for up to 8
 * solves. Each solve's arithmetic is the same alone or in a mix, so results do
 * not depend on what else is resident.
 * Thread safety: submit and wait may be called from any threads. */
#define ANOVA_SERVER_OPTS_VERSION 1
typedef struct anova_server_s* anova_server_t;

typedef struct {
    int32_t version;         /* ANOVA_SERVER_OPTS_VERSION                           */
    int32_t max_active;      /* resident solves at once, 1..64 (default 8)          */
    int64_t hbm_budget;      /* device bytes for resident solves; <= 0: 80% of the
                                free memory when the server is created (default)    */
    int32_t share_launches;  /* 1 (default): resident solves share matvec launches  */
    int32_t reserved;
    double  gather_us;       /* longest wait for more matvecs before a shared launch
                                (microseconds, default 200)                          */
} anova_server_opts;

typedef struct {
    const double*  X;        /* host, N x d FP64 row-major; copied by submit        */
    const double*  labels;   /* host, N FP64 in {-1, +1}; copied by submit          */
    const int32_t* windows;  /* host, P x 3 as for anova_plan_create; copied         */
    const double*  sigma;    /* host, P kernel widths; copied                        */
    int64_t N;
    int32_t d;
    int32_t P;
    double  C;
    const anova_opts*     nfft;  /* host or NULL (defaults); copied                 */
    const anova_ipm_opts* ipm;   /* host or NULL (defaults); copied                 */
} anova_request;

typedef struct {
    int32_t status;          /* the solve's status                                  */
    int32_t reserved;
    int64_t footprint;       /* bytes charged against the budget                    */
    double  queue_ms;        /* submit -> admission                                 */
    double  run_ms;          /* admission -> result on the host                     */
    double  latency_ms;      /* submit -> result on the host                        */
    double  lambda;          /* as svm_ipm_solve's lambda                           */
    anova_ipm_stats stats;
} anova_result;

/* Defaults: max_active = 8, hbm_budget = 0 (80% of free memory),
 * share_launches = 1, gather_us = 200. */
int anova_server_opts_default(anova_server_opts* o);

/* Start a server on HIP device `device` (scheduler and, with shared launches,
 * combiner threads). opts host or NULL. Errors: ANOVA_INVALID_ARG,
 * ANOVA_HIP_ERROR. */
int anova_server_create(const anova_server_opts* opts, int32_t device, anova_server_t* out);

/* Queue a solve; returns at once with a ticket (host out). The inputs are
 * copied, so the caller's buffers may be reused immediately. Errors:
 * ANOVA_INVALID_ARG (NULL fields, N < 2, d < 1, P < 1, C <= 0, option
 * version mismatch); problems found later (bad labels, windows) are reported
 * by anova_server_wait. */
int anova_server_submit(anova_server_t s, const anova_request* req, int64_t* ticket);

/* Block until the ticket's solve has finished, then copy alpha (host, N FP64,
 * may be NULL) and the result record (host, may be NULL); the ticket is
 * consumed. Returns the solve's status (ANOVA_OK, ANOVA_NOT_CONVERGED, or the
 * error it failed with, with the message in anova_last_error()). */
int anova_server_wait(anova_server_t s, int64_t ticket, double* alpha, anova_result* result);

/* Shared-launch counters since creation: launches made and matvecs served
 * (host outs; both 0 without shared launches). */
int anova_server_counters(anova_server_t s, int64_t* launches, int64_t* matvecs);

/* Finish every queued and resident solve, then stop. NULL is accepted.
 * Results not collected by anova_server_wait are dropped. */
int anova_server_destroy(anova_server_t s);

/* The device footprint the server charges for a request of this shape
 * (host out, bytes): inputs, plan, grids, iterates and preconditioner, with
 * a 25% margin. nfft and ipm host or NULL (defaults). */
int anova_request_footprint(int64_t N, int32_t d, int32_t P, const anova_opts* nfft,
                            const anova_ipm_opts* ipm, int64_t* bytes);

/* Decision values of a trained SVM at M new points (Section 2: the classifier
 * is f(x) = sum_j alpha_j y_j k(x, x_j) - lambda): the kernel sum with targets
 * other than its sources. One plan is built over the union of the training
 * and the new points, so that one torus map covers both, and one matvec of
 * [y * alpha ; 0] gives f at the new points.
 *   X       device, N x d FP64 training points, row i at X + i*ldx (ldx >= d).
 *   Xnew    device, M x d FP64 new points, row j at Xnew + j*ldn (ldn >= d).
 *   windows, P, sigma, eta, opts  as for anova_plan_create (the training plan's).
 *   labels, alpha  device, N FP64: the training labels and svm_ipm_solve's alpha.
 *   lambda  svm_ipm_solve's lambda.
 *   f       device, M FP64 output.
 * Synchronises `stream`. Errors as for anova_plan_create; ANOVA_OUT_OF_MEMORY. */
int anova_decision_function(const double* X, int64_t N, int64_t ldx, const double* Xnew, int64_t M,
                            int64_t ldn, int32_t d, const int32_t* windows, int32_t P, const double* sigma,
                            const double* eta, const anova_opts* opts, const double* labels,
                            const double* alpha, double lambda, double* f, void* stream);

/* ---- Hyperparameter grid -------------------------------------------------
 * Parameter search (Section 6.3 selects sigma and C by a search over
 * parameter combinations): many IPM solves that differ in the data (folds),
 * the kernel widths and C. One problem is one plan (a fold's training points
 * and one set of widths) with its labels and a list of C values. The low-rank
 * preconditioner depends on the kernel matrix only, so the solves of a
 * problem share one factor (built by the first of them). Up to max_active
 * solves run at once, each on its own stream and host thread; their matvecs
 * are collected and run together: the vectors of one plan in one 16-wide
 * batched pass when the plan is mixed precision with cutoff_m = 4 (any
 * number of them, one included, so each solve's arithmetic does not depend
 * on the other solves), other plans in shared one-vector launches. */
typedef struct {
    anova_plan_t plan;       /* each plan in at most one problem                     */
    const double* labels;    /* device, N of the plan, {-1, +1}                      */
    int32_t n_c;             /* number of C values, >= 1                             */
    int32_t reserved;
    const double* C;         /* host, n_c values > 0                                 */
    double* alpha;           /* device out, N x n_c column-major: column j for C[j]  */
    double* lambda;          /* host out, n_c                                        */
    anova_ipm_stats* stats;  /* host out, n_c; stats[j].status is that solve's
                                status (ANOVA_OK, ANOVA_NOT_CONVERGED or an error)  */
} anova_grid_problem;

/* Run every (problem, C) solve of the grid and return when all have
 * finished. Runs on the current HIP device, on streams of its own: the inputs
 * must be ready on the device before the call and the outputs are ready when
 * it returns. The plans must not be used by other calls meanwhile. opts as
 * for svm_ipm_solve (host or NULL). max_active in [1, 256]; gather_us: the
 * longest wait for more matvecs before a shared launch (microseconds, >= 0).
 * launches / matvecs (host, may be NULL): shared launches made and matvecs
 * served. Returns ANOVA_INVALID_ARG (NULL fields, n_c < 1, C <= 0, a plan in
 * two problems, bad options) before any solve starts, ANOVA_HIP_ERROR, or
 * ANOVA_OK with the per-solve outcome in stats[j].status. */
int anova_grid_solve(const anova_grid_problem* problems, int32_t n_problems, const anova_ipm_opts* opts,
                     int32_t max_active, double gather_us, int64_t* launches, int64_t* matvecs);

/* ---- Autotuner -------------------------------------------------------------
 * Chooses the fast-summation options for one data set and kernel widths: the
 * bandwidth N and cutoff m (Section 3 leaves both to the user: the error of
 * the NFFT-based sum falls and its cost grows with each), the precision and the
 * number of points per spreading work item. Every candidate plan multiplies a
 * seeded random block of `rhs` columns; its relative l2 error is measured
 * against an FP64 plan with bandwidth 64 and cutoff 4 (bandwidth 32 when the
 * data's occupied grid box does not fit), and the candidates within the target
 * are timed on `stream` (HIP events, `reps` calls each after one warm-up). The
 * fastest wins; a second pass tries two other work-item sizes for it.
 * Candidates: cutoff 2, 3, 4 x bandwidth 16, 24, 32, 48, 64 for each selected
 * precision. */
#define ANOVA_TUNE_OPTS_VERSION 1
typedef struct {
    int32_t  version;         /* ANOVA_TUNE_OPTS_VERSION                              */
    int32_t  rhs;             /* right-hand sides per timed matvec call, 1..64        */
    double   target_rel_err;  /* admissible relative l2 error (> 0)                   */
    int32_t  precisions;      /* bit 0: FP64 candidates, bit 1: mixed-precision ones   */
    int32_t  reps;            /* timed calls per admissible candidate, 1..100         */
    uint64_t seed;            /* the random test block                                */
} anova_tune_opts;

typedef struct {
    int32_t n_bw, cutoff_m, precision, seg_points;
    double  rel_err;          /* against the reference plan; < 0: the data set cannot
                                 use this size (the plan could not be built)          */
    double  ms;               /* mean time per call; < 0: not timed (error too large) */
} anova_tune_candidate;

/* rhs = 1, target_rel_err = 1e-4, both precisions, reps = 3, seed = 0. */
int anova_tune_opts_default(anova_tune_opts* t);

/* Run the search. Inputs as for anova_plan_create (X device; windows, sigma,
 * eta host); t host or NULL (defaults); best (host out) receives complete plan
 * options (defaults for the fields not searched). cands (host, may be NULL)
 * receives up to max_cands candidates in the order tried, *n_cands (host, may
 * be NULL) the number tried. Synchronises `stream`. Errors: ANOVA_INVALID_ARG,
 * ANOVA_NOT_CONVERGED (no candidate within the target; cands still filled),
 * ANOVA_OUT_OF_MEMORY, ANOVA_HIP_ERROR. */
int anova_autotune(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows, int32_t P,
                   const double* sigma, const double* eta, const anova_tune_opts* t, void* stream,
                   anova_opts* best, anova_tune_candidate* cands, int32_t max_cands, int32_t* n_cands);

/* ------------------------------------------------------------------ windows
 * Windows of features by mutual-information ranking (Section 3 builds the
 * windows W_l from the features' mutual-information scores). Each feature's
 * mutual information with the labels (nats) is estimated from a histogram of
 * `bins` equal-width bins over the feature's range [min, max] against the two
 * classes: bin floor((x - min) * (bins / (max - min))), clamped to bins - 1
 * (a constant feature falls in bin 0), and the estimate is
 * sum over n > 0 of (n / N) log(n N / (n_bin n_class)). The features are
 * ranked by it, largest first, ties to the lower index, and window l holds
 * the ranked features 3l, 3l + 1, 3l + 2 (the last window the remaining 1 or
 * 2 when 3P > d), so the windows cover the min(3P, d) best features.
 *   X        device, N x d row-major FP64, leading dimension ldx >= d; finite.
 *   labels   device, N FP64; a label > 0 is class +1, any other class -1.
 *   bins     2..1024.
 *   P        number of windows, 1 <= P <= ceil(d / 3).
 *   windows  host out, P x 3 int32, -1 padded (the layout anova_plan_create takes).
 *   mi       host out (may be NULL), d FP64: the estimate per feature.
 * Synchronises `stream`. Errors: ANOVA_INVALID_ARG (sizes, NaN/Inf in X),
 * ANOVA_OUT_OF_MEMORY, ANOVA_HIP_ERROR. */
int anova_mi_windows(const double* X, int64_t N, int32_t d, int64_t ldx, const double* labels, int32_t bins,
                     int32_t P, int32_t* windows, double* mi, void* stream);

/* Message describing the last failure on the calling thread ("" if none). */
const char* anova_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ANOVA_NFFT_H */
