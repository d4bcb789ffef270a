/*
 * ttfp.h -- C ABI of the tensor-train Fourier pricer for multi-asset options (gfx950).
 *
 * The library prices a European option on d assets that follow correlated geometric
 * Brownian motion (the market model of Sec. II.A of "A highly efficient tensor network
 * algorithm for multi-asset Fourier options pricing"). The price is the d-dimensional
 * shifted-contour Fourier integral of the characteristic function times the payoff
 * transform (Sec. III.B, Eq. maincont; Sec. III.C, Eq. main), discretised on a truncated
 * uniform grid (Sec. III.D, Eq. discr). The integrand tensor on that grid is built as a
 * tensor train by TT-cross (Sec. IV.B) and contracted against the quadrature weights
 * (Sec. IV.A); the cost is linear in d instead of N^d.
 *
 * Max/min payoffs are priced as a sum of d separable terms, one per asset that attains the
 * extreme; term j uses coordinates w_0 = x_j, w_l = x_l - x_j (x = log(S_T/K)).
 *
 * Conventions shared by every call:
 *  - All pointers in ttfp_option / ttfp_grid are HOST pointers owned by the caller; the
 *    library copies what it needs before returning. Output arrays are caller-owned host
 *    memory unless the name ends in _dev, in which case they are device pointers on the
 *    context's device (for example the storage of torch tensors).
 *  - A context owns its device workspaces and is bound to one device and one HIP stream.
 *    It is not thread-safe: calls on one context must not overlap.
 *  - Return codes: 0 = success; negative = hard error, nothing written to outputs;
 *    positive = warning, outputs written. No C++ exception crosses this boundary.
 *    ttfp_last_error() gives the text of the last error on a context.
 */
#ifndef TTFP_H
#define TTFP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TTFP_OK = 0,
    TTFP_EINVAL = -1,     /* invalid argument: d out of range, N < 2, S0/K/sigma/T <= 0, NaN,
                             correlation not symmetric / unit-diagonal / positive definite,
                             contour shift outside the payoff's strip, rank beyond limits */
    TTFP_ENOMEM = -2,     /* device allocation failed */
    TTFP_EDEVICE = -3,    /* HIP runtime error (text in ttfp_last_error) */
    TTFP_ENOTCONV = 1,    /* tolerance not met within max_sweeps or rank capped; price written */
    TTFP_EPRECISION = 2   /* cancellation factor times machine epsilon exceeds tol, or a
                             numerical failure (exactly singular maxvol start, non-finite
                             price); price written */
};

/* Payoffs (Sec. II.A uses the call on the minimum, Eq. minpayoff). The first three are priced
 * as d separable terms (see above). TTFP_CALL_MIN_STRIP is the call on the minimum in the
 * paper's own form (Sec. III.C, the min transform under Eq. main): one term in the asset
 * coordinates x with the joint transform (-1)^(d+1) / ((1 + i sum_k z_k) prod_k (i z_k)) on
 * Im z_k > 0, sum_k Im z_k > 1 (the transform as direct integration gives it; the printed one
 * differs by the phase i^(d-2)). Its automatic contour is alpha_k = a_k + 1/d (a_k the aliasing
 * distance); a scalar grid alpha puts +alpha on every coordinate (the paper uses 5/d). */
typedef enum { TTFP_CALL_MAX = 0, TTFP_PUT_MAX = 1, TTFP_CALL_MIN = 2, TTFP_CALL_MIN_STRIP = 3 } ttfp_payoff;

#define TTFP_MAX_D 32      /* largest number of assets */
#define TTFP_MAX_RANK 64   /* largest TT rank (plus enrichment columns <= 68) */

/* One option. S0[d], sigma[d] and corr[d*d] (row-major) are host arrays.
 * Jumps (Merton's model, the characteristic-function extension of Sec. VI): jump_rate > 0 adds a
 * compound-Poisson part with one clock at that rate per year and normally distributed log-jump
 * sizes of mean jump_mean[d] and covariance jump_cov[d*d] (symmetric, positive semidefinite); the
 * mean of ln S_T carries the compensator -jump_rate (e^{jump_mean_j + jump_cov_jj/2} - 1) T that
 * keeps the discounted prices martingales, and the characteristic function gains the factor
 * exp(jump_rate T (E[e^{i z.J}] - 1)). jump_rate = 0 (the pointers may be NULL): plain GBM.
 * Delta and vega keep their forms (the jump part does not depend on S0 or sigma). */
typedef struct {
    int32_t d;
    int32_t payoff;            /* ttfp_payoff */
    const double *S0;
    const double *sigma;
    const double *corr;
    double K, T, r;
    double jump_rate;
    const double *jump_mean;
    const double *jump_cov;
} ttfp_option;

/* Grid and TT-cross settings.
 *  N            nodes per coordinate, 2..1024: u_i = -L + (i + 1/2) 2L/N, i = 0..N-1
 *  L            > 0: the same half-width on every coordinate of every term; <= 0: automatic
 *  alpha        > 0: |contour shift| on every coordinate, signed by the coordinate's strip
 *               (call coordinate +alpha, which must exceed 1; put coordinate -alpha;
 *               max indicators -alpha; min indicators +alpha; TTFP_CALL_MIN_STRIP +alpha,
 *               with d alpha > 1); <= 0: automatic
 *  L_k, alpha_k optional [n_terms*d] per-term, per-coordinate values (alpha_k signed),
 *               overriding L / alpha when non-NULL (n_terms = d, or 1 when d = 1)
 *  tol          stop when the relative price change over a half sweep is <= tol
 *  rank_tol     relative pivot threshold for rank truncation; <= 0 means 0.1 tol / sqrt(d-1)
 *  max_rank     TT rank cap (<= TTFP_MAX_RANK); n_enrich random columns are added per step
 *  max_sweeps   at most this many forward+backward sweeps
 *  seed         seeds the counter-based generator for index sets and enrichment
 *  n_err_samples random grid points of the sampled error estimate of Sec. IV.B (the relative
 *               1-norm error of the tensor trains against the integrand), shared among the
 *               option's terms: > 0 that many, 0 the paper's 50 000, < 0 none (err_est NaN).
 *               Term t of an option with n_terms terms gets ceil(n / n_terms) points; coordinate
 *               k of its point s is the grid index rand(seed_t, 7, s, k, N), where
 *               rand(q, a, b, c, n) = ((h >> 32) * n) >> 32 with h = f(f(f(q ^ a) ^ b) ^ c), f the
 *               SplitMix64 finaliser (Steele, Lea and Flood 2014: add 0x9E3779B97F4A7C15, then
 *               xor-shift-multiply by 0xBF58476D1CE4E5B9 (30), 0x94D049BB133111EB (27), xor-shift 31),
 *               and seed_t = seed * 0x100000001B3 + t * 0x9E3779B97F4A7C15 + 1 (mod 2^64)
 *  certify      0: TTFP_OK means the half-sweep criterion above was met with no rank cap hit.
 *               1: TTFP_OK also needs err_est * kappa <= tol. The price is a positively weighted
 *               sum of the integrand over the grid, so |price error| / |price| <= (sum |TT - A|)
 *               / (sum |A|) * kappa, and err_est estimates that ratio from the samples: the
 *               product is a sampled bound on the price's relative error. An option that fails
 *               it returns TTFP_ENOTCONV (needs n_err_samples >= 0).                         */
typedef struct {
    int32_t N;
    double L, alpha;
    const double *L_k, *alpha_k;
    double tol, rank_tol;
    int32_t max_rank, max_sweeps, n_enrich;
    uint64_t seed;
    int32_t n_err_samples;
    int32_t certify;
} ttfp_grid;

/* Per-option diagnostics. */
typedef struct {
    double imag_rel;       /* |Im price| / |Re price| */
    double kappa;          /* cancellation factor: estimated sum |integrand| / |price| */
    double last_change;    /* relative price change over the last half sweep */
    int64_t n_evals;       /* integrand evaluations (the paper's oracle calls) */
    int64_t maxvol_swaps;  /* row swaps made by maxvol after its starting rows */
    int32_t sweeps;        /* half sweeps performed */
    int32_t rank_capped;   /* 1 if some bond hit max_rank (a capped cross also stops once its
                              change stops halving over a full sweep) */
    int32_t converged;     /* 1 if the tolerance was met */
    int64_t maxvol_full_starts; /* maxvol starts taken by pivoting over all rows because the
                              block of largest-norm rows was numerically rank deficient */
    double err_est;        /* the convergence measure of Sec. IV.B on the final tensor trains:
                              sum_t s_t sum_p |TT_t(x_p) - A_t(x_p)| / sum_t s_t sum_p |A_t(x_p)|
                              over the sample points of every term t (A_t its integrand, s_t > 0 its
                              quadrature scale K e^{-rT} prod_k eta_k / 2 pi); NaN without samples */
    int64_t err_samples;   /* sample points behind err_est (over all terms) */
} ttfp_diag;

typedef struct ttfp_ctx ttfp_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t,
 * NULL = the null stream). *out receives the context; the library owns it. */
int ttfp_create(ttfp_ctx **out, int device, void *hip_stream);
int ttfp_destroy(ttfp_ctx *ctx);

/* Host-only: the per-term grid the pricer would use (Sec. III.D truncation and contour
 * shift, with the automatic rule when L/alpha are not given). Writes n_terms, and
 * L_out / alpha_out [n_terms*d] (may be NULL). Returns TTFP_EINVAL for invalid input.
 * Needs no device. */
int ttfp_plan(const ttfp_option *opt, const ttfp_grid *grid, int32_t *n_terms,
              double *L_out, double *alpha_out);

/* Price one option. ranks (nullable) receives n_terms*(d+1) bond ranks, term-major.
 * diag is nullable. */
int ttfp_price(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, double *price,
               int32_t *ranks, ttfp_diag *diag);

/* Price n options in one batched pass (all terms of all options advance together).
 * grids[i] gives option i's settings. prices[n] receives prices; delta / vega (nullable)
 * receive sum_i d_i values each (option-major): dV/dS0_j and dV/dsigma_j at the fixed grid,
 * from the adjoint of the contraction against the frozen tensor-train cores. status[n]
 * (nullable) receives each option's return code. Returns the worst code. */
int ttfp_price_batch(ttfp_ctx *ctx, int32_t n, const ttfp_option *opts, const ttfp_grid *grids,
                     double *prices, double *delta, double *vega, int32_t *status);

/* Diagnostics of option i of the last ttfp_price_batch call on this context (the same fields
 * ttfp_price fills). TTFP_EINVAL when there is no such option. */
int ttfp_batch_diag(ttfp_ctx *ctx, int32_t i, ttfp_diag *diag);

/* Allocation-free variant of ttfp_price_batch, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc). Same arguments, outputs and return
 * codes as ttfp_price_batch, computed by the same kernels; it calls no hipMalloc / hipFree and
 * creates no events or graphs (like ttfp_price_batch it synchronises its stream between half
 * sweeps, so it cannot itself be captured into a graph). Its whole device workspace
 * (work-item array, activity flags, Greeks moments and every item's buffers) lives in one
 * static device array of TTFP_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs
 * on holds until the process ends. The batch is priced as one chunk; a batch whose workspace
 * exceeds that size returns TTFP_EINVAL before any kernel is launched, with the sizes in
 * ttfp_last_error. Every call on a GPU shares that GPU's array and the array keeps the last
 * call's contents (each call initialises what it reads): calls that overlap on one GPU, from
 * any context or stream, race and must not be made. The context's own buffers are untouched;
 * ttfp_tt_values / ttfp_tt_export do not see the tensor trains of this call. Returns
 * TTFP_EDEVICE when the array's device address could not be obtained at ttfp_create. */
#define TTFP_NOALLOC_SCRATCH_BYTES (128u << 20)
int ttfp_price_batch_noalloc(ttfp_ctx *ctx, int32_t n, const ttfp_option *opts, const ttfp_grid *grids,
                             double *prices, double *delta, double *vega, int32_t *status);

/* The two-train variant of Sec. IV (Eq. braket): each term's integrand is the product of the
 * characteristic function of w and the payoff transform; instead of one cross of the product, one
 * cross approximates the characteristic function (rank cap grid->max_rank, the paper's D_phi) and
 * another the payoff transform (rank cap payoff_rank, the paper's D_v; 0 = grid->max_rank), on the
 * same grid, and the price is their exact inner product (no conjugation) computed in tensor-train
 * form, scaled and summed over the terms. In exact arithmetic this is the grid sum of Eq. discr.
 * ranks_cf / ranks_payoff (nullable) receive n_terms*(d+1) bond ranks of each kind of train.
 * Status: TTFP_OK when both crosses met the tolerance without a rank cap (each by the relative
 * change of its own grid sum), else TTFP_ENOTCONV; TTFP_EPRECISION when the product's
 * cancellation factor kappa times the FP64 unit roundoff exceeds tol. diag (nullable): kappa of
 * the product, err_est the larger of the two trains' sampled errors, evaluations of both. */
int ttfp_price_two_trains(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t payoff_rank,
                          double *price, int32_t *ranks_cf, int32_t *ranks_payoff, ttfp_diag *diag);

/* Prices of one option at a ladder of market points that share its volatilities, correlation,
 * maturity and payoff: point p has spots S0_points[p*d .. p*d+d), strike K_points[p] and rate
 * r_points[p] (host arrays, n_points >= 1, at most TTFP_MAX_LADDER). One TT-cross builds the
 * integrand of the base option opt on its grid (the automatic rule of opt, or the given L/alpha),
 * which every point uses. A point's integrand differs from the base one only through the mean
 * of w: by exp(-i zeta . dm) with dm = m_w(point) - m_w(base), a product over the coordinates, so
 * its price is the contraction of the base tensor trains with one weight vector per coordinate
 * (Sec. IV.A contraction, the quadrature weights times exp(-i zeta_k dm_k)) times
 * K_p e^{-r_p T} / (K e^{-r T}). For each core the per-point contractions over the nodes form
 * one dense complex product (points x nodes by nodes x r_{k-1} r_k) on the FP64 matrix cores.
 * prices[n_points] (host) receives the prices; diag (nullable) the base cross's diagnostics.
 * Returns the base cross's status (TTFP_OK, TTFP_ENOTCONV, TTFP_EPRECISION: the same warning holds
 * for every point, whose accuracy is that of the base tensor trains scaled by |exp(alpha . dm)|);
 * TTFP_EINVAL for an invalid option, point or grid (no prices written). */
#define TTFP_MAX_LADDER 65536
int ttfp_price_ladder(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t n_points,
                      const double *S0_points, const double *K_points, const double *r_points, double *prices,
                      ttfp_diag *diag);

/* The integrand of term `term` of an option at npts grid multi-indices idx[npts*d]
 * (host, 0-based), evaluated by the GPU fiber kernel's device function. out[2*npts]
 * receives interleaved real/imaginary parts. */
int ttfp_eval_integrand(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t term,
                        int64_t npts, const int32_t *idx, double *out);

/* After the last ttfp_price on this context: the tensor train of term `term` evaluated at
 * npts multi-indices idx[npts*d] (host). out[2*npts] interleaved complex. */
int ttfp_tt_values(ttfp_ctx *ctx, int32_t term, int64_t npts, const int32_t *idx, double *out);

/* After the last ttfp_price on this context: the tensor train of term `term` (Sec. IV.A)
 * and the index sets its cross ended with (Sec. IV.B). Host buffers, owned by the caller:
 *   ranks[d+1]            bond ranks r_0 = 1, r_1, ..., r_d = 1
 *   cores (nullable)      the d cores one after another, core k as r_k x N x r_{k+1} complex
 *                         values (interleaved re/im) in index order [a][i][b]
 *   set_sizes (nullable)  [2(d+1)]: sizes of the left sets I_0..I_d, then of the right sets J_0..J_d
 *   left, right (nullable) [(d+1) x max_rank x d]: entry (k, a, c) holds coordinate c of the a-th
 *                         multi-index of I_k (c < k) or of J_k (c >= k); other entries are unused.
 * TTFP_EINVAL without a previous ttfp_price or for a term out of range. */
int ttfp_tt_export(ttfp_ctx *ctx, int32_t term, int32_t *ranks, double *cores, int32_t *set_sizes, int32_t *left,
                   int32_t *right);

/* Kernel-level entry points (same kernels as the pricer, exposed for verification).
 * ttfp_qr_r: upper-triangular factor R (n x n, row-major, interleaved complex) of a QR of
 * the m x n complex matrix A (row-major, interleaved), by the TSQR kernels; n <= 68.
 * ttfp_maxvol: rows[r] of a dominant r x r submatrix of the m x r complex matrix A and
 * B = A A[rows]^{-1} (m x r), by the maxvol kernel. All pointers host. */
int ttfp_qr_r(ttfp_ctx *ctx, int32_t m, int32_t n, const double *A, double *R);
int ttfp_maxvol(ttfp_ctx *ctx, int32_t m, int32_t r, const double *A, double delta, int32_t *rows,
                double *B);

/* Launch tuning of a context (chosen per workload shape by the autotuner in
 * paper_2203_02804_amd/tuning.py):
 *  TTFP_TUNE_MAXVOL_ROUNDS   refinement rounds of maxvol after its block start, 0..8 (default
 *                            3): each round swaps the rows of B beyond the dominance bound into
 *                            a new block and forms B again; more rounds give interpolation
 *                            nearer to dominant (and may change the result), at the cost of one
 *                            pass over B per round that moves a pivot
 *  TTFP_TUNE_TSQR_LDS_KB     LDS budget of a TSQR workgroup in KiB, 16..152 (default 152):
 *                            smaller budgets give shorter leaf blocks and merges of fewer
 *                            factors (a leaf keeps at least two groups of nc rows and a merge
 *                            at least two factors, whatever the budget)
 *  TTFP_TUNE_GRAPH           1 (default): capture each direction's half sweep (its kernels and
 *                            the on-device convergence test) in a hipGraph once per batch and
 *                            replay it, when the context's stream is not the null stream and
 *                            kernel timing is off; 0: launch eagerly. Either way the host only
 *                            reads one flag per half sweep, one half sweep behind the device
 *  TTFP_TUNE_QR              the fiber's triangular factor: shifted Cholesky QR with the Gram
 *                            and transform products on the FP64 matrix cores, 0 (default) with
 *                            two passes when every item's relative rank threshold is at least
 *                            1e-10 and three otherwise, 2 always two passes (singular values
 *                            resolved down to about 1e-12 of the largest, to 1e-5 relative above
 *                            1e-10), 3 always three (down to about 1e-16; ttfp_qr_r uses three
 *                            unless 2 is set); 1 Householder TSQR over LDS-resident row blocks
 *  TTFP_TUNE_MAXVOL_WARM     1 (default): from the second half sweep in a direction on, maxvol
 *                            starts from the pivots that the previous half sweep in that
 *                            direction chose at the same core (their multi-indices mapped onto
 *                            the current fiber's rows), when all r of them map and their block
 *                            is not near-singular, instead of eliminating on its candidate
 *                            block; 0: always the elimination start. Either start is followed
 *                            by the same swaps and refinement to dominance; the pivots found
 *                            (and so the result) may differ
 *  TTFP_TUNE_MM_WAVES        8 (default) or 16: 16-row panels per workgroup of the basis and
 *                            interpolation products on the matrix cores; the results are the same
 *                            bit for bit (a row's product does not depend on its workgroup)
 *  TTFP_TUNE_GRAM_THREADS    512 (default) or 1024 threads per workgroup of the Cholesky QR's Gram
 *                            products (two 16 x 16 tiles per wave or one); the same results bit
 *                            for bit (each tile sums the same rows in the same order)
 *  TTFP_TUNE_MM_PANELS       1 (default) or 2: 16-row panels per wave of the basis and
 *                            interpolation products (rows per workgroup = 16 x waves x panels);
 *                            the same results bit for bit
 *  TTFP_TUNE_INTERP_BOUND    1 (default): the checking passes of the interpolation matrix skip the
 *                            rows that cannot exceed the dominance bound, |B_ij|^2 <= |y_i|^2
 *                            max_j |A^-1 e_j|^2; 0: every row is formed. The same results bit for
 *                            bit (a skipped row could not have been marked)
 * Returns TTFP_EINVAL for an unknown parameter or value. */
enum { TTFP_TUNE_MAXVOL_ROUNDS = 0, TTFP_TUNE_TSQR_LDS_KB = 1, TTFP_TUNE_GRAPH = 2, TTFP_TUNE_QR = 3,
       TTFP_TUNE_MAXVOL_WARM = 4, TTFP_TUNE_MM_WAVES = 5, TTFP_TUNE_GRAM_THREADS = 6, TTFP_TUNE_MM_PANELS = 7,
       TTFP_TUNE_INTERP_BOUND = 8 };
int ttfp_set_tuning(ttfp_ctx *ctx, int param, int value);
int ttfp_get_tuning(ttfp_ctx *ctx, int param, int *value);

/* Kernel timing: when enabled, HIP events recorded on the context's stream bracket every
 * launch of each kernel family; ttfp_profile_read returns the number of launches, their
 * summed device time and the algorithmic work they did since the last enable (bytes written
 * for the fiber kernel: 16 per complex entry; FP64 flops for TSQR (8 m n^2 - 8 n^3 / 3), the
 * Cholesky QR's Gram products (4 m n^2 per pass: the Hermitian half of X^H X, m fiber rows,
 * n columns) and triangular transforms (4 m n^2 per pass: X R^{-1} with R^{-1} triangular),
 * basis (4 m r^2), maxvol on its candidate block of K rows (8 K r^2 for the block, 8 (K + r) r
 * per swap for the rank-one updates of the block and of A^{-1}, 8 r^3 per Gauss-Jordan inverse;
 * its refinement rounds on blocks of the pivots and violating rows are a family of their own)
 * and the interpolation matrix (8 m r^2), the ladder's per-point node contractions (8 S N r_{k-1} r_k
 * per core for S points); 0 where not counted). */
enum {
    TTFP_KERNEL_FIBER = 0, TTFP_KERNEL_TSQR = 1, TTFP_KERNEL_QRCP = 2, TTFP_KERNEL_BASIS = 3,
    TTFP_KERNEL_MAXVOL = 4, TTFP_KERNEL_FINISH = 5, TTFP_KERNEL_CORESUM = 6, TTFP_KERNEL_CONTRACT = 7,
    TTFP_KERNEL_INTERP = 8, TTFP_KERNEL_ERREST = 9, TTFP_KERNEL_GRAM = 10, TTFP_KERNEL_CHOL = 11,
    TTFP_KERNEL_XFORM = 12, TTFP_KERNEL_LADDER = 13, TTFP_KERNEL_REFINE = 14, TTFP_KERNEL_COUNT = 15
};
int ttfp_profile_enable(ttfp_ctx *ctx, int enable);
int ttfp_profile_read(ttfp_ctx *ctx, int kernel, int64_t *launches, double *total_ms, double *work);

/* ---------------------------------------------------------------------------------------
 * Price surrogate (an addition to the paper's method): an ensemble of n_models MLPs
 * n_in -> width (x depth, SiLU) -> 1 with BF16 weights and activations, FP32 accumulation
 * (MFMA), FP32 master weights and Adam, trained on prices produced by the TT path.
 * Parameters of one model, as a flat FP32 vector: for each layer l (depth hidden layers then
 * the head) W_l [out x in] row-major, then b_l [out].
 * x_dev / t_dev / y_dev are device pointers (FP32): x [batch x n_in] row-major, t and y
 * [batch]. The context owns its weights and activation buffers (sized for max_batch) and
 * enqueues on `stream`; calls on one context must not overlap.
 * ------------------------------------------------------------------------------------- */
typedef struct ttfp_mlp ttfp_mlp;
int ttfp_mlp_create(ttfp_mlp **out, int device, void *stream, int n_in, int width, int depth,
                    int n_models, int max_batch, uint64_t seed);
int ttfp_mlp_destroy(ttfp_mlp *m);
int ttfp_mlp_n_params(const ttfp_mlp *m, int64_t *n);
int ttfp_mlp_get_params(ttfp_mlp *m, int model, float *params);          /* host out */
int ttfp_mlp_set_params(ttfp_mlp *m, int model, const float *params);    /* host in; resets Adam */
/* y_dev[batch] = network(x_dev) for one model */
int ttfp_mlp_forward(ttfp_mlp *m, int model, int batch, const float *x_dev, float *y_dev);
/* gradient (host, n_params, nullable) and loss (host, nullable) of the mean squared error */
int ttfp_mlp_grad(ttfp_mlp *m, int model, int batch, const float *x_dev, const float *t_dev,
                  float *grad, float *loss);
/* one Adam step (beta 0.9 / 0.999) on the mean squared error; loss (host, nullable) before the step */
int ttfp_mlp_train_step(ttfp_mlp *m, int model, int batch, const float *x_dev, const float *t_dev,
                        float lr, float *loss);
/* Ensemble inference in one fused kernel (all layers of every model, activations in LDS) with
 * the gate on the device: for row b, price_m = cv_dev[b] + scale_dev[b] * y_m(x_b); mean_dev[b]
 * and spread_dev[b] receive the ensemble mean and standard deviation (ddof 1) of price_m, and
 * ok_dev[b] = (factor * spread <= gate * |mean|). All arrays are device arrays of `batch`
 * entries (x_dev: batch x n_in, FP32). Needs width <= 256, a multiple of 32. Asynchronous on the
 * model's stream; batch is not limited by max_batch. */
int ttfp_mlp_predict(ttfp_mlp *m, int batch, const float *x_dev, const float *cv_dev, const float *scale_dev,
                     float factor, float gate, float *mean_dev, float *spread_dev, int32_t *ok_dev);
/* The surrogate's control variate for the call on the maximum, max_j of the single-asset
 * Black-Scholes calls (Sec. II, Eq. BSexact), on the device: S0_dev, sigma_dev batch x d
 * row-major, K_dev, T_dev, r_dev [batch]; cv_dev [batch] receives it. */
int ttfp_mlp_control_variate(ttfp_mlp *m, int batch, int d, const float *S0_dev, const float *sigma_dev,
                             const float *K_dev, const float *T_dev, const float *r_dev, float *cv_dev);
const char *ttfp_mlp_last_error(const ttfp_mlp *m);

const char *ttfp_strerror(int code);
const char *ttfp_last_error(const ttfp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
