/*
 * ircur.h -- C ABI of libircur, IRCUR (Iterated Robust CUR) for robust PCA on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Cai, Hamm, Huang, Li, Wang, "Rapid Robust Principal Component
 * Analysis: CUR Accelerated Inexact Low Rank Estimation" (arXiv 2010.07422).
 * Given D = L + S (rank(L) <= r, S sparse; problem (1)), Algorithm 1 alternates
 *   Phase I  (section 3.2): [S_{k+1}] = T_zeta[D - L_k] on sampled rows I and
 *            columns J, with the hard threshold T_zeta of eq. (4) and the
 *            sampled low-rank estimate of eq. (5);
 *   Phase II (section 3.1): C = [D-S]_{:,J}, U = H_r([D-S]_{I,J}),
 *            R = [D-S]_{I,:} (eq. (2)) and L_{k+1} = C U^+ R (eq. (3)),
 * until the sampled residual e_k of eq. (6) is <= eps.  L is never formed:
 * the library keeps L_k = A_k B_k with A_k = C V_r Sigma_r^+ (n1 x r) and
 * B_k = W_r^T R (r x n2), where U = W_r Sigma_r V_r^T.
 *
 * Conventions
 *   - All functions are extern "C", return an int status (ircur_status), never
 *     throw, and validate every argument on the host before touching the GPU;
 *     an invalid argument returns IRCUR_ERR_ARG with no side effects.
 *   - "dev" pointers are HIP device pointers on the context's device; "host"
 *     pointers are ordinary host memory.  Matrices are row-major.
 *   - D (and its transpose, if given) is BORROWED: caller-owned device memory
 *     that must stay valid and unchanged until ircur_destroy.  The context and
 *     its workspace are owned by the library.
 *   - Work is enqueued on the stream given to ircur_init (a hipStream_t; NULL
 *     is the null stream).  Functions that return host values synchronise
 *     that stream; those that only fill device buffers do not.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Factor dtype: double when dtype == IRCUR_F64, float otherwise.
 */
#ifndef IRCUR_H
#define IRCUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ircur_ctx ircur_ctx;

enum ircur_status {
    IRCUR_OK = 0,
    IRCUR_NOT_CONVERGED = 1,        /* max_iter reached with e > eps (result valid) */
    IRCUR_WARN_RANK_DEFICIENT = 2,  /* a kept-rank test dropped components of U^+ */
    IRCUR_WARN_SVD_INEXACT = 3,     /* top-r SVD hit its iteration cap (sigma_r ~ sigma_{r+1}) */
    IRCUR_ERR_ARG = -1,
    IRCUR_ERR_ALLOC = -2,
    IRCUR_ERR_DEVICE = -3,          /* HIP error, or no usable device */
    IRCUR_ERR_SVD = -4,
    IRCUR_ERR_NONFINITE = -5,       /* NaN/Inf met in D or in the iterates */
    IRCUR_ERR_STATE = -6,           /* call not valid in the current state */
    IRCUR_ERR_UNSUPPORTED = -7      /* sizes beyond a documented kernel limit */
};

enum ircur_dtype { IRCUR_F64 = 0, IRCUR_F32 = 1, IRCUR_BF16 = 2 };

/* Largest supported rank r (the factor kernels are compiled for padded ranks). */
#define IRCUR_MAX_RANK 32

/*
 * Parameters of Algorithm 1 (its inputs: D, r, eps, zeta_0, gamma, |I|, |J|)
 * plus the implementation choices the paper leaves open.
 */
typedef struct {
    int64_t n1, n2;      /* D is n1 x n2 (n1, n2 >= 1)                              */
    int64_t ldD;         /* row stride of D in elements, ldD >= n2                  */
    int32_t r;           /* target rank, 1 <= r <= min(sI, sJ, IRCUR_MAX_RANK)      */
    int32_t sI, sJ;      /* |I| <= n1, |J| <= n2 (section 3.5: c r log n)            */
    int32_t dtype;       /* ircur_dtype of D: F64 computes in double; F32 and BF16
                            compute in float; the SVD of U is always double        */
    int32_t resample;    /* 1: IRCUR-R (new I, J every iteration), 0: IRCUR-F (3.4) */
    int32_t err_mode;    /* 0: e_k of eq. (6) read literally, with L_{k+1}, S_{k+1}
                            on the iteration's own I, J; 1: the below-threshold part
                            of D - L_k on the new I, J                            */
    double  zeta0;       /* initial threshold zeta_0 > 0 (0 allowed: removes all)  */
    double  gamma;       /* decay, zeta_{k+1} = gamma^k zeta_0, 0 < gamma <= 1      */
    double  eps;         /* stop when e_k <= eps (eps < 0: run max_iter iterations) */
    int32_t max_iter;    /* iteration cap, >= 1                                     */
    uint64_t seed;       /* index-sampler seed (SplitMix64 stream, see below)       */
    double  svd_tol;     /* residual tolerance of the top-r SVD (relative to the
                            smallest wanted Rayleigh quotient in the one-launch
                            SVD, to ||Q^T M^T M Q||_F in the general one); 0: default
                            (1e-13 for F64, 1e-9 for F32; for BF16
                            max(1e-7, 1e-2 e_k), e_k the stopping residual of the
                            iteration before, e_0 = 1)                              */
    int32_t svd_max_it;  /* cap on the products with M^T M of one top-r SVD; 0: the
                            default, 256 in the one-launch SVD (r <= 16), 64
                            subspace iterations in the general one              */
    int32_t svd_block;   /* least subspace width of the top-r SVD (r <= svd_block
                            <= 32); the width used is 16 or 32, the smaller one
                            at least max(svd_block, padded r); 0: from r alone.
                            Width 32 takes the general multi-launch SVD        */
    const double* zeta_sched; /* optional host array of max_iter thresholds (Algorithm
                            1, Phase I: any decreasing schedule zeta_{k+1}):
                            iteration k (0-based) thresholds with zeta_sched[k] in
                            place of gamma^k zeta_0; NULL: the geometric schedule.
                            Copied by ircur_init (the caller keeps ownership);
                            every entry finite and >= 0, else IRCUR_ERR_ARG.
                            Past the last iteration (ircur_sparse_full with
                            zeta < 0 after max_iter iterations) the last entry. */
} ircur_params;

/* Fill *p with defaults (gamma 0.7, eps 1e-5, max_iter 100, resample 1,
 * err_mode 0, dtype F64, everything else 0).  Sizes must still be set. */
int ircur_params_default(ircur_params* p);

/*
 * Create a context for D (device, dtype p->dtype, n1 x n2, row stride p->ldD).
 * Dt: optional device copy of D^T (n2 x n1, row stride ldDt >= n1, same dtype);
 * if NULL the library builds one (a transpose kernel; n1*n2 elements of
 * workspace).  The context starts at k = 0 with L_0 = S_0 = 0 (Algorithm 1).
 * stream: hipStream_t to enqueue on, or NULL.
 * Errors: IRCUR_ERR_ARG (any invalid size, pointer or parameter),
 * IRCUR_ERR_UNSUPPORTED (sizes beyond a kernel limit), IRCUR_ERR_DEVICE,
 * IRCUR_ERR_ALLOC.  On error *out is set to NULL.
 */
int ircur_init(ircur_ctx** out, const ircur_params* p, const void* D_dev,
               const void* Dt_dev, int64_t ldDt, void* stream);

/*
 * One iteration k -> k+1 of Algorithm 1 (Phase I, Phase II, e_{k+1}).
 * I_host, J_host: optional host arrays of sI / sJ distinct indices (any
 * order; they are sorted internally); if NULL the library's sampler draws
 * them (stream 0 for IRCUR-F, stream k for IRCUR-R).  Synchronises and writes
 * e_{k+1} to *e_out (may be NULL).  Returns IRCUR_ERR_STATE if the context has
 * already stopped (e <= eps or max_iter reached) unless ircur_reset was called.
 */
int ircur_step(ircur_ctx* ctx, const int32_t* I_host, const int32_t* J_host,
               double* e_out);

/*
 * Enqueue up to n_iter iterations with sampled index sets, without waiting.
 * A device-side stop flag turns the remaining launches into no-ops once
 * e <= eps or k = max_iter.  Use ircur_sync to read the outcome.
 */
int ircur_enqueue(ircur_ctx* ctx, int32_t n_iter);

/* Wait for enqueued work; report iterations done so far and the last e. */
int ircur_sync(ircur_ctx* ctx, int32_t* k_out, double* e_out);

/*
 * Run Algorithm 1 to the stop rule (e_k <= eps) or max_iter.  Writes the
 * number of iterations and the last e.  Returns IRCUR_OK or
 * IRCUR_NOT_CONVERGED (both with a valid result), or an error.  Iterations
 * are enqueued in chunks, two in flight; iterations enqueued past the
 * device-side stop return at once and change nothing.  Synchronises (returns
 * once every enqueued launch has finished).
 */
int ircur_solve(ircur_ctx* ctx, int32_t* iters_out, double* e_out);

/* Forget the stop state and restart from L_0 = 0, k = 0 (same D, params). */
int ircur_reset(ircur_ctx* ctx);

/*
 * Copy the current factors (L_k = A_k B_k): At_dev receives A_k^T (r x n1),
 * B_dev receives B_k (r x n2), both row-major in the factor dtype.  Either
 * pointer may be NULL.  Asynchronous on the context's stream.
 */
int ircur_get_factors(ircur_ctx* ctx, void* At_dev, void* B_dev);

/* Overwrite the factors (same layouts) and the iteration counter k. */
int ircur_set_factors(ircur_ctx* ctx, const void* At_dev, const void* B_dev,
                      int32_t k);

/* e_1 .. e_k of the run so far (host); *n_out = min(k, cap). Synchronises. */
int ircur_get_history(ircur_ctx* ctx, double* e_host, int32_t cap,
                      int32_t* n_out);

/* Index sets of the last completed iteration (host, sorted). Synchronises. */
int ircur_get_sets(ircur_ctx* ctx, int32_t* I_host, int32_t* J_host);

/*
 * Internals of the last completed iteration, for verification (device), all
 * double: M_dev = [D - S_k]_{I,J} (sI x sJ); Wt_dev (sI x r) and Q_dev
 * (sJ x r), orthonormal bases of the top-r left and right singular subspaces
 * of M; Kc_dev (r x r) with H_r(M) = Wt Kc Q^T, so the singular values of
 * H_r(M) are those of Kc (section 3.1).  Dropped components are zero.  Any
 * pointer may be NULL.  Asynchronous.
 */
int ircur_get_core(ircur_ctx* ctx, double* M_dev, double* Wt_dev,
                   double* Kc_dev, double* Q_dev);

/*
 * Output of Algorithm 1 (its C_k, U_k^+, R_k, eq. (2)-(3)) for the last
 * completed iteration k, recomputed from that iteration's input factors
 * (A_{k-1}, B_{k-1}), index sets (ircur_get_sets) and threshold zeta_k, with
 * the same arithmetic the iteration used (so the blocks are bitwise those it
 * used):  C_dev (n1 x sJ) = [D - S_k]_{:,J},  R_dev (sI x n2) = [D - S_k]_{I,:},
 * Upinv_dev (sJ x sI) = U_k^+ = V_r Sigma_r^+ W_r^T (so L_k = C U^+ R), and the
 * sparse blocks SI_dev = [S_k]_{I,:} (sI x n2), SJ_dev = [S_k]_{:,J} (n1 x sJ)
 * of Phase I (eq. (4)).  All row-major, factor dtype, device; any pointer may
 * be NULL.  Returns IRCUR_ERR_STATE if no iteration has completed since
 * ircur_init, ircur_reset, ircur_set_factors or ircur_set_state.  Synchronises.
 */
int ircur_get_cur(ircur_ctx* ctx, void* C_dev, void* Upinv_dev, void* R_dev,
                  void* SI_dev, void* SJ_dev);

/*
 * Algorithm 2 (CUR to SVD) applied to the current estimate in factored form,
 * L_k = A_k I_r B_k: QR of A_k and of B_k^T (Cholesky QR, twice, in FP64),
 * SVD of the r x r product of the triangular factors (one-sided Jacobi),
 * then W = Q_A U_M, V = Q_B V_M.  Outputs (device, double, row-major):
 * W_dev (n1 x r), sigma_dev (r, descending), V_dev (n2 x r), with
 * L_k = W diag(sigma) V^T; columns beyond the numerical rank of L_k are zero.
 * Any pointer may be NULL.  Synchronises.
 */
int ircur_to_svd(ircur_ctx* ctx, double* W_dev, double* sigma_dev, double* V_dev);

/*
 * ircur_to_svd for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same outputs, bit for bit, but the workspace
 * (Gram partials and the small maps) is a fixed array inside the library,
 * one per device, 4.03 MiB (enough for r <= IRCUR_MAX_RANK and any n1, n2),
 * set up by ircur_init; nothing is allocated or freed.  Calls on one device
 * share that array: calls that overlap on one device (other host threads,
 * other streams) race and must be serialised by the caller.  Every entry of
 * the workspace a call reads is written earlier in the same call, so nothing
 * carries over between calls.  IRCUR_ERR_UNSUPPORTED if the workspace would
 * exceed the array, IRCUR_ERR_STATE if ircur_init could not set it up on the
 * context's device.  Synchronises.
 */
int ircur_to_svd_noalloc(ircur_ctx* ctx, double* W_dev, double* sigma_dev, double* V_dev);

/*
 * Full sparse part S = T_zeta(D - A_k B_k) over all of D (the hard threshold
 * of eq. (4) applied to every entry; the foreground of the video application
 * of section 4.2), written to S_dev (n1 x n2, row stride ldS >= n2, dtype of D,
 * device).  zeta < 0 selects zeta_{k+1} = gamma^k zeta_0, the threshold the
 * next iteration would apply to D - L_k; zeta >= 0 is used as given.  The
 * number of nonzeros goes to *nnz_out (may be NULL; synchronises if not).
 */
int ircur_sparse_full(ircur_ctx* ctx, double zeta, void* S_dev, int64_t ldS,
                      int64_t* nnz_out);

/*
 * Checkpoint / resume.  The state is (k, stop flag, A_k, B_k, e history):
 * ircur_get_state with buf == NULL writes the required size to *bytes.
 * Resuming gives the same trajectory bit for bit.  Host buffers; synchronises.
 */
int ircur_get_state(ircur_ctx* ctx, void* buf, size_t* bytes);
int ircur_set_state(ircur_ctx* ctx, const void* buf, size_t bytes);

/* ---- Measurement entry points --------------------------------------------
 * The calls from here to ircur_time_sparse, and ircur_get_phase_profile(2)
 * below, are tooling for benchmarks and profiles: they compute nothing of
 * Algorithm 1 and leave the run's state as it was.  A solver needs none of
 * them. */

/*
 * Per-kernel timing with HIP events on the context's stream (for the
 * benchmark).  When enabled, every iteration records events around its
 * kernels; ircur_get_timing returns the accumulated milliseconds of the
 * core, svd, pass and finalize kernels and the number of timed iterations.
 */
int ircur_set_timing(ircur_ctx* ctx, int32_t enable);
int ircur_get_timing(ircur_ctx* ctx, double* ms4, int64_t* count);

/*
 * Duration of the fused row/column pass (Algorithm 1, Phase II: the products
 * of eq. (3) on the sampled rows and columns with the threshold of eq. (4)
 * applied in the same pass) measured with HIP events on the context's stream:
 * the pass of the last finished iteration k-1 is launched `reps` times back to
 * back between two events and the mean per launch, in microseconds, is
 * written to *us_out.  Each launch reads A_{k-1}, B_{k-1}, the iteration's
 * index sets and the svd's per-row data, all still in place, and rewrites
 * A_k, B_k and the stopping-test partial sums with the same values, so the
 * state is unchanged.  ERR_STATE if no iteration has finished since
 * init/reset/set_factors/set_state or the run has stopped; ERR_ARG for
 * reps < 1.  Synchronises.
 */
int ircur_time_pass(ircur_ctx* ctx, int32_t reps, double* us_out);

/*
 * Duration of the full sparse-part extraction of ircur_sparse_full (the
 * threshold of eq. (4) over all of D - A_k B_k, section 4.2's foreground)
 * measured with HIP events on the context's stream: the extraction into S_dev
 * (caller-owned device memory, n1 x n2 in D's storage type, leading
 * dimension ldS >= n2) is launched `reps` times back to back, without the
 * nonzero count, and the mean per launch in microseconds goes to *us_out.
 * zeta < 0 picks gamma^k zeta_0 as ircur_sparse_full does.  ERR_ARG for a
 * NULL pointer, ldS < n2, a NaN zeta or reps < 1.  Synchronises.
 */
int ircur_time_sparse(ircur_ctx* ctx, double zeta, void* S_dev, int64_t ldS, int32_t reps,
                      double* us_out);

/* Diagnostics of the last iteration: svd iterations, svd residual, the
 * estimated gap sigma_{r+1}/sigma_r, kept rank.  Synchronises. */
int ircur_get_info(ircur_ctx* ctx, int32_t* svd_iters, double* svd_resid,
                   double* gap, int32_t* kept);

/*
 * Per-iteration record of the top-r SVD of the core (section 3.1), for the
 * iterations completed since ircur_init, ircur_reset, ircur_set_factors or
 * ircur_set_state (entry i is iteration k_0 + i + 1): subspace iterations
 * used, the Ritz estimate of sigma_{r+1} / sigma_r (the gap that decides
 * whether H_r is unique; a lower bound once the wanted columns have
 * converged, from the extra columns' largest Rayleigh quotient; -1 when the
 * subspace block holds no column beyond r)
 * and the number of components kept by the pseudo-inverse rule.  Host arrays
 * of `cap` entries, any of them NULL; *n_out = entries written.
 * Synchronises.
 */
int ircur_get_svd_history(ircur_ctx* ctx, int32_t* iters_host, double* gap_host,
                          int32_t* kept_host, int32_t cap, int32_t* n_out);

/*
 * The sampler, on the host (no device needed): index sets of stream t.
 * Generator: SplitMix64 (Steele, Lea, Flood 2014) started from
 * mix(seed xor ((t+1) * 0xD1B54A32D192ED03)); bounded draws by 128-bit
 * multiply-shift; distinct sets by Floyd's algorithm; I drawn before J;
 * both sorted ascending.  IRCUR-F uses t = 0, IRCUR-R uses t = k at
 * iteration k+1.
 */
int ircur_sample(uint64_t seed, int64_t t, int64_t n1, int64_t n2, int32_t sI,
                 int32_t sJ, int32_t* I_host, int32_t* J_host);

/*
 * (Tooling.)  Accumulated phase times (microseconds) of the SVD kernel's
 * first workgroup, 16 slots, for builds compiled with IRCUR_PHASE_PROFILE
 * (zeros otherwise).  Synchronises.
 */
int ircur_get_phase_profile(ircur_ctx* ctx, double* us16);
/* Profile builds: the same timers for a second launch of the one-launch SVD
 * issued straight after the first with the same inputs (zeros otherwise). */
int ircur_get_phase_profile2(ircur_ctx* ctx, double* us16);

void        ircur_destroy(ircur_ctx* ctx);
const char* ircur_strerror(int status);
const char* ircur_last_error(const ircur_ctx* ctx);

/* ------------------------------------------------------------------------
 * Unrolled, differentiable mode.
 *
 * The paper's iteration uses the hard threshold of eq. (4) with the schedule
 * zeta_{k+1} = gamma^k zeta_0 (Algorithm 1).  This mode runs K iterations of
 * Algorithm 1 (resampled index sets, IRCUR-R) on a batch of independent
 * instances with one threshold zeta_k per iteration, shared by the batch,
 * and the gated sparse part S = x g, g = sigmoid((|x| - zeta_k) / (tau_rel
 * zeta_k)) in place of T_zeta (tau_rel = 0 is eq. (4) exactly).  Per instance
 *     loss_b = ||A_K B_K - W* V*^T||_F / ||W* V*^T||_F
 * against a target L* = W* V*^T.  ircur_backward returns d(sum_b w_b loss_b)
 * / d zeta_k through the factor products, the gate and the rank-r
 * pseudo-inverse of the core (first-order perturbation of the truncated SVD,
 * which needs sigma_r > sigma_{r+1}); the gathered rows and columns of D are
 * recomputed, not stored.
 * ---------------------------------------------------------------------- */
typedef struct ircur_unrolled ircur_unrolled;

typedef struct {
    int64_t n1, n2, ldD;   /* D: n1 x n2, row stride ldD >= n2                   */
    int32_t sI, sJ;        /* |I|, |J|: r <= sI <= min(n1, 176), r <= sJ <= min(n2, 176) */
    const void* D;         /* device, dtype of the batch; borrowed                 */
    const void* Dt;        /* optional device D^T (n2 x n1, row stride ldDt), or NULL */
    int64_t ldDt;
    const void* Wstar;     /* device, n1 x r, row-major, factor dtype: target W*   */
    const void* Vstar;     /* device, n2 x r: target V* (L* = W* V*^T)             */
    uint64_t seed;         /* sampler seed; step k uses stream k (see ircur_sample) */
} ircur_instance;

/*
 * Create a batch: nb instances, rank r (1..16), K steps, dtype IRCUR_F64 or
 * IRCUR_F32 (factors in the same type, the core SVD and its adjoint in
 * double), gate width tau_rel >= 0.  Draws and uploads every index set,
 * builds D^T where not given and allocates the tape.  Synchronises.
 * Errors: IRCUR_ERR_ARG, IRCUR_ERR_UNSUPPORTED (sizes beyond the limits
 * above), IRCUR_ERR_ALLOC, IRCUR_ERR_DEVICE.  On error *out is NULL.
 */
int ircur_unrolled_create(ircur_unrolled** out, const ircur_instance* inst, int32_t nb,
                          int32_t r, int32_t K, int32_t dtype, double tau_rel, void* stream);

/*
 * Forward pass from L_0 = 0 with thresholds zeta_dev[0..K-1] (device,
 * double; an FP32 parameter converts exactly).  Writes loss_b to loss_dev[b]
 * (device, nb doubles; may be NULL).  Asynchronous.
 */
int ircur_unrolled_forward(ircur_unrolled* u, const double* zeta_dev, double* loss_dev);

/*
 * Reverse sweep of the last forward pass: dzeta_dev[k] (device, K doubles)
 * = sum_b w_b d loss_b / d zeta_k with w = dloss_dev (device, nb doubles; NULL
 * means all ones).  Asynchronous.  IRCUR_ERR_STATE without a forward pass.
 */
int ircur_backward(ircur_unrolled* u, const double* dloss_dev, double* dzeta_dev);

/* Factors of instance b after step k (0..K): A_k^T (r x n1), B_k (r x n2). */
int ircur_unrolled_get_factors(ircur_unrolled* u, int32_t b, int32_t k, void* At_dev, void* B_dev);

/* Index sets of instance b at step k (host, sorted). */
int ircur_unrolled_get_sets(ircur_unrolled* u, int32_t b, int32_t k, int32_t* I_host, int32_t* J_host);

/*
 * Per-instance flags of the last passes (host, nb values): 1 a resolvent
 * solve of the backward stopped at its cap, 2 sigma_r ~ 0 in some core,
 * 4 an SVD hit its iteration cap, 8 the pinv rule dropped a component,
 * 16 SVD failure.  Synchronises.  Returns IRCUR_ERR_SVD if any has 16.
 */
int ircur_unrolled_status(ircur_unrolled* u, int32_t* flags_host);

void        ircur_unrolled_destroy(ircur_unrolled* u);
const char* ircur_unrolled_last_error(const ircur_unrolled* u);

#ifdef __cplusplus
}
#endif
#endif /* IRCUR_H */
