/*
 * bpmf.h -- C ABI of the MI355X (gfx950) BPMF Gibbs-sweep library.
 *
 * The method is the Gibbs sampler of Bayesian Probabilistic Matrix
 * Factorization as laid out in Vander Aa, Chakroun & Haber, "Distributed
 * Bayesian Probabilistic Matrix Factorization" (2017):
 *   - Sec. I: a sparse rating matrix R (M x N, users x movies) is approximated
 *     by U V^T with U: M x K and V: N x K, K << M, N.
 *   - Sec. II, Algorithm 1: each sampling iteration draws the movie
 *     hyperparameters from V, updates every movie from its ratings and the
 *     users who rated it (plus sampled noise), draws the user hyperparameters
 *     from U, updates every user likewise, then predicts every test point and
 *     computes the RMSE.
 *   - Sec. II: the per-item update is a few K x K matrix/vector operations and
 *     one K x K factorisation.
 * The model the paper cites (BPMF): r_ij ~ N(u_i . v_j, 1/alpha); rows of U
 * and V ~ N(mu, Lambda^-1) per side; (mu, Lambda) ~ Normal-Wishart(mu0,
 * beta0, W0, nu0).  Row draw: P = Lambda + alpha sum_j y_j y_j^T,
 * b = Lambda mu + alpha sum_j r'_ij y_j, P = L L^T, x = L^-T (L^-1 b + z).
 *
 * Conventions for every call:
 *   - All pointers are HOST pointers unless stated otherwise; the library
 *     copies what it needs before returning (inputs are borrowed only for the
 *     duration of the call).  Output buffers are allocated by the caller with
 *     the sizes stated.
 *   - Matrices are row-major.  Factors are rows x K.  Ratings are CSR with
 *     int64 row offsets, int32 column ids strictly increasing within a row
 *     and float32 values.
 *   - A context owns all device memory (hipMalloc) and its HIP streams (the
 *     Gibbs calls go to params.stream when the caller gives one); it is
 *     bound to the device that was current at bpmf_create.
 *   - Gibbs calls on one context must not run concurrently.
 *   - Every call returns BPMF_OK (0) or a negative status; on failure the
 *     context is unchanged (except after BPMF_E_DEVICE, which is sticky:
 *     only bpmf_destroy is then valid) and bpmf_last_error() describes it.
 *   - Randomness: every normal and chi-square draw is a function of
 *     (seed, counter) through Philox4x32-10 (Salmon et al., SC'11) with key
 *     (lo32(seed), hi32(seed)); row noise uses counter
 *     (row, t, stream<<24 | block, 0), so a draw depends only on
 *     (seed, t, side, row), never on launch order or thread count.
 */
#ifndef BPMF_H
#define BPMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bpmf_ctx bpmf_ctx;

enum {
    BPMF_OK = 0,
    BPMF_PENDING = 1,      /* fold-in result not ready yet */
    BPMF_E_INVAL = -1,     /* bad argument, or K out of range */
    BPMF_E_RANGE = -2,     /* an index outside [0, M) or [0, N) */
    BPMF_E_FORMAT = -3,    /* CSR not monotone, columns unsorted/duplicated, CSC not the transpose, non-finite value */
    BPMF_E_NOMEM = -4,     /* device allocation failed */
    BPMF_E_DEVICE = -5,    /* HIP error (sticky) */
    BPMF_E_BUSY = -6,      /* fold-in queue full; retry later */
    BPMF_E_TOOBIG = -7,    /* fold-in request larger than the memory pool */
    BPMF_E_NOSAMPLES = -8, /* fold-in before any bpmf_store_sample */
    BPMF_E_NOTFOUND = -9,  /* unknown fold-in request id */
    BPMF_E_NOTSPD = -10    /* a precision matrix was not positive definite in working precision
                              (row draw or hyper draw); not sticky, but the rows or
                              hyperparameters drawn by that call are undefined */
};

/* Sides of the factorisation: U holds the M users, V the N movies. */
enum { BPMF_SIDE_U = 0, BPMF_SIDE_V = 1 };

/* Arithmetic of the row update.
 *   BPMF_FP64      : factors, Gram, Cholesky and solves in FP64.
 *   BPMF_FP32      : factors FP32; Gram on FP32 matrix cores (MFMA) with FP32
 *                    accumulation; FP32 Cholesky and solves.
 *   BPMF_BF16_GRAM : as FP32, but the gathered factor rows are rounded to
 *                    BF16 and the Gram runs on BF16 MFMA with FP32
 *                    accumulation (rhs, Cholesky and solves stay FP32).
 * The hyperparameter draw is FP64 in every mode. */
enum { BPMF_FP64 = 0, BPMF_FP32 = 1, BPMF_BF16_GRAM = 2 };

typedef struct bpmf_params {
    int32_t K;            /* latent dimension, 1..128 */
    int32_t prec;         /* BPMF_FP64 / BPMF_FP32 / BPMF_BF16_GRAM */
    double alpha;         /* rating precision (default 2) */
    double beta0;         /* Normal-Wishart beta0 (default 2) */
    double nu0;           /* Wishart degrees of freedom (default K) */
    const double *mu0;    /* K values; NULL means 0 */
    const double *W0;     /* K x K SPD Wishart scale; NULL means identity */
    uint64_t seed;        /* Philox key */
    int32_t center;       /* 1: subtract the mean training rating (default 1) */
    int32_t burn_in;      /* sweeps t <= burn_in are left out of the running prediction mean */
    int32_t foldin_S;     /* fold-in sample ring size (default 16) */
    int32_t split_threshold; /* rows with more ratings are split across wavefronts (0: library
                                default, 2048 for K <= 64 and 8192 above) */
    uint64_t foldin_pool_bytes; /* fold-in device memory budget (0: 256 MiB) */
    void *stream;         /* hipStream_t the Gibbs calls are queued on (NULL: the context
                             creates its own); a caller's stream is borrowed, never destroyed,
                             and must outlive the context; it must not be the legacy null
                             stream (the sweep graph is captured on it) */
    int32_t reorder;      /* 1: hold users and movies in descending order of their rating
                             counts (ties by id), the reordering of R before partitioning
                             (Sec. IV-B), so the most-gathered factor rows lie together;
                             0 (default): keep the caller's order.  Every call still takes
                             and returns the caller's ids; only the "row" of the noise
                             counters, the initial factors' counters and the order of the
                             hyper draw's sums and of fold-in ties are the internal
                             position.  A relabelled context on R computes bit for bit
                             what an ordinary one computes on R relabelled the same way. */
} bpmf_params;

/* Fill *p with the defaults above for latent dimension K. */
void bpmf_default_params(bpmf_params *p, int32_t K);

/* Create a context from training ratings (CSR over the M users) and test
 * triples.  csc_* may be NULL: the transpose (columns ascending, rows
 * ascending within a column) is then built by the library; when given it
 * must be exactly that transpose (BPMF_E_FORMAT otherwise).  The factors
 * are initialised as X_ik = K^-1/4 z with z the Philox normals of counter
 * (row, 0, stream<<24 | block, 0), stream 5 for U and 6 for V.
 * Validation: ptr[0] = 0, ptr non-decreasing, ptr[M] = nnz; columns in
 * [0, N) and strictly increasing per row; values finite; test ids in range. */
int bpmf_create(int64_t M, int64_t N, const int64_t *csr_ptr, const int32_t *csr_col,
                const float *csr_val, const int64_t *csc_ptr, const int32_t *csc_row,
                const float *csc_val, int64_t nnz, const int32_t *test_row,
                const int32_t *test_col, const float *test_val, int64_t n_test,
                const bpmf_params *p, bpmf_ctx **out);

/* Algorithm 1, "sample hyper-parameters movies based on V" (side V) or
 * "users based on U" (side U), for sweep t: Normal-Wishart posterior draw in
 * FP64 on the device (Bartlett decomposition; chi-square counter
 * (k, t, stream<<24 | 0, attempt), lower normals (block, t, stream<<24 | 1, 0),
 * mu normals (block, t, stream<<24 | 2, 0), stream 3 for U, 4 for V). */
int bpmf_sample_hyper(bpmf_ctx *c, int32_t side, uint32_t t);

/* Algorithm 1, the item loop of one side for sweep t: every row of the side
 * is redrawn from its conditional given the other factor and the side's
 * current hyperparameters (row noise stream 1 for U, 2 for V).
 * BPMF_E_NOTSPD if some row's P = Lambda + alpha sum y y^T had a
 * non-positive pivot in working precision (those rows are undefined). */
int bpmf_update_side(bpmf_ctx *c, int32_t side, uint32_t t);

/* Algorithm 1 for sweeps t0 .. t0+n-1 (each: hyper V, update V, hyper U,
 * update U, predict), captured once as a HIP graph and replayed; the sweep
 * counter lives in device memory.  rmse_avg / rmse_last receive n values
 * each (either may be NULL): RMSE of the running mean prediction (sweeps
 * t > burn_in) and of the current sample. */
int bpmf_run_sweeps(bpmf_ctx *c, uint32_t t0, uint32_t n, double *rmse_avg, double *rmse_last);

/* Algorithm 1 for sweeps t0 .. t0+n-1 launched eagerly with HIP events
 * between its phases; phase_ms[7] receives the mean device time per sweep
 * of: hyper draw V, row kernel of V (all rows and split-row segments),
 * finishing of V's split rows, the same three for U, and prediction.  The chain advances exactly as with bpmf_run_sweeps
 * (n must not exceed the RMSE history size of an earlier bpmf_run_sweeps). */
int bpmf_profile_sweeps(bpmf_ctx *c, uint32_t t0, uint32_t n, double *phase_ms);

/* Algorithm 1, "predict rating and compute RMSE".  n == 0: predict the
 * registered test set with the current factors, fold the prediction into the
 * running mean as sweep t (if t > burn_in), and return the two RMSEs (t is
 * explicit here, as on every call that depends on the sweep index, so that
 * an eager sequence of calls reproduces bpmf_run_sweeps exactly).
 * n > 0: predict the n given (row, col) pairs into out[n] (float,
 * u_row . v_col + mean rating) without touching the running mean; the RMSE
 * pointers are then ignored. */
int bpmf_predict(bpmf_ctx *c, uint32_t t, int64_t n, const int32_t *row, const int32_t *col,
                 float *out, double *rmse_avg, double *rmse_last);

/* bpmf_predict with n > 0, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same predictions, bit for bit, of n (row, col) pairs
 * (host arrays; out[n] receives u_row . v_col + mean rating), staged through
 * a fixed device array of the library instead of buffers it allocates, so
 * the call allocates and frees nothing.  At most 524,288 pairs per call
 * (BPMF_E_TOOBIG above).  Each GPU holds one such array for the whole
 * process and every context on that GPU shares it: calls that overlap on one
 * GPU (from several threads or contexts) race and must be serialised by the
 * caller.  BPMF_E_RANGE for ids out of range. */
int bpmf_predict_noalloc(bpmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col, float *out);

/* Factor access: host buffer of rows x K values, float in FP32/BF16 modes and
 * double in FP64 mode (bpmf_get_factor_f64 / bpmf_set_factor_f64 convert). */
int bpmf_get_factor(bpmf_ctx *c, int32_t side, void *host);
int bpmf_set_factor(bpmf_ctx *c, int32_t side, const void *host);
int bpmf_get_factor_f64(bpmf_ctx *c, int32_t side, double *host);
int bpmf_set_factor_f64(bpmf_ctx *c, int32_t side, const double *host);

/* Hyperparameters of a side: mu (K) and Lambda (K x K), FP64. */
int bpmf_get_hyper(bpmf_ctx *c, int32_t side, double *mu, double *Lambda);
int bpmf_set_hyper(bpmf_ctx *c, int32_t side, const double *mu, const double *Lambda);

/* Chain state beyond the factors and hyperparameters, for checkpoint and
 * resume: the running sum of test predictions over the sweeps t > burn_in
 * (pred_sum[n_test], FP64, in the order the test pairs were given to
 * bpmf_create) and the number of sweeps in it (*n_avg).  Restoring it with
 * the factors lets a resumed chain report the same RMSE of the running mean
 * as an uninterrupted one (the next sweep index is passed explicitly to
 * bpmf_run_sweeps).  Either pointer may be NULL on get. */
int bpmf_get_chain_state(bpmf_ctx *c, double *pred_sum, uint32_t *n_avg);
int bpmf_set_chain_state(bpmf_ctx *c, const double *pred_sum, uint32_t n_avg);

/* The CSC the library uses (N+1 offsets, nnz row ids, nnz centred values as
 * stored: float, or double in FP64 mode, r - mean), in the caller's ids also
 * when params.reorder is set.  For verification. */
int bpmf_get_csc(bpmf_ctx *c, int64_t *ptr, int32_t *row, void *rc);

/* The degree plan of a side: perm[rows] = (caller's) row ids in processing order
 * (degree descending, ties by row id), n_split = number of rows split
 * across wavefronts (they come first in perm), n_low = number of rows on the
 * rank-one-update path (the last ones in perm).  Any pointer may be NULL. */
int bpmf_get_plan(bpmf_ctx *c, int32_t side, int32_t *perm, int64_t *n_split, int64_t *n_low);

/* Mean training rating subtracted from the ratings (0 when center = 0). */
double bpmf_mean_rating(const bpmf_ctx *c);

/* Block until all work queued on the context's stream has finished. */
int bpmf_synchronize(bpmf_ctx *c);

/* Device time (ms, HIP events on the context stream) of the most recent
 * bpmf_update_side / bpmf_sample_hyper / bpmf_run_sweeps call. */
int bpmf_last_time_ms(bpmf_ctx *c, double *ms);

/* Autotuning of the degree-bucket cut-offs and kernel family on the
 * context's own data.  The paper balances per-item work by degree with a
 * fixed cost plus a cost per rating and switches small items to a cheaper
 * serial method (Sec. III, Fig. 2, Sec. IV-B); here three cut-offs are chosen
 * by timing n_sweeps (1..64) graph sweeps per candidate:
 *   - the degree above which a row is split into segments across
 *     wavefronts: of 512, 1024, ... up to the first power of two at or above
 *     the largest degree, those within a factor of four of the workload
 *     model's threshold (or the one nearest it), and the current one.  The
 *     model: a row costs r + d rating-equivalents, r = 3K, and with W the sum
 *     over a side's rows and P the rows in flight on the GPU a row alone on
 *     its wave must not take more than half of the side's stage, so
 *     d* = W / (2P) - r, the smaller of the two sides';
 *   - for FP32 with 32 < K <= 64, whether rows take the column-per-lane
 *     (kmax 64) or the blocked (kmax 32) kernel;
 *   - for FP32 with K <= 64, the degree up to which rows take the rank-one
 *     update path (0 = off, 8, 16; a side uses it only where the saved
 *     factorisations outweigh transforming the gathered factor).
 * A candidate replaces the current plan only if it is at least 1% faster.
 * The chain state (factors, hyperparameters, running predictions, sweep
 * counter) is restored afterwards, so the chain continues as if no trial had
 * run; only the plan changes, and the sweep graph of the chosen plan is
 * captured before returning.  Outputs (each may be NULL): the chosen values,
 * the number of candidates tried (at most 64) and, per candidate, its values
 * and mean ms per sweep (caller arrays of 64). */
int bpmf_autotune(bpmf_ctx *c, uint32_t n_sweeps, int32_t *chosen_split, int32_t *chosen_kmax,
                  int32_t *chosen_low, int32_t *n_tried, int32_t *tried_split, int32_t *tried_kmax,
                  int32_t *tried_low, double *tried_ms);

/* Sets the plan the autotuner would choose, by hand: split_threshold
 * (1..2^24; rows with more ratings are cut into segments of
 * max(128, split_threshold / 2)), fast_kmax (0..64; FP32 factors with
 * K <= fast_kmax take the column-per-lane kernel, larger K the blocked one)
 * and lowrank_dmax (0, 4, 8 or 16; with FP32 factors and K <= 64 every row
 * with at most that many ratings takes the rank-one update path -- unlike the
 * autotuner, without weighing the transform of the gathered factor).  The
 * work items, finishing items and partial-sum workspace are rebuilt and the
 * sweep graph is re-captured (not launched) before returning; the chain
 * state is untouched and the samples do not depend on the plan beyond
 * rounding.  Used
 * to time each kernel family per degree (the per-item cost against degree
 * of Sec. III, Fig. 2).  BPMF_E_INVAL for a value out of range or the
 * rank-one path where it does not apply. */
int bpmf_set_plan(bpmf_ctx *c, int32_t split_threshold, int32_t fast_kmax, int32_t lowrank_dmax);

/* Mean device time (ms) of one side's row update (the item loop of
 * Algorithm 1: every work item -- segments of split rows, whole rows, rows on
 * the rank-one path -- and the finishing of split rows; not the BF16 shadow
 * copy) over the sweeps of the most recent bpmf_run_sweeps call: ms[0] for
 * the V side, ms[1] for the U side.  Measured inside the sweep graph with HIP
 * events recorded just before the side's first kernel and after its last
 * (both on the stream that joins the update's branches), one set per replay
 * (the first 1023 replays and the last).  Caller-owned ms[2].
 * BPMF_E_INVAL if no sweeps were timed. */
int bpmf_row_kernel_ms(bpmf_ctx *c, double *ms);

/* ---- Fold-in serving (not a step of Algorithm 1: new users against stored
 * posterior samples; requires BPMF_FP32 and K <= 64) ----
 *
 * For a new user with ratings {(j, r_j)}, each stored sample s gives one draw
 * from the same row conditional as Algorithm 1's user loop,
 *   P = Lambda_U^(s) + alpha sum_j v_j^(s) v_j^(s)T,
 *   b = Lambda_U^(s) mu_U^(s) + alpha sum_j (r_j - rbar) v_j^(s),
 *   u_s = L^-T (L^-1 b + z_s),  P = L L^T,
 * with z_s the Philox normals of counter (lo32(id), s, 7<<24 | block, hi32(id))
 * (id = the request id), then scores p_sj = u_s . v_j^(s) + rbar for every
 * movie.  The result is the top_n unrated movies by mean_j = (1/S) sum_s p_sj
 * (descending, ties to the smaller id -- the smaller internal position when
 * params.reorder is set), with mean_j and the predictive
 * variance var_j = 1/alpha + (1/S) sum_s (p_sj - mean_j)^2. */

/* Snapshot the current V and the user-side (mu_U, Lambda_U) into the next
 * slot of a device-resident ring of params.foldin_S samples (the oldest is
 * overwritten).  The first call allocates the ring and four batch slots
 * (each with its own stream) and starts the scheduler thread;
 * params.foldin_pool_bytes (default 256 MiB) bounds the rated movies in
 * flight: each batch admits requests while their ratings fit pool/32 (8 B
 * per rating, four batches).  Blocks until in-flight fold-in batches finished.  A Gibbs call: not concurrent with other Gibbs calls on
 * c, and the first call must return before any bpmf_foldin_submit. */
int bpmf_store_sample(bpmf_ctx *c);

/* Queue a request: n distinct movie ids in [0, N) with their ratings (host
 * arrays, copied), 1 <= top_n <= 1024.  *req_id receives the request id
 * (1, 2, ... in submission order on this context; also the noise key).
 * Thread-safe.  Errors: BPMF_E_NOSAMPLES before any stored sample,
 * BPMF_E_RANGE / BPMF_E_FORMAT for bad ids, duplicates or non-finite
 * ratings, BPMF_E_TOOBIG if n exceeds one batch's rating capacity,
 * BPMF_E_BUSY if 2^20 requests are pending.  Requests are batched by size
 * class as they arrive (continuous batching; up to four batches on the
 * device at once, each on its own stream); a request's result does not
 * depend on what it is batched with. */
int bpmf_foldin_submit(bpmf_ctx *c, int32_t n, const int32_t *movie, const float *rating,
                       int32_t top_n, uint64_t *req_id);

/* Thread-safe.  BPMF_PENDING while the request runs; BPMF_OK once done, after
 * copying top_n entries into movie_out / mean_out / var_out (caller-allocated,
 * any may be NULL; entries beyond the number of unrated movies are -1 / 0)
 * and the time from submission to completion into *latency_s; the request is
 * then forgotten (a second poll gives BPMF_E_NOTFOUND). */
int bpmf_foldin_poll(bpmf_ctx *c, uint64_t req_id, int32_t *movie_out, float *mean_out,
                     float *var_out, double *latency_s);

/* Block until every submitted request has completed. */
int bpmf_foldin_drain(bpmf_ctx *c);

/* Scheduler statistics since the first bpmf_store_sample (any pointer may
 * be NULL): batches launched, requests launched, the most requests in one
 * batch, and the most batches on the device at the same time (each staging
 * slot has its own stream, so batches overlap). */
int bpmf_foldin_stats(bpmf_ctx *c, int64_t *batches, int64_t *requests, int32_t *max_batch_requests,
                      int32_t *max_inflight_batches);

/* Number of samples currently in the ring. */
int bpmf_foldin_samples(const bpmf_ctx *c);

/* Ratings one batch can hold (0 before the first bpmf_store_sample). */
int64_t bpmf_foldin_capacity(const bpmf_ctx *c);

/* Message of the last failed call on c (or of the last failed create when c
 * is NULL). */
const char *bpmf_last_error(const bpmf_ctx *c);

void bpmf_destroy(bpmf_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* BPMF_H */
