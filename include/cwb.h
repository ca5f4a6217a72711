/*
 * cwb.h -- C ABI of the MI355X (gfx950) binned componentwise-boosting library.
 *
 * The library fits componentwise gradient boosting models (CWB), their
 * Nesterov-accelerated form (ACWB) and the hybrid of the two (HCWB) as
 * defined in "Accelerated Componentwise Gradient Boosting using Efficient
 * Data Representation and Momentum-based Optimization" (Schalk, Bischl,
 * Ruegamer, arXiv 2110.03513):
 *   - CWB:  appendix Algorithm A1 (Section 2.3);
 *   - binned features, index vectors and binMatVec / binMatMat:
 *           Section 3.1 and Algorithm 1;
 *   - ACWB: Algorithm 2 (Section 3.2), parameter bookkeeping Section 3.2.1;
 *   - HCWB: Algorithm 3 (Section 3.2.3);
 *   - P-spline and categorical ridge base learners with equal degrees of
 *     freedom: Section 2.2, Appendix A.2 and A.3.1; categorical features in
 *     the binary representation (one learner per class): Appendix A.3.2;
 *   - the fitted model and its learners' functions at new rows (Section
 *     2.3), single fits, batches of fits, a fit server, and K-fold
 *     cross-validation whose folds share one index matrix (Section 4.2).
 * Every iteration runs on the GPU in hand-written HIP kernels.  The one-off
 * FP64 setup in cwb_fit_create bins the features and counts the bins on the
 * GPU (or on host threads, see cwb_problem.setup); the host builds the
 * bases, Gram matrices, smoothing parameters and their factorisations.
 *
 * Conventions for every call:
 *   - Returns CWB_OK (0) or a negative CWB_E_* code; on error,
 *     cwb_last_error() returns a message for the calling thread.  No C++
 *     exception or abort crosses this boundary.
 *   - "host" pointers are ordinary CPU memory owned by the caller and only
 *     read during the call unless stated otherwise; "device" pointers are GPU
 *     memory (hipMalloc or a PyTorch CUDA tensor) owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All GPU work of a fit is enqueued on its stream.
 *   - A fit handle is not thread-safe; a server handle is.
 */
#ifndef CWB_H_
#define CWB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CWB_VERSION_MAJOR 1
#define CWB_VERSION_MINOR 0

/* status codes */
#define CWB_OK 0
#define CWB_E_INVALID_ARG -1  /* bad size, value, pointer or call argument */
#define CWB_E_UNSUPPORTED -2  /* valid request the library does not implement */
#define CWB_E_NO_MEMORY -3    /* workspace too small / memory budget exceeded */
#define CWB_E_DEVICE -4       /* HIP runtime error (message has the HIP text) */
#define CWB_E_NUMERIC -5      /* singular penalised Gram, non-finite model state */
#define CWB_E_AGAIN -6        /* result not ready yet (server poll) */
#define CWB_E_STATE -7        /* call out of order (e.g. run past M) */

/* losses (Section 2.1): L2 is (y - f)^2 / 2, so the pseudo-residual is
 * y - f; binomial uses y in {0, 1} and f = log-odds, L = log(1 + e^f) - y f. */
#define CWB_L2 0
#define CWB_BINOMIAL 1

/* variants */
#define CWB_CWB 0   /* appendix Algorithm A1 */
#define CWB_ACWB 1  /* Algorithm 2 */
#define CWB_HCWB 2  /* Algorithm 3 */

/* base-learner kinds */
#define CWB_PSPLINE 0    /* univariate B-spline basis with difference penalty (Sec. 2.2) */
#define CWB_RIDGE_CAT 1  /* categorical dummy basis with ridge penalty (App. A.3.1) */
#define CWB_BINARY_CAT 2 /* categorical feature in the binary representation
                            (App. A.3.2): one unpenalised learner per class,
                            the indicator of that class, with the class mean of
                            the signal as its estimate.  The feature's entry in
                            the traces is the class learner chosen: k is the
                            feature, and its coefficient row has one nonzero
                            entry, at the class.  df and lambda are ignored; a
                            class without fitted rows is never selected. */

/* One base learner per feature (Section 2.2: univariate learners, K = p); a
 * CWB_BINARY_CAT feature stands for its c_j class learners. */
typedef struct {
  int32_t kind;             /* CWB_PSPLINE, CWB_RIDGE_CAT or CWB_BINARY_CAT */
  int32_t degree;           /* P-spline degree, 1..3 (the paper uses 3) */
  int32_t n_interior_knots; /* equally spaced interior knots (the paper uses 20) */
  int32_t penalty_order;    /* difference order of the penalty (2) */
  double df;                /* > 0: lambda chosen so that trace of the hat matrix
                               equals df (App. A.2); <= 0: use `lambda` */
  double lambda;            /* smoothing parameter when df <= 0 (>= 0) */
  int32_t n_bins;           /* P-spline design points n* (Sec. 3.1.1), 2..65535;
                               -1 selects floor(sqrt(n)), -2 floor(n^(1/4))
                               (the smaller grid of App. B.3); 0 selects an unbinned
                               learner (each row's own basis, Sec. 2.2; cubic
                               only, and then every learner of the fit must be
                               unbinned: no categorical learners; not served) */
  int32_t n_levels;         /* categorical kinds: number of levels c_j (1..64) */
} cwb_learner_spec;

/* The fitting problem (all pointers are host memory, read during create). */
typedef struct {
  int64_t n;                     /* rows, >= 2 */
  int32_t p;                     /* features = base learners, >= 1 */
  const double* x;               /* n x p, COLUMN-major: x[j*ldx + i].  Ridge
                                    columns hold integer level codes 0..c_j-1. */
  const double* y;               /* n targets (binomial: 0 or 1) */
  int32_t loss;                  /* CWB_L2 or CWB_BINOMIAL */
  const cwb_learner_spec* specs; /* p entries */
  double nu;                     /* learning rate, > 0 */
  int32_t M;                     /* total boosting iterations, >= 1 */
  int32_t variant;               /* CWB_CWB, CWB_ACWB or CWB_HCWB */
  double gamma;                  /* momentum parameter (ACWB / HCWB), >= 0 */
  int32_t patience;              /* HCWB patience pat_0, >= 0 */
  const uint8_t* val_mask;       /* NULL, or n bytes with 1 = validation row.
                                    Required for HCWB.  CWB / ACWB then fit on
                                    the other rows and report validation risk. */
  int64_t ldx;                   /* column stride of x in elements: column j
                                    starts at x + j*ldx; 0 means n; else >= n */
  int32_t setup;                 /* where binning and bin counts run during
                                    create: CWB_SETUP_AUTO, CWB_SETUP_HOST or
                                    CWB_SETUP_DEVICE (binned fits with
                                    n < 2^31 only, else UNSUPPORTED).  Both
                                    give bitwise the same fit. */
} cwb_problem;

/* cwb_problem.setup */
#define CWB_SETUP_AUTO 0   /* device for binned fits with n < 2^31, else host
                              (the server alike: a request set up on the
                              device is binned and solved during its upload,
                              on the server's upload stream, overlapping the
                              running batch) */
#define CWB_SETUP_HOST 1   /* host threads bin every column (Sec. 3.1.1) */
#define CWB_SETUP_DEVICE 2 /* columns are copied to the workspace one at a
                              time and binned and counted on the GPU; the host
                              builds the bases from the ranges, and the GPU
                              the Gram matrices, smoothing parameters and
                              inverses of learners with at most 32 basis
                              functions from the counts (one block per
                              learner and row set; the host those of larger
                              ones) */

/* Sizes of a created fit (for sizing getter buffers). */
typedef struct {
  int64_t n;
  int32_t p;
  int32_t M;
  int32_t d_max;        /* largest basis size */
  int32_t sum_d;        /* total basis size (length of coefficient vectors) */
  int32_t nb_max;       /* largest bin / level count */
  int32_t iters_done;   /* iterations enqueued so far */
  int64_t n_train;      /* rows used by the training phase */
  double f0;            /* loss-optimal constant (intercept) */
} cwb_info;

int cwb_version(int* major, int* minor);

/* Message for the last non-zero status returned on this thread. */
const char* cwb_last_error(void);

/* Device bytes a fit of this problem needs (inputs in binned form, model
 * state, per-feature tables, traces, schedule and histogram partials) on the
 * current HIP device.  The caller allocates at least this many bytes of
 * device memory and passes them to cwb_fit_create. */
int cwb_workspace_bytes(const cwb_problem* pr, size_t* bytes);

/* Equal-grid binning of one numeric feature (Section 3.1.1), host only: n*
 * design points z_l = min + l (max - min)/(n* - 1) (z_{n*-1} = max exactly)
 * and the index of the closest design point for every value, ties to the
 * lower point -- the index vector cwb_fit_create builds for a P-spline
 * learner.  x: n host doubles; ind_out: n host uint16; z_out: n_bins host
 * doubles or NULL.  INVALID_ARG for n < 1, n_bins outside 2..65535, a
 * non-finite or constant x. */
int cwb_bin_feature(const double* x, int64_t n, int32_t n_bins, uint16_t* ind_out, double* z_out);

/* The smoothing parameter of a penalised learner for a target degrees of
 * freedom (App. A.2), host only: lambda >= 0 with
 * df(lambda) = trace((G + lambda D)^-1 G) = df, the computation
 * cwb_fit_create runs for every P-spline learner with a df target.  G, D:
 * d x d host doubles, row-major, symmetric (the learner's Gram matrix and
 * penalty).  INVALID_ARG for NULL pointers, d outside 1..64, df outside
 * (0, d) or a target the penalty's null space cannot reach; NUMERIC for a
 * degenerate G or D. */
int cwb_lambda_for_df(int32_t d, const double* G, const double* D, double df, double* lambda);

typedef struct cwb_fit cwb_fit;

/* Validate the problem, run the FP64 host setup (binning on an equal grid
 * with ties to the lower design point, Sec. 3.1.1; B-spline bases at the
 * design points; bin counts and Gram matrices by binMatMat, Alg. 1; the
 * smoothing parameter for the requested df by the Demmler-Reinsch
 * orthogonalisation, App. A.2; the inverse penalised Gram matrix, Sec. 2.4)
 * and copy everything to `dev_ws` on `stream`.  The library copies what it
 * needs, so the caller may free the host arrays on return.  `dev_ws` stays
 * owned by the caller and must outlive the fit.  Create then times the
 * histogram pass under each candidate tile shape on the fit's own data and
 * keeps the fastest (see cwb_tile; the environment variable CWB_AUTOTUNE=0
 * keeps the default shape).  Histograms are exact integer sums, so the
 * choice never changes a result.
 * Errors: INVALID_ARG (n < 2, p < 1, bins outside 2..65535, constant
 * feature, df <= 2 or df >= basis size for a P-spline, binomial y not 0/1,
 * nu <= 0, M < 1, NULL pointer, level code out of range, HCWB without a
 * validation row or training row), NO_MEMORY (ws_bytes too small),
 * NUMERIC (singular penalised Gram), DEVICE (HIP error). */
int cwb_fit_create(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream,
                   cwb_fit** out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): cwb_fit_create
 * with the fit's histogram partials (the scratch its histogram and select
 * passes exchange) in a 64 MiB array of the library's own device memory
 * instead of in `dev_ws`, which still holds every input and output.  The
 * call allocates no device memory: setup runs on the host threads, the
 * default tile shape is kept (no autotuning), and a workspace of
 * cwb_workspace_bytes() is always large enough.  Each GPU has its own copy
 * of the array, held until the process ends, and every fit created by this
 * call on a GPU shares it: runs of two such fits must not overlap on one
 * GPU (the caller orders them, e.g. on one stream), and batches, which keep
 * their own partials, are unaffected.  Errors as cwb_fit_create, plus
 * NO_MEMORY when the partials of the default tile exceed 64 MiB and
 * UNSUPPORTED for setup = CWB_SETUP_DEVICE. */
int cwb_fit_create_noalloc(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream,
                           cwb_fit** out);

/* Enqueue `iters` boosting iterations on the fit's stream and return
 * without waiting.  May be called repeatedly (the fit resumes where it
 * stopped); STATE if this would run past M. */
int cwb_fit_run(cwb_fit* f, int32_t iters);

/* Wait for the fit's stream; NUMERIC if the device flagged a non-finite
 * state, DEVICE on a HIP error. */
int cwb_fit_sync(cwb_fit* f);

int cwb_fit_info(const cwb_fit* f, cwb_info* info);

/* Traces for the iterations done so far (host buffers; any may be NULL):
 *   k[M]            selected learner per iteration (Alg. A1 / Alg. 2)
 *   theta[M*d_max]  its coefficients (zero padded to d_max)
 *   k_cor[M]        ACWB correction learner, -1 in CWB iterations
 *   theta_cor[M*d_max]
 *   train_risk[M+1] empirical risk of f^[m] on the training rows, m = 0..M
 *   val_risk[M+1]   empirical risk of f^[m] on the validation rows
 *   crit_gap[M]     runner-up minus best selection criterion (FP64), a
 *                   near-tie indicator
 *   switch_iter[1]  HCWB: first CWB iteration, or -1.
 * Synchronises the stream. */
int cwb_fit_get_trace(cwb_fit* f, int32_t* k, double* theta, int32_t* k_cor,
                      double* theta_cor, double* train_risk, double* val_risk,
                      double* crit_gap, int32_t* switch_iter);

/* Aggregated model (Section 2.3 and 3.2.1): intercept f0 and the summed
 * coefficients of each learner, concatenated in learner order (sum_d
 * values), for the primary model f and (ACWB / HCWB) the momentum model h.
 * coef_f includes the learning rate, so f = f0 + sum_k Z_k coef_f[k].
 * Synchronises the stream. */
int cwb_fit_get_model(cwb_fit* f, double* intercept, double* coef_f, double* coef_h);

/* Training-set predictions f^[m] (n floats, original row order) after the
 * iterations done so far.  Synchronises the stream. */
int cwb_fit_get_pred(cwb_fit* f, float* f_out);

/* The fitted primary model at new rows (Section 2.3: f0 plus every
 * learner's fitted function), enqueued on the fit's stream (the caller
 * synchronises, e.g. with cwb_fit_sync).  x: DEVICE array of n x p doubles,
 * column-major with column stride ldx >= n, raw feature values: P-spline
 * values are clamped to the learner's training range and evaluated with the
 * exact B-spline basis (not binned); categorical columns hold level codes
 * (an invalid code gives NaN).  out: DEVICE array of n doubles.  Both stay
 * owned by the caller.  INVALID_ARG for n < 0, ldx < n or NULL arrays. */
int cwb_fit_predict(cwb_fit* f, const double* x, int64_t n, int64_t ldx, double* out);

/* Partial effect of learner k (its fitted function alone, without f0) at n
 * values: x and out are DEVICE arrays of n doubles; otherwise as
 * cwb_fit_predict.  INVALID_ARG for k outside 0..p-1. */
int cwb_fit_partial_effect(cwb_fit* f, int32_t k, const double* x, int64_t n, double* out);

/* Checkpoint / resume: bytes of the mutable fit state (model vectors,
 * control block, traces, aggregated coefficients); save copies it to a host
 * buffer, load restores it into a fit created from the same problem. */
int cwb_fit_state_bytes(const cwb_fit* f, size_t* bytes);
int cwb_fit_save_state(cwb_fit* f, void* host_buf, size_t bytes);
int cwb_fit_load_state(cwb_fit* f, const void* host_buf, size_t bytes);

/* Per-kernel GPU timing with HIP events recorded on the fit's stream around
 * every launch of the selected kernels.  `mask` is a bit set: 1 = "hist"
 * (histogram pass), 2 = "state" (row pass), 4 = "select" (solve and
 * selection); 0 turns timing off.  Setting a mask resets the accumulation;
 * the query synchronises and returns the summed milliseconds and the number
 * of timed launches of the named kernel.  When the first fit of a batch has
 * timing on, the batch's eagerly launched iterations (not those replayed
 * from a captured graph) are timed into that fit's timer: the launches
 * then cover every fit of the batch. */
int cwb_fit_set_timing(cwb_fit* f, int32_t mask);
/* The same, timing only every `period`-th iteration (period >= 1): each
 * event pair costs a few microseconds of queue time, so sampling keeps the
 * timed run close to an untimed one. */
int cwb_fit_set_timing_period(cwb_fit* f, int32_t mask, int32_t period);
int cwb_fit_kernel_time(cwb_fit* f, const char* kernel, double* total_ms, int64_t* launches);

/* Histogram tile shape a fit or batch uses (Section 3.1.2's first stage:
 * each block accumulates the bin sums of `learners` learners over its rows
 * in LDS). */
typedef struct {
  int32_t threads;     /* threads per histogram block */
  int32_t learners;    /* learners per LDS histogram group */
  int32_t blocks;      /* histogram blocks per launch */
  int32_t candidates;  /* tile shapes timed at create (1: not tuned) */
  int32_t learners32;  /* learners (over all fits) whose LDS histograms take
                          32-bit words: their group's every learner holds
                          fewer than 2^acc32_bits rows in each bin */
  int32_t acc32_bits;  /* the fit's count bound (the largest over the batch's
                          fits); 0: int64 sums at the int64 scale */
  int32_t index_bits;  /* bits per bin index the histogram pass reads: 10 or
                          12 (a packed copy of the index matrix) or 16 (the
                          matrix itself); a batch reports the widest over
                          its fits */
  double tuned_us;     /* measured pass time of the chosen shape (0: not tuned) */
} cwb_tile;
int cwb_fit_tile(const cwb_fit* f, cwb_tile* out);

/* Free host-side objects; never frees the caller's device workspace. */
void cwb_fit_destroy(cwb_fit* f);

/* ---- batched fits: many independent fits advance together -------------
 * One launch per kernel per iteration covers every fit of the batch: the
 * row-tile pass, the histogram pass over all fits' bin-index matrices and
 * the per-feature solve / selection.  Fits keep their own workspaces; the
 * batch needs a workspace of its own for the combined schedule and
 * histogram partials.  All fits must have been created on `stream`'s device;
 * the batch enqueues on `stream`. */
typedef struct cwb_batch cwb_batch;
int cwb_batch_workspace_bytes(cwb_fit* const* fits, int32_t count, size_t* bytes);
/* Creates the combined schedule and autotunes its histogram tiles like
 * cwb_fit_create (the workspace is sized for every candidate shape). */
int cwb_batch_create(cwb_fit* const* fits, int32_t count, void* dev_ws, size_t ws_bytes,
                     void* stream, cwb_batch** out);
int cwb_batch_tile(const cwb_batch* b, cwb_tile* out);
/* Advance every fit by up to `iters` iterations (fits stop at their own M). */
int cwb_batch_run(cwb_batch* b, int32_t iters);
int cwb_batch_sync(cwb_batch* b);
void cwb_batch_destroy(cwb_batch* b);

/* ---- cross-validation: K folds sharing one index matrix ----------------
 * The folds of a K-fold cross-validation (the benchmark protocol of Sec.
 * 4.2) as K fits with 0/1 row weights: fold k trains on every row whose
 * fold id is not k and reports its risk on the held-out rows as its
 * validation risk.  The index matrix is binned once, with the rows grouped
 * by fold, and stored once; one histogram pass per iteration reads it once
 * for all folds, accumulating one histogram per fold (each fold leaves out
 * its own block of rows).  Every fold's selections, coefficients and risks are
 * those of a fit of the same problem with its fold as the validation mask,
 * up to the rounding of the FP32 model state (the histogram scale can
 * differ, since a fold's pass reads all n rows).
 * Rules: 2 <= n_folds <= 8; fold: n host int32 ids in [0, n_folds), every
 * fold with at least one row and two training rows; pr->val_mask NULL;
 * variant CWB or ACWB; binned learners; the folds' histograms of one learner
 * (n_folds x signals x bins x 8 bytes) within 152 KiB, else UNSUPPORTED.
 * Setup bins on host threads (pr->setup is not used). */
typedef struct cwb_cv cwb_cv;
int cwb_cv_workspace_bytes(const cwb_problem* pr, int32_t n_folds, const int32_t* fold,
                           size_t* bytes);
int cwb_cv_create(const cwb_problem* pr, int32_t n_folds, const int32_t* fold, void* dev_ws,
                  size_t ws_bytes, void* stream, cwb_cv** out);
/* Advance every fold by up to `iters` iterations (asynchronous). */
int cwb_cv_run(cwb_cv* cv, int32_t iters);
int cwb_cv_sync(cwb_cv* cv);
/* Fold k's fit, owned by the cross-validation: every cwb_fit_get_* call and
 * cwb_fit_predict / cwb_fit_partial_effect apply; do not destroy it. */
int cwb_cv_fold(cwb_cv* cv, int32_t k, cwb_fit** out);
/* Cross-validated risk: for m = 0..iterations done, the held-out loss summed
 * over all folds' held-out rows, divided by n (m + 1 doubles). */
int cwb_cv_risk(cwb_cv* cv, double* risk);
/* The histogram tile the folds' shared pass runs with (autotuned at create). */
int cwb_cv_tile(const cwb_cv* cv, cwb_tile* out);
void cwb_cv_destroy(cwb_cv* cv);

/* ---- serving: continuous batching of fit requests ---------------------
 * A request loop on its own host thread.  Requests are admitted while their
 * workspace fits in the device arena the caller hands in; admitted fits
 * advance together in batched iterations; requests that arrive while others
 * run join at the next scheduling quantum, and finished fits retire and free
 * their arena space.  submit never blocks; poll returns CWB_E_AGAIN until
 * the result is ready, then hands it over once (a second poll of the same
 * ticket is INVALID_ARG).  Requests that can never fit the arena finish
 * with status NO_MEMORY.  Destroy cancels requests not yet admitted
 * (status STATE) and finishes the admitted ones. */
typedef struct cwb_server cwb_server;
typedef struct {
  void* arena;          /* device memory for fit workspaces (caller-owned) */
  size_t arena_bytes;   /* its size: the HBM admission budget */
  int32_t max_slots;    /* most fits in flight at once */
  int32_t quantum;      /* iterations per scheduling round (e.g. 50) */
  void* stream;         /* hipStream_t for all server GPU work */
  int32_t setup_threads;/* host threads for request setup (0 = auto) */
} cwb_server_cfg;

typedef struct {
  int32_t status;       /* CWB_OK, or the error of this request */
  int32_t M;            /* iterations run */
  double latency_s;     /* submit -> result ready */
  double queue_s;       /* submit -> admitted */
  double intercept;
} cwb_result;

typedef struct {
  int64_t submitted, completed, rejected;
  int32_t in_flight, queued;
  double fits_per_s;    /* completed / seconds since the first submit */
  double p50_latency_s, p99_latency_s;
  size_t arena_in_use, arena_peak;
  double mean_setup_s;  /* per completed request: host setup plus upload
                           (the upload includes the device setup pass of a
                           request set up on the GPU) */
  double mean_queue_s;  /* submit -> admitted, per completed request */
  double round_s;       /* device-thread time inside rounds (launch to end of round) */
  double busy_s;        /* device-thread time from the first round to the last */
  int64_t rounds;       /* rounds run */
} cwb_stats;

int cwb_server_create(const cwb_server_cfg* cfg, cwb_server** out);
/* Queue a request and return at once; `ticket` identifies it.  The learner
 * specifications are copied; the arrays x, y and val_mask are read later by
 * the server's setup threads (x by its upload thread for a request set up on
 * the GPU), so the caller keeps them valid and unchanged
 * until poll has returned the request's result. */
int cwb_server_submit(cwb_server* s, const cwb_problem* pr, uint64_t* ticket);
/* CWB_E_AGAIN while pending; else fills `res` and, if the pointers are not
 * NULL, the training predictions (n floats) and k trace (M ints). */
int cwb_server_poll(cwb_server* s, uint64_t ticket, cwb_result* res, float* pred_out,
                    int32_t* k_out);
int cwb_server_stats(cwb_server* s, cwb_stats* st);
/* Stop accepting, finish in-flight work, join the thread. */
void cwb_server_destroy(cwb_server* s);

#ifdef __cplusplus
}
#endif
#endif /* CWB_H_ */
