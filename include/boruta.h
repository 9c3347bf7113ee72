/*
 * boruta.h -- C ABI of libboruta.so, a HIP (gfx950) implementation of the
 * Boruta feature-selection loop with GPU random forests, after
 * "Novel GPU Boruta algorithms for feature selection from high-dimensional
 * data" (arxiv 2605.09950).
 *
 * What one call computes (Algorithm 1, Sec. 2): starting from all features
 * undecided, each iteration t = 1, 2, ... while t <= max_iter and some
 * feature is undecided
 *   1. widens the quantile-binned matrix with shadow copies of the columns
 *      that are not rejected, doubled until there are at least five, each
 *      copy shuffled over the rows by its own keyed permutation;
 *   2. fits a random forest (bootstrap, per-node random feature draw, Gini
 *      split on bin thresholds) on the widened matrix;
 *   3. scores every widened column:
 *        TreeImp -- normalised mean impurity decrease (Algorithm 2, Sec. 2.1),
 *        Permut  -- out-of-bag accuracy drop when the column is permuted among
 *                   each tree's out-of-bag rows (Kursa's importance, Sec. 2;
 *                   permutation importance, Sec. 2.2);
 *        Permut-KL -- Algorithm 3: divergence (KL, bits) of the forest's
 *                   class probabilities on the full training matrix when the
 *                   column is permuted by one row permutation shared by all
 *                   columns, summed over the rows;
 *   4. adds a hit to each feature scoring strictly above the best shadow;
 *   5. confirms / rejects undecided features with a Bonferroni-corrected
 *      exact binomial test at level alpha;
 * and at the end ranks the features (Algorithm 1's final ranking; see
 * boruta_result.rank).
 * Results are a deterministic function of (inputs, seed, n_bins, n_perm):
 * identical across the plain and batched forms, the two split-ranking modes,
 * the launch tuning and batch composition (all scores are integers; hits
 * compare integers).
 *
 * Conventions: the caller owns every buffer; the library never frees caller
 * memory.  Entry points that allocate device memory (all but the ones given a
 * workspace) fail with BORUTA_E_OOM when the environment variable
 * BORUTA_FAIL_ALLOC is "1" (a hook for failure tests).  Host pointers unless stated otherwise.  All entry points are
 * blocking.  On error the return value is negative and boruta_last_error()
 * (thread-local) describes it; output buffers are then unspecified.
 */
#ifndef BORUTA_H
#define BORUTA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BORUTA_OK 0
#define BORUTA_E_INVALID_ARG -1 /* argument outside the ranges listed below           */
#define BORUTA_E_NONFINITE -2   /* NaN or Inf in X                                      */
#define BORUTA_E_OOM -3         /* device allocation failed or workspace too small      */
#define BORUTA_E_DEVICE -4      /* HIP runtime error or internal capacity check failed */
#define BORUTA_E_UNSUPPORTED -5 /* no usable gfx950 device                              */

enum { BORUTA_TREEIMP = 0, BORUTA_PERMUT = 1, BORUTA_PERMUT_KL = 2 };
enum { BORUTA_REJECTED = -1, BORUTA_TENTATIVE = 0, BORUTA_CONFIRMED = 1 };
enum { BORUTA_FORM_PLAIN = 0, BORUTA_FORM_BATCHED = 1 };
enum { BORUTA_RANK_EXACT = 0, BORUTA_RANK_FP32 = 1 };

/* Per-iteration record for the optional trace callback (host memory, valid
 * only during the call).  Nodes are listed in (tree, heap id) order; heap id
 * of the root is 1 and the children of h are 2h (left) and 2h+1. */
typedef struct {
    int32_t job;            /* index of the job in the batch (0 for boruta_fit)  */
    int32_t t;              /* iteration, 1-based                                */
    int32_t p_cur;          /* active original columns (state >= 0)              */
    int32_t n_sha;          /* shadow columns                                    */
    int32_t p_w;            /* widened width p_cur + n_sha                       */
    int32_t mtry;           /* features drawn per node this iteration            */
    int32_t n_trees;
    const int32_t* col_src; /* [p_w] original feature behind each widened column  */
    const int64_t* imp_int; /* [p_w] integer importance (see boruta_fit)         */
    const int32_t* hits;    /* [p] after this iteration                          */
    const int8_t* state;    /* [p] after this iteration's decision               */
    const int64_t* tree_stats; /* [n_trees][5]: tree, distinct in-bag rows, OOB
                                  rows, OOB correct (Permut only, else 0), nodes */
    int64_t n_nodes;
    const int64_t* nodes;   /* [n_nodes][6]: tree, heap id, widened feature (-1
                               leaf), threshold bin (leaf: class), weighted
                               count, Gini decrease in 2^-32 units (0 leaf)     */
} boruta_iter_trace;

typedef void (*boruta_trace_fn)(void* user, const boruta_iter_trace* tr);

/* Kernel timing of the dominant kernels, filled when boruta_options.stats is
 * non-null (times from HIP events recorded on the library's stream around
 * every launch of the kernel, so they include no host gaps). */
typedef struct {
    int64_t launches;       /* launches of the kernel                               */
    double ms;              /* summed event time                                    */
    double alg_bytes;       /* algorithmic bytes: sum over searched nodes of
                               rows x (features drawn + 6)                          */
} boruta_kernel_stat;

typedef struct {
    boruta_kernel_stat hist_large; /* node histogram + split scan, > 64 rows      */
    boruta_kernel_stat hist_small; /* wave-per-node split search, <= 64 rows      */
    boruta_kernel_stat finalize;   /* split choice + row partition, > 64 rows     */
    boruta_kernel_stat permut;     /* re-routing for the permutation importances  */
    double iter_ms;                /* device time of all iterations               */
    int64_t iterations;            /* job-iterations run                          */
    int64_t nodes;                 /* tree nodes grown                            */
    int64_t level_small[32];       /* nodes searched by the wave path, per depth  */
    int64_t level_large[32];       /* nodes searched by the tiled path, per depth */
    boruta_kernel_stat hist_col;   /* column-major histogram + split scan (levels
                                      >= col_level; hist_large covers the others) */
    double permut_visits;          /* tree nodes visited by the out-of-bag walks of
                                      Permut (base paths and re-routings)          */
} boruta_stats;

typedef struct {
    int32_t n_bins;       /* quantile bins, [2, 256]; default 256                  */
    int32_t n_perm;       /* Permut replicas per column, [1, 65535]; default 1     */
    int32_t split_rank;   /* BORUTA_RANK_EXACT or BORUTA_RANK_FP32 (FP32 ranking
                             with an exact recheck near the maximum); default FP32 */
    int32_t form;         /* BORUTA_FORM_PLAIN (one launch per tree node) or
                             BORUTA_FORM_BATCHED (all nodes of a tree level of all
                             trees and jobs per launch); default BATCHED           */
    int32_t graph;        /* batched form: 1 = capture one iteration's launch
                             sequence as a HIP graph on the first step and replay
                             it on every later step, 0 = launch eagerly; default 1.
                             Ignored (eager) when stats is set: kernel timing
                             needs events around every launch.  Results are
                             identical either way.                                 */
    /* Launch tuning (batched form; every choice gives identical results;
     * 0 = the library's default).                                                 */
    int32_t small_rows;   /* nodes with at most this many distinct rows (and a
                             weighted count below the packed-counter limit) take
                             the wavefront path, [2, 64]; default 32              */
    /* "needed" below: for the nodes tree level d can hold, at most the
     * plan's capacity and n_trees * 2^d; a chosen grid size is an upper
     * limit, lowered to what a level needs.                                */
    int32_t grid_small;   /* workgroups of the wavefront-path launch (4 nodes
                             each, grid-stride); default min(4096, needed)       */
    int32_t grid_hist;    /* workgroups of the histogram launch (4 items each),
                             rounded up to a multiple of 8; default
                             min(16384, needed)                                  */
    int32_t grid_finalize;/* workgroups of the split/partition launch (4 nodes
                             each, grid-stride); default min(4096, needed)       */
    int32_t col_level;    /* large nodes of tree levels >= col_level take the
                             column-major histogram path (items bucketed by bin
                             column, each column staged once per unit in LDS);
                             [1, 64], 64 = never; 0 (default) = automatic: level
                             5 when some job's widened bin matrix (2p columns of
                             n rounded up to 256 bytes) exceeds 128 MiB, else
                             never.  The path needs a whole bin column plus two
                             histograms in one workgroup's LDS; where it does
                             not fit, every level stays node-major.              */
    int32_t col_unit;     /* items (node, draw) per unit of that path, [1, 65536];
                             default 2048                                         */
    int32_t grid_col;     /* workgroups of its histogram launch (one unit at a
                             time, grid-stride); default min(2048, needed)      */
    int32_t kl_rows;      /* BORUTA_PERMUT_KL: rows per block of the divergence
                             step (its per-(column, row, class) buffer is sized
                             for one block), >= 0; default (0): as many rows as
                             keep that buffer within 256 MiB                     */
    /* Two options outside Algorithm 1, from Kursa's Boruta; the defaults keep
     * Algorithm 1 as written.                                                     */
    int32_t perc;         /* hit threshold: the perc-th percentile of the
                             iteration's shadow importances by the nearest-rank
                             rule (the ceil(perc n_sha / 100)-th smallest of the
                             n_sha shadows), [1, 100]; 0 or 100 (default) = the
                             maximum.  shadow_max reports this threshold.       */
    int32_t rough_fix;    /* 1: a feature still tentative when the results are
                             read is reported confirmed if the median of its
                             history entries exceeds the median of the shadow
                             thresholds of the same iterations, else rejected
                             (medians of an even count: mean of the middle two).
                             Only the reported decision and rank change; a
                             session's own state does not.  Default 0.          */
    boruta_trace_fn trace;/* nullable                                              */
    void* trace_user;
    boruta_stats* stats;  /* nullable                                              */
    /* Histogram shapes (launch tuning: every choice gives identical results). */
    int32_t hist_rb;      /* rows per lane per batch of the node-major histogram
                             kernel at tree levels below band_level (larger
                             nodes): 4, 8 or 16; default 8                        */
    int32_t hist_rb_deep; /* the same from band_level on; default 8                */
    int32_t band_level;   /* first tree level of the deep band, [1, 64]; default 6 */
    int32_t hist_fw;      /* drawn features per node-major histogram item: 0
                             (default: 2 for two classes, else 1), 1, 2 or 4;
                             reduced to at most 8 class rows of LDS per wavefront,
                             raised to 768 LDS words per wavefront for a batch
                             with a regression job, and 1 whenever the plan has
                             column-major levels                                  */
    int32_t col_waves;    /* wavefronts per workgroup of the column-major kernel,
                             [2, 16]; 0 (default) = as many as its LDS holds      */
    const char* tune_cache; /* nullable: path of a tuning cache written by the
                             project's autotuner (one line per workload: its
                             signature "B<bins>|R<replicas>" followed, per job, by
                             "|<n>x<p>K<classes or reg>T<trees>D<depth>m<mtry>
                             i<mode>", a tab, then "key=value" pairs separated
                             by spaces, keys among the launch tuning fields
                             above).  The entry of this call's workload sets every
                             tuning field left at its default; a missing file or
                             signature changes nothing.                           */
} boruta_options;

/* Fills *opt with the defaults above. */
void boruta_default_options(boruta_options* opt);

/* One Boruta run (Algorithm 1).
 *   X          [n][p] row-major float32, finite.  n in [2, 2^24], p in [1, 2^24].
 *   y          [n] class labels in [0, n_classes), n_classes in [2, 16].
 *   n_trees    [1, 65535]; max_depth in [1, 30] (root = depth 0).
 *   mtry       features drawn per node; 0 = floor(sqrt(p_w)) recomputed each
 *              iteration, otherwise min(mtry, p_w).
 *   importance_mode  BORUTA_TREEIMP (impurity decrease, Algorithm 2),
 *              BORUTA_PERMUT (out-of-bag accuracy drop under a column
 *              permutation per tree, Kursa's importance, Sec. 2) or
 *              BORUTA_PERMUT_KL (Algorithm 3: one row permutation per
 *              iteration shared by all columns, the forest's class
 *              probabilities on the full training matrix, KL divergence of
 *              the unpermuted from the permuted prediction).
 *   max_iter   [1, 1000]; alpha in (0, 0.5); seed keys every random draw.
 * Outputs (caller-allocated):
 *   decision_out    [p]  -1 rejected / 0 tentative / 1 confirmed.
 *   imp_history_out [max_iter][p]: row t-1 = reported importance of each
 *                   feature at iteration t (TreeImp: its share of the
 *                   renormalised impurity importance over all widened
 *                   columns; Permut: accuracy drop / (n_perm x OOB rows of
 *                   all trees); Permut-KL: mean divergence per row in bits),
 *                   NaN for features rejected before t; rows
 *                   at and past n_iter are left untouched.
 *   hits_out [p], shadow_max_out [max_iter]: nullable.
 *   n_iter_out      iterations run. */
int boruta_fit(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
               int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
               int32_t max_iter, double alpha, uint64_t seed, int8_t* decision_out,
               double* imp_history_out, int32_t* hits_out, double* shadow_max_out,
               int32_t* n_iter_out);

/* boruta_fit with options (opt nullable = defaults). */
int boruta_fit_ex(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                  int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                  int32_t max_iter, double alpha, uint64_t seed, const boruta_options* opt,
                  int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                  double* shadow_max_out, int32_t* n_iter_out);

/* Regression Boruta (the paper's regression experiments run Boruta on a
 * random-forest regressor with squared-error loss, Sec. 2.2 and Sec. 3):
 * importance_mode 0 (TreeImp), 1 (Permut) or 2 (Algorithm 3).  y: [n] float32
 * targets, finite (non-finite X or y: BORUTA_E_NONFINITE); n in [2, 2^24].
 * Each target is held exactly as the integer y_fix = rint(y 2^(38 - e)), e the
 * smallest integer with every |y| < 2^e (exact for |y| >= 2^(e - 15)).  A node
 * with bootstrap weights w has W = sum w and T = sum w y_fix; a split
 * maximises T_L^2/W_L + T_R^2/W_R exactly (ties to the earlier draw, then the
 * smaller bin) and needs a strictly positive decrease
 * D = (T_L W - T W_L)^2 / (W_L W_R W); Algorithm 2 accumulates
 * floor(D / 2^s_gain).  A leaf predicts floor(T / W).  Permut: a row scores
 * floor((y_fix - pred)^2 / 2^s_perm) and a column's drop is the increase of
 * the out-of-bag rows' summed score under its permutation, reported per OOB
 * row and replica in squared target units.  Algorithm 3: a row scores
 * floor(Dsum^2 / (n_trees^2 2^s_kl)), Dsum the change of its summed leaf
 * predictions under the iteration's shared row permutation, reported per row
 * in squared target units.  With R the range of y_fix, s_gain =
 * max(0, bits(n) + 2 bits(R) - 64), s_perm = max(0, bits(n_trees n_perm n) +
 * 2 bits(R + 1) - 63) and s_kl = max(0, bits(n) + 2 bits(R + 1) - 63) keep
 * every sum within 64 bits.  Arguments and outputs otherwise as boruta_fit_ex;
 * in a trace a node's weighted count is W, a leaf's class column holds its
 * prediction floor(T / W), and the OOB-correct count is 0.  Regression nodes
 * always take the histogram path (small_rows does not apply), and a batch
 * with a regression job keeps every tree level node-major (col_level does not
 * apply). */
int boruta_fit_regression(const float* X, const float* y, int64_t n, int64_t p, int32_t n_trees,
                          int32_t max_depth, int32_t mtry, int32_t importance_mode,
                          int32_t max_iter, double alpha, uint64_t seed, const boruta_options* opt,
                          int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                          double* shadow_max_out, int32_t* n_iter_out);

/* One job of a batch: the problem arguments of boruta_fit.  With y_reg set
 * the job is a regression job as in boruta_fit_regression: y_reg holds its
 * [n] float targets (host or device like X), y and n_classes are ignored. */
typedef struct {
    const float* X;
    const int32_t* y;
    int64_t n, p;
    int32_t n_classes, n_trees, max_depth, mtry, importance_mode, max_iter;
    double alpha;
    uint64_t seed;
    const float* y_reg;  /* nullable */
} boruta_job;

/* Caller-allocated outputs of one job (same meaning as boruta_fit). */
typedef struct {
    int8_t* decision;
    double* imp_history;
    int32_t* hits;       /* nullable */
    double* shadow_max;  /* nullable */
    int32_t* rank;       /* nullable: [p] Algorithm 1's final ranking -- 1 confirmed,
                            2 undecided, rejected features from 3 by descending
                            historical importance (mean of their history entries;
                            equal means share a rank).  After boruta_session_resume
                            the history counted starts at the resume point. */
    int32_t n_iter;      /* out */
    int32_t status;      /* out: BORUTA_OK or the job's own error code */
} boruta_result;

/* Many independent runs advanced together: every launch of an iteration step
 * covers the live jobs' trees and nodes.  Each job keeps its own seed, so its
 * results equal a boruta_fit of that job alone.  Returns the first error. */
int boruta_fit_batch(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                     boruta_result* results);

/* The repeated-seed protocol of the experiments (Results and Discussion,
 * Synthetic experiments and Experiments on Public Datasets: every method is
 * run with several random seeds and the median importance decides): one
 * problem run once per entry of seeds[n_seeds] (1..64 seeds), all runs
 * advanced together as one batch, each equal to a boruta_fit with that seed.
 * On the device, per feature j:
 *   median_importance_out[j] = median over the runs of the mean of the run's
 *     non-NaN history entries for j (0 if it has none); with an even count,
 *     the mean of the two middle values;
 *   decision_out[j] = the lower median of the runs' decisions (-1 < 0 < 1),
 *     i.e. confirmed only if more than half of the runs confirm it, rejected
 *     if at least half reject it.
 * Both are host arrays of p entries.  results (nullable) is an array of
 * n_seeds per-run outputs as for boruta_fit_batch; where its decision and
 * imp_history are set they receive the runs' own results.  Returns
 * BORUTA_E_INVALID_ARG for a missing output or a seed count out of range, or
 * the first run's error. */
int boruta_fit_seeds(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                     int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                     int32_t max_iter, double alpha, const uint64_t* seeds, int32_t n_seeds,
                     const boruta_options* opt, double* median_importance_out,
                     int8_t* decision_out, boruta_result* results);

/* boruta_fit_seeds for a regression problem (float targets y, as in
 * boruta_fit_regression). */
int boruta_fit_seeds_regression(const float* X, const float* y, int64_t n, int64_t p,
                                int32_t n_trees, int32_t max_depth, int32_t mtry,
                                int32_t importance_mode, int32_t max_iter, double alpha,
                                const uint64_t* seeds, int32_t n_seeds,
                                const boruta_options* opt, double* median_importance_out,
                                int8_t* decision_out, boruta_result* results);

/* Device bytes a call with these jobs needs (for boruta_fit_device). */
int boruta_workspace_size(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                          size_t* bytes);

/* boruta_fit on device-resident inputs: dX [n][p] float32 and dy [n] int32 are
 * DEVICE pointers; workspace is a device buffer of at least the size that
 * boruta_workspace_size reports for this problem (256-byte aligned); all
 * work is ordered on hip_stream (a hipStream_t, nullable = default stream).
 * The library allocates no device memory in this call.  Outputs are host
 * pointers as in boruta_fit. */
int boruta_fit_device(const float* dX, const int32_t* dy, int64_t n, int64_t p,
                      int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                      int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                      const boruta_options* opt, void* workspace, size_t ws_bytes,
                      void* hip_stream, int8_t* decision_out, double* imp_history_out,
                      int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out);

/* boruta_fit_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument; the library's own device scratch array
 * of 64 MiB (a file-scope array that each GPU the library runs on holds until
 * the process ends) serves as the workspace, and the call makes no hipMalloc,
 * creates no stream, event or graph and launches eagerly on hip_stream
 * (nullable = the default stream).  dX [n][p] float32 and dy [n] int32 are
 * device pointers, outputs host pointers, as in boruta_fit_device; results are
 * identical to it.  A problem whose boruta_workspace_size exceeds 64 MiB
 * returns BORUTA_E_INVALID_ARG (with the sizes in boruta_last_error()), and
 * so do options with kernel statistics (they need HIP events).  Every call on
 * one GPU uses that GPU's one scratch array: calls that overlap on one GPU (from
 * several threads or streams) race and give undefined results.  The scratch
 * keeps the previous call's contents; the call initialises whatever it reads. */
int boruta_fit_device_noalloc(const float* dX, const int32_t* dy, int64_t n, int64_t p,
                              int32_t n_classes, int32_t n_trees, int32_t max_depth,
                              int32_t mtry, int32_t importance_mode, int32_t max_iter,
                              double alpha, uint64_t seed, const boruta_options* opt,
                              void* hip_stream, int8_t* decision_out, double* imp_history_out,
                              int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out);

/* Incremental form of the same computation: create a session (upload,
 * validation, binning, decision thresholds), then advance every live job
 * one Boruta iteration per boruta_session_step, read results at any time,
 * and continue a job from a checkpoint (t, state, hits) with
 * boruta_session_resume -- Algorithm 1 keeps no other state between
 * iterations, and every random draw is keyed by (seed, t, ...), so a resumed
 * job reproduces an uninterrupted one exactly.
 *   inputs_on_device: X/y of the jobs are device pointers (see
 *   boruta_fit_device); workspace (nullable = allocated by the library, else
 *   at least boruta_workspace_size bytes) and hip_stream as there.  The
 *   options' trace/stats targets must outlive the session.  Returns the
 *   first job's error if any job fails validation (no session then). */
typedef struct boruta_session boruta_session;
int boruta_session_create(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                          int32_t inputs_on_device, void* workspace, size_t ws_bytes,
                          void* hip_stream, boruta_session** out);
/* One iteration of every live job; *n_live_out (nullable) = jobs still live. */
int boruta_session_step(boruta_session* s, int32_t* n_live_out);
/* Up to max_steps iterations of every live job, as many boruta_session_step
 * calls would run them, with the same results; with graph replay (and no
 * trace or statistics) the iterations are enqueued back to back, without a
 * host wait between them, and a job that finishes on the way is skipped by
 * the later ones.  *n_live_out and *job_iterations_out (nullable) = jobs
 * still live and the job-iterations run. */
int boruta_session_run(boruta_session* s, int32_t max_steps, int32_t* n_live_out,
                       int64_t* job_iterations_out);
/* Current decision/history/hits/shadow maximum of one job (caller buffers as
 * in boruta_result; n_iter = iterations done so far). */
int boruta_session_result(boruta_session* s, int32_t job, boruta_result* out);
/* Set job's state after iteration t (0 <= t < max_iter): state[p] in
 * {-1,0,1}, hits[p] in [0, t].  The next step runs iteration t + 1;
 * history rows before t are the caller's. */
int boruta_session_resume(boruta_session* s, int32_t job, int32_t t, const int8_t* state,
                          const int32_t* hits);
void boruta_session_destroy(boruta_session* s);

/* Streaming copy of `bytes` bytes between device buffers (calibration of
 * hardware byte counters); returns BORUTA_OK or an error code. */
int boruta_probe_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* The binning step alone (the quantile bins that every run starts from):
 * X [n][p] float32 host, row-major; bins_out [p][n] uint8 host, column-major:
 * per column, the order statistics of rank ceil(k n / n_bins) - 1 (k = 1 ..
 * n_bins - 1) are candidate cuts, the strictly increasing distinct ones form
 * the cut list U, and x gets bin #{u in U : u < x}.  Runs on the device;
 * BORUTA_E_NONFINITE for NaN/Inf in X. */
int boruta_bin(const float* X, int64_t n, int64_t p, int32_t n_bins, uint8_t* bins_out);

/* Message of the last error on the calling thread ("" if none). */
const char* boruta_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
