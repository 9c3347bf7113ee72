/*
 * boruta_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-definition CPU reference of one Boruta feature
 * selection run (Boruta main loop, Algorithm 1; impurity importance,
 * Algorithm 2 of Sec. 2.1; out-of-bag permutation importance in Kursa's
 * sense, Sec. 2), written to check the HIP implementation against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header or constant table with the GPU
 * library; both are written independently from the same stated definitions.
 *
 * All functions are thread-safe; none keeps global state.  Return codes:
 * 0 ok, -1 invalid argument, -2 non-finite value in X.
 */
#ifndef BORUTA_ORACLE_H
#define BORUTA_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-iteration record handed to a trace callback (host memory, valid only
 * during the call).  Nodes are listed in (tree, heap id) order. */
typedef struct {
    int32_t t;              /* iteration, 1-based                                  */
    int32_t p_cur;          /* active original columns (state >= 0)                */
    int32_t n_sha;          /* shadow columns                                      */
    int32_t p_w;            /* widened width p_cur + n_sha                         */
    int32_t mtry;           /* features drawn per node this iteration              */
    int32_t n_trees;        /* trees grown (all, or the requested subset)          */
    const int32_t* col_src; /* [p_w] original feature index behind widened column  */
    const int64_t* imp_int; /* [p_w] integer importance: TreeImp sum of per-tree
                               fixed-point shares, Permut accuracy-drop count, or
                               (mode 2) the sum over rows of the KL divergence in
                               bits with 32 fractional bits                        */
    const int32_t* hits;    /* [p] hit counts after this iteration                 */
    const int8_t* state;    /* [p] decisions after this iteration                  */
    const int64_t* tree_stats; /* [n_trees][5]: tree id, distinct in-bag rows,
                                  OOB rows, OOB correct, node count               */
    int64_t n_nodes;
    const int64_t* nodes;   /* [n_nodes][6]: tree, heap id, feature (-1 = leaf),
                               threshold bin (leaf: predicted class), weighted
                               count N, Gini decrease in 2^-32 units (0 leaf)      */
} oracle_iter_trace;

typedef void (*oracle_trace_fn)(void* user, const oracle_iter_trace* tr);

/* Philox4x32-10 block function: out = Philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Keyed bijection of [0, m) (Feistel over Philox, cycle walking). */
uint64_t oracle_keyed_perm(uint64_t seed, uint32_t stream, uint32_t t, uint32_t a,
                           uint32_t b, uint32_t c_hi, uint64_t m, uint64_t x);

/* Quantile binning of row-major X[n][p] into column-major bins[p][n]. */
int oracle_bin(const float* X, int64_t n, int64_t p, int32_t n_bins,
               uint8_t* bins_out, float* cuts_out /* [p][n_bins-1], nullable */,
               int32_t* ncuts_out /* [p], nullable */);

/* Bootstrap multiplicities of tree `tree` at iteration t: w_out[n]. */
void oracle_bootstrap(uint64_t seed, uint32_t t, uint32_t tree, int64_t n, uint32_t* w_out);

/* Best split of one node (exact rule, draw-order tie-break).  rows: the
 * node's distinct rows ascending; w: per-row multiplicity (indexed by row);
 * feats: candidate widened columns in draw order.  bins column-major
 * [p_w][n].  Writes {found, q, b, N_L, S_L, N_R, S_R, gain_fix} to out[8]
 * (found = 1 iff a valid candidate with strictly positive gain exists; q is
 * the position in feats; gain_fix = floor(2^32 * Gini decrease)). */
int oracle_best_split(const uint8_t* bins, int64_t n, const int32_t* y,
                      const uint32_t* w, const uint32_t* rows, int64_t n_rows,
                      const int32_t* feats, int32_t n_feats, int32_t n_classes,
                      int32_t n_bins, uint64_t out[8]);

/* Grow one tree on explicit binned data with explicit multiplicities w[n]
 * (rows with w = 0 are out of bag).  Feature draws use the MTRY stream
 * keyed by (seed, t, tree, heap id) over [0, p_w).  Writes up to
 * max_nodes rows of 6 int64 like oracle_iter_trace.nodes; returns the node
 * count (or a negative error).  gain_sum_out[p_w] (nullable) receives the
 * per-feature sum of fixed-point Gini decreases. */
int64_t oracle_grow_tree(const uint8_t* bins, int64_t n, int64_t p_w, const int32_t* y,
                         const uint32_t* w, int32_t n_classes, int32_t n_bins,
                         int32_t max_depth, int32_t mtry, uint64_t seed, uint32_t t,
                         uint32_t tree, int64_t* nodes_out, int64_t max_nodes,
                         uint64_t* gain_sum_out);

/* Exact Bonferroni binomial decision for one feature: returns 1 (confirm),
 * -1 (reject) or 0, for `hits` hits in t trials, p features, level alpha. */
int oracle_binom_decide(int32_t hits, int32_t t, int64_t p, double alpha);

/* 2^32 log2(x) by the squaring digit method (x >= 1; 0 for x = 0), and the
 * fixed-point KL divergence of mode 2 for K-class summed probabilities. */
uint64_t oracle_log2_fix32(uint64_t x);
int64_t oracle_kl_fix32(const uint64_t* S, const uint64_t* Sq, int32_t K);

/* Full run.  mode 0 = TreeImp, 1 = Permut (OOB accuracy drop), 2 = Algorithm
 * 3's prediction divergence (KL, full training matrix, one shared row
 * permutation per iteration).  n_threads 0 = all cores.
 * permut_naive = 1 re-traverses every (tree, column, replica, OOB row) in
 * full instead of only the columns on the row's path (same integers).
 * imp_history_out is [max_iter][p]; rows past n_iter are left untouched. */
int oracle_boruta_fit(const float* X, const int32_t* y, int64_t n, int64_t p,
                      int32_t n_classes, int32_t n_trees, int32_t max_depth,
                      int32_t mtry, int32_t importance_mode, int32_t max_iter,
                      double alpha, uint64_t seed, int32_t n_bins, int32_t n_perm,
                      int32_t n_threads, int32_t permut_naive,
                      int8_t* decision_out, double* imp_history_out,
                      int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out,
                      oracle_trace_fn trace, void* trace_user);

/* Algorithm 1's final ranking from a run's decision and history: 1
 * confirmed, 2 undecided, rejected from 3 by descending mean historical
 * importance (ties share a rank). */
void oracle_rank(const int8_t* decision, const double* imp_history, int64_t p, int32_t n_iter,
                 int32_t* rank_out);

/* One iteration t from a given (state, hits): the state machine of Algorithm
 * 1 is memoryless apart from these two vectors, so any iteration of a run
 * can be recomputed alone.  state/hits are updated in place.  tree_subset
 * (nullable) restricts growth to the listed trees; importances, hits and
 * the decision are then left untouched and only the trace's trees are
 * meaningful.  imp_row_out[p] / shadow_max_out[1] are nullable. */
int oracle_boruta_step(const float* X, const int32_t* y, int64_t n, int64_t p,
                       int32_t n_classes, int32_t n_trees, int32_t max_depth,
                       int32_t mtry, int32_t importance_mode, double alpha,
                       uint64_t seed, int32_t n_bins, int32_t n_perm, int32_t t,
                       int8_t* state, int32_t* hits, const int32_t* tree_subset,
                       int32_t n_subset, int32_t n_threads, int32_t permut_naive,
                       double* imp_row_out, double* shadow_max_out,
                       oracle_trace_fn trace, void* trace_user);

/* oracle_boruta_fit with the two options outside Algorithm 1 (from Kursa's
 * Boruta): perc in [1, 100] makes the hit threshold the perc-th percentile of
 * the shadow importances (nearest rank: the ceil(perc m / 100)-th smallest of
 * m; 100 = the maximum), and rough = 1 resolves the features still tentative
 * after the last iteration by oracle_rough_fix.  Returns -1 for perc or rough
 * out of range. */
int oracle_boruta_fit_ext(const float* X, const int32_t* y, int64_t n, int64_t p,
                          int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                          int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                          int32_t n_bins, int32_t n_perm, int32_t n_threads,
                          int32_t permut_naive, int32_t perc, int32_t rough,
                          int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                          double* shadow_max_out, int32_t* n_iter_out, oracle_trace_fn trace,
                          void* trace_user);

/* Regression Boruta (the paper's regression experiments run Boruta on a
 * random-forest regressor with squared-error loss): y [n] float32 targets,
 * finite (else -2).  Each target is held exactly as the integer
 * y_fix = rint(y 2^(38 - e)), e the smallest integer with every |y| < 2^e
 * (oracle_fix_targets).  A node with bootstrap weights w has W = sum w and
 * T = sum w y_fix; the split maximises T_L^2/W_L + T_R^2/W_R exactly (ties
 * to the earlier draw, then the smaller bin) and needs a strictly positive
 * decrease D = (T_L W - T W_L)^2 / (W_L W_R W); Algorithm 2 accumulates
 * floor(D / 2^s_gain).  A leaf predicts floor(T / W).  importance_mode 0
 * (TreeImp), 1 (Permut: a row scores floor((y_fix - pred)^2 / 2^s_perm); a
 * column's drop is the increase of the OOB rows' summed score under the
 * permutation, reported per OOB row and replica in squared target units) or
 * 2 (Algorithm 3: a row scores floor(Dsum^2 / (n_trees^2 2^s_kl)), Dsum the
 * change of its summed leaf predictions under the shared row permutation,
 * summed over rows and reported per row in squared target units).  The
 * shifts keep every sum within 64 bits (see oracle_fix_targets).  The
 * trace's node columns hold W as the weighted count and, for a leaf, its
 * prediction floor(T / W); its OOB-correct count is 0.  Other outputs as
 * oracle_boruta_fit. */
int oracle_boruta_fit_reg(const float* X, const float* y, int64_t n, int64_t p,
                          int32_t n_trees, int32_t max_depth, int32_t mtry,
                          int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                          int32_t n_bins, int32_t n_perm, int32_t n_threads,
                          int32_t permut_naive, int8_t* decision_out, double* imp_history_out,
                          int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out,
                          oracle_trace_fn trace, void* trace_user);

/* Fixed-point targets yfix_out[n] and the scale exponent e (returned); with
 * R = max y_fix - min y_fix, shifts_out (nullable) = s_gain = max(0, bits(n) +
 * 2 bits(R) - 64), s_perm = max(0, bits(n_trees n_perm n) + 2 bits(R + 1) -
 * 63), s_kl = max(0, bits(n) + 2 bits(R + 1) - 63), and R. */
int32_t oracle_fix_targets(const float* y, int64_t n, int32_t n_trees, int32_t n_perm,
                           int64_t* yfix_out, int64_t* shifts_out);

/* The regression split search of one node with fixed-point targets yfix:
 * out = found, draw position, bin, W_L, W_R, T_L, T_R, floor(D / 2^s_gain). */
int oracle_best_split_reg(const uint8_t* bins, int64_t n, const int64_t* yfix, const uint32_t* w,
                          const uint32_t* rows, int64_t n_rows, const int32_t* feats,
                          int32_t n_feats, int32_t n_bins, int32_t s_gain, int64_t out[8]);

/* Hit threshold over m >= 1 shadow importances at percentile perc (above). */
int64_t oracle_shadow_threshold(const int64_t* sha, int32_t m, int32_t perc);

/* Rough fix in place: each decision[j] == 0 becomes 1 when the median of
 * imp_history[t][j] over t < n_iter exceeds the median of shadow_max[t] over
 * t < n_iter, else -1 (medians of an even count: mean of the two middle
 * values).  n_iter == 0 changes nothing. */
void oracle_rough_fix(int8_t* decision, const double* imp_history, const double* shadow_max,
                      int64_t p, int32_t n_iter);

/* Multi-seed aggregate of n_runs finished runs of one problem: decisions
 * [n_runs][p], histories [n_runs][max_iter][p], n_iters [n_runs]; per
 * feature the median over runs of its mean history importance and the lower
 * median of its decisions. */
void oracle_seed_median(const int8_t* decisions, const double* histories, const int32_t* n_iters,
                        int64_t p, int32_t max_iter, int32_t n_runs, double* median_out,
                        int8_t* decision_out);

/* oracle_boruta_step with, for importance mode 2, only the listed widened
 * columns scored (the others read 0; hits and decisions are then
 * meaningless): checks of sampled columns at full size. */
int oracle_boruta_step_cols(const float* X, const int32_t* y, int64_t n, int64_t p,
                            int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                            int32_t importance_mode, double alpha, uint64_t seed, int32_t n_bins,
                            int32_t n_perm, int32_t t, int8_t* state, int32_t* hits,
                            const int32_t* tree_subset, int32_t n_subset, const int32_t* kl_cols,
                            int32_t n_kl_cols, int32_t n_threads, int32_t permut_naive,
                            double* imp_row_out, double* shadow_max_out, oracle_trace_fn trace,
                            void* trace_user);

#ifdef __cplusplus
}
#endif
#endif
