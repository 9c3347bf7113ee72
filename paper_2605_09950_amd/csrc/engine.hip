// engine.hip -- host orchestration of the Boruta loop and the C ABI of
// libboruta.so.  Every step of an iteration runs in the HIP kernels of
// k_prep.hip, k_forest.hip and k_importance.hip; this file plans device
// memory and launches them in order on one stream.  An iteration is a fixed
// launch sequence sized by plan-time bounds (the kernels read their real
// work counts on the device), followed by one read-back of the job records
// and level counters.
#include <algorithm>
#include <climits>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <stdexcept>
#include <string>
#include <vector>

#include "boruta.h"
#include "dev_common.hpp"

namespace boruta {

// launchers (k_prep.hip)
void launch_validate(const float*, size_t, const int32_t*, size_t, int, uint32_t*, hipStream_t);
void launch_validate_reg(const float*, size_t, const float*, size_t, uint32_t*, hipStream_t);
void launch_target_range(const float*, size_t, float*, hipStream_t);
void launch_target_fix(const float*, size_t, int, int64_t*, hipStream_t);
void launch_labels(const int32_t*, size_t, uint8_t*, hipStream_t);
void launch_binning(const float*, int64_t, int64_t, int, uint8_t*, int64_t, uint32_t*, int64_t,
                    hipStream_t);
void launch_thresholds(int32_t, int64_t, uint64_t, int32_t, int32_t*, int32_t*, hipStream_t);
void launch_active(JobDev*, int, hipStream_t);
void launch_shadow(JobDev*, int, int64_t, int, hipStream_t);
void launch_rowmaj(JobDev*, int, int64_t, int, hipStream_t);
uint32_t prepare_boot_draw(int64_t);
void launch_boot_draw(JobDev*, const TreeDev*, int, int64_t, uint32_t, hipStream_t);
void launch_fill_u32(uint32_t*, size_t, uint32_t, hipStream_t);
// k_forest.hip
void launch_boot_compact(const ForestDev&, uint32_t, hipStream_t);
void launch_split_small(const ForestDev&, int, uint32_t, uint32_t, uint32_t, hipStream_t);
void launch_hist_tile(const ForestDev&, int, uint32_t, uint32_t, uint32_t, int, hipStream_t);
void launch_split_finalize(const ForestDev&, int, uint32_t, uint32_t, uint32_t, hipStream_t);
void launch_draws(const ForestDev&, int, uint32_t, hipStream_t);
void launch_lists(const ForestDev&, int, uint32_t, hipStream_t);
void launch_col_sort(const ForestDev&, int, uint32_t, hipStream_t);
size_t hist_col_lds(int, int, uint32_t);
hipError_t prepare_hist_col(int, size_t);
void launch_hist_col(const ForestDev&, int, uint32_t, int, uint32_t, hipStream_t);
// k_importance.hip
void launch_tree_totals(JobDev*, const TreeDev*, int, uint64_t*, hipStream_t);
void launch_treeimp(JobDev*, const TreeDev*, int, const uint64_t*, int, hipStream_t);
void launch_permut(JobDev*, const TreeDev*, const NodeDev*, const uint32_t*, int, int, int64_t,
                   int, int, bool, unsigned long long*, hipStream_t);
void launch_hits_decide(JobDev*, int, int, hipStream_t);
void launch_rough_fix(const int8_t*, const double*, const double*, int64_t, int, int, int8_t*,
                      hipStream_t);
void launch_kl_block(JobDev*, int, const NodeDev*, const uint32_t*, int, uint32_t, int, int,
                     uint32_t, uint32_t, uint64_t*, uint32_t*, unsigned long long*, int,
                     hipStream_t);
void launch_copy(void*, const void*, size_t, hipStream_t);
void launch_ctr_sticky(LevelCtr*, int, hipStream_t);
void launch_seed_median(const JobDev*, const int8_t* const*, int, int64_t, double*, int8_t*,
                        hipStream_t);
void launch_rank(const int8_t*, const double*, int64_t, int, int, double*, int32_t*, hipStream_t);

namespace {

thread_local std::string g_err;

// LDS a gfx950 workgroup may allocate (checked against the device at set-up).
constexpr size_t kLdsPerWorkgroup = 160 * 1024;
// Column-major histogram path: the first tree level it serves when chosen
// automatically, the widened bin matrix of one job above which it is chosen
// (such a matrix no longer stays in the 256 MB last-level cache beside the
// row records, so node-major gathers pull whole lines from HBM), and the
// value that disables it.
constexpr int kColLevelAuto = 5;
constexpr size_t kColAutoBytes = size_t(128) << 20;
constexpr int kColNever = 64;
// KL importance: bound of its per-block difference buffer.
constexpr uint64_t kKlDeltaBytes = uint64_t(256) << 20;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPC(x)                                                                          \
    do {                                                                                 \
        const hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess)                                                            \
            throw Error(BORUTA_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Spec {
    const float* X;
    const int32_t* y;
    int64_t n, p;
    int K, T, D, mtry, mode, max_iter;
    double alpha;
    uint64_t seed;
    // regression: float targets [n] (y is null and K = 2: a node's weighted
    // target sum T is kept in its two class words); null for classification
    const float* yr = nullptr;
    // an earlier job of the same batch with the same inputs (X, y, n, p, K):
    // its input copy, labels and binned matrix serve this job too (-1: none)
    int share = -1;
};

// Jobs of one batch that pass the same input arrays (several seeds of one
// problem) are binned once.
void mark_shared_inputs(std::vector<Spec>& specs) {
    for (size_t j = 0; j < specs.size(); ++j) {
        specs[j].share = -1;
        for (size_t i = 0; i < j; ++i) {
            const Spec &a = specs[i], &b = specs[j];
            if (a.share < 0 && a.X == b.X && a.y == b.y && a.yr == b.yr && a.n == b.n &&
                a.p == b.p && a.K == b.K) {
                specs[j].share = (int)i;
                break;
            }
        }
    }
}

struct Opts {
    int B = 256, R = 1, split_rank = 1, form = 1, graph = 1;
    int small_rows = 32, grid_small = 0, grid_hist = 0, grid_finalize = 0;
    int col_level = 0, col_unit = 2048, grid_col = 0, kl_rows = 0;
    int perc = 100, rough_fix = 0;
    // histogram shapes: rows per lane per batch of the node-major kernel before
    // and from band_level on, its draws per item, and the waves per workgroup
    // of the column-major kernel (0 = the library's choice)
    int hist_rb = 8, hist_rb_deep = 8, band_level = 6, hist_fw = 0, col_waves = 0;
    // allocation-free calls: no second stream, no events, no graph
    bool no_alloc = false;
    boruta_trace_fn trace = nullptr;
    void* trace_user = nullptr;
    boruta_stats* stats = nullptr;
};

Opts read_opts(const boruta_options* o) {
    Opts r;
    if (o) {
        r.B = o->n_bins;
        r.R = o->n_perm;
        r.split_rank = o->split_rank;
        r.form = o->form;
        r.graph = o->graph;
        if (o->small_rows) r.small_rows = o->small_rows;
        r.grid_small = o->grid_small;
        r.grid_hist = o->grid_hist;
        r.grid_finalize = o->grid_finalize;
        if (o->col_level) r.col_level = o->col_level;
        if (o->col_unit) r.col_unit = o->col_unit;
        r.grid_col = o->grid_col;
        r.kl_rows = o->kl_rows;
        if (o->perc) r.perc = o->perc;
        r.rough_fix = o->rough_fix;
        if (o->hist_rb) r.hist_rb = o->hist_rb;
        if (o->hist_rb_deep) r.hist_rb_deep = o->hist_rb_deep;
        if (o->band_level) r.band_level = o->band_level;
        r.hist_fw = o->hist_fw;
        r.col_waves = o->col_waves;
        r.trace = o->trace;
        r.trace_user = o->trace_user;
        r.stats = o->stats;
    }
    if (r.B < 2 || r.B > 256) throw Error(BORUTA_E_INVALID_ARG, "n_bins outside [2, 256]");
    if (r.R < 1 || r.R > 65535) throw Error(BORUTA_E_INVALID_ARG, "n_perm outside [1, 65535]");
    if (r.split_rank != 0 && r.split_rank != 1)
        throw Error(BORUTA_E_INVALID_ARG, "split_rank must be 0 or 1");
    if (r.form != 0 && r.form != 1) throw Error(BORUTA_E_INVALID_ARG, "form must be 0 or 1");
    if (r.graph != 0 && r.graph != 1) throw Error(BORUTA_E_INVALID_ARG, "graph must be 0 or 1");
    if (r.small_rows < 2 || r.small_rows > kSmallRows)
        throw Error(BORUTA_E_INVALID_ARG, "small_rows outside [2, 64]");
    if (r.grid_small < 0 || r.grid_hist < 0 || r.grid_finalize < 0 || r.grid_small > 65536 ||
        r.grid_hist > 65536 || r.grid_finalize > 65536)
        throw Error(BORUTA_E_INVALID_ARG, "grid sizes outside [0, 65536]");
    if (r.col_level < 0 || r.col_level > kColNever)
        throw Error(BORUTA_E_INVALID_ARG, "col_level outside [0, 64]");
    if (r.col_unit < 1 || r.col_unit > 65536)
        throw Error(BORUTA_E_INVALID_ARG, "col_unit outside [1, 65536]");
    if (r.grid_col < 0 || r.grid_col > 65536)
        throw Error(BORUTA_E_INVALID_ARG, "grid_col outside [0, 65536]");
    if (r.kl_rows < 0) throw Error(BORUTA_E_INVALID_ARG, "kl_rows must be >= 0");
    if (r.perc < 1 || r.perc > 100) throw Error(BORUTA_E_INVALID_ARG, "perc outside [1, 100]");
    if (r.rough_fix != 0 && r.rough_fix != 1)
        throw Error(BORUTA_E_INVALID_ARG, "rough_fix must be 0 or 1");
    auto rb_ok = [](int v) { return v == 4 || v == 8 || v == 16; };
    if (!rb_ok(r.hist_rb) || !rb_ok(r.hist_rb_deep))
        throw Error(BORUTA_E_INVALID_ARG, "hist_rb and hist_rb_deep must be 4, 8 or 16");
    if (r.band_level < 1 || r.band_level > 64)
        throw Error(BORUTA_E_INVALID_ARG, "band_level outside [1, 64]");
    if (r.hist_fw != 0 && r.hist_fw != 1 && r.hist_fw != 2 && r.hist_fw != 4)
        throw Error(BORUTA_E_INVALID_ARG, "hist_fw must be 0, 1, 2 or 4");
    if (r.col_waves < 0 || r.col_waves > (int)kColWavesMax)
        throw Error(BORUTA_E_INVALID_ARG, "col_waves outside [0, 16]");
    return r;
}

// Workload signature of a tuning cache entry: "B<bins>|R<replicas>" and, per
// job, "|<n>x<p>K<classes or reg>T<trees>D<depth>m<mtry>i<mode>".
std::string tune_signature(const std::vector<Spec>& specs, const Opts& o) {
    std::string sig = "B" + std::to_string(o.B) + "|R" + std::to_string(o.R);
    for (const Spec& s : specs)
        sig += "|" + std::to_string(s.n) + "x" + std::to_string(s.p) + "K" +
               (s.yr ? std::string("reg") : std::to_string(s.K)) + "T" + std::to_string(s.T) +
               "D" + std::to_string(s.D) + "m" + std::to_string(s.mtry) + "i" +
               std::to_string(s.mode);
    return sig;
}

// The tuning cache's entry for this workload sets every launch tuning field
// that the caller left at its default (boruta_default_options); the values are
// validated as the caller's would be.  A missing file or signature changes
// nothing.
void apply_tune_cache(Opts& r, const boruta_options* o, const std::vector<Spec>& specs) {
    if (!o || !o->tune_cache) return;
    std::ifstream in(o->tune_cache);
    if (!in) return;
    const std::string sig = tune_signature(specs, r);
    boruta_options d;
    boruta_default_options(&d);
    std::string line;
    while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (line.empty() || line[0] == '#' || tab == std::string::npos) continue;
        if (line.compare(0, tab, sig) != 0 || tab != sig.size()) continue;
        std::istringstream kv(line.substr(tab + 1));
        std::string tok;
        while (kv >> tok) {
            const size_t eq = tok.find('=');
            if (eq == std::string::npos) continue;
            const std::string key = tok.substr(0, eq);
            int v = 0;
            try {
                v = std::stoi(tok.substr(eq + 1));
            } catch (...) {
                continue;
            }
            // a field the caller left at its default takes the cached value
#define BORUTA_TUNE_FIELD(name)                                        \
    if (key == #name) {                                                 \
        if (o->name == d.name) r.name = v;                              \
        continue;                                                       \
    }
            BORUTA_TUNE_FIELD(small_rows)
            BORUTA_TUNE_FIELD(grid_small)
            BORUTA_TUNE_FIELD(grid_hist)
            BORUTA_TUNE_FIELD(grid_finalize)
            BORUTA_TUNE_FIELD(col_level)
            BORUTA_TUNE_FIELD(col_unit)
            BORUTA_TUNE_FIELD(grid_col)
            BORUTA_TUNE_FIELD(kl_rows)
            BORUTA_TUNE_FIELD(hist_rb)
            BORUTA_TUNE_FIELD(hist_rb_deep)
            BORUTA_TUNE_FIELD(band_level)
            BORUTA_TUNE_FIELD(hist_fw)
            BORUTA_TUNE_FIELD(col_waves)
#undef BORUTA_TUNE_FIELD
        }
        break;
    }
    // a cached value must pass the checks the caller's value would
    boruta_options c = *o;
    c.small_rows = r.small_rows;
    c.grid_small = r.grid_small;
    c.grid_hist = r.grid_hist;
    c.grid_finalize = r.grid_finalize;
    c.col_level = r.col_level;
    c.col_unit = r.col_unit;
    c.grid_col = r.grid_col;
    c.kl_rows = r.kl_rows;
    c.hist_rb = r.hist_rb;
    c.hist_rb_deep = r.hist_rb_deep;
    c.band_level = r.band_level;
    c.hist_fw = r.hist_fw;
    c.col_waves = r.col_waves;
    c.tune_cache = nullptr;
    const Opts checked = read_opts(&c);
    const bool no_alloc = r.no_alloc;
    r = checked;
    r.no_alloc = no_alloc;
}

void check_spec(const Spec& s) {
    auto bad = [](const char* m) { throw Error(BORUTA_E_INVALID_ARG, m); };
    if (!s.X || (!s.y && !s.yr)) bad("X and y must be non-null");
    if (s.n < 2 || s.n > (int64_t(1) << 24)) bad("n outside [2, 2^24]");
    if (s.p < 1 || s.p > (int64_t(1) << 24)) bad("p outside [1, 2^24]");
    if (s.K < 2 || s.K > 16) bad("n_classes outside [2, 16]");
    if (s.T < 1 || s.T > 65535) bad("n_trees outside [1, 65535]");
    if (s.D < 1 || s.D > 30) bad("max_depth outside [1, 30]");
    if (s.mtry < 0) bad("mtry < 0");
    if (s.mode < 0 || s.mode > 2) bad("importance_mode must be 0, 1 or 2");
    if (s.max_iter < 1 || s.max_iter > 1000) bad("max_iter outside [1, 1000]");
    if (!(s.alpha > 0.0 && s.alpha < 0.5)) bad("alpha outside (0, 0.5)");
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int bit_len(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// Fixed-point scale of a regression job's float targets, from their minimum
// and maximum: e is the smallest integer with every |y| < 2^e and the
// targets are held as y_fix = rint(y 2^(38 - e)) (exact for |y| >= 2^(e-15));
// with R the range of y_fix, the split decreases, the Permut squared errors
// and the divergence scores are shifted right by s_gain, s_perm and s_kl bits
// so that a tree's decreases (at most n R^2 / 4), the n_trees n_perm n Permut
// terms and the n divergence terms (each at most (R + 1)^2) sum within 64 bits.
struct RegShift {
    int e = 0, s_gain = 0, s_perm = 0, s_kl = 0;
};

RegShift reg_shift(float lo, float hi, int64_t n, int T, int R) {
    RegShift r;
    const double m = std::max(std::fabs((double)lo), std::fabs((double)hi));
    if (m > 0.0) std::frexp(m, &r.e);
    const int64_t flo = (int64_t)std::rint(std::ldexp((double)lo, 38 - r.e));
    const int64_t fhi = (int64_t)std::rint(std::ldexp((double)hi, 38 - r.e));
    const uint64_t range = (uint64_t)(fhi - flo);
    r.s_gain = std::max(0, bit_len((uint64_t)n) + 2 * bit_len(range) - 64);
    r.s_perm = std::max(0, bit_len((uint64_t)T * (uint64_t)R * (uint64_t)n) +
                               2 * bit_len(range + 1) - 63);
    r.s_kl = std::max(0, bit_len((uint64_t)n) + 2 * bit_len(range + 1) - 63);
    return r;
}
int64_t pow2_at_least(int64_t v) {
    int64_t P = 1;
    while (P < v) P <<= 1;
    return P;
}
int isqrt_i(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (int)std::max<int64_t>(1, r);
}

// ---------------------------------------------------------------------------
// Device memory plan: one region, every buffer at a 256-byte aligned offset.
struct Region {
    size_t total = 0;
    size_t take(size_t bytes) {
        const size_t off = (total + 255) & ~size_t(255);
        total = off + std::max<size_t>(bytes, 1);
        return off;
    }
};

struct JobPlan {
    int64_t n_pad, P;
    size_t rowmaj = 0;        // row-major widened bins (column-path plans)
    uint32_t rm_stride = 0;
    uint32_t gbase;
    uint32_t kl_rb;  // KL importance: rows per block (0: the job does not use it)
    size_t rmean, rank;  // final ranking: per-feature mean history, rank
    size_t fixdec;       // decisions after the rough fix (when that option is set)
    int max_sha, pw_cap, mtry_max;
    size_t X, y32, y8, orig, sha, colptr, colsrc, act, state, hits, hist, smax, hconf, hrej, G,
        imp, wbuf, rec0, rec1, oob, tstat;
    size_t yfix = 0, yrange = 0;  // regression: fixed-point targets, target minimum/maximum
};

struct Plan {
    std::vector<JobPlan> jp;
    size_t keys, jobs, trees, tree_base, flags, nodes, cls, ngain, small0, small1, cand, cand_cl,
        feat, fcol, srec, kinds, chunk_sums, slot0, slot1, ctrs, alg, tot;
    size_t fcnt = 0, fpos = 0, fitems = 0, units = 0, gcolq = 0;
    size_t seed_med = 0, seed_dec = 0;  // multi-seed aggregate [p]
    size_t dec_ptrs = 0;                // per job: the decisions the aggregate reads
    size_t kl_S = 0, kl_pi = 0, kl_delta = 0;  // KL importance buffers (shared by its jobs)
    uint32_t node_cap = 0, slot_cap = 0, small_cap = 0;
    int kmax = 4, max_sha = 1, max_pw = 1, max_D = 1, T_total = 0, mtry_cap = 1,
        npi = 1, fw = 1;
    // column-major histogram path: levels >= col_level (col_level >= max_D: none)
    int col_level = kColNever, col_waves = 0;
    bool has_cls = false, has_reg = false;
    bool has_small_k = false;  // a classification job of at most 4 classes
    uint32_t n_gcol = 0, unit_cap = 0, gq_max = 0;
    int64_t max_n = 0;
    uint32_t boot_chunk = 0;  // rows per workgroup of the LDS bootstrap counts (0: atomics)
    size_t total = 0;
};

Plan make_plan(const std::vector<Spec>& specs, const Opts& o, bool inputs_on_device) {
    Plan pl;
    Region r;
    int maxK = 2;
    int64_t keys_words = 0;
    for (const Spec& s : specs) {
        maxK = std::max(maxK, s.K);
        keys_words = std::max<int64_t>(keys_words, s.p * pow2_at_least(s.n));
    }
    // class planes of the kernels: exactly 2, 3 or 4, else 8 or 16
    pl.kmax = maxK <= 4 ? maxK : (maxK <= 8 ? 8 : 16);
    pl.keys = r.take((size_t)keys_words * 4);
    uint64_t node_cap = 0, slot_cap = 0, small_cap = 0, n_gcol = 0;
    uint64_t kl_S = 0, kl_pi = 0, kl_delta = 0;
    for (const Spec& s : specs) {
        JobPlan j;
        const JobPlan* sh = s.share >= 0 ? &pl.jp[(size_t)s.share] : nullptr;
        j.n_pad = round_up(s.n, 256);
        j.P = pow2_at_least(s.n);
        j.max_sha = (int)std::max<int64_t>(s.p, 8);
        j.pw_cap = (int)(s.p + j.max_sha);
        j.gbase = (uint32_t)n_gcol;
        n_gcol += (uint64_t)j.pw_cap;
        pl.gq_max = std::max<uint32_t>(pl.gq_max, (uint32_t)(j.n_pad / 16));
        j.mtry_max = s.mtry > 0 ? std::min(s.mtry, j.pw_cap) : isqrt_i(j.pw_cap);
        const size_t n = (size_t)s.n, p = (size_t)s.p, T = (size_t)s.T;
        j.X = inputs_on_device || sh ? 0 : r.take(n * p * 4);
        j.y32 = inputs_on_device || sh ? 0 : r.take(n * 4);
        j.y8 = sh ? sh->y8 : r.take(n);
        j.orig = sh ? sh->orig : r.take(p * j.n_pad);
        j.sha = r.take((size_t)j.max_sha * j.n_pad);
        j.colptr = r.take((size_t)j.pw_cap * 8);
        j.colsrc = r.take((size_t)j.pw_cap * 4);
        j.act = r.take(p * 4);
        j.state = r.take(p);
        j.hits = r.take(p * 4);
        j.hist = r.take((size_t)s.max_iter * p * 8);
        j.smax = r.take((size_t)s.max_iter * 8);
        j.hconf = r.take((size_t)(s.max_iter + 1) * 4);
        j.hrej = r.take((size_t)(s.max_iter + 1) * 4);
        j.G = s.mode == 0 ? r.take(T * j.pw_cap * 8) : 0;
        j.imp = r.take((size_t)j.pw_cap * 8);
        j.wbuf = r.take(T * n * 4);
        j.rec0 = r.take(T * n * 8);
        j.rec1 = r.take(T * n * 8);
        if (s.yr) {
            j.yfix = sh ? sh->yfix : r.take(n * 8);
            j.yrange = sh ? sh->yrange : r.take(8);
        }
        j.oob = r.take(T * n * 4);
        j.tstat = r.take(T * 16);
        j.rmean = r.take(p * 8);
        j.rank = r.take(p * 4);
        j.fixdec = o.rough_fix ? r.take(p) : 0;
        // KL importance: the per-(column, row, class) leaf differences of a
        // block of rows are bounded by kKlDeltaBytes
        j.kl_rb = 0;
        if (s.mode == 2) {
            const uint64_t per_row = (uint64_t)j.pw_cap * s.K * 8;
            j.kl_rb = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>((uint64_t)s.n, kKlDeltaBytes / per_row));
            if (o.kl_rows) j.kl_rb = (uint32_t)std::min<int64_t>(s.n, o.kl_rows);
            kl_S = std::max<uint64_t>(kl_S, (uint64_t)j.kl_rb * (2 * s.K + 1) * 8);
            kl_pi = std::max<uint64_t>(kl_pi, (uint64_t)j.kl_rb * 4);
            kl_delta = std::max<uint64_t>(kl_delta, (uint64_t)j.kl_rb * per_row);
        }
        pl.jp.push_back(j);
        const uint64_t per_tree_nodes =
            std::min<uint64_t>((uint64_t(1) << (s.D + 1)) - 1, 2 * (uint64_t)s.n - 1);
        // every searched node reserves a pair of child slots (a leaf leaves its
        // pair unused), so the pool holds up to twice the nodes of the trees
        node_cap += T + 2 * T * per_tree_nodes;
        // a regression node of two or more distinct rows always takes the
        // histogram path
        const uint64_t large_per_tree = s.yr ? (uint64_t)(s.n + 1) / 2
                                             : (uint64_t)(s.n + o.small_rows) / (o.small_rows + 1);
        slot_cap += T * large_per_tree;
        small_cap += T * (uint64_t)((s.n + 1) / 2);
        pl.max_sha = std::max(pl.max_sha, j.max_sha);
        pl.max_pw = std::max(pl.max_pw, j.pw_cap);
        pl.mtry_cap = std::max(pl.mtry_cap, j.mtry_max);
        pl.max_D = std::max(pl.max_D, s.D);
        pl.max_n = std::max(pl.max_n, s.n);
        pl.T_total += s.T;
    }
    // The column-major path (batched form) stages a whole bin column in LDS
    // beside its waves' histograms: it is planned when a column and two
    // waves fit the workgroup's LDS, with up to kColWavesMax waves.  A plan
    // with a regression job stays node-major: its items need the node-major
    // item layout (an LDS region of at least 768 words per wave).
    bool any_reg = false;
    for (const Spec& s : specs) {
        any_reg |= s.yr != nullptr;
        pl.has_cls |= s.yr == nullptr;
        pl.has_small_k |= s.yr == nullptr && s.K <= 4;
    }
    pl.has_reg = any_reg;
    int col_level = any_reg ? kColNever : o.col_level;
    if (col_level == 0) {
        size_t widest = 0;
        for (const JobPlan& j : pl.jp) widest = std::max(widest, (size_t)j.pw_cap * j.n_pad);
        col_level = widest > kColAutoBytes ? kColLevelAuto : kColNever;
    }
    if (o.form == BORUTA_FORM_BATCHED && col_level < pl.max_D) {
        const size_t per_wave = (size_t)pl.kmax * 256 * 4, col = (size_t)pl.gq_max * 16;
        if (col + 2 * per_wave <= kLdsPerWorkgroup) {
            pl.col_level = col_level;
            pl.col_waves = (int)std::min<size_t>(kColWavesMax, (kLdsPerWorkgroup - col) / per_wave);
            if (o.col_waves >= 2) pl.col_waves = std::min(pl.col_waves, o.col_waves);
        }
    }
    // histogram items per large node: fw draws each (the column-major path
    // takes one draw per item, and both paths then share that layout).  A
    // chosen hist_fw is kept within 8 class rows of LDS per wave, and a plan
    // with a regression job keeps at least 768 words per wave (its items hold
    // 256 weights and 256 64-bit sums); none of this changes any result.
    if (pl.col_level < pl.max_D) {
        pl.fw = 1;
    } else {
        int fw = o.hist_fw ? o.hist_fw : hist_fw(pl.kmax);
        while (fw > 1 && fw * pl.kmax > 8) fw >>= 1;
        if (any_reg)
            while (fw * pl.kmax * 256 < 768) fw <<= 1;
        pl.fw = fw;
    }
    pl.npi = (pl.mtry_cap + pl.fw - 1) / pl.fw;
    if (node_cap >= 0xFFFFFFF0ull || slot_cap * (uint64_t)pl.mtry_cap + n_gcol >= 0xFFFFFFF0ull ||
        small_cap >= 0xFFFFFFF0ull)
        throw Error(BORUTA_E_INVALID_ARG, "problem too large: more than 2^32 tree nodes");
    pl.node_cap = (uint32_t)node_cap;
    pl.slot_cap = (uint32_t)slot_cap;
    pl.small_cap = (uint32_t)small_cap;
    pl.jobs = r.take(specs.size() * sizeof(JobDev));
    pl.trees = r.take((size_t)pl.T_total * sizeof(TreeDev));
    pl.tree_base = r.take(specs.size() * 4);
    pl.flags = r.take(64);
    pl.nodes = r.take((size_t)pl.node_cap * sizeof(NodeDev));
    pl.cls = r.take((size_t)pl.node_cap * pl.kmax * 4);
    pl.ngain = r.take((size_t)pl.node_cap * 8);
    pl.small0 = r.take((size_t)pl.small_cap * 4);
    pl.small1 = r.take((size_t)pl.small_cap * 4);
    pl.cand = r.take((size_t)pl.slot_cap * pl.npi * sizeof(Cand));
    pl.cand_cl = r.take((size_t)pl.slot_cap * pl.npi * pl.kmax * 4);
    pl.feat = r.take((size_t)pl.slot_cap * pl.mtry_cap * 4);
    pl.fcol = r.take((size_t)pl.slot_cap * pl.mtry_cap * 8);
    pl.srec = r.take((size_t)pl.slot_cap * sizeof(SlotRec));
    pl.kinds = r.take((size_t)pl.small_cap + pl.slot_cap);
    pl.chunk_sums = r.take(((size_t)pl.small_cap + pl.slot_cap + 4095) / 4096 * 8);
    pl.slot0 = r.take((size_t)pl.slot_cap * 4);
    pl.slot1 = r.take((size_t)pl.slot_cap * 4);
    // level d < max_D reads ctrs[d] and appends to ctrs[d + 1]
    pl.ctrs = r.take((size_t)(pl.max_D + 2) * sizeof(LevelCtr));
    pl.alg = r.take(4 * kAlgWords * 8);  // algorithmic bytes [3][..], Permut node visits
    pl.tot = r.take((size_t)pl.T_total * 8);
    {
        int64_t pmax = 1;
        for (const Spec& sp : specs) pmax = std::max<int64_t>(pmax, sp.p);
        pl.seed_med = r.take((size_t)pmax * 8);
        pl.seed_dec = r.take((size_t)pmax);
        pl.dec_ptrs = r.take(specs.size() * sizeof(void*));
    }
    if (kl_delta) {
        pl.kl_S = r.take(kl_S);
        pl.kl_pi = r.take(kl_pi);
        pl.kl_delta = r.take(kl_delta);
    }
    if (pl.col_level < pl.max_D) {
        const uint64_t items = slot_cap * (uint64_t)pl.mtry_cap;
        pl.n_gcol = (uint32_t)n_gcol;
        // units: at most one partial run per column plus the full runs
        pl.unit_cap = (uint32_t)std::min<uint64_t>(items / (uint64_t)o.col_unit + n_gcol + 1,
                                                   0xFFFFFFF0ull);
        pl.fcnt = r.take(n_gcol * 4);
        pl.fpos = r.take((items + n_gcol) * 4);
        pl.fitems = r.take(items * 4);
        pl.units = r.take((size_t)pl.unit_cap * sizeof(ColUnit));
        pl.gcolq = r.take(n_gcol * 4);
        // small nodes gather many drawn columns at few rows: a row-major copy
        // puts a row's columns in a few cache lines
        for (JobPlan& j : pl.jp) {
            j.rm_stride = (uint32_t)((j.pw_cap + 63) / 64 * 64);
            j.rowmaj = r.take((size_t)j.n_pad * j.rm_stride);
        }
    }
    pl.total = r.total + 256;
    return pl;
}

struct Out {
    int8_t* decision;
    double* hist;
    int32_t* hits;
    double* smax;
    int32_t* rank = nullptr;
    int32_t n_iter = 0;
};

// HIP event pairs around launches, recorded without host waits and read
// after the synchronisation that ends the iteration.
class KernelClock {
public:
    explicit KernelClock(bool on) : on_(on) {}
    ~KernelClock() {
        for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
    }
    KernelClock(const KernelClock&) = delete;
    KernelClock& operator=(const KernelClock&) = delete;
    // Returns the handle that end() takes.
    size_t begin(boruta_kernel_stat* k, hipStream_t st) {
        if (!on_) return 0;
        Rec r;
        r.k = k;
        r.a = take();
        r.b = take();
        HIPC(hipEventRecord(r.a, st));
        recs_.push_back(r);
        return recs_.size() - 1;
    }
    void end(size_t h, hipStream_t st) {
        if (on_) HIPC(hipEventRecord(recs_[h].b, st));
    }
    // Every recorded event must have completed (the stream was synchronised).
    // keep: the records belong to a captured graph and are recorded again by
    // every replay.
    void collect(bool keep) {
        for (const Rec& r : recs_) {
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, r.a, r.b));
            r.k->ms += ms;
            r.k->launches += 1;
        }
        if (!keep) {
            recs_.clear();
            next_ = 0;
        }
    }

private:
    struct Rec {
        boruta_kernel_stat* k;
        hipEvent_t a, b;
    };
    hipEvent_t take() {
        if (next_ == pool_.size()) {
            hipEvent_t e = nullptr;
            HIPC(hipEventCreate(&e));
            pool_.push_back(e);
        }
        return pool_[next_++];
    }
    bool on_;
    std::vector<hipEvent_t> pool_;
    size_t next_ = 0;
    std::vector<Rec> recs_;
};

// ---------------------------------------------------------------------------
class Engine {
public:
    Engine(const std::vector<Spec>& specs, const Opts& o, bool dev_inputs, char* base,
           hipStream_t st)
        : S(specs), O(o), dev_in(dev_inputs), base(base), st(st), clock(o.stats != nullptr) {
        pl = make_plan(specs, o, dev_inputs);
    }
    ~Engine() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;

    template <class T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(base + off);
    }

    void d2h(void* dst, const void* src, size_t bytes) {
        HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
    }
    void h2d(void* dst, const void* src, size_t bytes) {
        HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    }

    // Whole run: setup, iterations until no job is live, results.
    void run(std::vector<Out>& outs, std::vector<int>& status);
    // Upload/validate/bin every job; status[j] receives each job's code.
    void setup(std::vector<int>& status);
    // One iteration of every live job; returns the number still live.
    int step();
    // Up to k iterations enqueued back to back (graph replays, no host wait
    // between them); returns the job-iterations run and the jobs still live.
    int64_t run_steps(int k, int* n_live);
    void result(int j, Out& o);
    const int8_t* decisions(int j);
    // Continue job j from a checkpoint: the next iteration is t + 1.
    void resume(int j, int t, const int8_t* state, const int32_t* hits);
    void flush_stats();
    const JobDev& job(int j) const { return hj[j]; }
    // Multi-seed aggregate over all jobs (runs of one problem with p features).
    void seed_median(int64_t p, double* med, int8_t* dec) {
        // the kernel sorts each feature's values of at most 64 runs in registers
        if (S.size() > 64) throw Error(BORUTA_E_INVALID_ARG, "multi-seed aggregate: > 64 runs");
        std::vector<const int8_t*> ptrs(S.size());
        for (size_t j = 0; j < S.size(); ++j) ptrs[j] = decisions((int)j);
        h2d(at<void>(pl.dec_ptrs), ptrs.data(), ptrs.size() * sizeof(void*));
        launch_seed_median(at<JobDev>(pl.jobs), at<const int8_t*>(pl.dec_ptrs), (int)S.size(), p,
                           at<double>(pl.seed_med), at<int8_t>(pl.seed_dec), st);
        d2h(med, at<double>(pl.seed_med), (size_t)p * 8);
        d2h(dec, at<int8_t>(pl.seed_dec), (size_t)p);
    }

private:
    void iteration(const std::vector<int>& live);
    void enqueue_iteration();
    ForestDev forest() const;
    void grow_level_plain(const ForestDev& F, int level);
    void emit_trace(const std::vector<int>& live, uint32_t n_nodes);

    std::vector<Spec> S;
    Opts O;
    bool dev_in;
    char* base;
    hipStream_t st;
    Plan pl;
    KernelClock clock;
    boruta_kernel_stat iter_stat{};  // event time of whole iterations
    hipGraph_t graph = nullptr;      // captured iteration (batched form)
    hipGraphExec_t gexec = nullptr;
    hipStream_t side = nullptr;      // second stream of the batched form
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<JobDev> hj;       // host mirror of the job records
    std::vector<int> tree_base;   // first tree of each job in the static tree table
    std::vector<int> hist_t0;     // first history row computed here (after a resume: t)
    bool any_treeimp = false, any_permut = false, any_kl = false;
};

void Engine::setup(std::vector<int>& status) {
    const int nj = (int)S.size();
    if (O.form == BORUTA_FORM_BATCHED && !O.no_alloc) {
        HIPC(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        HIPC(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        HIPC(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }
    hj.assign(nj, JobDev{});
    hist_t0.assign(nj, 0);
    uint32_t* flags = at<uint32_t>(pl.flags);
    for (int j = 0; j < nj; ++j) {
        const Spec& s = S[j];
        const JobPlan& jp = pl.jp[j];
        if (s.share >= 0) {
            // inputs validated, labelled and binned with job s.share
            status[j] = status[(size_t)s.share];
            if (status[j] != BORUTA_OK) continue;
        } else {
            const float* X = dev_in ? s.X : at<float>(jp.X);
            // classification labels, or the regression targets (same buffer size)
            const int32_t* y = dev_in ? s.y : at<int32_t>(jp.y32);
            const float* yr = dev_in ? s.yr : at<float>(jp.y32);
            if (!dev_in) {
                h2d((void*)X, s.X, (size_t)s.n * s.p * 4);
                if (s.yr)
                    h2d((void*)yr, s.yr, (size_t)s.n * 4);
                else
                    h2d((void*)y, s.y, (size_t)s.n * 4);
            }
            launch_fill_u32(flags, 1, 0u, st);
            if (s.yr)
                launch_validate_reg(X, (size_t)s.n * s.p, yr, (size_t)s.n, flags, st);
            else
                launch_validate(X, (size_t)s.n * s.p, y, (size_t)s.n, s.K, flags, st);
            uint32_t f = 0;
            d2h(&f, flags, 4);
            if (f & 1u) {
                status[j] = BORUTA_E_NONFINITE;
                continue;
            }
            if (f & 2u) {
                status[j] = BORUTA_E_INVALID_ARG;
                continue;
            }
            if (s.yr) {
                // the targets' range picks the fixed-point scale
                launch_target_range(yr, (size_t)s.n, at<float>(jp.yrange), st);
                float lh[2];
                d2h(lh, at<float>(jp.yrange), 8);
                const RegShift rs = reg_shift(lh[0], lh[1], s.n, s.T, O.R);
                launch_target_fix(yr, (size_t)s.n, 38 - rs.e, at<int64_t>(jp.yfix), st);
            } else {
                launch_labels(y, (size_t)s.n, at<uint8_t>(jp.y8), st);
            }
            launch_binning(X, s.n, s.p, O.B, at<uint8_t>(jp.orig), jp.n_pad,
                           at<uint32_t>(pl.keys), jp.P, st);
        }
        int ex = 0;
        const double fr = std::frexp(s.alpha, &ex);
        const uint64_t am = (uint64_t)std::ldexp(fr, 53);
        launch_thresholds(s.max_iter, s.p, am, ex - 53, at<int32_t>(jp.hconf),
                          at<int32_t>(jp.hrej), st);
        JobDev& J = hj[j];
        J.n = (int32_t)s.n;
        J.n_pad = (int32_t)jp.n_pad;
        J.p = (int32_t)s.p;
        J.K = s.K;
        J.B = O.B;
        J.T = s.T;
        J.D = s.D;
        J.mtry_opt = s.mtry;
        J.mode = s.mode;
        J.R = O.R;
        J.max_iter = s.max_iter;
        J.seed_lo = (uint32_t)s.seed;
        J.seed_hi = (uint32_t)(s.seed >> 32);
        J.max_sha = jp.max_sha;
        J.pw_cap = jp.pw_cap;
        J.gbase = jp.gbase;
        J.gq = (uint32_t)(jp.n_pad / 16);
        J.reg = s.yr ? 1 : 0;
        J.rstride = (uint32_t)s.n;
        J.yfix = s.yr ? at<int64_t>(jp.yfix) : nullptr;
        J.s_gain = J.s_perm = J.s_kl = J.rep_exp = 0;
        if (s.yr) {
            float lh[2];
            d2h(lh, at<float>(jp.yrange), 8);
            const RegShift rs = reg_shift(lh[0], lh[1], s.n, s.T, O.R);
            J.s_gain = rs.s_gain;
            J.s_perm = rs.s_perm;
            J.s_kl = rs.s_kl;
            // reported regression scores in squared target units
            J.rep_exp = s.mode == 1 ? rs.s_perm - 2 * (38 - rs.e)
                                    : (s.mode == 2 ? rs.s_kl - 2 * (38 - rs.e) : 0);
        }
        J.y = at<uint8_t>(jp.y8);
        J.orig = at<uint8_t>(jp.orig);
        J.sha = at<uint8_t>(jp.sha);
        J.colptr = at<const uint8_t*>(jp.colptr);
        J.col_src = at<int32_t>(jp.colsrc);
        J.act = at<int32_t>(jp.act);
        J.state = at<int8_t>(jp.state);
        J.hits = at<int32_t>(jp.hits);
        J.hist = at<double>(jp.hist);
        J.shadow_max = at<double>(jp.smax);
        J.h_conf = at<int32_t>(jp.hconf);
        J.h_rej = at<int32_t>(jp.hrej);
        J.G = s.mode == 0 ? at<uint64_t>(jp.G) : nullptr;
        J.imp = at<int64_t>(jp.imp);
        J.wbuf = at<uint32_t>(jp.wbuf);
        J.rec[0] = at<uint64_t>(jp.rec0);
        J.rec[1] = at<uint64_t>(jp.rec1);
        J.oob = at<uint32_t>(jp.oob);
        J.tstat = at<int32_t>(jp.tstat);
        J.rowmaj = jp.rm_stride ? at<uint8_t>(jp.rowmaj) : nullptr;
        J.rm_stride = jp.rm_stride;
        J.t = 0;
        J.live = 1;
        launch_fill_u32((uint32_t*)J.state, ((size_t)s.p + 3) / 4, 0u, st);
        launch_fill_u32((uint32_t*)J.hits, (size_t)s.p, 0u, st);
        if (s.mode == 0)
            launch_fill_u32((uint32_t*)J.G, (size_t)s.T * jp.pw_cap * 2, 0u, st);
        // bootstrap multiplicities: zero here, then cleared by their reader
        launch_fill_u32(J.wbuf, (size_t)s.T * s.n, 0u, st);
        status[j] = BORUTA_OK;
    }
    for (int j = 0; j < nj; ++j)
        if (status[j] != BORUTA_OK) hj[j].live = 0;
    // static tree table: the trees of every job in job order; the kernels
    // skip the trees of jobs that are no longer live
    std::vector<TreeDev> trees;
    tree_base.assign(nj, 0);
    for (int j = 0; j < nj; ++j) {
        tree_base[j] = (int)trees.size();
        for (int tau = 0; tau < S[j].T; ++tau) trees.push_back(TreeDev{j, tau});
        any_treeimp |= S[j].mode == 0;
        any_permut |= S[j].mode == 1;
        any_kl |= S[j].mode == 2;
    }
    h2d(at<TreeDev>(pl.trees), trees.data(), trees.size() * sizeof(TreeDev));
    h2d(at<int32_t>(pl.tree_base), tree_base.data(), tree_base.size() * 4);
    launch_fill_u32(at<uint32_t>(pl.alg), 8 * kAlgWords, 0u, st);
    // KL importance differences start at zero; each block's reader clears them
    if (any_kl) {
        size_t words = 0;
        for (int j = 0; j < nj; ++j)
            if (pl.jp[j].kl_rb)
                words = std::max(words, (size_t)pl.jp[j].kl_rb * pl.jp[j].pw_cap * S[j].K * 2);
        launch_fill_u32(at<uint32_t>(pl.kl_delta), words, 0u, st);
    }
    pl.boot_chunk = prepare_boot_draw(pl.max_n);
    if (pl.col_level < pl.max_D) {
        int dev = 0, lds_max = 0;
        HIPC(hipGetDevice(&dev));
        HIPC(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t lds = hist_col_lds(pl.kmax, pl.col_waves, pl.gq_max);
        if ((size_t)lds_max < lds || prepare_hist_col(pl.kmax, lds) != hipSuccess) {
            (void)hipGetLastError();
            pl.col_level = kColNever;  // node-major at every level (same item layout)
        } else {
            std::vector<uint32_t> gq(pl.n_gcol, 0u);
            for (int j = 0; j < nj; ++j)
                for (int f = 0; f < pl.jp[j].pw_cap; ++f)
                    gq[pl.jp[j].gbase + f] = (uint32_t)(pl.jp[j].n_pad / 16);
            h2d(at<uint32_t>(pl.gcolq), gq.data(), gq.size() * 4);
            // per-column counts start at zero; each level's scan clears them
            launch_fill_u32(at<uint32_t>(pl.fcnt), pl.n_gcol, 0u, st);
        }
    }
    h2d(at<JobDev>(pl.jobs), hj.data(), hj.size() * sizeof(JobDev));
    // level counters, and the accumulated capacity flags after them
    launch_fill_u32(at<uint32_t>(pl.ctrs), (size_t)(pl.max_D + 2) * sizeof(LevelCtr) / 4, 0u, st);
    HIPC(hipStreamSynchronize(st));
}

ForestDev Engine::forest() const {
    ForestDev F;
    std::memset(&F, 0, sizeof(F));
    F.jobs = at<JobDev>(pl.jobs);
    F.trees = at<TreeDev>(pl.trees);
    F.nodes = at<NodeDev>(pl.nodes);
    F.cls = at<uint32_t>(pl.cls);
    F.ngain = at<uint64_t>(pl.ngain);
    F.cand = at<Cand>(pl.cand);
    F.cand_cl = at<uint32_t>(pl.cand_cl);
    F.feat = at<uint32_t>(pl.feat);
    F.fcol = at<const uint8_t*>(pl.fcol);
    F.srec = at<SlotRec>(pl.srec);
    F.kinds = at<uint8_t>(pl.kinds);
    F.chunk_sums = at<unsigned long long>(pl.chunk_sums);
    F.npi = pl.npi;
    F.fw = pl.fw;
    if (pl.col_level < pl.max_D) {
        F.fcnt = at<uint32_t>(pl.fcnt);
        F.fpos = at<uint32_t>(pl.fpos);
        F.fitems = at<uint32_t>(pl.fitems);
        F.units = at<ColUnit>(pl.units);
        F.gcol_q = at<uint32_t>(pl.gcolq);
        F.n_gcol = pl.n_gcol;
        F.unit_cap = pl.unit_cap;
        F.col_unit = (uint32_t)O.col_unit;
    }
    F.small_rows = (uint32_t)O.small_rows;
    F.mtry_cap = pl.mtry_cap;
    F.draw_seg = 1;
    while (F.draw_seg < (uint32_t)pl.mtry_cap && F.draw_seg < 64u) F.draw_seg <<= 1;
    // round tables of (256 / draw_seg) node segments, at most 48 KB of LDS:
    // 1536 entries from 16 lanes per node, 768 for 8 lanes, none below
    F.draw_tab = F.draw_seg >= 16u ? kDrawTab : (F.draw_seg == 8u ? kDrawTab / 2 : 0u);
    F.ctrs = at<LevelCtr>(pl.ctrs);
    F.ctr = F.ctrs;
    F.n_roots = (uint32_t)pl.T_total;
    F.alg_bytes = O.stats ? at<uint64_t>(pl.alg) : nullptr;
    F.node_cap = pl.node_cap;
    F.slot_cap = pl.slot_cap;
    F.small_cap = pl.small_cap;
    F.kmax = pl.kmax;
    F.split_rank = O.split_rank;
    F.has_cls = pl.has_cls ? 1 : 0;
    F.has_reg = pl.has_reg ? 1 : 0;
    F.split_k = pl.kmax > 4 && pl.has_small_k ? 1 : 0;
    // the wave path packs class counters in 32/kmax-bit fields up to 4 classes
    // (16-bit for 2, 10-bit for 3, 8-bit for 4), 16-bit fields beyond
    F.small_ncap = pl.kmax == 4 ? 256u : (pl.kmax == 3 ? 1024u : 65536u);
    return F;
}

void Engine::grow_level_plain(const ForestDev& F, int level) {
    // One launch (or, for a large node, one histogram launch over its column
    // groups and one finalize launch) per node: the level's counters are read
    // back and each node is its own launch.
    LevelCtr c;
    d2h(&c, F.ctrs + level, sizeof(c));
    if (c.overflow) return;  // reported after the iteration
    for (uint32_t i = 0; i < c.n_small; ++i) launch_split_small(F, level, i, 1, 1, st);
    if (c.n_slots) launch_draws(F, level, 1, st);
    for (uint32_t sl = 0; sl < c.n_slots; ++sl) {
        launch_hist_tile(F, level, sl * pl.npi, pl.npi, (pl.npi + 3) / 4,
                         level < O.band_level ? O.hist_rb : O.hist_rb_deep, st);
        launch_split_finalize(F, level, sl, 1, 1, st);
    }
    const uint32_t chunks = (c.n_small + c.n_slots + 4095) / 4096;
    if (chunks && level + 1 < pl.max_D) launch_lists(F, level, chunks, st);
}

namespace {
// Grid of a grid-stride level kernel: enough workgroups to fill the 256 CUs
// several times over, never more than the level's capacity can use.
uint32_t level_grid(uint64_t cap_units, uint32_t per_wg, uint32_t limit) {
    const uint64_t g = (cap_units + per_wg - 1) / per_wg;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, limit));
}
constexpr uint32_t kAll = 0xFFFFFFFFu;  // level kernels: work count read on the device
}  // namespace

// The launch sequence of one iteration of every live job.  Work sizes come
// from plan-time bounds; every kernel reads its real work count on the device,
// so the sequence is the same for every iteration (and capturable), except in
// the plain form, which reads each level's node list back.
void Engine::enqueue_iteration() {
    const int nj = (int)S.size();
    const uint32_t n_trees = (uint32_t)pl.T_total;
    JobDev* djobs = at<JobDev>(pl.jobs);
    TreeDev* dtrees = at<TreeDev>(pl.trees);
    boruta_stats* stats = O.stats;
    const size_t h_whole = clock.begin(&iter_stat, st);
    launch_active(djobs, nj, st);
    launch_shadow(djobs, nj, pl.max_n, pl.max_sha, st);
    if (pl.col_level < pl.max_D) launch_rowmaj(djobs, nj, pl.max_n, pl.max_pw, st);
    launch_boot_draw(djobs, dtrees, (int)n_trees, pl.max_n, pl.boot_chunk, st);

    ForestDev F = forest();
    // levels 0 .. max_D - 1 search splits; nodes of depth max_D are leaves
    const int n_levels = pl.max_D;
    launch_fill_u32((uint32_t*)F.ctrs, (size_t)(n_levels + 1) * sizeof(LevelCtr) / 4, 0u, st);
    uint32_t* slots[2] = {at<uint32_t>(pl.slot0), at<uint32_t>(pl.slot1)};
    uint32_t* small[2] = {at<uint32_t>(pl.small0), at<uint32_t>(pl.small1)};
    // the roots go to the level-0 lists (parity 0)
    F.small_out = small[0];
    F.slot_node_out = slots[0];
    launch_boot_compact(F, n_trees, st);
    const uint32_t g_col = O.grid_col ? (uint32_t)O.grid_col : level_grid(pl.unit_cap, 1, 2048);
    for (int d = 0; d < n_levels; ++d) {
        // Level d holds at most n_trees * 2^d nodes: the shallow levels launch
        // no more workgroups than that bound can use (a chosen grid size is
        // an upper limit), the deep ones are held to the plan's capacities.
        const auto at_level = [&](uint64_t cap) {
            return d < 32 ? std::min<uint64_t>(cap, (uint64_t)n_trees << d) : cap;
        };
        const uint64_t lv_small = at_level(pl.small_cap), lv_slots = at_level(pl.slot_cap);
        const auto capped = [](int chosen, uint32_t need) {
            return chosen ? std::min<uint32_t>((uint32_t)chosen, need) : need;
        };
        const uint32_t g_small = capped(O.grid_small, level_grid(lv_small, 4, 4096));
        // a multiple of 8: workgroup b serves the node slots congruent to b mod 8
        const uint32_t g_tile =
            (capped(O.grid_hist, level_grid(lv_slots * pl.npi, 4, 16384)) + 7) / 8 * 8;
        // k_draws serves 64 / draw_seg nodes per wavefront, four wavefronts per workgroup
        const uint32_t g_draw = level_grid(lv_slots, 4 * (64u / F.draw_seg), 16384);
        const uint32_t g_list = level_grid(lv_small + lv_slots, 4096, 1024);
        const uint32_t g_fin = capped(O.grid_finalize, level_grid(lv_slots, 4, 4096));
        // lists, slots and row records of level d are read from parity d & 1
        // and the children of level d go to the other parity
        F.small_in = small[d & 1];
        F.slot_node_in = slots[d & 1];
        F.small_out = small[(d + 1) & 1];
        F.slot_node_out = slots[(d + 1) & 1];
        F.parity = d & 1;
        if (O.form == BORUTA_FORM_PLAIN) {
            grow_level_plain(F, d);
            continue;
        }
        // The small nodes and the large nodes of a level touch disjoint
        // nodes, child pairs, row segments and kinds entries: without kernel
        // statistics the small-node launch runs on a second stream, beside
        // the large-node kernels, and rejoins before the lists are built.
        // Regression nodes all take the histogram path: a plan of regression
        // jobs alone has no small-node work.
        const bool fork = !stats && side != nullptr && pl.has_cls;
        hipStream_t ss = st;
        if (fork) {
            HIPC(hipEventRecord(ev_fork, st));
            HIPC(hipStreamWaitEvent(side, ev_fork, 0));
            ss = side;
        }
        size_t h = 0;
        if (pl.has_cls) {
            h = clock.begin(stats ? &stats->hist_small : nullptr, ss);
            launch_split_small(F, d, 0, kAll, g_small, ss);
            clock.end(h, ss);
        }
        if (fork) HIPC(hipEventRecord(ev_join, side));
        const bool col = d >= pl.col_level;
        if (col) {
            // items bucketed by column, one LDS-staged column per unit
            ForestDev Fc = F;
            Fc.col_count = pl.n_gcol <= kColCountLds ? 2 : 1;
            launch_draws(Fc, d, g_draw, st);
            launch_col_sort(Fc, d, level_grid(lv_slots, 4, 16384), st);
            h = clock.begin(stats ? &stats->hist_col : nullptr, st);
            launch_hist_col(F, d, g_col, pl.col_waves, pl.gq_max, st);
            HIPC(hipGetLastError());  // a refused launch would leave stale candidates
            clock.end(h, st);
        } else {
            launch_draws(F, d, g_draw, st);
            h = clock.begin(stats ? &stats->hist_large : nullptr, st);
            launch_hist_tile(F, d, 0, kAll, g_tile, d < O.band_level ? O.hist_rb : O.hist_rb_deep,
                             st);
            clock.end(h, st);
        }
        h = clock.begin(stats ? &stats->finalize : nullptr, st);
        launch_split_finalize(F, d, 0, kAll, g_fin, st);
        clock.end(h, st);
        if (fork) HIPC(hipStreamWaitEvent(st, ev_join, 0));
        // the children of the last level are all leaves (maximum depth)
        if (d + 1 < n_levels) launch_lists(F, d, g_list, st);
    }

    // importance
    if (any_treeimp) {
        launch_tree_totals(djobs, dtrees, (int)n_trees, at<uint64_t>(pl.tot), st);
        launch_treeimp(djobs, dtrees, (int)n_trees, at<uint64_t>(pl.tot), pl.max_pw, st);
    }
    if (any_permut) {
        const size_t h = clock.begin(stats ? &stats->permut : nullptr, st);
        bool any_reg = false;
        for (const Spec& sp : S) any_reg |= sp.yr != nullptr;
        launch_permut(djobs, dtrees, F.nodes, F.cls, pl.kmax, (int)n_trees, pl.max_n, pl.max_D,
                      pl.max_pw, any_reg,
                      stats ? (unsigned long long*)at<uint64_t>(pl.alg) + 3 * kAlgWords : nullptr,
                      st);
        clock.end(h, st);
    }
    if (any_kl) {
        // per job of mode 2, blocks of rows (the kernels skip finished jobs)
        const size_t h = clock.begin(stats ? &stats->permut : nullptr, st);
        for (int j = 0; j < (int)S.size(); ++j) {
            const uint32_t rb = pl.jp[j].kl_rb;
            if (!rb) continue;
            for (int64_t r0 = 0; r0 < S[j].n; r0 += rb)
                launch_kl_block(djobs, j, F.nodes, F.cls, pl.kmax, (uint32_t)tree_base[j], S[j].T,
                                pl.jp[j].pw_cap, (uint32_t)r0, rb, at<uint64_t>(pl.kl_S),
                                at<uint32_t>(pl.kl_pi), at<unsigned long long>(pl.kl_delta),
                                pl.max_D, st);
        }
        clock.end(h, st);
    }
    launch_hits_decide(djobs, nj, O.perc, st);
    launch_ctr_sticky(at<LevelCtr>(pl.ctrs), pl.max_D, st);
    clock.end(h_whole, st);
}

void Engine::iteration(const std::vector<int>& live) {
    // Kernel timing needs events around each launch, which a replayed graph
    // cannot report: with stats the sequence is launched eagerly.
    const bool use_graph = O.graph && O.form == BORUTA_FORM_BATCHED && !O.stats;
    if (use_graph) {
        if (!gexec) {
            // Captured on a private stream (the caller's stream may be the
            // null stream, which cannot be captured); replays go to the
            // caller's stream.
            hipStream_t user = st, cs = nullptr;
            HIPC(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            st = cs;
            try {
                HIPC(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
                try {
                    enqueue_iteration();
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(cs, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HIPC(hipStreamEndCapture(cs, &graph));
                HIPC(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            } catch (...) {
                st = user;
                (void)hipStreamDestroy(cs);
                throw;
            }
            st = user;
            (void)hipStreamDestroy(cs);
        }
        HIPC(hipGraphLaunch(gexec, st));
    } else {
        enqueue_iteration();
    }
    const int n_levels = pl.max_D;
    std::vector<LevelCtr> c(n_levels + 2);  // levels, then the accumulated flags
    HIPC(hipMemcpyAsync(c.data(), at<LevelCtr>(pl.ctrs), c.size() * sizeof(LevelCtr),
                        hipMemcpyDeviceToHost, st));
    d2h(hj.data(), at<JobDev>(pl.jobs), hj.size() * sizeof(JobDev));
    clock.collect(use_graph);
    uint32_t overflow = 0;
    uint64_t n_nodes = (uint32_t)pl.T_total;
    for (int d = 0; d <= n_levels + 1; ++d) {
        overflow |= c[d].overflow;
        if (d < n_levels) n_nodes += 2ull * (c[d].n_small + c[d].n_slots);
    }
    if (overflow)
        throw Error(BORUTA_E_DEVICE,
                    "internal capacity exceeded (flags " + std::to_string(overflow) + ")");
    if (n_nodes > pl.node_cap) throw Error(BORUTA_E_DEVICE, "node pool too small");
    boruta_stats* stats = O.stats;
    if (stats) {
        stats->iter_ms += iter_stat.ms;
        stats->nodes += (int64_t)n_nodes;
        stats->iterations += (int64_t)live.size();
        for (int d = 0; d < n_levels && d < 32; ++d) {
            stats->level_small[d] += c[d].n_small;
            stats->level_large[d] += c[d].n_slots;
        }
    }
    iter_stat.ms = 0.0;
    if (O.trace) emit_trace(live, (uint32_t)n_nodes);
}

void Engine::emit_trace(const std::vector<int>& live, uint32_t n_nodes) {
    // Called after the decision kernel: importances and trees are those of
    // this iteration, hits and states already include its decision.
    std::vector<NodeDev> nodes(n_nodes);
    std::vector<uint64_t> gains(n_nodes);
    d2h(nodes.data(), at<NodeDev>(pl.nodes), (size_t)n_nodes * sizeof(NodeDev));
    d2h(gains.data(), at<uint64_t>(pl.ngain), (size_t)n_nodes * 8);
    // regression leaves report their prediction floor(T / W), T in the
    // node's first two class words
    bool any_reg = false;
    for (int j : live) any_reg |= hj[j].reg != 0;
    std::vector<uint32_t> cls;
    if (any_reg) {
        cls.resize((size_t)n_nodes * pl.kmax);
        d2h(cls.data(), at<uint32_t>(pl.cls), cls.size() * 4);
    }
    for (size_t li = 0; li < live.size(); ++li) {
        const int j = live[li];
        const JobDev& J = hj[j];
        std::vector<int32_t> col_src(J.p_w), hits(J.p), tstat((size_t)J.T * 4);
        std::vector<int64_t> imp(J.p_w);
        std::vector<int8_t> state(J.p);
        d2h(col_src.data(), J.col_src, (size_t)J.p_w * 4);
        d2h(imp.data(), J.imp, (size_t)J.p_w * 8);
        d2h(hits.data(), J.hits, (size_t)J.p * 4);
        d2h(state.data(), J.state, (size_t)J.p);
        d2h(tstat.data(), J.tstat, tstat.size() * 4);
        const int g0 = tree_base[j];
        std::vector<std::vector<uint32_t>> idx(J.T);
        for (uint32_t i = 0; i < n_nodes; ++i) {
            if (nodes[i].tree == 0xFFFFFFFFu) continue;  // unused child pair of a leaf
            const int g = (int)nodes[i].tree;
            if (g >= g0 && g < g0 + J.T) idx[g - g0].push_back(i);
        }
        std::vector<int64_t> rows, stats;
        for (int tau = 0; tau < J.T; ++tau) {
            auto& v = idx[tau];
            std::sort(v.begin(), v.end(),
                      [&](uint32_t a, uint32_t b) { return nodes[a].heap < nodes[b].heap; });
            for (uint32_t i : v) {
                const NodeDev& nd = nodes[i];
                int64_t leaf = nd.leaf_class;
                if (J.reg && nd.feat < 0) {
                    const int64_t T = (int64_t)((uint64_t)cls[(size_t)i * pl.kmax] |
                                                ((uint64_t)cls[(size_t)i * pl.kmax + 1] << 32));
                    const int64_t W = (int64_t)nd.n;
                    leaf = T / W;
                    if (leaf * W != T && T < 0) --leaf;  // floor
                }
                rows.insert(rows.end(), {(int64_t)tau, (int64_t)nd.heap, (int64_t)nd.feat,
                                         (int64_t)(nd.feat >= 0 ? nd.thr : leaf), (int64_t)nd.n,
                                         (int64_t)gains[i]});
            }
            stats.insert(stats.end(), {(int64_t)tau, (int64_t)tstat[tau * 4 + 0],
                                       (int64_t)tstat[tau * 4 + 1],
                                       (int64_t)(J.mode == 1 ? tstat[tau * 4 + 2] : 0),
                                       (int64_t)v.size()});
        }
        boruta_iter_trace tr;
        tr.job = j;
        tr.t = J.t;
        tr.p_cur = J.p_cur;
        tr.n_sha = J.n_sha;
        tr.p_w = J.p_w;
        tr.mtry = J.mtry;
        tr.n_trees = J.T;
        tr.col_src = col_src.data();
        tr.imp_int = imp.data();
        tr.hits = hits.data();
        tr.state = state.data();
        tr.tree_stats = stats.data();
        tr.n_nodes = (int64_t)(rows.size() / 6);
        tr.nodes = rows.data();
        O.trace(O.trace_user, &tr);
    }
}

int Engine::step() {
    std::vector<int> live;
    for (int j = 0; j < (int)S.size(); ++j)
        if (hj[j].live) live.push_back(j);
    if (live.empty()) return 0;
    iteration(live);
    int n = 0;
    for (const JobDev& J : hj) n += J.live != 0;
    return n;
}

int64_t Engine::run_steps(int k, int* n_live) {
    std::vector<int32_t> t0(hj.size());
    for (size_t j = 0; j < hj.size(); ++j) t0[j] = hj[j].t;
    const bool replay = O.graph && O.form == BORUTA_FORM_BATCHED && !O.stats && !O.trace;
    for (int i = 0; i < k; ++i) {
        std::vector<int> live;
        for (int j = 0; j < (int)S.size(); ++j)
            if (hj[j].live) live.push_back(j);
        if (live.empty()) break;
        if (!replay || !gexec) {
            iteration(live);  // with a host read-back (and the graph's capture)
            continue;
        }
        // The host's view of liveness stays as it was: a job that finishes
        // on the device is skipped by every kernel of the later replays.
        HIPC(hipGraphLaunch(gexec, st));
    }
    if (replay) {
        std::vector<LevelCtr> c(pl.max_D + 2);
        HIPC(hipMemcpyAsync(c.data(), at<LevelCtr>(pl.ctrs), c.size() * sizeof(LevelCtr),
                            hipMemcpyDeviceToHost, st));
        d2h(hj.data(), at<JobDev>(pl.jobs), hj.size() * sizeof(JobDev));
        if (c[pl.max_D + 1].overflow)
            throw Error(BORUTA_E_DEVICE, "internal capacity exceeded (flags " +
                                             std::to_string(c[pl.max_D + 1].overflow) + ")");
    }
    int64_t done = 0;
    int n = 0;
    for (size_t j = 0; j < hj.size(); ++j) {
        done += hj[j].t - t0[j];
        n += hj[j].live != 0;
    }
    if (n_live) *n_live = n;
    return done;
}

void Engine::flush_stats() {
    if (!O.stats) return;
    std::vector<uint64_t> ab(4 * kAlgWords);
    d2h(ab.data(), at<uint64_t>(pl.alg), ab.size() * 8);
    for (uint32_t i = 0; i < kAlgWords; ++i) {
        O.stats->hist_large.alg_bytes += (double)ab[i];
        O.stats->hist_small.alg_bytes += (double)ab[kAlgWords + i];
        O.stats->hist_col.alg_bytes += (double)ab[2 * kAlgWords + i];
        O.stats->permut_visits += (double)ab[3 * kAlgWords + i];
    }
    launch_fill_u32(at<uint32_t>(pl.alg), 8 * kAlgWords, 0u, st);
}

// Decisions of job j as reported: the live state, or after the rough fix of
// the tentative features over the iterations run here.
const int8_t* Engine::decisions(int j) {
    const JobDev& J = hj[j];
    if (!O.rough_fix || J.t <= hist_t0[j]) return J.state;
    int8_t* out = at<int8_t>(pl.jp[j].fixdec);
    launch_rough_fix(J.state, J.hist, J.shadow_max, S[j].p, hist_t0[j], J.t, out, st);
    return out;
}

void Engine::result(int j, Out& o) {
    const Spec& s = S[j];
    const JobDev& J = hj[j];
    HIPC(hipStreamSynchronize(st));
    const int8_t* dec = decisions(j);
    d2h(o.decision, dec, (size_t)s.p);
    if (J.t > 0 && o.hist) d2h(o.hist, J.hist, (size_t)J.t * s.p * 8);
    if (o.hits) d2h(o.hits, J.hits, (size_t)s.p * 4);
    if (o.smax && J.t > 0) d2h(o.smax, J.shadow_max, (size_t)J.t * 8);
    if (o.rank) {
        const JobPlan& jp = pl.jp[j];
        launch_rank(dec, J.hist, s.p, hist_t0[j], J.t, at<double>(jp.rmean),
                    at<int32_t>(jp.rank), st);
        d2h(o.rank, at<int32_t>(jp.rank), (size_t)s.p * 4);
    }
    o.n_iter = J.t;
}

void Engine::resume(int j, int t, const int8_t* state, const int32_t* hits) {
    const Spec& s = S[j];
    if (t < 0 || t >= s.max_iter) throw Error(BORUTA_E_INVALID_ARG, "resume: t outside [0, max_iter)");
    for (int64_t i = 0; i < s.p; ++i) {
        if (state[i] < -1 || state[i] > 1) throw Error(BORUTA_E_INVALID_ARG, "resume: bad state");
        if (hits[i] < 0 || hits[i] > t) throw Error(BORUTA_E_INVALID_ARG, "resume: bad hits");
    }
    JobDev& J = hj[j];
    h2d(J.state, state, (size_t)s.p);
    h2d(J.hits, hits, (size_t)s.p * 4);
    bool und = false;
    for (int64_t i = 0; i < s.p; ++i) und |= state[i] == 0;
    J.t = t;
    J.live = und ? 1 : 0;
    hist_t0[j] = t;  // history rows before t are the caller's
    h2d(at<JobDev>(pl.jobs) + j, &J, sizeof(JobDev));
    HIPC(hipStreamSynchronize(st));
}

void Engine::run(std::vector<Out>& outs, std::vector<int>& status) {
    setup(status);
    while (step() > 0) {
    }
    flush_stats();
    for (int j = 0; j < (int)S.size(); ++j)
        if (status[j] == BORUTA_OK) result(j, outs[j]);
}

struct DeviceRegion {
    char* p = nullptr;
    ~DeviceRegion() {
        if (p) (void)hipFree(p);
    }
};

void require_device() {
    int count = 0;
    const hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1)
        throw Error(BORUTA_E_UNSUPPORTED, std::string("no HIP device available (") +
                                              hipGetErrorName(e) + ", " + std::to_string(count) +
                                              " devices)");
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw Error(BORUTA_E_UNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                              ", this library is built for gfx950");
}

// Device region, stream and engine of one set of jobs (a boruta_fit call or
// a session).
struct Context {
    std::vector<Spec> specs;
    hipStream_t st = nullptr;
    bool own_stream = false;
    DeviceRegion reg;
    std::unique_ptr<Engine> eng;
    std::vector<int> status;
    ~Context() {
        eng.reset();
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
};

std::unique_ptr<Context> prepare(const std::vector<Spec>& specs, const boruta_options* opt,
                                 bool dev_inputs, void* ws, size_t ws_bytes,
                                 hipStream_t user_stream, bool no_alloc = false) {
    Opts o = read_opts(opt);
    apply_tune_cache(o, opt, specs);
    if (no_alloc) {
        if (o.stats)
            throw Error(BORUTA_E_INVALID_ARG,
                        "kernel statistics need HIP events: not in the allocation-free call");
        o.no_alloc = true;
        o.graph = 0;  // launched eagerly: no graph is instantiated
    }
    for (const Spec& s : specs) {
        check_spec(s);
    }
    require_device();
    std::unique_ptr<Context> c(new Context);
    c->specs = specs;
    mark_shared_inputs(c->specs);
    c->st = user_stream;
    if (!ws && !c->st) {
        HIPC(hipStreamCreate(&c->st));
        c->own_stream = true;
    }
    const size_t need = make_plan(c->specs, o, dev_inputs).total;
    char* base = nullptr;
    if (ws) {
        if (ws_bytes < need) throw Error(BORUTA_E_OOM, "workspace smaller than boruta_workspace_size");
        base = (char*)ws;
    } else {
        // BORUTA_FAIL_ALLOC=1 in the environment makes this allocation fail
        // (failure tests: the call must return BORUTA_E_OOM and leak nothing)
        const char* fail = std::getenv("BORUTA_FAIL_ALLOC");
        if ((fail && std::strcmp(fail, "1") == 0) ||
            hipMalloc(&c->reg.p, need) != hipSuccess) {
            (void)hipGetLastError();
            c->reg.p = nullptr;
            throw Error(BORUTA_E_OOM, "hipMalloc of " + std::to_string(need) + " bytes failed");
        }
        base = c->reg.p;
    }
    base = (char*)(((uintptr_t)base + 255) & ~uintptr_t(255));
    c->eng.reset(new Engine(c->specs, o, dev_inputs, base, c->st));
    c->status.assign(specs.size(), BORUTA_OK);
    return c;
}

int run_jobs(const std::vector<Spec>& specs, const boruta_options* opt, std::vector<Out>& outs,
             std::vector<int>& status, bool dev_inputs, void* ws, size_t ws_bytes,
             hipStream_t user_stream, bool no_alloc = false) {
    g_err.clear();
    try {
        std::unique_ptr<Context> c =
            prepare(specs, opt, dev_inputs, ws, ws_bytes, user_stream, no_alloc);
        c->eng->run(outs, status);
        HIPC(hipStreamSynchronize(c->st));
        for (int s : status)
            if (s != BORUTA_OK) {
                g_err = "a job failed validation";
                return s;
            }
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

Spec spec_from(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t K, int32_t T,
               int32_t D, int32_t mtry, int32_t mode, int32_t max_iter, double alpha,
               uint64_t seed) {
    return Spec{X, y, n, p, K, T, D, mtry, mode, max_iter, alpha, seed};
}

int finish_single(int rc, const std::vector<Out>& outs, int32_t* n_iter_out) {
    if (n_iter_out) *n_iter_out = outs[0].n_iter;
    return rc;
}


// The repeated-seed protocol: one problem (classification labels y, or
// regression targets y_reg) run once per seed as one batch, then the median
// aggregate on the device.
int fit_seeds(const float* X, const int32_t* y, const float* y_reg, int64_t n, int64_t p,
              int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
              int32_t importance_mode, int32_t max_iter, double alpha, const uint64_t* seeds,
              int32_t n_seeds, const boruta_options* opt, double* median_importance_out,
              int8_t* decision_out, boruta_result* results) {
    g_err.clear();
    if (!seeds || n_seeds < 1 || n_seeds > 64 || !median_importance_out || !decision_out) {
        g_err = "seeds (1..64 of them), median_importance_out and decision_out are required";
        return BORUTA_E_INVALID_ARG;
    }
    if (p < 1) {
        g_err = "p must be positive";
        return BORUTA_E_INVALID_ARG;
    }
    std::vector<Spec> specs;
    for (int i = 0; i < n_seeds; ++i) {
        specs.push_back(spec_from(X, y, n, p, n_classes, n_trees, max_depth, mtry,
                                  importance_mode, max_iter, alpha, seeds[i]));
        specs.back().yr = y_reg;
    }
    // per-run outputs: the caller's, or a decision scratch (the aggregate reads
    // the histories on the device)
    std::vector<std::vector<int8_t>> dec_s((size_t)n_seeds);
    std::vector<Out> outs(n_seeds);
    for (int i = 0; i < n_seeds; ++i) {
        if (results && results[i].decision && results[i].imp_history) {
            outs[i].decision = results[i].decision;
            outs[i].hist = results[i].imp_history;
            outs[i].hits = results[i].hits;
            outs[i].smax = results[i].shadow_max;
            outs[i].rank = results[i].rank;
        } else {
            dec_s[i].resize((size_t)p);
            outs[i].decision = dec_s[i].data();
            outs[i].hist = nullptr;
        }
    }
    std::vector<int> status(n_seeds, BORUTA_OK);
    try {
        std::unique_ptr<Context> c = prepare(specs, opt, false, nullptr, 0, nullptr);
        c->eng->run(outs, status);
        if (results)
            for (int i = 0; i < n_seeds; ++i) {
                results[i].n_iter = outs[i].n_iter;
                results[i].status = status[i];
            }
        for (int s2 : status)
            if (s2 != BORUTA_OK) {
                g_err = "the problem failed validation";
                return s2;
            }
        c->eng->seed_median(p, median_importance_out, decision_out);
        HIPC(hipStreamSynchronize(c->st));
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}
}  // namespace
}  // namespace boruta

using namespace boruta;

extern "C" {

void boruta_default_options(boruta_options* opt) {
    if (!opt) return;
    opt->n_bins = 256;
    opt->n_perm = 1;
    opt->split_rank = BORUTA_RANK_FP32;
    opt->form = BORUTA_FORM_BATCHED;
    opt->graph = 1;
    opt->small_rows = 32;
    opt->grid_small = 0;
    opt->grid_hist = 0;
    opt->grid_finalize = 0;
    opt->col_level = 0;
    opt->col_unit = 2048;
    opt->grid_col = 0;
    opt->kl_rows = 0;
    opt->perc = 100;
    opt->rough_fix = 0;
    opt->trace = nullptr;
    opt->trace_user = nullptr;
    opt->stats = nullptr;
    opt->hist_rb = 8;
    opt->hist_rb_deep = 8;
    opt->band_level = 6;
    opt->hist_fw = 0;
    opt->col_waves = 0;
    opt->tune_cache = nullptr;
}

int boruta_fit_ex(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                  int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                  int32_t max_iter, double alpha, uint64_t seed, const boruta_options* opt,
                  int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                  double* shadow_max_out, int32_t* n_iter_out) {
    if (!decision_out || !imp_history_out || !n_iter_out) {
        g_err = "decision_out, imp_history_out and n_iter_out must be non-null";
        return BORUTA_E_INVALID_ARG;
    }
    std::vector<Spec> specs{spec_from(X, y, n, p, n_classes, n_trees, max_depth, mtry,
                                      importance_mode, max_iter, alpha, seed)};
    std::vector<Out> outs(1);
    outs[0].decision = decision_out;
    outs[0].hist = imp_history_out;
    outs[0].hits = hits_out;
    outs[0].smax = shadow_max_out;
    std::vector<int> status(1, BORUTA_OK);
    const int rc = run_jobs(specs, opt, outs, status, false, nullptr, 0, nullptr);
    return finish_single(rc, outs, n_iter_out);
}

int boruta_fit_regression(const float* X, const float* y, int64_t n, int64_t p, int32_t n_trees,
                          int32_t max_depth, int32_t mtry, int32_t importance_mode,
                          int32_t max_iter, double alpha, uint64_t seed, const boruta_options* opt,
                          int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                          double* shadow_max_out, int32_t* n_iter_out) {
    if (!decision_out || !imp_history_out || !n_iter_out) {
        g_err = "decision_out, imp_history_out and n_iter_out must be non-null";
        return BORUTA_E_INVALID_ARG;
    }
    Spec sp = spec_from(X, nullptr, n, p, 2, n_trees, max_depth, mtry, importance_mode, max_iter,
                        alpha, seed);
    sp.yr = y;
    std::vector<Spec> specs{sp};
    std::vector<Out> outs(1);
    outs[0].decision = decision_out;
    outs[0].hist = imp_history_out;
    outs[0].hits = hits_out;
    outs[0].smax = shadow_max_out;
    std::vector<int> status(1, BORUTA_OK);
    const int rc = run_jobs(specs, opt, outs, status, false, nullptr, 0, nullptr);
    return finish_single(rc, outs, n_iter_out);
}


int boruta_fit_seeds(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                     int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                     int32_t max_iter, double alpha, const uint64_t* seeds, int32_t n_seeds,
                     const boruta_options* opt, double* median_importance_out,
                     int8_t* decision_out, boruta_result* results) {
    return fit_seeds(X, y, nullptr, n, p, n_classes, n_trees, max_depth, mtry, importance_mode,
                     max_iter, alpha, seeds, n_seeds, opt, median_importance_out, decision_out,
                     results);
}

int boruta_fit_seeds_regression(const float* X, const float* y, int64_t n, int64_t p,
                                int32_t n_trees, int32_t max_depth, int32_t mtry,
                                int32_t importance_mode, int32_t max_iter, double alpha,
                                const uint64_t* seeds, int32_t n_seeds,
                                const boruta_options* opt, double* median_importance_out,
                                int8_t* decision_out, boruta_result* results) {
    return fit_seeds(X, nullptr, y, n, p, 2, n_trees, max_depth, mtry, importance_mode, max_iter,
                     alpha, seeds, n_seeds, opt, median_importance_out, decision_out, results);
}

int boruta_fit(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
               int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
               int32_t max_iter, double alpha, uint64_t seed, int8_t* decision_out,
               double* imp_history_out, int32_t* hits_out, double* shadow_max_out,
               int32_t* n_iter_out) {
    return boruta_fit_ex(X, y, n, p, n_classes, n_trees, max_depth, mtry, importance_mode,
                         max_iter, alpha, seed, nullptr, decision_out, imp_history_out, hits_out,
                         shadow_max_out, n_iter_out);
}

static std::vector<Spec> specs_of(const boruta_job* jobs, int32_t n_jobs) {
    std::vector<Spec> specs;
    for (int i = 0; i < n_jobs; ++i) {
        const boruta_job& b = jobs[i];
        Spec sp = spec_from(b.X, b.y_reg ? nullptr : b.y, b.n, b.p, b.y_reg ? 2 : b.n_classes,
                            b.n_trees, b.max_depth, b.mtry, b.importance_mode, b.max_iter,
                            b.alpha, b.seed);
        sp.yr = b.y_reg;
        specs.push_back(sp);
    }
    return specs;
}

int boruta_fit_batch(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                     boruta_result* results) {
    g_err.clear();
    if (!jobs || !results || n_jobs < 1) {
        g_err = "jobs/results must be non-null and n_jobs >= 1";
        return BORUTA_E_INVALID_ARG;
    }
    std::vector<Spec> specs = specs_of(jobs, n_jobs);
    std::vector<Out> outs(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        if (!results[i].decision || !results[i].imp_history) {
            g_err = "every result needs decision and imp_history buffers";
            return BORUTA_E_INVALID_ARG;
        }
        outs[i].decision = results[i].decision;
        outs[i].hist = results[i].imp_history;
        outs[i].hits = results[i].hits;
        outs[i].smax = results[i].shadow_max;
        outs[i].rank = results[i].rank;
    }
    std::vector<int> status(n_jobs, BORUTA_OK);
    const int rc = run_jobs(specs, opt, outs, status, false, nullptr, 0, nullptr);
    for (int i = 0; i < n_jobs; ++i) {
        results[i].n_iter = outs[i].n_iter;
        results[i].status = rc == BORUTA_OK ? status[i] : (status[i] != BORUTA_OK ? status[i] : rc);
    }
    return rc;
}

int boruta_workspace_size(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                          size_t* bytes) {
    g_err.clear();
    if (!jobs || n_jobs < 1 || !bytes) {
        g_err = "jobs and bytes must be non-null, n_jobs >= 1";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        Opts o = read_opts(opt);
        std::vector<Spec> specs = specs_of(jobs, n_jobs);
        apply_tune_cache(o, opt, specs);
        for (const Spec& s : specs) {
            if (s.n < 2 || s.n > (int64_t(1) << 24) || s.p < 1 || s.p > (int64_t(1) << 24) ||
                s.T < 1 || s.D < 1 || s.D > 30 || s.max_iter < 1 || s.max_iter > 1000 ||
                s.K < 2 || s.K > 16 || s.mode < 0 || s.mode > 2 || s.mtry < 0)
                throw Error(BORUTA_E_INVALID_ARG, "job arguments out of range");
        }
        *bytes = make_plan(specs, o, true).total;
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    }
}

int boruta_fit_device(const float* dX, const int32_t* dy, int64_t n, int64_t p,
                      int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                      int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                      const boruta_options* opt, void* workspace, size_t ws_bytes,
                      void* hip_stream, int8_t* decision_out, double* imp_history_out,
                      int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out) {
    if (!decision_out || !imp_history_out || !n_iter_out || !workspace) {
        g_err = "decision_out, imp_history_out, n_iter_out and workspace must be non-null";
        return BORUTA_E_INVALID_ARG;
    }
    std::vector<Spec> specs{spec_from(dX, dy, n, p, n_classes, n_trees, max_depth, mtry,
                                      importance_mode, max_iter, alpha, seed)};
    std::vector<Out> outs(1);
    outs[0].decision = decision_out;
    outs[0].hist = imp_history_out;
    outs[0].hits = hits_out;
    outs[0].smax = shadow_max_out;
    std::vector<int> status(1, BORUTA_OK);
    const int rc = run_jobs(specs, opt, outs, status, true, workspace, ws_bytes,
                            (hipStream_t)hip_stream);
    return finish_single(rc, outs, n_iter_out);
}

}  // extern "C"

namespace {

// Scratch of the allocation-free entry point: a file-scope device array of
// kScratchBytes that every GPU the library runs on holds until the process
// ends.  Host code never uses the array's name as an address (on the host it
// only stands in for the symbol); the device address is taken once per device,
// with that device current, by hipGetSymbolAddress and kept in g_scratch.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch;  // [device] scratch's device address (null: not yet taken)

void* scratch_address() {
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[(size_t)dev]) {
        void* p = nullptr;
        HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(BORUTA_E_DEVICE, "hipGetSymbolAddress returned no address");
        g_scratch[(size_t)dev] = p;
    }
    return g_scratch[(size_t)dev];
}

}  // namespace

extern "C" {

int boruta_fit_device_noalloc(const float* dX, const int32_t* dy, int64_t n, int64_t p,
                              int32_t n_classes, int32_t n_trees, int32_t max_depth,
                              int32_t mtry, int32_t importance_mode, int32_t max_iter,
                              double alpha, uint64_t seed, const boruta_options* opt,
                              void* hip_stream, int8_t* decision_out, double* imp_history_out,
                              int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out) {
    g_err.clear();
    if (!decision_out || !imp_history_out || !n_iter_out) {
        g_err = "decision_out, imp_history_out and n_iter_out must be non-null";
        return BORUTA_E_INVALID_ARG;
    }
    std::vector<Spec> specs{spec_from(dX, dy, n, p, n_classes, n_trees, max_depth, mtry,
                                      importance_mode, max_iter, alpha, seed)};
    void* ws = nullptr;
    try {
        Opts o = read_opts(opt);
        apply_tune_cache(o, opt, specs);
        check_spec(specs[0]);
        require_device();
        // the problem must fit the scratch (the workspace plan of boruta_fit_device,
        // plus the alignment slack of its base)
        const size_t need = make_plan(specs, o, true).total;
        if (need > kScratchBytes)
            throw Error(BORUTA_E_INVALID_ARG,
                        "problem needs " + std::to_string(need) +
                            " bytes of device scratch; the allocation-free call holds " +
                            std::to_string(kScratchBytes));
        ws = scratch_address();
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    }
    std::vector<Out> outs(1);
    outs[0].decision = decision_out;
    outs[0].hist = imp_history_out;
    outs[0].hits = hits_out;
    outs[0].smax = shadow_max_out;
    std::vector<int> status(1, BORUTA_OK);
    const int rc = run_jobs(specs, opt, outs, status, true, ws, kScratchBytes,
                            (hipStream_t)hip_stream, true);
    return finish_single(rc, outs, n_iter_out);
}

int boruta_bin(const float* X, int64_t n, int64_t p, int32_t n_bins, uint8_t* bins_out) {
    g_err.clear();
    if (!X || !bins_out || n < 1 || n > (int64_t(1) << 24) || p < 1 ||
        p > (int64_t(1) << 24) || n_bins < 2 || n_bins > 256) {
        g_err = "X and bins_out non-null, n and p in [1, 2^24], n_bins in [2, 256]";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        require_device();
        const int64_t n_pad = round_up(n, 256), P = pow2_at_least(n);
        const size_t bx = (size_t)n * p * 4, bk = (size_t)p * P * 4, bb = (size_t)p * n_pad;
        DeviceRegion reg;
        const char* fail = std::getenv("BORUTA_FAIL_ALLOC");
        if ((fail && std::strcmp(fail, "1") == 0) ||
            hipMalloc(&reg.p, bx + bk + bb + 256) != hipSuccess) {
            (void)hipGetLastError();
            reg.p = nullptr;
            throw Error(BORUTA_E_OOM, "hipMalloc for the binning failed");
        }
        float* dX = reinterpret_cast<float*>(reg.p);
        uint32_t* keys = reinterpret_cast<uint32_t*>(reg.p + bx);
        uint8_t* bins = reinterpret_cast<uint8_t*>(reg.p + bx + bk);
        uint32_t* flags = reinterpret_cast<uint32_t*>(reg.p + ((bx + bk + bb + 3) & ~size_t(3)));
        hipStream_t st = nullptr;
        HIPC(hipMemcpyAsync(dX, X, bx, hipMemcpyHostToDevice, st));
        launch_fill_u32(flags, 1, 0u, st);
        launch_validate_reg(dX, (size_t)n * p, dX, 0, flags, st);  // X finite
        uint32_t f = 0;
        HIPC(hipMemcpyAsync(&f, flags, 4, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        if (f) throw Error(BORUTA_E_NONFINITE, "X holds NaN or Inf");
        launch_binning(dX, n, p, n_bins, bins, n_pad, keys, P, st);
        HIPC(hipMemcpy2DAsync(bins_out, (size_t)n, bins, (size_t)n_pad, (size_t)n, (size_t)p,
                              hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

int boruta_probe_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
    g_err.clear();
    if (!dst || !src || bytes % 16) {
        g_err = "dst/src must be non-null and bytes a multiple of 16";
        return BORUTA_E_INVALID_ARG;
    }
    launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_err = hipGetErrorString(e);
        return BORUTA_E_DEVICE;
    }
    return BORUTA_OK;
}

}  // extern "C"

struct boruta_session {
    std::unique_ptr<boruta::Context> ctx;
};

extern "C" {

int boruta_session_create(const boruta_job* jobs, int32_t n_jobs, const boruta_options* opt,
                          int32_t inputs_on_device, void* workspace, size_t ws_bytes,
                          void* hip_stream, boruta_session** out) {
    g_err.clear();
    if (!jobs || n_jobs < 1 || !out) {
        g_err = "jobs and out must be non-null, n_jobs >= 1";
        return BORUTA_E_INVALID_ARG;
    }
    *out = nullptr;
    try {
        std::unique_ptr<boruta_session> s(new boruta_session);
        s->ctx = prepare(specs_of(jobs, n_jobs), opt, inputs_on_device != 0, workspace, ws_bytes,
                         (hipStream_t)hip_stream);
        s->ctx->eng->setup(s->ctx->status);
        for (int32_t j = 0; j < n_jobs; ++j)
            if (s->ctx->status[j] != BORUTA_OK) {
                g_err = "job " + std::to_string(j) + " failed validation";
                return s->ctx->status[j];
            }
        *out = s.release();
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

int boruta_session_step(boruta_session* s, int32_t* n_live_out) {
    g_err.clear();
    if (!s) {
        g_err = "null session";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        const int n = s->ctx->eng->step();
        s->ctx->eng->flush_stats();
        if (n_live_out) *n_live_out = n;
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

int boruta_session_run(boruta_session* s, int32_t max_steps, int32_t* n_live_out,
                       int64_t* job_iterations_out) {
    g_err.clear();
    if (!s || max_steps < 0) {
        g_err = "null session or max_steps < 0";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        int n = 0;
        const int64_t done = s->ctx->eng->run_steps(max_steps, &n);
        s->ctx->eng->flush_stats();
        if (n_live_out) *n_live_out = n;
        if (job_iterations_out) *job_iterations_out = done;
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

int boruta_session_result(boruta_session* s, int32_t job, boruta_result* out) {
    g_err.clear();
    if (!s || !out || job < 0 || job >= (int32_t)s->ctx->specs.size() || !out->decision) {
        g_err = "bad session, job index or result buffers";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        Out o;
        o.decision = out->decision;
        o.hist = out->imp_history;
        o.hits = out->hits;
        o.smax = out->shadow_max;
        o.rank = out->rank;
        s->ctx->eng->result(job, o);
        out->n_iter = o.n_iter;
        out->status = BORUTA_OK;
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

int boruta_session_resume(boruta_session* s, int32_t job, int32_t t, const int8_t* state,
                          const int32_t* hits) {
    g_err.clear();
    if (!s || !state || !hits || job < 0 || job >= (int32_t)s->ctx->specs.size()) {
        g_err = "bad session, job index or checkpoint buffers";
        return BORUTA_E_INVALID_ARG;
    }
    try {
        s->ctx->eng->resume(job, t, state, hits);
        return BORUTA_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return BORUTA_E_DEVICE;
    }
}

void boruta_session_destroy(boruta_session* s) { delete s; }

const char* boruta_last_error(void) { return g_err.c_str(); }

}  // extern "C"
