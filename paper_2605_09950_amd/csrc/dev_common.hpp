// dev_common.hpp -- types and device helpers shared by the HIP kernels and
// the host engine of libboruta.so (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace boruta {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// Random streams.  Every random draw of a run is Philox4x32-10 (Salmon et al.,
// SC'11) keyed by the job's 64-bit seed, at a counter that names what is
// drawn: word0 = stream<<28 | feistel_round<<24 | iteration, then (a, b, c).
enum : uint32_t { kBoot = 1, kMtry = 2, kShadow = 3, kOobPerm = 4, kFlush = 5 };

struct Philox4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ uint32_t ctr_word0(uint32_t stream, uint32_t round,
                                                       uint32_t t) {
    return (stream << 28) | (round << 24) | (t & 0xFFFFFFu);
}

// Keyed bijection of [0, m): balanced Feistel network over the smallest even
// bit width k >= 2 with 2^k >= m, halves of h = k/2 bits, max(6, ceil(24/h))
// rounds with round function word 0 of Philox(word0(stream, r, t), a, b,
// c_hi | R) masked to h bits, cycle-walked back into [0, m).
struct KeyedPerm {
    uint32_t k0, k1, w0, a, b, c_hi;
    uint32_t half, mask, rounds;
    uint64_t m;
};

__host__ __device__ __forceinline__ KeyedPerm make_perm(uint32_t k0, uint32_t k1,
                                                        uint32_t stream, uint32_t t, uint32_t a,
                                                        uint32_t b, uint32_t c_hi, uint64_t m) {
    KeyedPerm P;
    P.k0 = k0;
    P.k1 = k1;
    P.w0 = ctr_word0(stream, 0, t);
    P.a = a;
    P.b = b;
    P.c_hi = c_hi;
    P.m = m;
    uint32_t k = 0;
    while ((uint64_t(1) << k) < m) ++k;
    if (k < 2) k = 2;
    k += k & 1u;
    P.half = k >> 1;
    P.mask = (1u << P.half) - 1u;
    const uint32_t r = (24u + P.half - 1u) / P.half;
    P.rounds = r > 6u ? r : 6u;
    return P;
}

__device__ __forceinline__ uint32_t perm_round(const KeyedPerm& P, uint32_t r, uint32_t right) {
    return philox4x32_10(P.w0 | (r << 24), P.a, P.b, P.c_hi | right, P.k0, P.k1).x & P.mask;
}

__device__ __forceinline__ uint32_t perm_apply(const KeyedPerm& P, uint32_t x) {
    if (P.m <= 1) return 0;
    do {
        uint32_t left = x >> P.half, right = x & P.mask;
        for (uint32_t r = 0; r < P.rounds; ++r) {
            const uint32_t f = perm_round(P, r, right);
            const uint32_t nl = right;
            right = left ^ f;
            left = nl;
        }
        x = (left << P.half) | right;
    } while ((uint64_t)x >= P.m);
    return x;
}

// One pass of the Feistel network (no cycle walking): perm_apply repeats it
// from x until the value falls below m.
__device__ __forceinline__ uint32_t perm_pass(const KeyedPerm& P, uint32_t x) {
    uint32_t left = x >> P.half, right = x & P.mask;
    for (uint32_t r = 0; r < P.rounds; ++r) {
        const uint32_t f = perm_round(P, r, right);
        const uint32_t nl = right;
        right = left ^ f;
        left = nl;
    }
    return (left << P.half) | right;
}

// Same bijection with the round functions tabulated: tab[r << half | R].
__device__ __forceinline__ uint32_t perm_apply_tab(const KeyedPerm& P, const uint16_t* tab,
                                                   uint32_t x) {
    if (P.m <= 1) return 0;
    do {
        uint32_t left = x >> P.half, right = x & P.mask;
        for (uint32_t r = 0; r < P.rounds; ++r) {
            const uint32_t f = tab[(r << P.half) | right];
            const uint32_t nl = right;
            right = left ^ f;
            left = nl;
        }
        x = (left << P.half) | right;
    } while ((uint64_t)x >= P.m);
    return x;
}

// Load through the global address space (the pointers here are generic; the
// cast lets the compiler issue global loads that overlap instead of flat
// loads that also wait on LDS traffic).
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

// Row record i of a node's len >= 1 records, 0 (weight 0) past the end: the
// load itself is unconditional (clamped to the last record), so a batch of
// them issues back to back instead of one branch per load.
__device__ __forceinline__ uint64_t rec_at(const uint64_t* recs, uint32_t i, uint32_t len) {
    const uint64_t v = ldg(recs + (i < len ? i : len - 1u));
    return i < len ? v : 0ull;
}
// The same load without the mask, for records loaded ahead of their use (a
// prefetch): the caller masks past-the-end records when it uses them, so the
// load need not complete at the point of the call.
__device__ __forceinline__ uint64_t rec_raw(const uint64_t* recs, uint32_t i, uint32_t len) {
    return ldg(recs + (i < len ? i : len - 1u));
}

// Wave-uniform values: the compiler cannot see that e.g. threadIdx.x / 64 is
// the same in every lane; readfirstlane moves such values to scalar registers.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
// Value of lane `src` (a wave-uniform index) as a scalar.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Exact integer helpers.
__device__ __forceinline__ int clz128(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return hi ? __clzll(hi) : 64 + (lo ? __clzll(lo) : 64);
}

__device__ __forceinline__ double u128_to_double(u128 v) {
    return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v;
}

// floor(num / den), exact, for quotients below 2^62 (larger ones saturate).
// A double-precision estimate (relative error ~2^-51: a few units for the
// quotients used here) is corrected with 128-bit remainders; if it is off by
// more than 64 units, shift-subtract long division is used instead, so the
// loop count is bounded for every input.
__device__ __forceinline__ uint64_t udiv128(u128 num, u128 den) {
    if (den == 0 || num < den) return 0;
    if ((num >> 62) >= den) return (uint64_t)1 << 62;  // quotient >= 2^62: saturate
    const double qd = u128_to_double(num) / u128_to_double(den);
    uint64_t q = (uint64_t)(qd < 4.0e18 ? qd : 4.0e18);
    u128 prod = (u128)q * den;  // q < 2^62 and den <= num < 2^62 den: no overflow
    for (int step = 0; step < 64; ++step) {
        if (prod > num) {
            --q;
            prod -= den;
        } else if (num - prod >= den) {
            ++q;
            prod += den;
        } else {
            return q;
        }
    }
    const int shift = clz128(den) - clz128(num);
    u128 d = den << shift, r = num;
    q = 0;
    for (int i = 0; i <= shift; ++i) {
        q <<= 1;
        if (r >= d) {
            r -= d;
            q |= 1;
        }
        d >>= 1;
    }
    return q;
}

// ---------------------------------------------------------------------------
// Split candidate: threshold b of the feature at draw position q (widened
// column f); left/right weighted counts N and sums of squared class counts S.
struct Cand {
    int32_t q, f, b;
    uint32_t nl, nr, pad;
    uint64_t sl, sr;
};

// Q_a > Q_b exactly, with Q = S_L/N_L + S_R/N_R (cross-multiplied in 128 bits;
// every product stays below 2^121 for N < 2^24).
__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
    const u128 na = (u128)a.sl * a.nr + (u128)a.sr * a.nl;
    const u128 nb = (u128)b.sl * b.nr + (u128)b.sr * b.nl;
    const uint64_t da = (uint64_t)a.nl * a.nr, db = (uint64_t)b.nl * b.nr;
    return na * db > nb * da;
}

// Q > S/N exactly (strictly positive Gini decrease).
__device__ __forceinline__ bool cand_positive(const Cand& c, uint64_t s, uint64_t n) {
    const u128 num = (u128)c.sl * c.nr + (u128)c.sr * c.nl;
    return num * n > (u128)s * ((uint64_t)c.nl * c.nr);
}

// floor(2^32 * (Q - S/N)).
__device__ __forceinline__ uint64_t cand_gain_fix(const Cand& c, uint64_t s, uint64_t n) {
    const uint64_t lr = (uint64_t)c.nl * c.nr;
    const u128 num = ((u128)c.sl * c.nr + (u128)c.sr * c.nl) * n - (u128)s * lr;
    const u128 den = (u128)lr * n;
    return udiv128(num << 32, den);
}

// FP32 score used only to rank candidates: S_L * rcp(N_L) + S_R * rcp(N_R)
// with the hardware reciprocal (1 ulp).  Relative error <= 5u, u = 2^-24:
// u converting S, 2u the reciprocal, u the product, u the sum (N < 2^24 is
// exact in FP32).
__device__ __forceinline__ float cand_q32(const Cand& c) {
    return (float)c.sl * __builtin_amdgcn_rcpf((float)c.nl) +
           (float)c.sr * __builtin_amdgcn_rcpf((float)c.nr);
}

// ---------------------------------------------------------------------------
// Device-resident run state.
struct JobDev {
    // fixed for the run
    int32_t n, n_pad, p, K, B, T, D, mtry_opt, mode, R, max_iter;
    uint32_t seed_lo, seed_hi;
    int32_t max_sha;       // shadow column capacity
    int32_t pw_cap;        // p + max_sha
    uint32_t gbase;        // first global column id of the job (column-major histogram path)
    uint32_t gq;           // 16-byte words of one bin column (n_pad / 16)
    uint32_t rstride;      // row records per tree (n)
    int32_t reg;           // regression job: targets in yfix, labels unused
    // regression: fixed-point shifts of the decrease, the Permut and the
    // divergence scores, and the binary exponent of the reported importance
    int32_t s_gain, s_perm, s_kl, rep_exp;
    const int64_t* yfix;   // [n] regression: targets rint(y 2^(38 - e))
    const uint8_t* y;      // [n] class labels
    uint8_t* orig;         // [p][n_pad] binned originals
    uint8_t* sha;          // [max_sha][n_pad] shadows of the current iteration
    const uint8_t** colptr;// [pw_cap] widened column -> bins
    int32_t* col_src;      // [pw_cap]
    int32_t* act;          // [p] active originals, ascending
    int8_t* state;         // [p]
    int32_t* hits;         // [p]
    double* hist;          // [max_iter][p]
    double* shadow_max;    // [max_iter]
    int32_t* h_conf;       // [max_iter + 1] smallest hit count that confirms at t
    int32_t* h_rej;        // [max_iter + 1] largest hit count that rejects at t
    uint64_t* G;           // [T][pw_cap] per-tree fixed-point Gini decreases
    int64_t* imp;          // [pw_cap] integer importance of the iteration
    uint32_t* wbuf;        // [T][n] bootstrap multiplicities
    uint64_t* rec[2];      // [T][rstride] row records, ping-pong by level parity
    uint32_t* oob;         // [T][n] out-of-bag rows, ascending
    int32_t* tstat;        // [T][4] distinct in-bag, OOB rows, OOB correct, spare
    uint8_t* rowmaj;       // [n_pad][rm_stride] the widened bins row-major, rebuilt every
                           // iteration (null: the job keeps none)
    uint32_t rm_stride;    // pw_cap rounded up to 64
    uint32_t pad_rm;
    // per iteration, written on the device
    int32_t t, p_cur, n_sha, p_w, mtry, pad_i, n_undecided, live;
};

struct TreeDev {
    int32_t job, tau;
};

// One tree node.  Roots of the iteration's trees are nodes [0, n_trees).
struct NodeDev {
    uint32_t tree;   // global tree index of the iteration
    uint32_t heap;   // heap id: root 1, children 2h, 2h+1
    uint32_t seg;    // first row record (within the tree's record block)
    uint32_t len;    // distinct rows
    uint32_t n;      // weighted rows
    int32_t feat;    // widened column, -1 for a leaf
    uint32_t left;   // index of the left child; the right one is left + 1
    uint16_t thr;    // threshold bin (left iff bin <= thr)
    uint8_t leaf_class;
    uint8_t depth;
};

// What a histogram item needs of its large node, gathered once per node and
// level so that an item's first loads do not depend on each other.
struct SlotRec {
    const uint64_t* recs;  // the node's row records (this level's parity)
    const int64_t* yfix;   // regression job: its fixed-point targets (else null)
    uint32_t id;           // node index
    uint32_t len, n;       // distinct rows, weighted rows
    uint32_t mtry;         // features drawn this iteration
    uint32_t B, reg;       // bins; 1 for a regression job
    uint32_t K, pad;       // the job's classes
    uint32_t cnode[16];    // weighted class counts (zero past K); regression: the
                           // weighted target sum T in words 0 (low) and 1 (high)
};

// Per-level counters: the lists of tree level d (small nodes, large-node
// slots) are counted in ctrs[d]; they are zeroed once per iteration.
struct LevelCtr {
    uint32_t unused[2];
    uint32_t n_slots;   // large nodes
    uint32_t n_small;   // small nodes
    uint32_t overflow;  // a capacity check failed
    uint32_t n_units;   // column units of the column-major histogram path
    uint32_t pad[2];
};

// Row record: row | weight << 32 | label << 48.
__device__ __forceinline__ uint64_t rec_pack(uint32_t row, uint32_t w, uint32_t y) {
    return (uint64_t)row | ((uint64_t)w << 32) | ((uint64_t)y << 48);
}
__device__ __forceinline__ uint32_t rec_row(uint64_t r) { return (uint32_t)r; }
__device__ __forceinline__ uint32_t rec_w(uint64_t r) { return (uint32_t)(r >> 32) & 0xFFFFu; }
__device__ __forceinline__ uint32_t rec_y(uint64_t r) { return (uint32_t)(r >> 48) & 0xFFu; }

// k_col_count: columns counted in LDS (64 KB) and its workgroups
constexpr uint32_t kColCountLds = 16384;
constexpr uint32_t kColCountGrid = 512;
// Keyed-permutation round tables in LDS: 16-bit entries per table, rounds
// << half for halves of at most 8 bits (6 rounds of 256 entries at most)
constexpr uint32_t kDrawTab = 1536;
constexpr int kSmallRows = 64;  // nodes with at most this many distinct rows take the wave path
constexpr int kWave = 64;
constexpr uint32_t kAlgWords = 1024;  // statistics words per kernel

// Draws per histogram work item (one wavefront, LDS histogram of
// hist_fw * kmax rows of 256 bins): 4 KB per wave up to 4 classes.
__host__ __device__ constexpr int hist_fw(int kmax) { return kmax <= 4 ? 4 / kmax : 1; }

// Column-major histogram path: a unit is a run of items (node, draw) of one
// bin column; the column is staged once per unit in LDS.
struct ColUnit {
    uint32_t begin, end;  // items [begin, end) of the feature-sorted item list
    uint32_t gq;          // 16-byte words of the column
    uint32_t pad;
};
constexpr uint32_t kColWavesMax = 16;  // waves per workgroup of the column path

struct ForestDev {
    JobDev* jobs;
    const TreeDev* trees;
    NodeDev* nodes;
    uint32_t* cls;        // [node][kmax] weighted class counts
    uint64_t* ngain;      // [node] fixed-point Gini decrease of a split node
    Cand* cand;           // [slot][npi] best candidate of each histogram item
    uint32_t* cand_cl;    // [slot][npi][kmax] left class counts of that candidate
    uint32_t* feat;       // [slot][mtry_cap] the node's drawn features, draw order
    const uint8_t** fcol; // [slot][mtry_cap] their bin columns
    SlotRec* srec;        // [slot] the large nodes of the level
    uint8_t* kinds;       // [searched node of the level] what its two children need
                          // next (2 bits each: leaf, wave path, histogram path)
    unsigned long long* chunk_sums;  // [chunk] (wave-path, histogram-path) children
    const uint32_t* slot_node_in;  // [slot] node of each large-node slot of this level
    uint32_t* slot_node_out;       // [slot] the same for the next level
    const uint32_t* small_in;
    uint32_t* small_out;
    LevelCtr* ctr;        // counters the current launch appends to (set per kernel)
    LevelCtr* ctrs;       // [levels + 1]: ctrs[d] counts the lists of tree level d
    uint32_t n_roots;     // trees of the iteration (= root nodes [0, n_roots))
    uint64_t* alg_bytes;  // [3][kAlgWords] algorithmic bytes (node-major large, small,
                          // column-major large), nullable;
                          // the words per kernel spread the atomics
    uint32_t node_cap, slot_cap, small_cap;
    uint32_t next_base;   // first node index of the next level
    uint32_t n_small_cur; // small nodes searched in this level
    uint32_t small_ncap;  // a node takes the wave path only below this weighted count
    int32_t kmax, parity, split_rank;
    int32_t has_cls, has_reg;  // the plan holds classification / regression jobs
    int32_t split_k;      // a plan of more than 4 class planes that also holds jobs of at
                          // most 4 classes: their node-major items take the 4-plane kernel
    int32_t npi;          // histogram items per large node (draw positions / fw)
    int32_t fw;           // draws per histogram item
    uint32_t small_rows;  // a node takes the wave path only up to this many distinct rows
    int32_t mtry_cap;     // row stride of feat
    uint32_t draw_seg;    // lanes per node in k_draws: mtry_cap rounded up to a power
                          // of two, at most 64
    uint32_t draw_tab;    // k_draws: round-table entries per node segment (0: no tables;
                          // a permutation with more entries is walked directly)
    // column-major histogram path (null when the plan has none)
    uint32_t* fcnt;       // [n_gcol] items per global column, zero between levels
    uint32_t* fpos;       // [slot][mtry_cap] an item's place within its column's items,
                          // then [n_gcol] the columns' offsets in fitems
    const uint32_t* gcol_q;  // [n_gcol] 16-byte words of each column
    uint32_t* fitems;     // [slot * mtry_cap] items sorted by column
    ColUnit* units;       // [unit_cap]
    uint32_t n_gcol, unit_cap, col_unit;  // columns, unit capacity, items per unit
    int32_t col_count;    // this level takes the column path: its items' places in their
                          // columns are counted by k_draws (1) or k_col_count (2)
};

}  // namespace boruta
