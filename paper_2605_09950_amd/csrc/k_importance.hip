// k_importance.hip -- importance scores, hits and decisions (gfx950).
//
//   * TreeImp (Algorithm 2, Sec. 2.1): per tree, each widened column's summed
//     fixed-point Gini decrease G (accumulated at split time) is normalised
//     to floor(2^44 G / sum_f G) and the shares are summed over trees; the
//     mean's 1/T cancels in the final renormalisation.
//   * Permut (Kursa's accuracy drop, Sec. 2; Sec. 2.2): for every tree, OOB
//     row j, column f on the row's path and replica r, the row is re-routed
//     with f's bin taken from OOB row pi(j), pi the keyed permutation of the
//     tree's OOB rows for (t, tree, f, r); the drop in correct predictions is
//     summed per column.  Columns off the path cannot change the prediction,
//     so only path columns are re-routed, from their first node on the path.
//   * KL permutation importance (Algorithm 3, Sec. 2.2; importance mode 2):
//     the forest's class distribution for row r is the sum over trees of
//     floor(2^32 c_k / N) at the leaf r reaches; one keyed row permutation
//     pi per iteration serves every column, whose bin at row r is replaced
//     by the bin at row pi(r); the column scores the sum over rows of
//     KL(P || Q) in bits with 32 fractional bits (a class Q misses while P
//     has it counts one unit).  Again only the columns on a row's path in a
//     tree can move it to another leaf of that tree: per (row, tree) those
//     columns are re-routed and the leaf differences accumulated per
//     (column, row); rows are taken in blocks that bound that buffer.
//   * hits (strictly above the best shadow) and the binomial decision;
//   * Algorithm 1's final ranking: confirmed 1, undecided 2, rejected from 3
//     by descending historical importance (the mean of the feature's finite
//     history entries, summed in iteration order; equal means share a rank).
#include "dev_common.hpp"
#include "reg_dev.hpp"

namespace boruta {

// Per tree: total fixed-point decrease over its columns.
__global__ __launch_bounds__(256) void k_tree_totals(JobDev* jobs, const TreeDev* trees,
                                                     uint64_t* tot) {
    __shared__ unsigned long long s[4];
    const TreeDev tr = trees[blockIdx.x];
    const JobDev& J = jobs[tr.job];
    if (!J.live || J.mode != 0) return;  // finished job, or Permut job of a mixed batch
    const uint64_t* G = J.G + (size_t)tr.tau * J.pw_cap;
    unsigned long long v = 0;
    for (int f = threadIdx.x; f < J.p_w; f += 256) v += G[f];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) tot[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Per (column, tree): I_f += floor(2^44 G[tree][f] / total of the tree),
// summed with 64-bit integer atomics (exact in any order).  G is cleared
// behind the read, ready for the next iteration.
__global__ __launch_bounds__(256) void k_treeimp(JobDev* jobs, const TreeDev* trees,
                                                 const uint64_t* tot) {
    const uint32_t g = blockIdx.y;
    const TreeDev tr = trees[g];
    JobDev& J = jobs[tr.job];
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (!J.live || J.mode != 0 || f >= J.p_w) return;
    uint64_t* Gp = J.G + (size_t)tr.tau * J.pw_cap + f;
    const uint64_t gv = ldg(Gp);
    if (gv == 0) return;
    *Gp = 0;
    atomicAdd((unsigned long long*)&J.imp[f],
              (unsigned long long)udiv128((u128)gv << 44, (u128)tot[g]));
}

// Permut: one thread per (tree, OOB row).  When the job's widened width is
// at most lds_cols, the drops are summed per column in LDS and each
// workgroup adds its nonzero sums to the importances: once most columns are
// decided, few remain and per-row atomics would all meet on them (with many
// columns the per-row atomics are spread out and cheaper than a flush per
// workgroup).  For a regression job a row's score is the negated squared
// error against its leaf's prediction, sq_error_fix below, and the
// per-column sums in LDS are 64-bit.
// Prediction of a regression leaf: floor(T / W), T in the node's first two
// class words and W its weighted count.
__device__ __forceinline__ long long leaf_pred(const NodeDev* nodes, const uint32_t* cls, int kmax,
                                               uint32_t node) {
    const int64_t T = (int64_t)((uint64_t)cls[(size_t)node * kmax] |
                                ((uint64_t)cls[(size_t)node * kmax + 1] << 32));
    return (long long)reg_pred(T, nodes[node].n);
}

// floor((y_fix - pred)^2 / 2^s_perm) (|y_fix - pred| < 2^40).
__device__ __forceinline__ long long sq_error_fix(const NodeDev* nodes, const uint32_t* cls,
                                                  int kmax, uint32_t node, long long yfix,
                                                  int s_perm) {
    const long long e = yfix - leaf_pred(nodes, cls, kmax, node);
    const u128 a = (u128)(uint64_t)(e < 0 ? -e : e);
    return (long long)((a * a) >> s_perm);
}

// (path column, replica) pairs whose OOB sources are walked together
constexpr int kPermGroup = 8;

__global__ __launch_bounds__(256) void k_permut(JobDev* jobs, const TreeDev* trees,
                                                const NodeDev* nodes, const uint32_t* cls,
                                                int kmax, int max_depth, int lds_cols,
                                                int lds_words, unsigned long long* visits) {
    // [2][max_depth][256]: node, feature; [lds_words]: the column drops
    // (lds_cols of them); [kPermGroup][256]: a group's source rows
    extern __shared__ uint32_t s_path[];
    const uint32_t g = blockIdx.y;
    const TreeDev tr = trees[g];
    JobDev& J = jobs[tr.job];
    if (!J.live || J.mode != 1) return;  // finished job, or TreeImp job of a mixed batch
    const int tid = threadIdx.x;
    const uint32_t m = (uint32_t)J.tstat[tr.tau * 4 + 1];
    const uint32_t j = blockIdx.x * 256u + tid;
    if (blockIdx.x * 256u >= m) return;
    int* s_drop = reinterpret_cast<int*>(s_path + 2 * max_depth * 256);
    long long* s_drop64 = reinterpret_cast<long long*>(s_drop);  // regression jobs
    const bool reg = J.reg != 0;
    const bool lds = J.p_w <= lds_cols;  // uniform: one tree per workgroup
    if (lds) {
        for (int c = tid; c < J.p_w; c += 256) {
            if (reg)
                s_drop64[c] = 0;
            else
                s_drop[c] = 0;
        }
        __syncthreads();
    }
    const bool active = j < m;
    const uint32_t* oob = J.oob + (size_t)tr.tau * J.n;
    const uint32_t row = active ? oob[j] : 0u;
    const uint32_t yv = reg ? 0u : (uint32_t)J.y[row];
    const long long yfv = reg ? (long long)J.yfix[row] : 0ll;
    uint32_t* pn = s_path;
    uint32_t* pf = s_path + max_depth * 256;
    int len = 0;
    uint32_t node = g;
    bool base_ok = false;
    long long base_err = 0;
    unsigned long long nv = 0;  // node visits (statistics)
    if (active) {
        NodeDev nd = nodes[node];
        while (nd.feat >= 0) {
            pn[len * 256 + tid] = node;
            pf[len * 256 + tid] = (uint32_t)nd.feat;
            ++len;
            node = (int)J.colptr[nd.feat][row] <= (int)nd.thr ? nd.left : nd.left + 1;
            nd = nodes[node];
        }
        nv += (unsigned long long)len + 1u;
        if (reg)
            base_err = sq_error_fix(nodes, cls, kmax, node, yfv, J.s_perm);
        else
            base_ok = nd.leaf_class == yv;
    }
    const unsigned long long okm = __ballot(active && base_ok);
    if ((tid & 63) == 0 && okm) atomicAdd(&J.tstat[tr.tau * 4 + 2], (int)__popcll(okm));
    // The row's (path column, replica) pairs in order -- path positions in
    // order, a column already on the path skipped, replicas 0..R-1 -- taken
    // kPermGroup at a time.  First the group's source rows, pi(j) of each
    // pair's keyed OOB permutation, by walks interleaved in one loop (a lane
    // starts its next pair's walk as soon as one ends, so the wave waits for
    // the lane with the longest total rather than for the longest walk of
    // every pair), kept in LDS; then each pair's re-routing.
    uint32_t* g_src = s_path + 2 * max_depth * 256 + lds_words;  // [kPermGroup][256]
    const int R = J.R;
    // next pair at or after (pi, r): a column already on the path is skipped
    auto next_pair = [&](int& pi, int& r) {
        if (++r < R) return;
        r = 0;
        for (++pi; pi < len; ++pi) {
            const uint32_t f = pf[pi * 256 + tid];
            bool dup = false;
            for (int pj = 0; pj < pi; ++pj) dup |= pf[pj * 256 + tid] == f;
            if (!dup) return;
        }
    };
    auto pair_perm = [&](int pi, int r) {
        return make_perm(J.seed_lo, J.seed_hi, kOobPerm, (uint32_t)J.t, (uint32_t)tr.tau,
                         pf[pi * 256 + tid], (uint32_t)r << 16, (uint64_t)m);
    };
    int cpi = 0, cr = 0;  // the next pair to score (position 0 is never a duplicate)
    while (active && cpi < len) {
        // walks of the group's pairs
        int wpi = cpi, wr = cr, k = 0;
        KeyedPerm P = pair_perm(wpi, wr);
        uint32_t x = j;
        while (k < kPermGroup && wpi < len) {
            if (m > 1u) x = perm_pass(P, x);
            if (m <= 1u || x < m) {
                g_src[k * 256 + tid] = m <= 1u ? 0u : x;
                ++k;
                next_pair(wpi, wr);
                x = j;
                if (wpi < len) P = pair_perm(wpi, wr);
            }
        }
        // re-routing of the group's pairs; a column's drops are added when
        // its pairs end or the group does
        int drop = 0;
        long long drop_sq = 0;  // regression: increase of the squared error
        for (int g = 0; g < k; ++g) {
            const uint32_t f = pf[cpi * 256 + tid];
            const int sb = J.colptr[f][oob[g_src[g * 256 + tid]]];
            uint32_t nd_i = pn[cpi * 256 + tid];
            NodeDev nd = nodes[nd_i];
            ++nv;
            while (nd.feat >= 0) {
                const int b = (uint32_t)nd.feat == f ? sb : (int)J.colptr[nd.feat][row];
                nd_i = b <= (int)nd.thr ? nd.left : nd.left + 1;
                nd = nodes[nd_i];
                ++nv;
            }
            if (reg)
                drop_sq += sq_error_fix(nodes, cls, kmax, nd_i, yfv, J.s_perm) - base_err;
            else
                drop += (int)base_ok - (int)(nd.leaf_class == yv);
            const int opi = cpi;
            next_pair(cpi, cr);
            if (cpi != opi || g + 1 == k) {
                if (drop_sq) {
                    if (lds)
                        atomicAdd((unsigned long long*)&s_drop64[f], (unsigned long long)drop_sq);
                    else
                        atomicAdd((unsigned long long*)&J.imp[f], (unsigned long long)drop_sq);
                }
                if (drop) {
                    if (lds)
                        atomicAdd(&s_drop[f], drop);
                    else
                        atomicAdd((unsigned long long*)&J.imp[f],
                                  (unsigned long long)(int64_t)drop);
                }
                drop = 0;
                drop_sq = 0;
            }
        }
    }
    if (lds) {
        __syncthreads();
        for (int c = tid; c < J.p_w; c += 256) {
            const long long v = reg ? s_drop64[c] : (long long)s_drop[c];
            if (v) atomicAdd((unsigned long long*)&J.imp[c], (unsigned long long)v);
        }
    }
    if (visits) {
        for (int m = 1; m < 64; m <<= 1) nv += __shfl_xor(nv, m);
        if ((tid & 63) == 0 && nv)
            atomicAdd(visits + ((blockIdx.x * 4u + (uint32_t)(tid >> 6)) & (kAlgWords - 1)), nv);
    }
}

// ---------------------------------------------------------------------------
// KL permutation importance.

// Fixed-point class frequency of a leaf: floor(2^32 c_k / N).
__device__ __forceinline__ uint64_t leaf_freq(const uint32_t* cls, int kmax, uint32_t node,
                                              int k, uint32_t N) {
    return ((uint64_t)cls[(size_t)node * kmax + k] << 32) / N;
}

__device__ __forceinline__ uint32_t leaf_weight(const uint32_t* cls, int kmax, uint32_t node,
                                                int K) {
    uint32_t N = 0;
    for (int k = 0; k < K; ++k) N += cls[(size_t)node * kmax + k];
    return N;
}

// 2^32 log2(x), 1 <= x < 2^62: bit length, then 32 digits of the fraction
// from successive squares of the mantissa (62 fractional bits, truncated).
__device__ __forceinline__ uint64_t lg2_q32(uint64_t x) {
    const int e = 63 - __builtin_clzll(x);
    uint64_t m = x << (62 - e);
    uint64_t frac = 0;
    for (int i = 0; i < 32; ++i) {
        const uint64_t hi = __umul64hi(m, m), lo = m * m;
        m = (hi << 2) | (lo >> 62);
        const uint64_t top = m >> 63;
        frac = (frac << 1) | top;
        m >>= top;
    }
    return ((uint64_t)e << 32) | frac;
}

// KL(P || Q) in 2^-32 bits for summed fixed-point frequencies S (P) and
// Sq (Q), Q's missing classes raised to one unit where P has them:
// floor(sum_k S_k (lg S_k - lg Q_k) / sum S) + lg sum Q - lg sum S.
// lgS[k] = lg S_k (where S_k > 0) and lgsum = lg sum S come with P: a row's
// P is shared by every column.
template <int KMAX>
__device__ int64_t kl_q32(const uint64_t* S, const uint64_t* lgS, uint64_t lgsum,
                          const uint64_t* Sq, int K) {
    u128 pos = 0, neg = 0;
    uint64_t sp = 0, sq = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= K) break;
        const uint64_t q = (Sq[k] == 0 && S[k] != 0) ? 1 : Sq[k];
        sp += S[k];
        sq += q;
        if (S[k]) {
            const uint64_t a = lgS[k], b = q == S[k] ? a : lg2_q32(q);
            if (a >= b)
                pos += (u128)S[k] * (a - b);
            else
                neg += (u128)S[k] * (b - a);
        }
    }
    int64_t first;
    if (pos >= neg) {
        first = (int64_t)udiv128(pos - neg, (u128)sp);
    } else {  // floor of a negative quotient
        const u128 m = neg - pos;
        const uint64_t qt = udiv128(m, (u128)sp);
        first = -(int64_t)qt - (((u128)qt * sp != m) ? 1 : 0);
    }
    return first + (int64_t)(sq == sp ? lgsum : lg2_q32(sq)) - (int64_t)lgsum;
}

// Rows [r0, r0 + rb) of job J: one wavefront per row, lanes over the job's
// trees; writes the row's summed leaf frequencies S_k, their lg S_k and
// lg sum S (S[row][2K + 1]), and pi(row).
template <int KMAX>
__global__ __launch_bounds__(256) void k_kl_base(JobDev* jobs, int j, const NodeDev* nodes,
                                                 const uint32_t* cls, int kmax, uint32_t tree0,
                                                 uint32_t r0, uint32_t rb, uint64_t* S,
                                                 uint32_t* pi) {
    const JobDev& J = jobs[j];
    if (!J.live) return;
    const int lane = threadIdx.x & 63;
    const uint32_t rr = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (rr >= rb || r0 + rr >= (uint32_t)J.n) return;
    const uint32_t row = r0 + rr;
    const int K = J.K;
    if (J.reg) {  // regression: the loss depends on the change of the prediction only
        if (lane == 0) {
            const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kFlush, (uint32_t)J.t, 0u, 0u,
                                          0u, (uint64_t)J.n);
            pi[rr] = perm_apply(P, row);
        }
        return;
    }
    uint64_t acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = 0;
    for (int tau = lane; tau < J.T; tau += 64) {
        uint32_t node = tree0 + (uint32_t)tau;
        NodeDev nd = nodes[node];
        while (nd.feat >= 0) {
            node = (int)J.colptr[nd.feat][row] <= (int)nd.thr ? nd.left : nd.left + 1;
            nd = nodes[node];
        }
        const uint32_t N = leaf_weight(cls, kmax, node, K);
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K) acc[k] += leaf_freq(cls, kmax, node, k, N);
    }
    uint64_t mine = 0, sum = 0;  // lane k < K keeps S_k
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        uint64_t v = acc[k];
        for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
        if (lane == k) mine = v;
        if (k < K) sum += v;
    }
    uint64_t* row_out = S + (size_t)rr * (2 * K + 1);
    if (lane < K) {
        row_out[lane] = mine;
        row_out[K + lane] = mine ? lg2_q32(mine) : 0ull;
    }
    if (lane == K) row_out[2 * K] = lg2_q32(sum);
    if (lane == 0) {
        const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kFlush, (uint32_t)J.t, 0u, 0u, 0u,
                                      (uint64_t)J.n);
        pi[rr] = perm_apply(P, row);
    }
}

// One thread per (tree, row of the block), rows fastest so that a wave
// walks one tree for 64 rows (its node and bin loads and its atomics then
// spread over rows, not over trees meeting at one column): the row's path;
// for each column on it (first occurrence), the row is re-routed from that
// node with the column's bin taken from row pi(row), and a different leaf
// adds its frequency difference to delta[column][row][k] (64-bit two's
// complement).
__global__ __launch_bounds__(256) void k_kl_delta(JobDev* jobs, int j, const NodeDev* nodes,
                                                  const uint32_t* cls, int kmax, uint32_t tree0,
                                                  uint32_t r0, uint32_t rb, const uint32_t* pi,
                                                  unsigned long long* delta, int max_depth) {
    extern __shared__ uint32_t s_path[];  // [2][max_depth][256]: node, column
    const JobDev& J = jobs[j];
    if (!J.live) return;
    const int tid = threadIdx.x;
    const uint64_t gi = (uint64_t)blockIdx.x * 256u + (uint64_t)tid;
    const uint32_t T = (uint32_t)J.T;
    const uint32_t tau = (uint32_t)(gi / rb), rr = (uint32_t)(gi % rb);
    if (tau >= T || r0 + rr >= (uint32_t)J.n) return;
    const uint32_t row = r0 + rr, src = pi[rr];
    const int K = J.K;
    uint32_t* pn = s_path;
    uint32_t* pf = s_path + max_depth * 256;
    int len = 0;
    uint32_t node = tree0 + tau;
    NodeDev nd = nodes[node];
    while (nd.feat >= 0) {
        pn[len * 256 + tid] = node;
        pf[len * 256 + tid] = (uint32_t)nd.feat;
        ++len;
        node = (int)J.colptr[nd.feat][row] <= (int)nd.thr ? nd.left : nd.left + 1;
        nd = nodes[node];
    }
    const uint32_t leaf0 = node;
    const uint32_t N0 = leaf_weight(cls, kmax, leaf0, K);
    for (int a = 0; a < len; ++a) {
        const uint32_t f = pf[a * 256 + tid];
        bool dup = false;
        for (int b = 0; b < a; ++b) dup |= pf[b * 256 + tid] == f;
        if (dup) continue;
        const int sb = J.colptr[f][src];
        uint32_t ni = pn[a * 256 + tid];
        NodeDev x = nodes[ni];
        while (x.feat >= 0) {
            const int bin = (uint32_t)x.feat == f ? sb : (int)J.colptr[x.feat][row];
            ni = bin <= (int)x.thr ? x.left : x.left + 1;
            x = nodes[ni];
        }
        if (ni == leaf0) continue;
        unsigned long long* d = delta + ((size_t)f * rb + rr) * K;
        if (J.reg) {  // change of the leaf's prediction, in the first slot
            const long long dv = leaf_pred(nodes, cls, kmax, ni) - leaf_pred(nodes, cls, kmax, leaf0);
            if (dv) atomicAdd(d, (unsigned long long)dv);
            continue;
        }
        const uint32_t N1 = leaf_weight(cls, kmax, ni, K);
        for (int k = 0; k < K; ++k) {
            const uint64_t dv = leaf_freq(cls, kmax, ni, k, N1) - leaf_freq(cls, kmax, leaf0, k, N0);
            if (dv) atomicAdd(d + k, (unsigned long long)dv);
        }
    }
}

// One thread per (column, row of the block): the row's divergence for the
// column from S and S + delta (zero when delta is), delta cleared behind the
// read; one 64-bit atomic per workgroup into the column's importance.
template <int KMAX>
__global__ __launch_bounds__(256) void k_kl_reduce(JobDev* jobs, int j, uint32_t r0, uint32_t rb,
                                                   uint32_t row_groups, const uint64_t* S,
                                                   unsigned long long* delta) {
    __shared__ long long s_sum[4];
    JobDev& J = jobs[j];
    if (!J.live) return;
    const uint32_t f = blockIdx.x / row_groups;
    const uint32_t rr = (blockIdx.x % row_groups) * 256u + threadIdx.x;
    const int K = J.K;
    long long kl = 0;
    if (J.reg && f < (uint32_t)J.p_w && rr < rb && r0 + rr < (uint32_t)J.n) {
        // regression: floor(D^2 / n_trees^2) >> s_kl, D the change of the summed
        // leaf predictions (|D| < 2^56); the 128-bit quotient by 32-bit limbs
        unsigned long long* d = delta + ((size_t)f * rb + rr) * K;
        const long long D = (long long)d[0];
        if (D) {
            const uint64_t a = (uint64_t)(D < 0 ? -D : D), T2 = (uint64_t)J.T * (uint64_t)J.T;
            const u128 num = (u128)a * a;
            u128 q = 0;
            uint64_t rem = 0;
            for (int i = 3; i >= 0; --i) {
                const uint64_t cur = (rem << 32) | (uint32_t)(num >> (32 * i));
                q |= (u128)(cur / T2) << (32 * i);
                rem = cur % T2;
            }
            kl = (long long)(q >> J.s_kl);
            d[0] = 0;
        }
    } else if (f < (uint32_t)J.p_w && rr < rb && r0 + rr < (uint32_t)J.n) {
        unsigned long long* d = delta + ((size_t)f * rb + rr) * K;
        uint64_t base[KMAX], lg[KMAX], q[KMAX];
        const uint64_t* row_in = S + (size_t)rr * (2 * K + 1);
        bool moved = false;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            base[k] = q[k] = lg[k] = 0;
            if (k < K) {
                const uint64_t dv = d[k];
                moved |= dv != 0;
                base[k] = row_in[k];
                q[k] = base[k] + dv;
            }
        }
        if (moved) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < K) lg[k] = row_in[K + k];
            kl = kl_q32<KMAX>(base, lg, row_in[2 * K], q, K);
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < K) d[k] = 0;
        }
    }
    for (int m = 1; m < 64; m <<= 1) kl += __shfl_xor(kl, m);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = kl;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long v = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        if (v) atomicAdd((unsigned long long*)&J.imp[f], (unsigned long long)v);
    }
}

// Selection of the k-th smallest (0-based) of the job's n_sha shadow
// importances by a most-significant-digit radix select over the order-
// preserving unsigned keys (sign bit flipped): eight passes of an 8-bit
// digit histogram in LDS.  All 256 threads call it.
__device__ long long shadow_select(const JobDev& J, int k, unsigned* s_hist, int* s_sel) {
    const int tid = threadIdx.x;
    const int p_cur = J.p_cur, p_w = J.p_w;
    unsigned long long prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        s_hist[tid] = 0u;
        __syncthreads();
        for (int c = p_cur + tid; c < p_w; c += 256) {
            const unsigned long long u = (unsigned long long)J.imp[c] ^ (1ull << 63);
            if ((u & mask) == prefix) atomicAdd(&s_hist[(u >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int d = 0;
            unsigned below = 0;
            while (d < 255 && below + s_hist[d] <= (unsigned)k) below += s_hist[d++];
            s_sel[0] = d;
            s_sel[1] = k - (int)below;
        }
        __syncthreads();
        prefix |= (unsigned long long)s_sel[0] << shift;
        mask |= 0xFFull << shift;
        k = s_sel[1];
        __syncthreads();  // s_sel and s_hist are rewritten by the next pass
    }
    return (long long)(prefix ^ (1ull << 63));
}

// Per job: hits, history row, shadow threshold, decisions, liveness.  The
// hit threshold is the maximum shadow importance (perc = 100) or the
// ceil(perc n_sha / 100)-th smallest one.
__global__ __launch_bounds__(256) void k_hits_decide(JobDev* jobs, int perc) {
    __shared__ long long s_max[4], s_sum[4];
    __shared__ int s_und[4];
    __shared__ unsigned s_hist[256];
    __shared__ int s_sel[2];
    JobDev& J = jobs[blockIdx.x];
    if (!J.live) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t = J.t, p_cur = J.p_cur, p_w = J.p_w;
    long long mx = LLONG_MIN, sum = 0;
    for (int c = tid; c < p_w; c += 256) {
        const long long v = J.imp[c];
        if (c >= p_cur) mx = v > mx ? v : mx;
        sum += v;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const long long o = __shfl_xor(mx, m);
        mx = o > mx ? o : mx;
        sum += __shfl_xor(sum, m);
    }
    if (lane == 0) {
        s_max[wave] = mx;
        s_sum[wave] = sum;
    }
    __syncthreads();
    long long best = s_max[0], total = s_sum[0];
    for (int v = 1; v < 4; ++v) {
        best = s_max[v] > best ? s_max[v] : best;
        total += s_sum[v];
    }
    if (perc < 100) {
        const int rank = (int)(((long long)perc * J.n_sha + 99) / 100);  // 1-based
        best = shadow_select(J, rank - 1, s_hist, s_sel);
    }
    // reported value = ldexp(v / denom, rep_exp): regression scores come back
    // to squared target units (rep_exp is 0 for classification and TreeImp)
    double denom;
    if (J.mode == 0) {
        denom = (double)total;
    } else if (J.mode == 2) {  // mean divergence per row, in bits
        denom = (double)J.n * (J.reg ? 1.0 : 4294967296.0);
    } else {
        long long oob = 0;
        for (int tau = 0; tau < J.T; ++tau) oob += J.tstat[tau * 4 + 1];
        denom = (double)((long long)J.R * oob);
    }
    const int rexp = J.reg ? J.rep_exp : 0;
    double* hrow = J.hist + (size_t)(t - 1) * J.p;
    for (int j = tid; j < J.p; j += 256)
        if (J.state[j] < 0) hrow[j] = __longlong_as_double(0x7FF8000000000000ll);
    for (int c = tid; c < p_cur; c += 256) {
        const int j = J.act[c];
        const long long v = J.imp[c];
        hrow[j] = denom > 0.0 ? ldexp((double)v / denom, rexp) : 0.0;
        if (v > best) J.hits[j] += 1;
    }
    if (tid == 0) J.shadow_max[t - 1] = denom > 0.0 ? ldexp((double)best / denom, rexp) : 0.0;
    __syncthreads();
    int und = 0;
    const int hc = J.h_conf[t], hr = J.h_rej[t];
    for (int j = tid; j < J.p; j += 256) {
        int8_t s = J.state[j];
        if (s == 0) {
            const int h = J.hits[j];
            if (h >= hc)
                s = 1;
            else if (h <= hr)
                s = -1;
            J.state[j] = s;
        }
        und += s == 0;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) und += __shfl_xor(und, m);
    if (lane == 0) s_und[wave] = und;
    __syncthreads();
    if (tid == 0) {
        const int u = s_und[0] + s_und[1] + s_und[2] + s_und[3];
        J.n_undecided = u;
        J.live = (u > 0 && t < J.max_iter) ? 1 : 0;
    }
}

// Final ranking, step 1: one thread per feature; a rejected feature's mean
// over its finite history entries of iterations [t0, t1).
__global__ __launch_bounds__(256) void k_rank_mean(const int8_t* state, const double* hist,
                                                   int64_t p, int t0, int t1, double* mean) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= p) return;
    double s = 0.0, m = 0.0;
    int c = 0;
    if (state[j] == -1) {
        for (int t = t0; t < t1; ++t) {
            const double v = hist[(size_t)t * p + j];
            if (v != v) continue;  // NaN: not active in iteration t
            s += v;
            ++c;
        }
        m = c ? s / c : 0.0;
    }
    mean[j] = m;
}

// Step 2: one thread per feature; a rejected feature ranks 3 plus the number
// of rejected features with a strictly larger mean.
__global__ __launch_bounds__(256) void k_rank_count(const int8_t* state, const double* mean,
                                                    int64_t p, int32_t* rank) {
    __shared__ double s_m[256];
    __shared__ int8_t s_s[256];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int8_t sj = j < p ? state[j] : (int8_t)0;
    const double mj = j < p ? mean[j] : 0.0;
    int above = 0;
    for (int64_t g0 = 0; g0 < p; g0 += 256) {
        __syncthreads();
        const int64_t g = g0 + threadIdx.x;
        s_m[threadIdx.x] = g < p ? mean[g] : 0.0;
        s_s[threadIdx.x] = g < p ? state[g] : (int8_t)0;
        __syncthreads();
        const int lim = (int)(p - g0 < 256 ? p - g0 : 256);
        for (int i = 0; i < lim; ++i) above += (s_s[i] == -1 && s_m[i] > mj) ? 1 : 0;
    }
    if (j < p) rank[j] = sj == 1 ? 1 : (sj == 0 ? 2 : 3 + above);
}

// Multi-seed aggregate over the n_jobs runs of one problem (same p): one
// thread per feature; per run the mean of the feature's finite history
// entries (summed in iteration order), then the median over runs (mean of
// the middle pair for an even count) and the lower median of the decisions.
__global__ __launch_bounds__(256) void k_seed_median(const JobDev* jobs,
                                                     const int8_t* const* decisions, int n_jobs,
                                                     int64_t p, double* med, int8_t* dec) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= p) return;
    double v[64];
    int dv[64];
    for (int r = 0; r < n_jobs; ++r) {
        const JobDev& J = jobs[r];
        double s = 0.0;
        int c = 0;
        for (int t = 0; t < J.t; ++t) {
            const double x = J.hist[(size_t)t * p + j];
            if (x != x) continue;  // NaN: rejected before iteration t + 1
            s += x;
            ++c;
        }
        const double m = c ? s / c : 0.0;
        const int d = decisions[r][j];
        int i = r;  // insertion into the sorted prefixes
        while (i > 0 && v[i - 1] > m) {
            v[i] = v[i - 1];
            --i;
        }
        v[i] = m;
        i = r;
        while (i > 0 && dv[i - 1] > d) {
            dv[i] = dv[i - 1];
            --i;
        }
        dv[i] = d;
    }
    med[j] = n_jobs % 2 ? v[n_jobs / 2] : (v[n_jobs / 2 - 1] + v[n_jobs / 2]) / 2.0;
    dec[j] = (int8_t)dv[(n_jobs - 1) / 2];
}

// Rough fix of the features still tentative (an option outside Algorithm 1,
// from Kursa's Boruta): one workgroup per feature.  A tentative feature is
// confirmed when the median of its history entries of iterations [t0, t1)
// exceeds the median of the shadow thresholds of those iterations, else
// rejected; other decisions are copied.  Medians by rank counting in LDS
// (t1 - t0 <= 1000 values); an even count takes the mean of the middle two.
__device__ double lds_median(const double* v, int m, double* s_mid) {
    // the element of rank r (0-based) is v[i] with #{v < v[i]} + #{v[j] ==
    // v[i], j < i} == r: one writer per rank
    const int r0 = (m - 1) / 2, r1 = m / 2;
    for (int i = threadIdx.x; i < m; i += 256) {
        int less = 0, eq_before = 0;
        for (int j = 0; j < m; ++j) {
            less += v[j] < v[i];
            eq_before += j < i && v[j] == v[i];
        }
        const int r = less + eq_before;
        if (r == r0) s_mid[0] = v[i];
        if (r == r1) s_mid[1] = v[i];
    }
    __syncthreads();
    const double med = m % 2 ? s_mid[0] : (s_mid[0] + s_mid[1]) / 2.0;
    __syncthreads();  // s_mid is rewritten by the next call
    return med;
}

__global__ __launch_bounds__(256) void k_rough_fix(const int8_t* state, const double* hist,
                                                   const double* smax, int64_t p, int t0, int t1,
                                                   int8_t* out) {
    __shared__ double s_v[1000];
    __shared__ double s_mid[2];
    const int64_t j = blockIdx.x;
    const int8_t st = state[j];
    if (st != 0) {
        if (threadIdx.x == 0) out[j] = st;
        return;
    }
    const int m = t1 - t0;
    for (int i = threadIdx.x; i < m; i += 256) s_v[i] = smax[t0 + i];
    __syncthreads();
    const double ms = lds_median(s_v, m, s_mid);
    for (int i = threadIdx.x; i < m; i += 256) s_v[i] = hist[(size_t)(t0 + i) * p + j];
    __syncthreads();
    const double mf = lds_median(s_v, m, s_mid);
    if (threadIdx.x == 0) out[j] = mf > ms ? (int8_t)1 : (int8_t)-1;
}

// Capacity flags of an iteration's tree levels, accumulated into the word
// after them, which only the session set-up clears: iterations enqueued back
// to back then report a failure of any one of them.
__global__ void k_ctr_sticky(LevelCtr* c, int n_levels) {
    if (threadIdx.x != 0) return;
    uint32_t o = 0;
    for (int d = 0; d <= n_levels; ++d) o |= c[d].overflow;
    c[n_levels + 1].overflow |= o;
}

void launch_ctr_sticky(LevelCtr* c, int n_levels, hipStream_t st) {
    hipLaunchKernelGGL(k_ctr_sticky, dim3(1), dim3(64), 0, st, c, n_levels);
}

// Streaming copy used to calibrate hardware byte counters.
__global__ void k_copy(uint4* dst, const uint4* src, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

void launch_tree_totals(JobDev* jobs, const TreeDev* trees, int n_trees, uint64_t* tot,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_tree_totals, dim3(n_trees), dim3(256), 0, st, jobs, trees, tot);
}

void launch_treeimp(JobDev* jobs, const TreeDev* trees, int n_trees, const uint64_t* tot,
                    int max_pw, hipStream_t st) {
    hipLaunchKernelGGL(k_treeimp, dim3((unsigned)((max_pw + 255) / 256), (unsigned)n_trees),
                       dim3(256), 0, st, jobs, trees, tot);
}

void launch_permut(JobDev* jobs, const TreeDev* trees, const NodeDev* nodes, const uint32_t* cls,
                   int kmax, int n_trees, int64_t max_n, int max_depth, int max_pw,
                   bool any_reg, unsigned long long* visits, hipStream_t st) {
    // per-column drop sums in LDS for jobs of at most 1024 widened columns
    // (64-bit when the batch has a regression job)
    const int lds_cols = max_pw < 1024 ? max_pw : 1024;
    const int lds_words = lds_cols * (any_reg ? 2 : 1);
    const size_t lds = ((size_t)2 * max_depth * 256 + lds_words + (size_t)kPermGroup * 256) *
                       sizeof(uint32_t);
    hipLaunchKernelGGL(k_permut, dim3((unsigned)((max_n + 255) / 256), (unsigned)n_trees),
                       dim3(256), lds, st, jobs, trees, nodes, cls, kmax, max_depth, lds_cols,
                       lds_words, visits);
}

// The KL importance of job j over rows [r0, r0 + rb): base, deltas, reduce.
void launch_kl_block(JobDev* jobs, int j, const NodeDev* nodes, const uint32_t* cls, int kmax,
                     uint32_t tree0, int T, int p_w_cap, uint32_t r0, uint32_t rb, uint64_t* S,
                     uint32_t* pi, unsigned long long* delta, int max_depth, hipStream_t st) {
    const dim3 b256(256);
    const unsigned g_base = (rb + 3) / 4;
    switch (kmax) {
        case 2: hipLaunchKernelGGL(k_kl_base<2>, dim3(g_base), b256, 0, st, jobs, j, nodes, cls, kmax, tree0, r0, rb, S, pi); break;
        case 3: hipLaunchKernelGGL(k_kl_base<3>, dim3(g_base), b256, 0, st, jobs, j, nodes, cls, kmax, tree0, r0, rb, S, pi); break;
        case 4: hipLaunchKernelGGL(k_kl_base<4>, dim3(g_base), b256, 0, st, jobs, j, nodes, cls, kmax, tree0, r0, rb, S, pi); break;
        case 8: hipLaunchKernelGGL(k_kl_base<8>, dim3(g_base), b256, 0, st, jobs, j, nodes, cls, kmax, tree0, r0, rb, S, pi); break;
        default: hipLaunchKernelGGL(k_kl_base<16>, dim3(g_base), b256, 0, st, jobs, j, nodes, cls, kmax, tree0, r0, rb, S, pi); break;
    }
    const size_t lds = (size_t)2 * max_depth * 256 * sizeof(uint32_t);
    const unsigned g_delta = (unsigned)(((uint64_t)rb * T + 255) / 256);
    hipLaunchKernelGGL(k_kl_delta, dim3(g_delta), b256, lds, st, jobs, j, nodes, cls, kmax, tree0,
                       r0, rb, pi, delta, max_depth);
    const uint32_t groups = (rb + 255) / 256;
    const unsigned g_red = (unsigned)(groups * (uint64_t)p_w_cap);
    switch (kmax) {
        case 2: hipLaunchKernelGGL(k_kl_reduce<2>, dim3(g_red), b256, 0, st, jobs, j, r0, rb, groups, S, delta); break;
        case 3: hipLaunchKernelGGL(k_kl_reduce<3>, dim3(g_red), b256, 0, st, jobs, j, r0, rb, groups, S, delta); break;
        case 4: hipLaunchKernelGGL(k_kl_reduce<4>, dim3(g_red), b256, 0, st, jobs, j, r0, rb, groups, S, delta); break;
        case 8: hipLaunchKernelGGL(k_kl_reduce<8>, dim3(g_red), b256, 0, st, jobs, j, r0, rb, groups, S, delta); break;
        default: hipLaunchKernelGGL(k_kl_reduce<16>, dim3(g_red), b256, 0, st, jobs, j, r0, rb, groups, S, delta); break;
    }
}

void launch_hits_decide(JobDev* jobs, int n_jobs, int perc, hipStream_t st) {
    hipLaunchKernelGGL(k_hits_decide, dim3(n_jobs), dim3(256), 0, st, jobs, perc);
}

void launch_rough_fix(const int8_t* state, const double* hist, const double* smax, int64_t p,
                      int t0, int t1, int8_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_rough_fix, dim3((unsigned)p), dim3(256), 0, st, state, hist, smax, p, t0,
                       t1, out);
}

void launch_rank(const int8_t* state, const double* hist, int64_t p, int t0, int t1,
                 double* mean, int32_t* rank, hipStream_t st) {
    const unsigned g = (unsigned)((p + 255) / 256);
    hipLaunchKernelGGL(k_rank_mean, dim3(g), dim3(256), 0, st, state, hist, p, t0, t1, mean);
    hipLaunchKernelGGL(k_rank_count, dim3(g), dim3(256), 0, st, state, mean, p, rank);
}

void launch_seed_median(const JobDev* jobs, const int8_t* const* decisions, int n_jobs, int64_t p,
                        double* med, int8_t* dec, hipStream_t st) {
    hipLaunchKernelGGL(k_seed_median, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, jobs,
                       decisions, n_jobs, p, med, dec);
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)dst,
                       (const uint4*)src, n16);
}

}  // namespace boruta
