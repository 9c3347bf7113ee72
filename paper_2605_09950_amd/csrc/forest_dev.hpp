// forest_dev.hpp -- device functions shared by the tree-growth kernels:
// node creation / classification and wave-level candidate reductions.
#pragma once

#include <climits>

#include "dev_common.hpp"
#include "reg_dev.hpp"

namespace boruta {

// Lane-ordered comparison of two candidates of ONE feature: higher Q first,
// then the smaller threshold (the smallest b of an equal-score partition).
// Invalid candidates (nl == 0) lose to everything.
__device__ __forceinline__ bool cand_wins_same_feature(const Cand& a, const Cand& b) {
    if (b.nl == 0) return a.nl != 0 || a.b < b.b;
    if (a.nl == 0) return false;
    if (cand_better(a, b)) return true;
    if (cand_better(b, a)) return false;
    return a.b < b.b;
}

__device__ __forceinline__ Cand shfl_cand(const Cand& c, int src) {
    Cand o;
    o.q = __shfl(c.q, src);
    o.f = __shfl(c.f, src);
    o.b = __shfl(c.b, src);
    o.nl = __shfl(c.nl, src);
    o.nr = __shfl(c.nr, src);
    o.pad = 0;
    o.sl = __shfl(c.sl, src);
    o.sr = __shfl(c.sr, src);
    return o;
}

__device__ __forceinline__ Cand shfl_xor_cand(const Cand& c, int m) {
    return shfl_cand(c, (int)((threadIdx.x & 63) ^ m));
}

// Exact wave-wide best of one feature's candidates (all lanes get it).
__device__ __forceinline__ Cand wave_best_exact(Cand c) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Cand o = shfl_xor_cand(c, m);
        if (cand_wins_same_feature(o, c)) c = o;
    }
    return c;
}

// Wave-wide scans through DPP row shifts (within rows of 16 lanes) and row
// broadcasts (lane 15 -> next row, lane 31 -> rows 2-3); lanes whose DPP
// source is outside the pattern take the identity.  No LDS traffic.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Maximum over the wave (a max-scan; lane 63 ends with the total), as a
// wave-uniform value.  The values must be >= -1 (the "no candidate" mark).
__device__ __forceinline__ float wave_max_f_dpp(float v) {
    const int lo = __float_as_int(-2.0f);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x111, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x112, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x114, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x118, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x142, 0xa, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x143, 0xc, 0xf, false)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = fmaxf(v, __shfl_xor(v, m));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = min(v, __shfl_xor(v, m));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = max(v, __shfl_xor(v, m));
    return v;
}

// Margin of the FP32 ranking.  An FP32 score is within eps of its exact value
// Q: eps = 5u (u = 2^-24) for cand_q32 and (K + 4)u <= 20u for hist_q32
// below.  The exact best then scores at least (1 - 2 eps) * FP32 max, so
// every candidate at or above (1 - 2^-18) * FP32 max (64u > 2 * 20u plus the
// rounding of this product) is re-ranked exactly, and the FP32-ranked choice
// equals the exact one.  Two scores farther apart than this margin are in
// exact order.
__device__ __forceinline__ float fp32_floor(float qmax) { return qmax * (1.0f - 0x1.0p-18f); }

// FP32 score straight from the left class counts of a threshold:
// S_L = sum cl_k^2 and S_R = sum (c_k - cl_k)^2 by FMA chains (K roundings
// each; the counts are exact in FP32 below 2^24), then S_L rcp(N_L) +
// S_R rcp(N_R).  Relative error <= (K + 4)u.  Returns -1 when one side is
// empty.
template <int KMAX>
__device__ __forceinline__ float hist_q32(const uint32_t* cl, const uint32_t* cnode, uint32_t N) {
    float nl = 0.0f, sl = 0.0f, sr = 0.0f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const float l = (float)cl[k], r = (float)(cnode[k] - cl[k]);
        nl += l;
        sl = fmaf(l, l, sl);
        sr = fmaf(r, r, sr);
    }
    const float nr = (float)N - nl;
    if (nl == 0.0f || nr == 0.0f) return -1.0f;
    return sl * __builtin_amdgcn_rcpf(nl) + sr * __builtin_amdgcn_rcpf(nr);
}

// Best of one feature's candidates with FP32 ranking and exact recheck of the
// finalists.  q32 < 0 marks an invalid candidate.
__device__ __forceinline__ Cand wave_best_fp32(const Cand& c, float q32) {
    const float qmax = wave_max_f(q32);
    Cand out;
    out.nl = 0;
    out.b = 0x7FFFFFFF;
    if (qmax < 0.0f) return out;  // no valid candidate in the wave
    const bool fin = q32 >= fp32_floor(qmax);
    const int bmin = wave_min_i(fin ? c.b : 0x7FFFFFFF);
    const int bmax = wave_max_i(fin ? c.b : -1);
    if (bmin == bmax) {
        // one threshold among the finalists: the same candidate in every finalist lane
        const unsigned long long mask = __ballot(fin && c.b == bmin);
        return shfl_cand(c, (int)__ffsll(mask) - 1);
    }
    Cand f = c;
    if (!fin) {
        f.nl = 0;
        f.b = 0x7FFFFFFF;
    }
    return wave_best_exact(f);
}

// Total order over candidates of different features: higher Q, then the
// earlier draw position q, then the smaller threshold b (equal (q, b) is the
// same candidate).  The winner over a set is the sequential rule's choice.
__device__ __forceinline__ bool cand_wins_total(const Cand& a, const Cand& b) {
    if (b.nl == 0) return a.nl != 0;
    if (a.nl == 0) return false;
    if (cand_better(a, b)) return true;
    if (cand_better(b, a)) return false;
    return a.q < b.q || (a.q == b.q && a.b < b.b);
}

__device__ __forceinline__ Cand wave_best_total_exact(Cand c) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Cand o = shfl_xor_cand(c, m);
        if (cand_wins_total(o, c)) c = o;
    }
    return c;
}

__device__ __forceinline__ long long wave_min_ll(long long v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const long long o = __shfl_xor(v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ long long wave_max_ll(long long v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const long long o = __shfl_xor(v, m);
        v = o > v ? o : v;
    }
    return v;
}

// The same with FP32 ranking: exact comparisons only among the finalists,
// and none when all finalists are one candidate (the common case).
__device__ __forceinline__ Cand wave_best_total_fp32(const Cand& c, float q32) {
    const float qmax = wave_max_f(q32);
    Cand out;
    out.nl = 0;
    out.b = 0x7FFFFFFF;
    out.q = 0x7FFFFFFF;
    if (qmax < 0.0f) return out;
    const bool fin = q32 >= fp32_floor(qmax);
    const long long key = ((long long)c.q << 9) | (long long)(c.b & 511);
    const long long kmin = wave_min_ll(fin ? key : LLONG_MAX);
    const long long kmax = wave_max_ll(fin ? key : -1ll);
    if (kmin == kmax) {
        const unsigned long long mask = __ballot(fin && key == kmin);
        return shfl_cand(c, (int)__ffsll(mask) - 1);
    }
    Cand f = c;
    if (!fin) {
        f.nl = 0;
        f.b = 0x7FFFFFFF;
    }
    return wave_best_total_exact(f);
}

enum : int { kLeaf = 0, kSmall = 1, kLarge = 2 };

// Children of tree level d start at n_roots + 2 * (searched nodes of levels
// 0..d-1): every searched node owns a pair of child slots.
__device__ __forceinline__ uint32_t level_next_base(const ForestDev& F, int level) {
    uint64_t b = F.n_roots;
    for (int e = 0; e < level; ++e) b += 2ull * ((uint64_t)F.ctrs[e].n_small + F.ctrs[e].n_slots);
    return b < F.node_cap ? (uint32_t)b : F.node_cap;  // past the pool: splits flag overflow
}

// Work lists of tree level `level` as counted on the device; empty once a
// capacity overflow has been flagged for the level (the host reports it).
__device__ __forceinline__ uint32_t level_small(const ForestDev& F, int level) {
    const LevelCtr& c = F.ctrs[level];
    return c.overflow ? 0u : min(c.n_small, F.small_cap);
}
__device__ __forceinline__ uint32_t level_slots(const ForestDev& F, int level) {
    const LevelCtr& c = F.ctrs[level];
    return c.overflow ? 0u : min(c.n_slots, F.slot_cap);
}

// The launch-local view of the forest for tree level `level`: appends go to
// the next level's counters.
__device__ __forceinline__ ForestDev level_view(const ForestDev& F, int level) {
    ForestDev L = F;
    L.ctr = F.ctrs + level + 1;
    L.next_base = level_next_base(F, level);
    L.n_small_cur = F.ctrs[level].n_small;
    return L;
}

// Write a new node record -- a leaf until a split search turns it into a
// split -- and return what it needs next: nothing (final leaf: maximum depth,
// fewer than two distinct rows or a single class), the wave path (<= 64
// distinct rows) or the tiled histogram path.
__device__ inline int write_node(const ForestDev& F, const JobDev& J, uint32_t idx, uint32_t tree,
                                 uint32_t heap, uint32_t seg, uint32_t len, uint32_t n,
                                 uint32_t depth, const uint32_t* counts) {
    uint32_t arg = 0, nonzero = 0;
    for (int k = 0; k < J.K; ++k) {
        F.cls[(size_t)idx * F.kmax + k] = counts[k];
        if (counts[k] > counts[arg]) arg = k;
        nonzero += counts[k] != 0;
    }
    NodeDev nd;
    nd.tree = tree;
    nd.heap = heap;
    nd.seg = seg;
    nd.len = len;
    nd.n = n;
    nd.feat = -1;
    nd.left = 0;
    nd.thr = 0;
    nd.leaf_class = (uint8_t)arg;
    nd.depth = (uint8_t)depth;
    F.nodes[idx] = nd;
    F.ngain[idx] = 0;
    if ((int)depth >= J.D || len < 2 || nonzero <= 1) return kLeaf;
    return (len <= F.small_rows && n < F.small_ncap) ? kSmall : kLarge;
}

// Regression node: weight W and weighted target sum T (kept in the node's
// first two class words); it is a final leaf at the maximum depth or with
// fewer than two distinct rows, else it takes the histogram path (its split
// search ranks exact weighted target sums, which the wave path does not keep).
// A leaf's prediction floor(T / W) is read from these fields.
__device__ inline int write_node_reg(const ForestDev& F, const JobDev& J, uint32_t idx,
                                     uint32_t tree, uint32_t heap, uint32_t seg, uint32_t len,
                                     uint32_t W, int64_t T, uint32_t depth) {
    F.cls[(size_t)idx * F.kmax] = (uint32_t)(uint64_t)T;
    F.cls[(size_t)idx * F.kmax + 1] = (uint32_t)((uint64_t)T >> 32);
    NodeDev nd;
    nd.tree = tree;
    nd.heap = heap;
    nd.seg = seg;
    nd.len = len;
    nd.n = W;
    nd.feat = -1;
    nd.left = 0;
    nd.thr = 0;
    nd.leaf_class = 0;
    nd.depth = (uint8_t)depth;
    F.nodes[idx] = nd;
    F.ngain[idx] = 0;
    if ((int)depth >= J.D || len < 2) return kLeaf;
    return kLarge;
}

// Weighted target sum of a regression node from its class words.
__device__ __forceinline__ int64_t node_tsum(const uint32_t* cls, int kmax, uint32_t idx) {
    return (int64_t)((uint64_t)cls[(size_t)idx * kmax] |
                     ((uint64_t)cls[(size_t)idx * kmax + 1] << 32));
}

// Place node idx in the next level's lists at already reserved positions.
__device__ inline void put_small(const ForestDev& F, uint32_t pos, uint32_t idx) {
    if (pos < F.small_cap)
        F.small_out[pos] = idx;
    else
        atomicOr(&F.ctr->overflow, 1u);
}

__device__ inline void put_large(const ForestDev& F, uint32_t slot, uint32_t idx) {
    if (slot >= F.slot_cap) {
        atomicOr(&F.ctr->overflow, 2u);
        return;
    }
    F.slot_node_out[slot] = idx;
}

// Reserve list positions for up to two new nodes (one atomic per list) and
// place them.
__device__ inline void enqueue_nodes(const ForestDev& F, const JobDev& J, uint32_t idx0,
                                     const int* kinds, int count) {
    uint32_t ns = 0, nl = 0;
    for (int c = 0; c < count; ++c) {
        ns += kinds[c] == kSmall;
        nl += kinds[c] == kLarge;
    }
    uint32_t ps = ns ? atomicAdd(&F.ctr->n_small, ns) : 0u;
    uint32_t pl = nl ? atomicAdd(&F.ctr->n_slots, nl) : 0u;
    for (int c = 0; c < count; ++c) {
        if (kinds[c] == kSmall) put_small(F, ps++, idx0 + c);
        if (kinds[c] == kLarge) put_large(F, pl++, idx0 + c);
    }
}

// Children of the i-th searched node of a level (small nodes first, then
// large-node slots) live at next_base + 2 i: no allocation counter.  A
// searched node that stays a leaf marks its pair unused.
__device__ inline void mark_unused_pair(const ForestDev& F, uint32_t child) {
    if (child + 2 <= F.node_cap) {
        F.nodes[child].tree = 0xFFFFFFFFu;
        F.nodes[child + 1].tree = 0xFFFFFFFFu;
    }
}

// Turn node `id` into a split on (best.f, best.b) and write both children
// at child, child + 1; kinds[] receives what each child needs next.
__device__ inline void split_node(const ForestDev& F, JobDev& J, const TreeDev& tr, uint32_t id,
                                  const NodeDev& nd, const Cand& best, uint32_t nl_rows,
                                  const uint32_t* cl, const uint32_t* cr, uint64_t gain,
                                  uint32_t child, int* kinds) {
    kinds[0] = kinds[1] = kLeaf;
    if (child + 2 > F.node_cap) {
        atomicOr(&F.ctr->overflow, 4u);
        return;  // stays a leaf; the host reports the failure
    }
    F.nodes[id].feat = best.f;
    F.nodes[id].thr = (uint16_t)best.b;
    F.nodes[id].left = child;
    F.ngain[id] = gain;
    if (J.mode == 0)
        atomicAdd((unsigned long long*)&J.G[(size_t)tr.tau * J.pw_cap + best.f],
                  (unsigned long long)gain);
    kinds[0] = write_node(F, J, child, nd.tree, 2 * nd.heap, nd.seg, nl_rows, best.nl,
                          nd.depth + 1u, cl);
    kinds[1] = write_node(F, J, child + 1, nd.tree, 2 * nd.heap + 1, nd.seg + nl_rows,
                          nd.len - nl_rows, best.nr, nd.depth + 1u, cr);
}

// Regression form of split_node: the children's weights and target sums
// come from the winning candidate.
__device__ inline void split_node_reg(const ForestDev& F, JobDev& J, const TreeDev& tr,
                                      uint32_t id, const NodeDev& nd, const Cand& best,
                                      uint32_t nl_rows, uint64_t gain, uint32_t child,
                                      int* kinds) {
    kinds[0] = kinds[1] = kLeaf;
    if (child + 2 > F.node_cap) {
        atomicOr(&F.ctr->overflow, 4u);
        return;
    }
    F.nodes[id].feat = best.f;
    F.nodes[id].thr = (uint16_t)best.b;
    F.nodes[id].left = child;
    F.ngain[id] = gain;
    if (J.mode == 0)
        atomicAdd((unsigned long long*)&J.G[(size_t)tr.tau * J.pw_cap + best.f],
                  (unsigned long long)gain);
    kinds[0] = write_node_reg(F, J, child, nd.tree, 2 * nd.heap, nd.seg, nl_rows, best.nl,
                              reg_tl(best), nd.depth + 1u);
    kinds[1] = write_node_reg(F, J, child + 1, nd.tree, 2 * nd.heap + 1, nd.seg + nl_rows,
                              nd.len - nl_rows, best.nr, reg_tr(best), nd.depth + 1u);
}

}  // namespace boruta
