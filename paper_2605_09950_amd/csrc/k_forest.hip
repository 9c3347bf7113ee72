// k_forest.hip -- random-forest growth kernels (gfx950).
//
// Trees grow level by level, all trees of all live jobs in the same launch:
//   * k_boot_compact  per tree: in-bag row records and OOB rows from the
//                     bootstrap multiplicities, root node;
//   * k_split_small   one wavefront per node with <= small_rows distinct
//                     rows: the rows sit in lanes and every threshold's left
//                     class counts come from an in-register all-pairs sum;
//   * k_draws         one wavefront per large node: its drawn features and
//                     their columns, and the node's slot record;
//   * k_hist_tile     node-major: one wavefront per (large node, fw drawn
//                     features): LDS class-count histogram [feature][class]
//                     [bin] built with LDS atomics from batched global bin
//                     gathers, then a wave prefix scan per feature; writes
//                     the item's best candidate;
//   * k_col_scan, k_col_scatter, k_hist_col  column-major (deep levels of
//                     large matrices): the level's items bucketed by bin
//                     column, each column staged once per unit in LDS, the
//                     same histogram and scan per item from the staged bins;
//   * k_split_finalize one wavefront per large node: best over the node's
//                     items, then a partition of its rows;
//   * k_lists_count, k_lists_write  the next level's node lists, in parent
//                     order, without atomics.
// The split rule (reading of the Gini forest of Sec. 2.1): maximise
// Q = S_L/N_L + S_R/N_R over drawn features and thresholds "bin <= b",
// exact rational comparison, ties to the earlier draw then the smaller b;
// split only on a strictly positive decrease Q - S/N.
#include <type_traits>

#include "forest_dev.hpp"

namespace boruta {

// ---------------------------------------------------------------------------
// Per tree: compact the in-bag rows (multiplicity > 0, ascending) into row
// records and the out-of-bag rows into a list; create the root node.  The
// multiplicities are cleared behind the read.  A regression root keeps its
// bootstrap weight W and weighted fixed-point target sum T.
__global__ __launch_bounds__(1024) void k_boot_compact(ForestDev F0) {
    __shared__ uint32_t s_win[16], s_wout[16], s_rin[16];
    __shared__ uint32_t s_cls[16];
    __shared__ unsigned long long s_tsum;
    __shared__ uint32_t s_base_in, s_base_out, s_base_rows;
    ForestDev F = F0;
    F.ctr = F0.ctrs;  // the roots form the lists of level 0
    const uint32_t g = blockIdx.x;
    const TreeDev tr = F.trees[g];
    JobDev& J = F.jobs[tr.job];
    if (!J.live) {  // finished job: its tree slots stay empty
        if (threadIdx.x == 0) F.nodes[g].tree = 0xFFFFFFFFu;
        return;
    }
    const uint32_t n = (uint32_t)J.n;
    const bool reg = J.reg != 0;
    uint32_t* w = J.wbuf + (size_t)tr.tau * n;
    uint64_t* recs = J.rec[0] + (size_t)tr.tau * J.rstride;
    uint32_t* oob = J.oob + (size_t)tr.tau * n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 16) s_cls[tid] = 0;
    if (tid == 0) {
        s_tsum = 0;
        s_base_in = 0;
        s_base_out = 0;
        s_base_rows = 0;
    }
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + tid;
        const uint32_t wi = i < n ? w[i] : 0u;
        if (i < n) w[i] = 0;  // multiplicities start from zero next iteration
        const bool inb = i < n && wi > 0, isoob = i < n && wi == 0;
        const uint32_t yi = inb && !reg ? (uint32_t)J.y[i] : 0u;
        const uint64_t mi = __ballot(inb), mo = __ballot(isoob);
        if (lane == 0) {
            s_win[wave] = __popcll(mi);
            s_wout[wave] = __popcll(mo);
            s_rin[wave] = __popcll(mi);
        }
        __syncthreads();
        uint32_t pin = s_base_in, pout = s_base_out;
        for (int v = 0; v < wave; ++v) {
            pin += s_win[v];
            pout += s_wout[v];
        }
        if (inb) {
            if (wi > 0xFFFFu) atomicOr(&F.ctr->overflow, 8u);
            recs[pin + __popcll(mi & below)] = rec_pack(i, wi, yi);
            atomicAdd(&s_cls[yi], wi);
        }
        if (reg) {  // the root's weighted target sum: one LDS atomic per wave
            long long tv = inb ? (long long)wi * (long long)ldg(J.yfix + i) : 0ll;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) tv += __shfl_xor(tv, m);
            if (lane == 0 && tv) atomicAdd(&s_tsum, (unsigned long long)tv);
        }
        if (isoob) oob[pout + __popcll(mo & below)] = i;
        __syncthreads();
        if (tid == 0) {
            uint32_t ti = 0, to = 0, tr_ = 0;
            for (int v = 0; v < 16; ++v) {
                ti += s_win[v];
                to += s_wout[v];
                tr_ += s_rin[v];
            }
            s_base_in += ti;
            s_base_out += to;
            s_base_rows += tr_;
        }
        __syncthreads();
    }
    if (tid == 0) {
        J.tstat[tr.tau * 4 + 0] = (int32_t)s_base_rows;
        J.tstat[tr.tau * 4 + 1] = (int32_t)s_base_out;
        J.tstat[tr.tau * 4 + 2] = 0;
        uint32_t counts[16], tot = 0;
        for (int k = 0; k < 16; ++k) {
            counts[k] = s_cls[k];
            tot += s_cls[k];
        }
        const int kind = reg ? write_node_reg(F, J, g, g, 1u, 0u, s_base_in, tot,
                                              (int64_t)s_tsum, 0u)
                             : write_node(F, J, g, g, 1u, 0u, s_base_in, tot, 0u, counts);
        enqueue_nodes(F, J, g, &kind, 1);
    }
}

// ---------------------------------------------------------------------------
// Small nodes: one wavefront per node.  With W = the node's row count rounded
// up to a power of two, the wave is split into 64/W segments of W lanes; a
// segment holds the node's rows (one per lane) and evaluates one drawn
// feature, so 64/W features are scored per pass.  The left class counts of
// the threshold at a lane's own bin come from an all-pairs sum over the
// segment; the bins of the next pass are gathered while this one computes.
struct SmallOut {
    int kinds[2];
    uint32_t child;
    uint64_t alg;
};

// Packed per-class counters of the wave path: KMAX <= 4 classes fit one
// 32-bit word (16-bit fields for 2 classes, 8-bit for 4; the node's weighted
// count stays below the field range), more classes use 64-bit words of four
// 16-bit fields.
template <int KMAX>
struct Pack {
    static constexpr bool kU32 = KMAX <= 4;
    typedef typename std::conditional<kU32, uint32_t, uint64_t>::type word;
    static constexpr int kPer = kU32 ? KMAX : 4;         // fields per word
    static constexpr int kBits = kU32 ? 32 / KMAX : 16;  // bits per field
    static constexpr int kWords = kU32 ? 1 : KMAX / 4;
    static __device__ __forceinline__ uint32_t field(word w, int k) {
        return (uint32_t)(w >> (kBits * (k % kPer))) & ((1u << kBits) - 1u);
    }
};

__device__ __forceinline__ uint32_t readlane_w(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ uint64_t readlane_w(uint64_t v, int src) { return readlane64(v, src); }

// tab: the wave's kDrawTab-entry LDS region for the node's permutation
// round table (as in k_draws); scnt: the wave's 64 LDS words for the rows'
// one-word class counters
template <int KMAX>
__device__ void small_node(const ForestDev& F, uint32_t idx, SmallOut& out, uint16_t* tab,
                           uint32_t* scnt) {
    typedef Pack<KMAX> PK;
    typedef typename PK::word word;
    const int lane = threadIdx.x & 63;
    out.kinds[0] = out.kinds[1] = kLeaf;
    out.child = F.next_base + 2u * idx;
    const uint32_t id = uniform(F.small_in[idx]);
    const NodeDev nd = F.nodes[id];
    const TreeDev tr = F.trees[nd.tree];
    JobDev& J = F.jobs[tr.job];
    const int B = J.B;
    const size_t tbase = (size_t)tr.tau * J.rstride + nd.seg;
    const uint64_t* rin = J.rec[F.parity] + tbase;
    uint64_t* rout = J.rec[F.parity ^ 1] + tbase;
    const int len = (int)uniform(nd.len);
    int W = 2;
    while (W < len) W <<= 1;
    const int G = 64 / W;                // features per pass
    const int seg = lane / W, i = lane & (W - 1);
    const bool valid = i < len;
    const uint64_t rec = valid ? ldg(rin + i) : 0ull;
    const uint32_t row = rec_row(rec), wt = rec_w(rec), yv = rec_y(rec);
    // class counter word of this lane's row; zero outside segment 0 so that
    // reading lane j >= len (any segment) contributes nothing
    word cv[PK::kWords];
#pragma unroll
    for (int w = 0; w < PK::kWords; ++w)
        cv[w] = (seg == 0 && valid && (int)yv / PK::kPer == w)
                    ? ((word)wt << (PK::kBits * ((int)yv % PK::kPer)))
                    : (word)0;
    uint32_t cnode[KMAX];
    uint64_t S = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        cnode[k] = k < J.K ? F.cls[(size_t)id * F.kmax + k] : 0u;
        S += (uint64_t)cnode[k] * cnode[k];
    }
    const uint32_t N = nd.n;
    const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kMtry, (uint32_t)J.t, (uint32_t)tr.tau,
                                  nd.heap, 0u, (uint64_t)J.p_w);
    // the wave tabulates the round functions once, evenly, instead of every
    // lane walking its draw through all rounds (halves of up to 8 bits)
    const bool use_tab = (P.rounds << P.half) <= kDrawTab;
    if (use_tab) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the previous node's lookups
        for (uint32_t e = (uint32_t)lane; e < (P.rounds << P.half); e += 64u)
            tab[e] = (uint16_t)perm_round(P, e >> P.half, e & P.mask);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // Each lane keeps the best of its own candidates over the passes (they
    // arrive in increasing draw position, so an exact tie keeps the earlier
    // one); one wave-wide reduction per node picks the winner.  With FP32
    // ranking, two candidates are compared exactly only when their FP32
    // scores are within the ranking margin of each other.
    Cand lb;
    lb.nl = 0;
    lb.q = 0x7FFFFFFF;
    lb.b = 0x7FFFFFFF;
    lb.f = 0;
    lb.nr = 0;
    lb.pad = 0;
    lb.sl = lb.sr = 0;
    float lq = -1.0f;
    const bool fp32 = F.split_rank != 0;
    const int abase = (lane - i) << 2;  // ds_bpermute byte address of the segment's lane 0
    if constexpr (PK::kWords == 1) {
        // row j's counter word at scnt[j] (lane j holds row j in segment 0;
        // every other lane holds zero): the passes read four rows' counters
        // per LDS broadcast instead of one lane read per row
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the previous node's reads
        scnt[lane] = (uint32_t)cv[0];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    for (int q0 = 0; q0 < J.mtry; q0 += 64) {
        const int nq = min(64, J.mtry - q0);
        const int myf =
            lane < nq ? (int)(use_tab ? perm_apply_tab(P, tab, (uint32_t)(q0 + lane))
                                      : perm_apply(P, (uint32_t)(q0 + lane)))
                      : 0;
        const unsigned long long mycol =
            lane < nq ? (unsigned long long)ldg(J.colptr + myf) : 0ull;
        const int passes = (nq + G - 1) / G;
        // The bin load is unconditional (lanes without a row read row 0, lanes
        // past the drawn features read the first one) so that blocks of loads
        // issue back to back; eval() masks what does not count.
        auto gather = [&](int pass) {
            const int qq = pass * G + seg;
            if (J.rowmaj) {  // the row's drawn columns share cache lines
                const int fq = __shfl(myf, qq < nq ? qq : 0);
                return (int)ldg(J.rowmaj + (size_t)row * J.rm_stride + (uint32_t)fq);
            }
            const uint8_t* col = (const uint8_t*)__shfl(mycol, qq < nq ? qq : 0);
            return (int)ldg(col + row);
        };
        auto eval = [&](int pass, int raw) {
            const int qq = pass * G + seg;
            const bool act = qq < nq;
            const int b = (valid && act) ? raw : 0x7FFF;
            // left counts of threshold b: the segment's rows j with bin <= b.
            // Bins by lane permute, counters of row j read from lane j as
            // scalars; rows j >= len read zero counters.
            word acc[PK::kWords];
#pragma unroll
            for (int w = 0; w < PK::kWords; ++w) acc[w] = 0;
            for (int j0 = 0; j0 < len; j0 += 8) {
                int bj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    bj[u] = __builtin_amdgcn_ds_bpermute(abase + ((j0 + u) << 2), b);
                if constexpr (PK::kWords == 1) {
                    const uint4 c0 = *reinterpret_cast<const uint4*>(scnt + j0);
                    const uint4 c1 = *reinterpret_cast<const uint4*>(scnt + j0 + 4);
                    const uint32_t cj[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[0] += bj[u] <= b ? (word)cj[u] : (word)0;
                    continue;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool take = bj[u] <= b;
#pragma unroll
                    for (int w = 0; w < PK::kWords; ++w) {
                        const word o = readlane_w(cv[w], j0 + u);
                        acc[w] += take ? o : (word)0;
                    }
                }
            }
            Cand c;
            c.q = q0 + qq;
            c.f = __shfl(myf, act ? qq : 0);
            c.b = b;
            c.pad = 0;
            uint32_t nl = 0;
            uint64_t sl = 0, sr = 0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const uint32_t l = PK::field(acc[k / PK::kPer], k);
                const uint32_t r = cnode[k] - l;
                nl += l;
                sl += (uint64_t)l * l;
                sr += (uint64_t)r * r;
            }
            c.nl = nl;
            c.nr = N - nl;
            c.sl = sl;
            c.sr = sr;
            const bool ok = valid && act && b <= B - 2 && nl > 0 && nl < N;
            const bool has = lb.nl != 0;
            bool better;
            float qc = -1.0f;
            if (fp32) {
                qc = ok ? cand_q32(c) : -1.0f;
                const bool near = ok && has && qc >= fp32_floor(lq) && lq >= fp32_floor(qc);
                bool exact = false;
                if (__ballot(near)) exact = cand_better(c, lb);
                better = ok && (!has || (near ? exact : qc > lq));
            } else {
                better = ok && (!has || cand_better(c, lb));
            }
            if (better) {
                lb = c;
                lq = qc;
            }
        };
        // bins of kPF passes are in flight while the previous kPF are scored
        constexpr int kPF = 2;
        int bq[kPF];
#pragma unroll
        for (int u = 0; u < kPF; ++u) bq[u] = gather(u);
        for (int pb = 0; pb < passes; pb += kPF) {
            int bn[kPF];
            if (pb + kPF < passes) {
#pragma unroll
                for (int u = 0; u < kPF; ++u) bn[u] = gather(pb + kPF + u);
            }
#pragma unroll
            for (int u = 0; u < kPF; ++u)
                if (pb + u < passes) eval(pb + u, bq[u]);
#pragma unroll
            for (int u = 0; u < kPF; ++u) bq[u] = bn[u];
        }
    }
    const Cand best = fp32 ? wave_best_total_fp32(lb, lb.nl != 0 ? lq : -1.0f)
                           : wave_best_total_exact(lb);
    out.alg = (uint64_t)len * (uint64_t)(J.mtry + 6);
    if (best.nl == 0 || !cand_positive(best, S, N)) {  // stays the leaf it was created as
        if (lane == 0) mark_unused_pair(F, out.child);
        return;
    }
    // partition with the lanes of segment 0
    const bool mine = seg == 0 && valid;
    const uint8_t* col = ldg(J.colptr + best.f);
    const bool left = mine && (int)ldg(col + row) <= best.b;
    const uint64_t lm = __ballot(left), vm = __ballot(mine);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nl_rows = (uint32_t)__popcll(lm);
    if (mine) {
        const uint32_t pos = left ? (uint32_t)__popcll(lm & below)
                                  : nl_rows + (uint32_t)__popcll(vm & ~lm & below);
        rout[pos] = rec;
    }
    word lc[PK::kWords];
#pragma unroll
    for (int w = 0; w < PK::kWords; ++w) {
        word v = left ? cv[w] : (word)0;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
        lc[w] = v;
    }
    if (lane == 0) {
        uint32_t cl[16], cr[16];
        for (int k = 0; k < 16; ++k) {
            cl[k] = k < KMAX ? PK::field(lc[k / PK::kPer], k) : 0u;
            cr[k] = (k < KMAX ? cnode[k] : 0u) - cl[k];
        }
        split_node(F, J, tr, id, nd, best, nl_rows, cl, cr, cand_gain_fix(best, S, N),
                   out.child, out.kinds);
    }
}

// One wavefront per node (grid-stride over the level's small-node list).
// The small nodes of tree level `level`: all of them (count from the level's
// counters, grid-stride) or, with an explicit count, list entries
// [first, first + count).
template <int KMAX>
__global__ __launch_bounds__(256) void k_split_small(ForestDev F0, int level, uint32_t first,
                                                     uint32_t count) {
    const ForestDev F = level_view(F0, level);
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_small(F0, level);
    }
    extern __shared__ uint16_t stab[];  // [4][kDrawTab] permutation round tables
    __shared__ __align__(16) uint32_t s_cnt[4][64];  // per wave: the node's row counters
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    unsigned long long alg = 0;  // statistics
    for (uint32_t li = blockIdx.x * 4u + (uint32_t)wave; li < count; li += gridDim.x * 4u) {
        SmallOut o;
        o.kinds[0] = o.kinds[1] = kLeaf;
        o.child = 0;
        o.alg = 0;
        small_node<KMAX>(F, first + li, o, stab + (size_t)wave * kDrawTab, s_cnt[wave]);
        // what the children need next; the next level's lists are built from these
        if (lane == 0) F.kinds[first + li] = (uint8_t)(o.kinds[0] | o.kinds[1] << 2);
        alg += o.alg;
    }
    // one atomic per wave for the statistics
    if (F.alg_bytes && lane == 0 && alg)
        atomicAdd((unsigned long long*)&F.alg_bytes[kAlgWords + ((blockIdx.x * 4u + wave) &
                                                                 (kAlgWords - 1))], alg);
}

// ---------------------------------------------------------------------------
// Best threshold of one feature from its LDS histogram h[KMAX][256] (class
// rows of 256 bins; bins >= B stay zero).  Lane l owns bins 4l .. 4l+3, read
// as one 16-byte word per class (consecutive lanes, consecutive words: no
// bank conflicts); class prefix sums come from a DPP wave scan.
template <int KMAX>
__device__ Cand feature_best(const uint32_t* h, int B, int q, int f, const uint32_t* cnode,
                             uint32_t N, int split_rank) {
    constexpr bool kRegs = KMAX <= 4;  // keep the lane's counts in registers
    const int lane = threadIdx.x & 63;
    const int b0 = lane * 4;
    uint32_t hv[kRegs ? KMAX : 1][4];
    uint32_t excl[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const uint4 v = *reinterpret_cast<const uint4*>(h + k * 256 + b0);
        if constexpr (kRegs) {
            hv[k][0] = v.x;
            hv[k][1] = v.y;
            hv[k][2] = v.z;
            hv[k][3] = v.w;
        }
        const uint32_t a = v.x + v.y + v.z + v.w;
        excl[k] = wave_incl_sum(a) - a;
    }
    auto hval = [&](int k, int u) -> uint32_t {
        if constexpr (kRegs)
            return hv[k][u];
        else
            return h[k * 256 + b0 + u];
    };
    // candidates of this lane, in ascending threshold order
    auto make = [&](int b, const uint32_t* cl) {
        Cand c;
        c.q = q;
        c.f = f;
        c.b = b;
        c.pad = 0;
        uint32_t nl = 0;
        uint64_t sl = 0, sr = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t r = cnode[k] - cl[k];
            nl += cl[k];
            sl += (uint64_t)cl[k] * cl[k];
            sr += (uint64_t)r * r;
        }
        c.nl = nl;
        c.nr = N - nl;
        c.sl = sl;
        c.sr = sr;
        return c;
    };
    Cand lb;
    lb.nl = 0;
    lb.b = 0x7FFFFFFF;
    lb.q = q;
    lb.f = f;
    lb.nr = 0;
    lb.pad = 0;
    lb.sl = lb.sr = 0;
    uint32_t cl[KMAX];
    if (!split_rank) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) cl[k] = excl[k];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u;
            uint32_t add = 0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const uint32_t v = hval(k, u);
                cl[k] += v;
                add += v;
            }
            // an empty bin repeats the previous threshold's partition, which the
            // smaller threshold already represents
            if (b > B - 2 || add == 0) continue;
            const Cand c = make(b, cl);
            if (c.nl == 0 || c.nl == N) continue;
            if (lb.nl == 0 || cand_better(c, lb)) lb = c;
        }
        return wave_best_exact(lb);
    }
    // FP32 ranking: the lane's best and second-best FP32 scores; finalists
    // are the lanes whose best is within the margin of the wave maximum.  A
    // finalist lane whose second-best is also within it re-ranks its bins
    // exactly; otherwise its finalist is the best bin alone.
    float q1 = -1.0f, q2 = -1.0f;
    int u1 = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) cl[k] = excl[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int b = b0 + u;
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t v = hval(k, u);
            cl[k] += v;
            add += v;
        }
        if (b > B - 2 || add == 0) continue;
        const float qc = hist_q32<KMAX>(cl, cnode, N);
        if (qc < 0.0f) continue;
        if (qc > q1) {
            q2 = q1;
            q1 = qc;
            u1 = u;
        } else if (qc > q2) {
            q2 = qc;
        }
    }
    const float qmax = wave_max_f_dpp(q1);
    if (qmax < 0.0f) return lb;
    const float floor32 = fp32_floor(qmax);
    const bool fin = q1 >= floor32;
    const bool multi = fin && q2 >= floor32;
    if (__ballot(multi)) {
        if (multi) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) cl[k] = excl[k];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int b = b0 + u;
                uint32_t add = 0;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    const uint32_t v = hval(k, u);
                    cl[k] += v;
                    add += v;
                }
                if (b > B - 2 || add == 0) continue;
                const float qc = hist_q32<KMAX>(cl, cnode, N);
                if (qc < floor32) continue;  // includes the empty-side -1
                const Cand c = make(b, cl);
                if (lb.nl == 0 || cand_better(c, lb)) lb = c;
            }
        }
    }
    if (fin && !multi) {
        // class counts left of bin b0 + u1
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            uint32_t v = excl[k];
#pragma unroll
            for (int u = 0; u < 4; ++u) v += u <= u1 ? hval(k, u) : 0u;
            cl[k] = v;
        }
        lb = make(b0 + u1, cl);
    }
    const unsigned long long finm = __ballot(lb.nl != 0);
    if (__popcll(finm) == 1) return shfl_cand(lb, (int)__ffsll(finm) - 1);
    return wave_best_exact(lb);
}

// Best threshold of one feature, compacted form (up to 4 classes): as
// feature_best, but the thresholds worth scoring (a non-empty bin below
// B - 1 with rows on both sides) are first packed into a dense list, so a
// node with few distinct bins costs one scoring round instead of four.  The
// list overwrites the feature's histogram h (read first); each entry is
// KMAX words, the bin in the top byte of the first (counts stay below 2^24).
// cl_out receives the winner's left class counts.
template <int KMAX>
__device__ Cand feature_best_compact(uint32_t* h, int B, int q, int f, const uint32_t* cnode,
                                     uint32_t N, int split_rank, uint32_t* cl_out) {
    static_assert(KMAX <= 4, "compact scan keeps four bins per class in registers");
    const int lane = threadIdx.x & 63;
    const int b0 = lane * 4;
    uint32_t hv[KMAX][4], excl[KMAX], a[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const uint4 v = *reinterpret_cast<const uint4*>(h + k * 256 + b0);
        hv[k][0] = v.x;
        hv[k][1] = v.y;
        hv[k][2] = v.z;
        hv[k][3] = v.w;
        a[k] = v.x + v.y + v.z + v.w;
    }
    bool packed = false;
    if constexpr (KMAX == 4) {
        if (N < 65536u) {
            // every prefix of a class count is below N: two classes per word,
            // one wave scan per pair (measured faster for four classes only)
#pragma unroll
            for (int k = 0; k < 4; k += 2) {
                const uint32_t pk = a[k] | (a[k + 1] << 16);
                const uint32_t ex = wave_incl_sum(pk) - pk;
                excl[k] = ex & 0xFFFFu;
                excl[k + 1] = ex >> 16;
            }
            packed = true;
        }
    }
    if (!packed) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) excl[k] = wave_incl_sum(a[k]) - a[k];
    }
    // the lane's thresholds worth scoring: a non-empty bin below B - 1 with
    // rows on both sides (prefix counts are rebuilt in the writing pass)
    uint32_t okm = 0, cnt = 0;
    {
        uint32_t nl = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) nl += excl[k];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t add = 0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) add += hv[k][u];
            nl += add;
            const bool ok = b0 + u <= B - 2 && add != 0 && nl != 0 && nl != N;
            okm |= (uint32_t)ok << u;
            cnt += ok;
        }
    }
    const uint32_t incl = wave_incl_sum(cnt);
    const int total = __builtin_amdgcn_readlane((int)incl, 63);
    uint32_t pos = incl - cnt;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // h has been read
    {
        uint32_t cl[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) cl[k] = excl[k];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) cl[k] += hv[k][u];
            if (okm >> u & 1u) {
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    h[pos * KMAX + k] = cl[k] | (k == 0 ? (uint32_t)(b0 + u) << 24 : 0u);
                ++pos;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    auto entry = [&](int e, uint32_t* c) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) c[k] = h[e * KMAX + k];
        const int b = (int)(c[0] >> 24);
        c[0] &= 0xFFFFFFu;
        return b;
    };
    auto make = [&](int b, const uint32_t* c) {
        Cand x;
        x.q = q;
        x.f = f;
        x.b = b;
        x.pad = 0;
        uint32_t nl = 0;
        uint64_t sl = 0, sr = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t r = cnode[k] - c[k];
            nl += c[k];
            sl += (uint64_t)c[k] * c[k];
            sr += (uint64_t)r * r;
        }
        x.nl = nl;
        x.nr = N - nl;
        x.sl = sl;
        x.sr = sr;
        return x;
    };
    Cand lb;
    lb.nl = 0;
    lb.b = 0x7FFFFFFF;
    lb.q = q;
    lb.f = f;
    lb.nr = 0;
    lb.pad = 0;
    lb.sl = lb.sr = 0;
    uint32_t lcl[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) lcl[k] = 0;
    if (!split_rank) {
        // exact: each lane ranks its entries (ascending thresholds: a strictly
        // better score replaces, so ties keep the smaller threshold)
        for (int e = lane; e < total; e += 64) {
            uint32_t c[KMAX];
            const int b = entry(e, c);
            const Cand x = make(b, c);
            if (lb.nl == 0 || cand_better(x, lb)) {
                lb = x;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) lcl[k] = c[k];
            }
        }
    } else {
        float q1 = -1.0f, q2 = -1.0f;
        int e1 = 0;
        for (int e = lane; e < total; e += 64) {
            uint32_t c[KMAX];
            (void)entry(e, c);
            const float qc = hist_q32<KMAX>(c, cnode, N);
            if (qc > q1) {
                q2 = q1;
                q1 = qc;
                e1 = e;
            } else if (qc > q2) {
                q2 = qc;
            }
        }
        const float qmax = wave_max_f_dpp(q1);
        if (qmax < 0.0f) return lb;
        const float floor32 = fp32_floor(qmax);
        const bool fin = q1 >= floor32;
        const bool multi = fin && q2 >= floor32;
        if (__ballot(multi)) {
            if (multi) {
                for (int e = lane; e < total; e += 64) {
                    uint32_t c[KMAX];
                    const int b = entry(e, c);
                    if (hist_q32<KMAX>(c, cnode, N) < floor32) continue;
                    const Cand x = make(b, c);
                    if (lb.nl == 0 || cand_better(x, lb)) {
                        lb = x;
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) lcl[k] = c[k];
                    }
                }
            }
        }
        if (fin && !multi) {
            uint32_t c[KMAX];
            const int b = entry(e1, c);
            lb = make(b, c);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) lcl[k] = c[k];
        }
    }
    const unsigned long long finm = __ballot(lb.nl != 0);
    if (!finm) return lb;
    int src;
    Cand w;
    if (__popcll(finm) == 1) {
        src = (int)__ffsll(finm) - 1;
        w = shfl_cand(lb, src);
    } else {
        w = wave_best_exact(lb);
        const unsigned long long m = __ballot(lb.nl != 0 && lb.b == w.b);
        src = (int)__ffsll(m) - 1;
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        cl_out[k] = (uint32_t)__builtin_amdgcn_readlane((int)lcl[k], src);
    return w;
}

// ---------------------------------------------------------------------------
// Regression items (a job of the float-target regressor).  For each of the
// item's drawn features in turn: an LDS histogram of the bootstrap weights
// W[256] (32-bit) and the weighted fixed-point target sums T[256] (64-bit LDS
// atomics, two's complement) over the node's rows, then the threshold scan.
// Lane l owns bins 4l .. 4l+3; prefix sums over the lanes give each
// threshold's left (W_L, T_L).  Thresholds are ranked by the FP64 score
// g^2 / (W_L W_R) (g = T_L W_R - T_R W_L) and every threshold within the
// ranking margin of the maximum is compared exactly (reg_better); with exact
// ranking every valid threshold is.
__device__ __forceinline__ long long wave_excl_sum64(long long x) {
    long long incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long o = __shfl_up(incl, d);
        if ((int)(threadIdx.x & 63) >= d) incl += o;
    }
    return incl - x;
}

__device__ __forceinline__ Cand reg_feature_best(const uint32_t* hw, const long long* ht, int B,
                                                 int q, int f, uint32_t W, int64_t T,
                                                 int split_rank) {
    const int lane = threadIdx.x & 63;
    const uint4 wv = reinterpret_cast<const uint4*>(hw)[lane];
    const uint32_t w4[4] = {wv.x, wv.y, wv.z, wv.w};
    long long t4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t4[u] = ht[lane * 4 + u];
    const uint32_t wsum = w4[0] + w4[1] + w4[2] + w4[3];
    const long long tsum = t4[0] + t4[1] + t4[2] + t4[3];
    uint32_t wl = wave_incl_sum(wsum) - wsum;
    long long tl = wave_excl_sum64(tsum);
    Cand c[4];
    double qc[4];
    double q1 = -1.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        wl += w4[u];
        tl += t4[u];
        const int b = lane * 4 + u;
        c[u].q = q;
        c[u].f = f;
        c[u].b = b;
        c[u].pad = 0;
        const bool ok = b <= B - 2 && w4[u] != 0 && wl != 0 && wl != W;
        c[u].nl = ok ? wl : 0u;
        c[u].nr = W - wl;
        c[u].sl = (uint64_t)tl;
        c[u].sr = (uint64_t)(T - (int64_t)tl);
        qc[u] = ok ? reg_q64(c[u]) : -1.0;
        q1 = qc[u] > q1 ? qc[u] : q1;
    }
    double qmax = q1;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const double o = __shfl_xor(qmax, m);
        qmax = o > qmax ? o : qmax;
    }
    Cand lb;
    lb.nl = 0;
    lb.b = 0x7FFFFFFF;
    lb.q = q;
    lb.f = f;
    lb.nr = 0;
    lb.pad = 0;
    lb.sl = lb.sr = 0;
    if (qmax < 0.0) return lb;
    const double floor64 = split_rank ? fp64_floor(qmax) : 0.0;
    // the lane's finalists in ascending threshold order: a strictly better
    // one replaces, so ties keep the smaller threshold
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (c[u].nl != 0 && qc[u] >= floor64 && (lb.nl == 0 || reg_better(c[u], lb))) lb = c[u];
    const unsigned long long finm = __ballot(lb.nl != 0);
    if (__popcll(finm) == 1) return shfl_cand(lb, (int)__ffsll(finm) - 1);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Cand o = shfl_xor_cand(lb, m);
        if (reg_wins_same_feature(o, lb)) lb = o;
    }
    return lb;
}

// One regression item: draws q0 .. q0 + nf - 1 of the node, one after the
// other in the wave's LDS region (256 words of W, then 256 64-bit sums).
template <int RB>
__device__ __forceinline__ Cand reg_item(const ForestDev& F, const SlotRec& sr, int q0, int nf,
                                         const int* fq, const uint8_t* const* col,
                                         uint32_t* hist) {
    const int lane = threadIdx.x & 63;
    uint32_t* hw = hist;
    long long* ht = reinterpret_cast<long long*>(hist + 256);
    const int64_t T = (int64_t)((uint64_t)sr.cnode[0] | ((uint64_t)sr.cnode[1] << 32));
    const uint32_t W = sr.n, len = sr.len;
    const int64_t* yfix = sr.yfix;
    const uint64_t* recs = sr.recs;
    Cand best;
    best.nl = 0;
    for (int v = 0; v < nf; ++v) {
        reinterpret_cast<uint4*>(hw)[lane] = make_uint4(0u, 0u, 0u, 0u);
        reinterpret_cast<uint4*>(ht)[2 * lane] = make_uint4(0u, 0u, 0u, 0u);
        reinterpret_cast<uint4*>(ht)[2 * lane + 1] = make_uint4(0u, 0u, 0u, 0u);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (uint32_t i0 = 0; i0 < len; i0 += 64 * RB) {
            uint64_t r[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const uint32_t i = i0 + u * 64 + lane;
                r[u] = rec_at(recs, i, len);
            }
            uint32_t b[RB];
            long long yv[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                b[u] = ldg(col[v] + rec_row(r[u]));
                yv[u] = ldg(yfix + rec_row(r[u]));
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const uint32_t w = rec_w(r[u]);  // padding rows: w = 0
                if (w) {
                    atomicAdd(&hw[b[u]], w);
                    atomicAdd(reinterpret_cast<unsigned long long*>(&ht[b[u]]),
                              (unsigned long long)((long long)w * yv[u]));
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const Cand fb = reg_feature_best(hw, ht, (int)sr.B, q0 + v, fq[v], W, T, F.split_rank);
        // draws in order: a strictly better score replaces
        if (fb.nl != 0 && (best.nl == 0 || reg_better(fb, best))) best = fb;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the next draw rewrites
    }
    return best;
}

// Large nodes, phase 0: each node's mtry drawn features (the keyed
// permutation of its heap id, in draw order), their bin columns and the
// node's slot record.  A wavefront serves 64 / S nodes at once, S = the
// plan's draws per node rounded up to a power of two (at most 64): lane l
// takes the draws l mod S, l mod S + S, ... of node l / S, so few draws per
// node do not leave most of the lanes idle.  When the permutation's round
// functions fit the segment's table (rounds << half 16-bit entries, at most
// F.draw_tab: halves of up to 8 bits, at most 2^16 widened columns), the
// node's lane segment first tabulates them in LDS: each lane then evaluates
// a few round functions, uniformly, instead of every round of every
// cycle-walking step of its draws, where the segment waits for its longest
// walk.
__global__ __launch_bounds__(256) void k_draws(ForestDev F, int level) {
    extern __shared__ uint16_t dtab[];  // [256 / S][F.draw_tab]
    const uint32_t count = level_slots(F, level);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t S = F.draw_seg, G = 64u / S;
    const uint32_t sub = lane / S, ql = lane % S;
    const uint32_t w0 = blockIdx.x * 4u + uniform(threadIdx.x >> 6);
    uint16_t* tab = dtab + (size_t)(threadIdx.x / S) * F.draw_tab;
    for (uint32_t base = w0 * G; base < count; base += gridDim.x * 4u * G) {
        const uint32_t slot = base + sub;
        if (slot >= count) continue;
        const uint32_t id = F.slot_node_in[slot];
        const NodeDev nd = F.nodes[id];
        const TreeDev tr = F.trees[nd.tree];
        const JobDev& J = F.jobs[tr.job];
        const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kMtry, (uint32_t)J.t,
                                      (uint32_t)tr.tau, nd.heap, 0u, (uint64_t)J.p_w);
        uint32_t* out = F.feat + (size_t)slot * F.mtry_cap;
        const uint8_t** oc = F.fcol + (size_t)slot * F.mtry_cap;
        uint32_t* pos = F.fpos + (size_t)slot * F.mtry_cap;
        const bool use_tab = (P.rounds << P.half) <= F.draw_tab;  // uniform over the segment
        if (use_tab) {
            // the previous node's lookups of this segment are done (program order)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            for (uint32_t e = ql; e < (P.rounds << P.half); e += S)
                tab[e] = (uint16_t)perm_round(P, e >> P.half, e & P.mask);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        for (uint32_t q = ql; q < (uint32_t)J.mtry; q += S) {
            const uint32_t f = use_tab ? perm_apply_tab(P, tab, q) : perm_apply(P, q);
            out[q] = f;
            oc[q] = ldg(J.colptr + f);
            // column-major path without k_col_count: the item's place among
            // its column's items
            if (F.col_count == 1) pos[q] = atomicAdd(F.fcnt + J.gbase + f, 1u);
        }
        SlotRec* sr = F.srec + slot;
        for (uint32_t c = ql; c < 16u; c += S)
            sr->cnode[c] = c < (uint32_t)J.K ? F.cls[(size_t)id * F.kmax + c] : 0u;
        if (ql == 0) {
            sr->recs = J.rec[F.parity] + (size_t)tr.tau * J.rstride + nd.seg;
            sr->yfix = J.reg ? J.yfix : nullptr;
            sr->id = id;
            sr->len = nd.len;
            sr->n = nd.n;
            sr->mtry = (uint32_t)J.mtry;
            sr->B = (uint32_t)J.B;
            sr->reg = (uint32_t)J.reg;
            sr->K = (uint32_t)J.K;
        }
    }
}

// Large nodes, phase 1: one wavefront per (node, FW consecutive draws)
// item, with its own LDS histogram [FW][KMAX][256] (4 KB up to 4 classes,
// 8 KB / 16 KB for 5-8 / 9-16 classes).  The wave gathers the bins of its features at the node's rows,
// accumulates the weighted class counts with LDS atomics (class-major rows
// spread a wave's atomics over the banks by bin), scans each feature and
// writes the item's best candidate and its left class counts.  No barriers:
// the four waves of a workgroup are independent.
// Regression item of a node with at most kRegWaveRows distinct rows: lane i
// holds row i (its weight w_i and w_i y_fix_i), and for each drawn feature
// the left sums of the threshold at lane i's bin, (W_L, T_L) = the sums of
// (w_j, w_j y_fix_j) over the rows j with bin <= b_i, come from one pass over
// the rows with their values broadcast -- no histogram to clear and scan.
// The thresholds scored are the occupied bins, as in reg_feature_best, and
// ranking, margin and tie-breaks are the same, so both give one candidate.
constexpr uint32_t kRegWaveRows = 24;

__device__ __forceinline__ Cand reg_item_wave(const ForestDev& F, const SlotRec& sr, int q0,
                                              int nf, const int* fq,
                                              const uint8_t* const* col) {
    const int lane = threadIdx.x & 63;
    const uint32_t len = sr.len, W = sr.n;
    const int64_t T = (int64_t)((uint64_t)sr.cnode[0] | ((uint64_t)sr.cnode[1] << 32));
    const bool have = (uint32_t)lane < len;
    const uint64_t r = have ? ldg(sr.recs + lane) : 0ull;
    const uint32_t row = rec_row(r), w = have ? rec_w(r) : 0u;
    const int64_t yw = have ? (int64_t)w * ldg(sr.yfix + row) : 0;
    Cand best;
    best.nl = 0;
    for (int v = 0; v < nf; ++v) {
        const int b = have ? (int)ldg(col[v] + row) : 0x7FFF;
        uint32_t wl = 0;
        int64_t tl = 0;
        for (uint32_t j = 0; j < len; ++j) {
            const int bj = __builtin_amdgcn_readlane(b, (int)j);
            const uint32_t wj = readlane_w(w, (int)j);
            const int64_t tj = (int64_t)readlane64((uint64_t)yw, (int)j);
            if (bj <= b) {
                wl += wj;
                tl += tj;
            }
        }
        Cand c;
        c.q = q0 + v;
        c.f = fq[v];
        c.b = b;
        c.pad = 0;
        const bool ok = have && b <= (int)sr.B - 2 && wl != W;  // wl >= w_i > 0
        c.nl = ok ? wl : 0u;
        c.nr = W - wl;
        c.sl = (uint64_t)tl;
        c.sr = (uint64_t)(T - tl);
        const double qc = ok ? reg_q64(c) : -1.0;
        double qmax = qc;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const double o = __shfl_xor(qmax, m);
            qmax = o > qmax ? o : qmax;
        }
        if (qmax < 0.0) continue;
        const double floor64 = F.split_rank ? fp64_floor(qmax) : 0.0;
        if (!(ok && qc >= floor64)) {
            c.nl = 0;
            c.b = 0x7FFFFFFF;
        }
        const unsigned long long finm = __ballot(c.nl != 0);
        Cand fb;
        if (__popcll(finm) == 1) {
            fb = shfl_cand(c, (int)__ffsll(finm) - 1);
        } else {
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const Cand o = shfl_xor_cand(c, m);
                if (reg_wins_same_feature(o, c)) c = o;
            }
            fb = c;
        }
        // draws in order: a strictly better score replaces
        if (fb.nl != 0 && (best.nl == 0 || reg_better(fb, best))) best = fb;
    }
    return best;
}

// Work of a level for the node-major histogram kernels: node slots [0, n)
// with npi items each.  Workgroup b takes the slots congruent to b mod 8 (the
// grid is a multiple of 8), and its waves walk those slots' items in order,
// so a node's items run side by side in one XCD and share its records
// through that XCD's L2 when the hardware deals workgroups round-robin to the
// 8 XCDs (any mapping gives the same results: every item is visited once).
// With an explicit count, items [first, first + count) are walked directly
// (plain form).
struct ItemWalk {
    bool dyn;
    uint32_t x, r, R, m_end, first, npi;
    __device__ ItemWalk(const ForestDev& F, int level, uint32_t first_, uint32_t count,
                        uint32_t wave) {
        npi = (uint32_t)F.npi;
        first = first_;
        dyn = count == 0xFFFFFFFFu;
        x = 0;
        r = blockIdx.x * 4u + wave;
        R = gridDim.x * 4u;
        m_end = count;
        if (dyn) {
            const uint32_t n_slots = level_slots(F, level);
            x = blockIdx.x % 8u;
            r = (blockIdx.x / 8u) * 4u + wave;
            R = (gridDim.x / 8u) * 4u;
            m_end = n_slots > x ? (n_slots - x + 7u) / 8u * npi : 0u;
        }
    }
    __device__ uint32_t item(uint32_t cur) const {
        return dyn ? (8u * (cur / npi) + x) * npi + cur % npi : first + cur;
    }
};

// Regression nodes of the node-major levels: one wavefront per (node, F.fw
// consecutive draws) item, the histograms and scan of reg_item in the wave's
// LDS region (F.fw * F.kmax * 256 words, at least 768).  Items of
// classification nodes are left to k_hist_tile, which in turn skips these:
// the regression item's registers and code stay out of the classification
// kernel.
template <int RB>
__global__ __launch_bounds__(256) void k_hist_reg(ForestDev F, int level, uint32_t first,
                                                  uint32_t count) {
    extern __shared__ uint4 lds_raw[];
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    const int fw = F.fw;
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds_raw) + (size_t)wave * fw * F.kmax * 256;
    const ItemWalk wk(F, level, first, count, (uint32_t)wave);
    unsigned long long alg = 0;
    for (uint32_t cur = wk.r; cur < wk.m_end; cur += wk.R) {
        const uint32_t item = wk.item(cur);
        const uint32_t slot = item / wk.npi, j = item % wk.npi;
        const SlotRec& sr = F.srec[slot];
        if (!sr.reg) continue;  // a classification node: k_hist_tile
        const int q0 = (int)j * fw;
        const int mtry = (int)sr.mtry;
        if (q0 >= mtry) continue;  // the job draws fewer features this iteration
        const int nf = min(fw, mtry - q0);
        const uint32_t* drawn = F.feat + (size_t)slot * F.mtry_cap + q0;
        const uint8_t* const* dcol = F.fcol + (size_t)slot * F.mtry_cap + q0;
        int fq[4];
        const uint8_t* col[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            fq[u] = (int)drawn[u < nf ? u : 0];
            col[u] = dcol[u < nf ? u : 0];
        }
        const Cand best = sr.len <= kRegWaveRows ? reg_item_wave(F, sr, q0, nf, fq, col)
                                                 : reg_item<RB>(F, sr, q0, nf, fq, col, hist);
        if (lane == 0) F.cand[item] = best;
        alg += (unsigned long long)sr.len * (unsigned long long)(nf + (j == 0 ? 6 : 0));
    }
    if (F.alg_bytes && lane == 0 && alg)
        atomicAdd((unsigned long long*)&F.alg_bytes[(blockIdx.x * 4u + wave) & (kAlgWords - 1)],
                  alg);
}

template <int KMAX, int FW, int RB>
__global__ __launch_bounds__(256) void k_hist_tile(ForestDev F, int level, uint32_t first,
                                                   uint32_t count) {
    // RB rows per lane per batch: RB record loads and RB * FW bin gathers in
    // flight (a launch tuning choice; every RB gives the same histograms)
    constexpr int WORDS = FW * KMAX * 256;
    extern __shared__ uint4 lds_raw[];
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds_raw) + wave * WORDS;
    const ItemWalk wk(F, level, first, count, (uint32_t)wave);
    const uint32_t npi = wk.npi;
    unsigned long long alg = 0;
    for (uint32_t cur = wk.r; cur < wk.m_end; cur += wk.R) {
        const uint32_t item = wk.item(cur);
        const uint32_t slot = item / npi, j = item % npi;
        const SlotRec& sr = F.srec[slot];
        if (sr.reg) continue;  // a regression node: k_hist_reg
        // with split_k, jobs of at most 4 classes take the 4-plane instance
        if (F.split_k && ((sr.K <= 4u) != (KMAX <= 4))) continue;
        const int q0 = (int)j * FW;
        const int mtry = (int)sr.mtry;
        if (q0 >= mtry) continue;  // the job draws fewer features this iteration
        const int nf = min(FW, mtry - q0);
        const uint32_t* drawn = F.feat + (size_t)slot * F.mtry_cap + q0;
        const uint8_t* const* dcol = F.fcol + (size_t)slot * F.mtry_cap + q0;
        int fq[FW];
        const uint8_t* col[FW];
#pragma unroll
        for (int u = 0; u < FW; ++u) {
            fq[u] = (int)drawn[u < nf ? u : 0];
            col[u] = dcol[u < nf ? u : 0];
        }
#pragma unroll
        for (int i = 0; i < WORDS / 256; ++i)
            reinterpret_cast<uint4*>(hist)[i * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
        const uint64_t* recs = sr.recs;
        const uint32_t len = sr.len;
        // (loading the next batch's records ahead of this batch's gathers was
        // measured slower here: the other waves of the SIMD hide the latency)
        for (uint32_t i0 = 0; i0 < len; i0 += 64 * RB) {
            uint64_t r[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const uint32_t i = i0 + u * 64 + lane;
                r[u] = i < len ? ldg(recs + i) : 0ull;
            }
            uint32_t b[RB][FW];
#pragma unroll
            for (int u = 0; u < RB; ++u)
#pragma unroll
                for (int v = 0; v < FW; ++v) b[u][v] = ldg(col[v] + rec_row(r[u]));
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const uint32_t w = rec_w(r[u]), y = rec_y(r[u]);  // padding rows: w = 0
#pragma unroll
                for (int v = 0; v < FW; ++v)
                    if (v < nf && w) atomicAdd(&hist[(v * KMAX + y) * 256 + b[u][v]], w);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        uint32_t cnode[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) cnode[c] = sr.cnode[c];
        const uint32_t N = sr.n;
        const int B = (int)sr.B;
        Cand best;
        best.nl = 0;
        int bi = 0;
        uint32_t best_cl[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) best_cl[c] = 0;
#pragma unroll
        for (int v = 0; v < FW; ++v) {
            if (v >= nf) break;
            Cand fb;
            uint32_t fcl[KMAX];
            if constexpr (KMAX <= 4)
                fb = feature_best_compact<KMAX>(hist + v * KMAX * 256, B, q0 + v, fq[v], cnode,
                                                N, F.split_rank, fcl);
            else
                fb = feature_best<KMAX>(hist + v * KMAX * 256, B, q0 + v, fq[v], cnode, N,
                                        F.split_rank);
            // draws in order: a strictly better score replaces
            if (fb.nl != 0 && (best.nl == 0 || cand_better(fb, best))) {
                best = fb;
                bi = v;
                if constexpr (KMAX <= 4) {
#pragma unroll
                    for (int c = 0; c < KMAX; ++c) best_cl[c] = fcl[c];
                }
            }
        }
        // left class counts of the item's best, for the partition step
        uint32_t* out = F.cand_cl + (size_t)item * F.kmax;
        if constexpr (KMAX <= 4) {
            if (lane < KMAX) {
#pragma unroll
                for (int c = 0; c < KMAX; ++c)
                    if (lane == c) out[c] = best.nl != 0 ? best_cl[c] : 0u;
            } else if (lane < F.kmax) {
                out[lane] = 0u;  // the plan's class planes past this instance's
            }
        } else {
            const int bt = best.nl != 0 ? best.b : -1;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                const uint4 v4 =
                    *reinterpret_cast<const uint4*>(hist + (bi * KMAX + c) * 256 + lane * 4);
                const int bl = lane * 4;
                const uint32_t a = (bl <= bt ? v4.x : 0u) + (bl + 1 <= bt ? v4.y : 0u) +
                                   (bl + 2 <= bt ? v4.z : 0u) + (bl + 3 <= bt ? v4.w : 0u);
                const uint32_t tot =
                    (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(a), 63);
                if (lane == c) out[c] = tot;
            }
        }
        if (lane == 0) F.cand[item] = best;
        alg += (unsigned long long)len * (unsigned long long)(nf + (j == 0 ? 6 : 0));
        // the histogram is rewritten by the wave's next item
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // one atomic per wave for the statistics
    if (F.alg_bytes && lane == 0 && alg)
        atomicAdd((unsigned long long*)&F.alg_bytes[(blockIdx.x * 4u + wave) & (kAlgWords - 1)],
                  alg);
}

// ---------------------------------------------------------------------------
// Column-major histogram path.  At deep levels the nodes are small and a
// node-major gather pulls one cache line per row and drawn feature from a
// column far larger than the node; here the items (node, draw) of a level are
// bucketed by bin column instead, and each workgroup stages one column in LDS
// once and serves the histograms of a run of that column's items from it.
//
// k_col_scan (one workgroup): exclusive offsets of the per-column item counts
// that k_draws accumulated, the units (runs of at most col_unit items of one
// column), and zero counts for the next level.
__global__ __launch_bounds__(256) void k_col_scan(ForestDev F, int level) {
    __shared__ uint32_t s_i[4], s_u[4];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t G = F.n_gcol, U = F.col_unit;
    const uint32_t C = (G + 255u) / 256u;
    const uint32_t a = min(G, tid * C), b = min(G, a + C);
    uint32_t si = 0, su = 0;
    for (uint32_t g = a; g < b; ++g) {
        const uint32_t c = F.fcnt[g];
        si += c;
        su += (c + U - 1u) / U;
    }
    const uint32_t ii = wave_incl_sum(si), iu = wave_incl_sum(su);
    if (lane == 63) {
        s_i[wave] = ii;
        s_u[wave] = iu;
    }
    __syncthreads();
    uint32_t oi = ii - si, ou = iu - su, tu = 0;
    for (uint32_t v = 0; v < 4; ++v) {
        if (v < wave) {
            oi += s_i[v];
            ou += s_u[v];
        }
        tu += s_u[v];
    }
    for (uint32_t g = a; g < b; ++g) {
        const uint32_t c = F.fcnt[g];
        F.fcnt[g] = 0;
        F.fpos[(size_t)F.slot_cap * F.mtry_cap + g] = oi;  // column offsets follow the places
        const uint32_t gq = F.gcol_q[g];
        for (uint32_t k = 0; k * U < c; ++k) {
            if (ou < F.unit_cap) {
                ColUnit cu;
                cu.begin = oi + k * U;
                cu.end = oi + min(c, (k + 1u) * U);
                cu.gq = gq;
                cu.pad = 0;
                F.units[ou] = cu;
            }
            ++ou;
        }
        oi += c;
    }
    if (tid == 0) {
        if (tu > F.unit_cap) atomicOr(&F.ctrs[level].overflow, 16u);
        F.ctrs[level].n_units = min(tu, F.unit_cap);
    }
}

// k_col_count: the items' places within their columns, counted per workgroup
// in LDS.  Workgroup w takes a contiguous run of the level's node slots,
// ranks each item among the workgroup's items of its column (LDS atomics),
// reserves one run per touched column in the global per-column counts (one
// global atomic per column and workgroup, not one per item), then adds the
// run's start to its items' places.  The places of a column's items are
// unique and dense; their order is immaterial.
__global__ __launch_bounds__(256) void k_col_count(ForestDev F, int level) {
    extern __shared__ uint32_t lcnt[];  // [n_gcol]
    const uint32_t count = level_slots(F, level);
    const uint32_t G = F.n_gcol;
    const uint32_t per = (count + gridDim.x - 1u) / gridDim.x;
    const uint32_t s0 = min(count, blockIdx.x * per), s1 = min(count, s0 + per);
    if (s0 >= s1) return;  // the whole workgroup: no barrier is skipped by part of it
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) lcnt[g] = 0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = uniform(threadIdx.x >> 6);
    for (uint32_t slot = s0 + wave; slot < s1; slot += 4u) {
        const SlotRec& sr = F.srec[slot];
        const NodeDev nd = F.nodes[uniform(sr.id)];
        const uint32_t gb = F.jobs[F.trees[nd.tree].job].gbase;
        const size_t row = (size_t)slot * F.mtry_cap;
        for (uint32_t q = lane; q < sr.mtry; q += 64u)
            F.fpos[row + q] = atomicAdd(&lcnt[gb + F.feat[row + q]], 1u);
    }
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
        const uint32_t c = lcnt[g];
        lcnt[g] = c ? atomicAdd(F.fcnt + g, c) : 0u;
    }
    __syncthreads();
    for (uint32_t slot = s0 + wave; slot < s1; slot += 4u) {
        const SlotRec& sr = F.srec[slot];
        const NodeDev nd = F.nodes[uniform(sr.id)];
        const uint32_t gb = F.jobs[F.trees[nd.tree].job].gbase;
        const size_t row = (size_t)slot * F.mtry_cap;
        for (uint32_t q = lane; q < sr.mtry; q += 64u)
            F.fpos[row + q] += lcnt[gb + F.feat[row + q]];
    }
}

// k_col_scatter: one wavefront per large node; each drawn item goes to its
// column's run of the sorted list (order within a run is immaterial: every
// item writes only its own candidate).
__global__ __launch_bounds__(256) void k_col_scatter(ForestDev F, int level) {
    const uint32_t count = level_slots(F, level);
    const int lane = threadIdx.x & 63;
    const uint32_t* off = F.fpos + (size_t)F.slot_cap * F.mtry_cap;
    for (uint32_t slot = blockIdx.x * 4u + uniform(threadIdx.x >> 6); slot < count;
         slot += gridDim.x * 4u) {
        const SlotRec& sr = F.srec[slot];
        const NodeDev nd = F.nodes[uniform(sr.id)];
        const uint32_t gb = F.jobs[F.trees[nd.tree].job].gbase;
        const size_t row = (size_t)slot * F.mtry_cap;
        for (uint32_t q = lane; q < sr.mtry; q += 64) {
            const uint32_t dst = off[gb + F.feat[row + q]] + F.fpos[row + q];
            F.fitems[dst] = (uint32_t)(row + q);
        }
    }
}

// k_hist_col: grid-stride over units.  The workgroup copies the unit's bin
// column into LDS (16-byte loads, the whole column once), then each wave
// takes the unit's items in turn: an LDS class-count histogram [KMAX][256]
// from the node's row records and the staged bins, the prefix scan, and the
// item's candidate and left class counts (item = slot * mtry_cap + draw).
template <int KMAX>
__global__ __launch_bounds__(1024) void k_hist_col(ForestDev F, int level) {
    constexpr int WORDS = KMAX * 256;
    constexpr int RB = 8;
    extern __shared__ uint4 lds_raw[];
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds_raw) + wave * WORDS;
    uint4* colq = lds_raw + nw * (WORDS / 4);
    const uint8_t* colb = reinterpret_cast<const uint8_t*>(colq);
    const LevelCtr& lc = F.ctrs[level];
    const uint32_t n_units = lc.overflow ? 0u : min(lc.n_units, F.unit_cap);
    const uint32_t mc = (uint32_t)F.mtry_cap;
    unsigned long long alg = 0;
    for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const ColUnit cu = F.units[u];
        const uint4* src = reinterpret_cast<const uint4*>(F.fcol[F.fitems[cu.begin]]);
        for (uint32_t i = threadIdx.x; i < cu.gq; i += blockDim.x) colq[i] = src[i];
        __syncthreads();
        // The wave's items are k0 + t * nw; their node records are loaded
        // one per lane, 64 at a time, and read back with readlane.
        for (uint32_t k0 = cu.begin + (uint32_t)wave; k0 < cu.end; k0 += 64u * nw) {
            const uint32_t kk = k0 + (uint32_t)lane * nw;
            const bool have = kk < cu.end;
            const uint32_t my_item = have ? F.fitems[kk] : 0u;
            const SlotRec* msr = F.srec + my_item / mc;
            const uint64_t my_recs = have ? reinterpret_cast<uint64_t>(msr->recs) : 0ull;
            const uint32_t my_len = have ? msr->len : 0u, my_n = have ? msr->n : 0u;
            const uint32_t my_B = have ? msr->B : 0u, my_f = have ? F.feat[my_item] : 0u;
            uint32_t my_cn[KMAX];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) my_cn[c] = have ? msr->cnode[c] : 0u;
            const uint32_t n_here = min(64u, (cu.end - k0 + nw - 1u) / nw);
            // Record batches stream one ahead: while a batch is counted, the
            // next one is in flight -- the item's next batch, or after its
            // last batch the first batch of the wave's next item (hidden
            // behind that item's scan).
            uint64_t rn[RB];
            {
                const uint64_t* recs = reinterpret_cast<const uint64_t*>(readlane64(my_recs, 0));
                const uint32_t len = readlane_w(my_len, 0);
#pragma unroll
                for (int v = 0; v < RB; ++v) {
                    const uint32_t i = v * 64 + lane;
                    rn[v] = rec_raw(recs, i, len);
                }
            }
            for (uint32_t t = 0; t < n_here; ++t) {
                const uint32_t item = readlane_w(my_item, (int)t);
                const uint32_t q = item - (item / mc) * mc;
                const uint64_t* recs = reinterpret_cast<const uint64_t*>(readlane64(my_recs, (int)t));
                const uint32_t len = readlane_w(my_len, (int)t);
#pragma unroll
                for (int i = 0; i < WORDS / 256; ++i)
                    reinterpret_cast<uint4*>(hist)[i * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
                for (uint32_t i0 = 0;;) {
                    uint64_t r[RB];
#pragma unroll
                    for (int v = 0; v < RB; ++v) r[v] = rn[v];
                    // all bins of the batch first (records past the node's end
                    // repeat its last record and are masked below), then the
                    // atomics: one LDS round trip for the batch, not one per row
                    uint32_t bb[RB];
#pragma unroll
                    for (int v = 0; v < RB; ++v) bb[v] = colb[rec_row(r[v])];
                    const uint32_t i1 = i0 + 64 * RB;
                    if (i1 < len) {
#pragma unroll
                        for (int v = 0; v < RB; ++v) rn[v] = rec_raw(recs, i1 + v * 64 + lane, len);
                    } else if (t + 1 < n_here) {
                        const uint64_t* nrecs =
                            reinterpret_cast<const uint64_t*>(readlane64(my_recs, (int)t + 1));
                        const uint32_t nlen = readlane_w(my_len, (int)t + 1);
#pragma unroll
                        for (int v = 0; v < RB; ++v) rn[v] = rec_raw(nrecs, v * 64 + lane, nlen);
                    }
#pragma unroll
                    for (int v = 0; v < RB; ++v) {
                        if (i0 + (uint32_t)(v * 64 + lane) < len)
                            atomicAdd(&hist[rec_y(r[v]) * 256 + bb[v]], rec_w(r[v]));
                    }
                    if (i1 >= len) break;
                    i0 = i1;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                uint32_t cnode[KMAX];
#pragma unroll
                for (int c = 0; c < KMAX; ++c) cnode[c] = readlane_w(my_cn[c], (int)t);
                const int B = (int)readlane_w(my_B, (int)t), fq = (int)readlane_w(my_f, (int)t);
                const uint32_t N = readlane_w(my_n, (int)t);
                Cand best;
                uint32_t* out = F.cand_cl + (size_t)item * F.kmax;
                if constexpr (KMAX <= 4) {
                    uint32_t cl[KMAX];
                    best = feature_best_compact<KMAX>(hist, B, (int)q, fq, cnode, N, F.split_rank,
                                                      cl);
                    if (lane < KMAX) {
#pragma unroll
                        for (int c = 0; c < KMAX; ++c)
                            if (lane == c) out[c] = best.nl != 0 ? cl[c] : 0u;
                    }
                } else {
                    best = feature_best<KMAX>(hist, B, (int)q, fq, cnode, N, F.split_rank);
                    const int bt = best.nl != 0 ? best.b : -1;
#pragma unroll
                    for (int c = 0; c < KMAX; ++c) {
                        const uint4 v4 =
                            *reinterpret_cast<const uint4*>(hist + c * 256 + lane * 4);
                        const int bl = lane * 4;
                        const uint32_t a = (bl <= bt ? v4.x : 0u) + (bl + 1 <= bt ? v4.y : 0u) +
                                           (bl + 2 <= bt ? v4.z : 0u) + (bl + 3 <= bt ? v4.w : 0u);
                        const uint32_t tot =
                            (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(a), 63);
                        if (lane == c) out[c] = tot;
                    }
                }
                if (lane == 0) F.cand[item] = best;
                alg += (unsigned long long)len * (unsigned long long)(1u + (q == 0 ? 6u : 0u));
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
        __syncthreads();  // the column is replaced by the next unit's
    }
    if (F.alg_bytes && lane == 0 && alg)
        atomicAdd((unsigned long long*)&F.alg_bytes[2 * kAlgWords +
                                                    ((blockIdx.x * nw + wave) & (kAlgWords - 1))],
                  alg);
}

// Partition of a split node's first `len` row records in one pass: left rows
// (bin <= b) from the front in row order, right rows from the back in reverse
// row order (no result depends on a node's row order, and each child segment
// stays monotone in row index for the next level's gathers); returns the
// left rows.  len = 0 when neither child is searched again.  AHEAD: the next
// block's records are loaded while a block is placed (classification nodes;
// the regression finalize, at more registers, measured slower with it).
template <bool AHEAD>
__device__ uint32_t partition_rows(const ForestDev& F, const JobDev& J, const TreeDev& tr,
                                   const NodeDev& nd, const SlotRec& sr, const Cand& best,
                                   uint32_t len) {
    const int lane = threadIdx.x & 63;
    const uint8_t* col = ldg(J.colptr + best.f);
    const uint64_t* recs = sr.recs;
    uint64_t* rout = J.rec[F.parity ^ 1] + (size_t)tr.tau * J.rstride + nd.seg;
    constexpr int kR = 8;  // rows per lane per block: lane l owns rows [l kR, l kR + kR)
    uint32_t runl = 0, runr = 0;
    uint64_t rn[kR];  // with AHEAD: the next block's records, loaded one block ahead
    if constexpr (AHEAD) {
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            const uint32_t i = (uint32_t)lane * kR + u;
            rn[u] = i < len ? ldg(recs + i) : 0ull;
        }
    }
    for (uint32_t blk = 0; blk < len; blk += 64 * kR) {
        const uint32_t i0 = blk + (uint32_t)lane * kR;
        uint64_t r[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            if constexpr (AHEAD)
                r[u] = rn[u];
            else
                r[u] = i0 + u < len ? ldg(recs + i0 + u) : 0ull;
        }
        int bb[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) bb[u] = i0 + u < len ? (int)ldg(col + rec_row(r[u])) : 0x7FFF;
        if constexpr (AHEAD) {
            // the next block's records are in flight while this block is placed
            const uint32_t j0 = i0 + 64 * kR;
#pragma unroll
            for (int u = 0; u < kR; ++u) rn[u] = j0 + u < len ? ldg(recs + j0 + u) : 0ull;
        }
        uint32_t nlm = 0, nrm = 0;
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            nlm += bb[u] <= best.b;
            nrm += i0 + u < len && bb[u] > best.b;
        }
        // exclusive prefix of (left, right) over the lanes, both packed in one
        // word (a block holds 512 rows)
        const uint32_t mine = nlm | (nrm << 16);
        const uint32_t incl = wave_incl_sum(mine);
        const uint32_t pre = incl - mine;
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        uint32_t lrow = runl + (pre & 0xFFFFu), rrow = runr + (pre >> 16);
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            if (i0 + u >= len) break;
            if (bb[u] <= best.b)
                rout[lrow++] = r[u];
            else
                rout[len - 1 - rrow++] = r[u];
        }
        runl += tot & 0xFFFFu;
        runr += tot >> 16;
    }
    return runl;
}

// Regression form of the split choice and partition: the node's best
// candidate (exact total order), a split when its gap is nonzero, the rows
// partitioned as for classification when the children are searched next.
__device__ void finalize_reg(const ForestDev& F, JobDev& J, const TreeDev& tr, uint32_t slot,
                             const SlotRec& sr, const NodeDev& nd, Cand c) {
    const int lane = threadIdx.x & 63;
    if (F.split_rank) {
        // FP64 ranking: only the candidates within the margin of the wave's
        // maximum take part in the exact comparison
        const double q = c.nl != 0 ? reg_q64(c) : -1.0;
        double qmax = q;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const double o = __shfl_xor(qmax, m);
            qmax = o > qmax ? o : qmax;
        }
        if (c.nl != 0 && q < fp64_floor(qmax)) c.nl = 0;
        const unsigned long long fin = __ballot(c.nl != 0);
        if (__popcll(fin) == 1) {
            c = shfl_cand(c, (int)__ffsll(fin) - 1);
        } else {
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const Cand o = shfl_xor_cand(c, m);
                if (reg_wins_total(o, c)) c = o;
            }
        }
    } else {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const Cand o = shfl_xor_cand(c, m);
            if (reg_wins_total(o, c)) c = o;
        }
    }
    const Cand best = c;
    const uint32_t child = F.next_base + 2u * (F.n_small_cur + slot);
    if (best.nl == 0 || reg_gap(best) == 0) {  // no decrease: stays the leaf it was created as
        if (lane == 0) {
            mark_unused_pair(F, child);
            F.kinds[F.n_small_cur + slot] = 0;
        }
        return;
    }
    const bool part = (int)nd.depth + 1 < J.D;
    const uint32_t runl = partition_rows<false>(F, J, tr, nd, sr, best, part ? sr.len : 0u);
    if (lane == 0) {
        int kinds[2];
        split_node_reg(F, J, tr, sr.id, nd, best, runl, reg_gain_fix(best, J.s_gain), child,
                       kinds);
        F.kinds[F.n_small_cur + slot] = (uint8_t)(kinds[0] | kinds[1] << 2);
    }
}

// Large nodes, phase 2: one wavefront per node (four per workgroup, no
// barriers).  The node's split is the best of its histogram items' candidates
// (exact score, then draw position, then threshold); a strictly positive
// decrease splits the node and its rows are partitioned in one pass: left
// rows from the front in row order, right rows from the back in reverse row
// order.  No result depends on the order of a node's rows, and each child
// segment stays monotone in row index for the next level's gathers.
// Phase 2 for the regression nodes of a level (k_split_finalize skips them,
// so that the 256-bit arithmetic stays out of the classification kernel).
__global__ __launch_bounds__(256) void k_split_finalize_reg(ForestDev F0, int level,
                                                            uint32_t first, uint32_t count) {
    const ForestDev F = level_view(F0, level);
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_slots(F0, level);
    }
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    for (uint32_t k = blockIdx.x * 4u + (uint32_t)wave; k < count; k += gridDim.x * 4u) {
        const uint32_t slot = first + k;
        const SlotRec& sr = F.srec[slot];
        if (!sr.reg) continue;  // a classification node: k_split_finalize
        const NodeDev nd = F.nodes[sr.id];
        const TreeDev tr = F.trees[nd.tree];
        JobDev& J = F.jobs[tr.job];
        // rank the items' candidates: each lane keeps the best of its items
        const int ni = ((int)sr.mtry + F.fw - 1) / F.fw;
        Cand c;
        c.nl = 0;
        c.q = 0x7FFFFFFF;
        c.b = 0x7FFFFFFF;
        c.f = 0;
        c.nr = 0;
        c.pad = 0;
        c.sl = c.sr = 0;
        for (int t = lane; t < ni; t += 64) {
            const Cand d = F.cand[(size_t)slot * F.npi + t];
            if (d.nl != 0 && (c.nl == 0 || reg_wins_total(d, c))) c = d;
        }
        finalize_reg(F, J, tr, slot, sr, nd, c);
    }
}

template <int KMAX>
__global__ __launch_bounds__(256) void k_split_finalize(ForestDev F0, int level, uint32_t first,
                                                        uint32_t count) {
    const ForestDev F = level_view(F0, level);
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_slots(F0, level);
    }
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    for (uint32_t k = blockIdx.x * 4u + (uint32_t)wave; k < count; k += gridDim.x * 4u) {
        const uint32_t slot = first + k;
        const SlotRec& sr = F.srec[slot];
        if (sr.reg) continue;  // a regression node: k_split_finalize_reg
        const uint32_t id = sr.id;
        const NodeDev nd = F.nodes[id];
        const TreeDev tr = F.trees[nd.tree];
        JobDev& J = F.jobs[tr.job];
        uint32_t cnode[KMAX];
        uint64_t S = 0;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            cnode[c] = sr.cnode[c];
            S += (uint64_t)cnode[c] * cnode[c];
        }
        const uint32_t N = sr.n;
        // rank the items' candidates: each lane keeps the best of its items
        const int ni = ((int)sr.mtry + F.fw - 1) / F.fw;
        Cand c;
        c.nl = 0;
        c.q = 0x7FFFFFFF;
        c.b = 0x7FFFFFFF;
        c.f = 0;
        c.nr = 0;
        c.pad = 0;
        c.sl = c.sr = 0;
        int ci = -1;
        for (int t = lane; t < ni; t += 64) {
            const Cand d = F.cand[(size_t)slot * F.npi + t];
            if (d.nl != 0 && (c.nl == 0 || cand_wins_total(d, c))) {
                c = d;
                ci = t;
            }
        }
        // FP32 ranking with the exact recheck of the finalists (as in the
        // histogram scans), or exact throughout
        const Cand best = F.split_rank ? wave_best_total_fp32(c, c.nl != 0 ? cand_q32(c) : -1.0f)
                                       : wave_best_total_exact(c);
        const unsigned long long hit =
            __ballot(best.nl != 0 && c.nl != 0 && c.q == best.q && c.b == best.b);
        const int bt = hit ? __shfl(ci, (int)__ffsll(hit) - 1) : -1;
        const uint32_t child = F.next_base + 2u * (F.n_small_cur + slot);
        const bool split = bt >= 0 && cand_positive(best, S, N);
        if (!split) {  // stays the leaf it was created as
            if (lane == 0) {
                mark_unused_pair(F, child);
                F.kinds[F.n_small_cur + slot] = 0;
            }
            continue;
        }
        const uint32_t* clt = F.cand_cl + ((size_t)slot * F.npi + bt) * F.kmax;
        uint32_t cl[16], cr[16];
        int nzl = 0, nzr = 0;
#pragma unroll
        for (int c2 = 0; c2 < 16; ++c2) {
            cl[c2] = c2 < KMAX ? clt[c2] : 0u;
            cr[c2] = (c2 < KMAX ? cnode[c2] : 0u) - cl[c2];
            nzl += cl[c2] != 0;
            nzr += cr[c2] != 0;
        }
        // Rows are partitioned only for a child that is searched next: below
        // the maximum depth with two or more classes (which implies two or
        // more distinct rows); other children are final leaves.
        const bool part = (int)nd.depth + 1 < J.D && (nzl >= 2 || nzr >= 2);
        const uint32_t runl = partition_rows<true>(F, J, tr, nd, sr, best, part ? sr.len : 0u);
        if (lane == 0) {
            int kinds[2];
            split_node(F, J, tr, id, nd, best, runl, cl, cr, cand_gain_fix(best, S, N), child,
                       kinds);
            F.kinds[F.n_small_cur + slot] = (uint8_t)(kinds[0] | kinds[1] << 2);
        }
    }
}

// ---------------------------------------------------------------------------
// Next-level lists, without atomics: searched node i of level d (the small
// nodes first, then the large-node slots) owns the child pair at
// next_base + 2i, and its children's kinds were recorded in kinds[i].  Two
// passes over chunks of kListChunk nodes: count the wave-path and the
// histogram-path children per chunk, then let every chunk add up the counts
// of the chunks before it and write its children to the lists in node order.
constexpr uint32_t kListChunk = 4096;  // 1024 threads x 4 nodes

__device__ __forceinline__ uint32_t level_searched(const ForestDev& F, int level) {
    return level_small(F, level) + level_slots(F, level);
}

// Packed (wave path | histogram path << 16) children of 4 nodes from i0.
__device__ __forceinline__ uint32_t kinds4(const ForestDev& F, uint32_t i0, uint32_t n,
                                           uint32_t* kd) {
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        kd[u] = i0 + u < n ? F.kinds[i0 + u] : 0u;
        const uint32_t a = kd[u] & 3u, b = kd[u] >> 2;
        c += (a == (uint32_t)kSmall) + (b == (uint32_t)kSmall) +
             (((a == (uint32_t)kLarge) + (b == (uint32_t)kLarge)) << 16);
    }
    return c;
}

// Sum over the workgroup of 1024 threads (16 waves); all threads get it.
__device__ __forceinline__ unsigned long long block_sum64(unsigned long long v,
                                                          unsigned long long* s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
    if (lane == 0) s_w[wave] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < 16; ++w) t += s_w[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(1024) void k_lists_count(ForestDev F, int level) {
    __shared__ unsigned long long s_w[16];
    const uint32_t n = level_searched(F, level);
    const uint32_t nchunks = (n + kListChunk - 1) / kListChunk;
    for (uint32_t b = blockIdx.x; b < nchunks; b += gridDim.x) {
        uint32_t kd[4];
        const uint32_t c = kinds4(F, b * kListChunk + threadIdx.x * 4u, n, kd);
        const unsigned long long t =
            block_sum64((unsigned long long)(c & 0xFFFFu) | ((unsigned long long)(c >> 16) << 32),
                        s_w);
        if (threadIdx.x == 0) F.chunk_sums[b] = t;
    }
}

__global__ __launch_bounds__(1024) void k_lists_write(ForestDev F0, int level) {
    __shared__ unsigned long long s_w[16];
    __shared__ uint32_t s_wc[16];
    const ForestDev F = level_view(F0, level);  // appends describe level + 1
    const uint32_t n = level_searched(F0, level);
    const uint32_t nchunks = (n + kListChunk - 1) / kListChunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t b = blockIdx.x; b < nchunks; b += gridDim.x) {
        // children of the chunks before this one
        unsigned long long pre = 0;
        for (uint32_t e = threadIdx.x; e < b; e += 1024) pre += F.chunk_sums[e];
        pre = block_sum64(pre, s_w);
        uint32_t kd[4];
        const uint32_t i0 = b * kListChunk + threadIdx.x * 4u;
        const uint32_t c = kinds4(F0, i0, n, kd);
        const uint32_t incl = wave_incl_sum(c);  // per field < 2^16: 4096 nodes, 2 children
        if (lane == 63) s_wc[wave] = incl;
        __syncthreads();
        uint32_t off = incl - c;
        for (int w = 0; w < wave; ++w) off += s_wc[w];
        uint32_t ps = (uint32_t)pre + (off & 0xFFFFu), pl = (uint32_t)(pre >> 32) + (off >> 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                const uint32_t k = (kd[u] >> (2 * ch)) & 3u;
                const uint32_t node = F.next_base + 2u * (i0 + u) + ch;
                if (k == (uint32_t)kSmall) {
                    if (ps < F.small_cap)
                        F.small_out[ps] = node;
                    else
                        atomicOr(&F.ctr->overflow, 1u);
                    ++ps;
                } else if (k == (uint32_t)kLarge) {
                    if (pl < F.slot_cap)
                        F.slot_node_out[pl] = node;
                    else
                        atomicOr(&F.ctr->overflow, 2u);
                    ++pl;
                }
            }
        }
        if (b == nchunks - 1 && threadIdx.x == 1023) {  // the last node's totals
            F.ctr->n_small = min(ps, F.small_cap);
            F.ctr->n_slots = min(pl, F.slot_cap);
        }
        __syncthreads();  // shared sums are reused by the next chunk
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
void launch_boot_compact(const ForestDev& F, uint32_t n_trees, hipStream_t st) {
    hipLaunchKernelGGL(k_boot_compact, dim3(n_trees), dim3(1024), 0, st, F);
}

// count == 0xFFFFFFFF: the whole level, sized on the device (grid-stride).
void launch_split_small(const ForestDev& F, int level, uint32_t first, uint32_t count,
                        uint32_t grid_wg, hipStream_t st) {
    if (!count) return;
    const dim3 grid(grid_wg);
    const size_t lds = (size_t)4 * kDrawTab * sizeof(uint16_t);  // four waves' round tables
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_split_small<2>, grid, dim3(256), lds, st, F, level, first, count); break;
        case 3: hipLaunchKernelGGL(k_split_small<3>, grid, dim3(256), lds, st, F, level, first, count); break;
        case 4: hipLaunchKernelGGL(k_split_small<4>, grid, dim3(256), lds, st, F, level, first, count); break;
        case 8: hipLaunchKernelGGL(k_split_small<8>, grid, dim3(256), lds, st, F, level, first, count); break;
        default: hipLaunchKernelGGL(k_split_small<16>, grid, dim3(256), lds, st, F, level, first, count); break;
    }
}

void launch_lists(const ForestDev& F, int level, uint32_t grid_wg, hipStream_t st) {
    hipLaunchKernelGGL(k_lists_count, dim3(grid_wg), dim3(1024), 0, st, F, level);
    hipLaunchKernelGGL(k_lists_write, dim3(grid_wg), dim3(1024), 0, st, F, level);
}

void launch_draws(const ForestDev& F, int level, uint32_t grid_wg, hipStream_t st) {
    const size_t lds = (size_t)(256u / F.draw_seg) * F.draw_tab * sizeof(uint16_t);
    hipLaunchKernelGGL(k_draws, dim3(grid_wg), dim3(256), lds, st, F, level);
}

template <int KMAX, int FW>
static void launch_tile_rb(const ForestDev& F, int level, uint32_t first, uint32_t count,
                           dim3 grid, size_t lds, int rb, hipStream_t st) {
    switch (rb) {
        case 4: hipLaunchKernelGGL((k_hist_tile<KMAX, FW, 4>), grid, dim3(256), lds, st, F, level, first, count); break;
        case 16: hipLaunchKernelGGL((k_hist_tile<KMAX, FW, 16>), grid, dim3(256), lds, st, F, level, first, count); break;
        default: hipLaunchKernelGGL((k_hist_tile<KMAX, FW, 8>), grid, dim3(256), lds, st, F, level, first, count); break;
    }
}

// rb: rows per lane per batch (4, 8 or 16); F.fw draws per item with
// F.fw * F.kmax <= 8 (the engine validates both).  Regression items run in
// k_hist_reg, classification items in k_hist_tile: two launches over the
// same items for a plan holding both kinds of job.
void launch_hist_tile(const ForestDev& F, int level, uint32_t first, uint32_t count,
                      uint32_t grid_wg, int rb, hipStream_t st) {
    if (!count) return;
    // four waves of fw * KMAX * 256 words
    const size_t lds = (size_t)4 * F.fw * F.kmax * 256 * sizeof(uint32_t);
    const dim3 grid(grid_wg);
    if (F.has_reg) {
        switch (rb) {
            case 4: hipLaunchKernelGGL((k_hist_reg<4>), grid, dim3(256), lds, st, F, level, first, count); break;
            case 16: hipLaunchKernelGGL((k_hist_reg<16>), grid, dim3(256), lds, st, F, level, first, count); break;
            default: hipLaunchKernelGGL((k_hist_reg<8>), grid, dim3(256), lds, st, F, level, first, count); break;
        }
    }
    if (!F.has_cls) return;
    if (F.split_k) {  // the items of jobs of at most 4 classes (FW = 1 for these plans)
        const size_t lds4 = (size_t)4 * F.fw * 4 * 256 * sizeof(uint32_t);
        if (F.fw == 1) launch_tile_rb<4, 1>(F, level, first, count, grid, lds4, rb, st);
        else launch_tile_rb<4, 2>(F, level, first, count, grid, lds4, rb, st);
    }
    switch (F.kmax * 8 + F.fw) {
        case 2 * 8 + 4: launch_tile_rb<2, 4>(F, level, first, count, grid, lds, rb, st); break;
        case 2 * 8 + 2: launch_tile_rb<2, 2>(F, level, first, count, grid, lds, rb, st); break;
        case 2 * 8 + 1: launch_tile_rb<2, 1>(F, level, first, count, grid, lds, rb, st); break;
        case 3 * 8 + 2: launch_tile_rb<3, 2>(F, level, first, count, grid, lds, rb, st); break;
        case 3 * 8 + 1: launch_tile_rb<3, 1>(F, level, first, count, grid, lds, rb, st); break;
        case 4 * 8 + 2: launch_tile_rb<4, 2>(F, level, first, count, grid, lds, rb, st); break;
        case 4 * 8 + 1: launch_tile_rb<4, 1>(F, level, first, count, grid, lds, rb, st); break;
        case 8 * 8 + 1: launch_tile_rb<8, 1>(F, level, first, count, grid, lds, rb, st); break;
        default: launch_tile_rb<16, 1>(F, level, first, count, grid, lds, rb, st); break;
    }
}

size_t hist_col_lds(int kmax, int waves, uint32_t gq_max) {
    return (size_t)waves * kmax * 256 * sizeof(uint32_t) + (size_t)gq_max * 16;
}

// F.col_count == 2: the places are counted by k_col_count (n_gcol <= kColCountLds)
void launch_col_sort(const ForestDev& F, int level, uint32_t grid_wg, hipStream_t st) {
    if (F.col_count == 2)
        hipLaunchKernelGGL(k_col_count, dim3(kColCountGrid), dim3(256),
                           (size_t)F.n_gcol * sizeof(uint32_t), st, F, level);
    hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(256), 0, st, F, level);
    hipLaunchKernelGGL(k_col_scatter, dim3(grid_wg), dim3(256), 0, st, F, level);
}

// Allows the column path's dynamic LDS (above the default per-launch limit)
// for the instantiation of kmax classes.
hipError_t prepare_hist_col(int kmax, size_t lds) {
    const void* fn;
    switch (kmax) {
        case 2: fn = reinterpret_cast<const void*>(&k_hist_col<2>); break;
        case 3: fn = reinterpret_cast<const void*>(&k_hist_col<3>); break;
        case 4: fn = reinterpret_cast<const void*>(&k_hist_col<4>); break;
        case 8: fn = reinterpret_cast<const void*>(&k_hist_col<8>); break;
        default: fn = reinterpret_cast<const void*>(&k_hist_col<16>); break;
    }
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

void launch_hist_col(const ForestDev& F, int level, uint32_t grid_wg, int waves, uint32_t gq_max,
                     hipStream_t st) {
    const size_t lds = hist_col_lds(F.kmax, waves, gq_max);
    const dim3 grid(grid_wg), block(64 * waves);
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_hist_col<2>, grid, block, lds, st, F, level); break;
        case 3: hipLaunchKernelGGL(k_hist_col<3>, grid, block, lds, st, F, level); break;
        case 4: hipLaunchKernelGGL(k_hist_col<4>, grid, block, lds, st, F, level); break;
        case 8: hipLaunchKernelGGL(k_hist_col<8>, grid, block, lds, st, F, level); break;
        default: hipLaunchKernelGGL(k_hist_col<16>, grid, block, lds, st, F, level); break;
    }
}

void launch_split_finalize(const ForestDev& F, int level, uint32_t first, uint32_t count,
                           uint32_t grid_wg, hipStream_t st) {
    if (!count) return;
    const dim3 grid(grid_wg);
    if (F.has_reg)
        hipLaunchKernelGGL(k_split_finalize_reg, grid, dim3(256), 0, st, F, level, first, count);
    if (!F.has_cls) return;
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_split_finalize<2>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 3: hipLaunchKernelGGL(k_split_finalize<3>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 4: hipLaunchKernelGGL(k_split_finalize<4>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 8: hipLaunchKernelGGL(k_split_finalize<8>, grid, dim3(256), 0, st, F, level, first, count); break;
        default: hipLaunchKernelGGL(k_split_finalize<16>, grid, dim3(256), 0, st, F, level, first, count); break;
    }
}

}  // namespace boruta
