// k_forest.hip -- random-forest growth kernels (gfx950).
//
// Trees grow level by level, all trees of all live jobs in the same launch:
//   * k_boot_compact  per tree: in-bag row records and OOB rows from the
//                     bootstrap multiplicities, root node;
//   * k_split_small   one wavefront per node with <= 64 distinct rows: the
//                     rows sit in lanes and every threshold's left class
//                     counts come from an in-register all-pairs sum;
//   * k_hist_tile     one workgroup per (node, tile of drawn features):
//                     LDS class-count histogram [feature][class][bin] built
//                     with LDS atomics from batched global gathers, then a
//                     wave prefix scan over the bins per feature; writes the
//                     tile's best candidate;
//   * k_split_finalize one workgroup per large node: best over the node's
//                     tiles, then a stable partition of its rows.
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
// multiplicities are cleared behind the read.
__global__ __launch_bounds__(1024) void k_boot_compact(ForestDev F0) {
    __shared__ uint32_t s_win[16], s_wout[16];
    __shared__ uint32_t s_cls[16];
    __shared__ uint32_t s_base_in, s_base_out;
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
    uint32_t* w = J.wbuf + (size_t)tr.tau * n;
    uint64_t* recs = J.rec[0] + (size_t)tr.tau * n;
    uint32_t* oob = J.oob + (size_t)tr.tau * n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 16) s_cls[tid] = 0;
    if (tid == 0) {
        s_base_in = 0;
        s_base_out = 0;
    }
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + tid;
        const uint32_t wi = i < n ? w[i] : 0u;
        if (i < n) w[i] = 0;  // multiplicities start from zero next iteration
        const bool inb = i < n && wi > 0, isoob = i < n && wi == 0;
        const uint64_t mi = __ballot(inb), mo = __ballot(isoob);
        if (lane == 0) {
            s_win[wave] = __popcll(mi);
            s_wout[wave] = __popcll(mo);
        }
        __syncthreads();
        uint32_t pin = s_base_in, pout = s_base_out;
        for (int v = 0; v < wave; ++v) {
            pin += s_win[v];
            pout += s_wout[v];
        }
        if (inb) {
            const uint32_t yi = J.y[i];
            if (wi > 0xFFFFu) atomicOr(&F.ctr->overflow, 8u);
            recs[pin + __popcll(mi & below)] = rec_pack(i, wi, yi);
            atomicAdd(&s_cls[yi], wi);
        }
        if (isoob) oob[pout + __popcll(mo & below)] = i;
        __syncthreads();
        if (tid == 0) {
            uint32_t ti = 0, to = 0;
            for (int v = 0; v < 16; ++v) {
                ti += s_win[v];
                to += s_wout[v];
            }
            s_base_in += ti;
            s_base_out += to;
        }
        __syncthreads();
    }
    if (tid == 0) {
        J.tstat[tr.tau * 4 + 0] = (int32_t)s_base_in;
        J.tstat[tr.tau * 4 + 1] = (int32_t)s_base_out;
        J.tstat[tr.tau * 4 + 2] = 0;
        uint32_t counts[16], tot = 0;
        for (int k = 0; k < 16; ++k) {
            counts[k] = s_cls[k];
            tot += s_cls[k];
        }
        const int kind = write_node(F, J, g, g, 1u, 0u, s_base_in, tot, 0u, counts);
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
    uint32_t ntiles;
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

template <int KMAX>
__device__ void small_node(const ForestDev& F, uint32_t idx, SmallOut& out) {
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
    const size_t tbase = (size_t)tr.tau * J.n + nd.seg;
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
    for (int q0 = 0; q0 < J.mtry; q0 += 64) {
        const int nq = min(64, J.mtry - q0);
        const int myf = lane < nq ? (int)perm_apply(P, (uint32_t)(q0 + lane)) : 0;
        const unsigned long long mycol =
            lane < nq ? (unsigned long long)ldg(J.colptr + myf) : 0ull;
        const int passes = (nq + G - 1) / G;
        // The bin load is unconditional (lanes without a row read row 0, lanes
        // past the drawn features read the first one) so that blocks of loads
        // issue back to back; eval() masks what does not count.
        auto gather = [&](int pass) {
            const int qq = pass * G + seg;
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
        // bins of eight passes are in flight while the previous eight are scored
        int bq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bq[u] = gather(u);
        for (int pb = 0; pb < passes; pb += 8) {
            int bn[8];
            if (pb + 8 < passes) {
#pragma unroll
                for (int u = 0; u < 8; ++u) bn[u] = gather(pb + 8 + u);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (pb + u < passes) eval(pb + u, bq[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u) bq[u] = bn[u];
        }
    }
    const Cand best = fp32 ? wave_best_total_fp32(lb, lb.nl != 0 ? lq : -1.0f)
                           : wave_best_total_exact(lb);
    out.ntiles = (uint32_t)J.ntiles;
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

// Four nodes per workgroup (one per wave); the children's list positions are
// reserved with one atomic per list for the whole workgroup.
// The small nodes of tree level `level`: all of them (count from the level's
// counters, grid-stride) or, with an explicit count, list entries
// [first, first + count).
template <int KMAX>
__global__ __launch_bounds__(256) void k_split_small(ForestDev F0, int level, uint32_t first,
                                                     uint32_t count) {
    __shared__ uint32_t s_ns[4], s_nl[4], s_ni[4], s_base[3];
    __shared__ unsigned long long s_alg[4];
    const ForestDev F = level_view(F0, level);
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_small(F0, level);
    }
    const int lane = threadIdx.x & 63, wave = (int)uniform(threadIdx.x >> 6);
    for (uint32_t base = blockIdx.x * 4u; base < count; base += gridDim.x * 4u) {
    const uint32_t li = base + wave;
    SmallOut o;
    o.kinds[0] = o.kinds[1] = kLeaf;
    o.child = 0;
    o.ntiles = 0;
    o.alg = 0;
    if (li < count) small_node<KMAX>(F, first + li, o);
    if (lane == 0) {
        s_ns[wave] = (o.kinds[0] == kSmall) + (o.kinds[1] == kSmall);
        s_nl[wave] = (o.kinds[0] == kLarge) + (o.kinds[1] == kLarge);
        s_ni[wave] = s_nl[wave] * o.ntiles;
        s_alg[wave] = o.alg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t ts = s_ns[0] + s_ns[1] + s_ns[2] + s_ns[3];
        const uint32_t tl = s_nl[0] + s_nl[1] + s_nl[2] + s_nl[3];
        const uint32_t ti = s_ni[0] + s_ni[1] + s_ni[2] + s_ni[3];
        s_base[0] = ts ? atomicAdd(&F.ctr->n_small, ts) : 0u;
        s_base[1] = tl ? atomicAdd(&F.ctr->n_slots, tl) : 0u;
        s_base[2] = ti ? atomicAdd(&F.ctr->n_items, ti) : 0u;
        if (F.alg_bytes)
            atomicAdd((unsigned long long*)&F.alg_bytes[64 + (blockIdx.x & 63)],
                      s_alg[0] + s_alg[1] + s_alg[2] + s_alg[3]);
    }
    __syncthreads();
    if (lane == 0 && li < count) {
        uint32_t ps = s_base[0], pl = s_base[1], pi = s_base[2];
        for (int v = 0; v < wave; ++v) {
            ps += s_ns[v];
            pl += s_nl[v];
            pi += s_ni[v];
        }
        for (int c = 0; c < 2; ++c) {
            if (o.kinds[c] == kSmall) put_small(F, ps++, o.child + c);
            if (o.kinds[c] == kLarge) {
                put_large(F, pl++, pi, o.ntiles, o.child + c);
                pi += o.ntiles;
            }
        }
    }
    __syncthreads();  // the shared counts are reused by the next batch
    }
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
        const Cand c = make(b, cl);
        if (c.nl == 0 || c.nl == N) continue;
        const float qc = cand_q32(c);
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
                const Cand c = make(b, cl);
                if (c.nl == 0 || c.nl == N) continue;
                if (cand_q32(c) < floor32) continue;
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

// Large nodes, phase 1: one workgroup per (node, feature tile).  FT columns
// per tile keep the LDS histogram at FT * KMAX * 256 * 4 = 32 KB; the class-
// major rows spread a wave's atomics over the banks by bin.
template <int KMAX>
__global__ __launch_bounds__(256) void k_hist_tile(ForestDev F, int level, uint32_t first,
                                                   uint32_t count) {
    constexpr int FT = 32 / KMAX;
    extern __shared__ uint4 hist_raw[];  // [FT][KMAX][256] class counts (16-byte aligned)
    uint32_t* hist = reinterpret_cast<uint32_t*>(hist_raw);
    __shared__ const uint8_t* s_col[FT];
    __shared__ int s_feat[FT];
    __shared__ Cand s_fbest[FT];
    __shared__ int s_bi;
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_items(F, level);
    }
    for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
    const uint32_t item = first + k;
    const Item it = F.items_in[item];
    const NodeDev nd = F.nodes[it.node];
    const TreeDev tr = F.trees[nd.tree];
    const JobDev& J = F.jobs[tr.job];
    const int B = J.B, tid = threadIdx.x, lane = tid & 63, wave = (int)uniform(tid >> 6);
    const int q0 = (int)it.tile * FT;
    const int nf = min(FT, J.mtry - q0);
    if (tid < nf) {
        const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kMtry, (uint32_t)J.t,
                                      (uint32_t)tr.tau, nd.heap, 0u, (uint64_t)J.p_w);
        const int f = (int)perm_apply(P, (uint32_t)(q0 + tid));
        s_feat[tid] = f;
        s_col[tid] = ldg(J.colptr + f);
    }
    for (int i = tid; i < FT * KMAX * 64; i += 256)
        reinterpret_cast<uint4*>(hist)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const uint8_t* col[FT];
#pragma unroll
    for (int q = 0; q < FT; ++q) col[q] = q < nf ? s_col[q] : s_col[0];
    const uint64_t* recs = J.rec[F.parity] + (size_t)tr.tau * J.n + nd.seg;
    const uint32_t len = nd.len;
    // two rows per thread per pass: up to 2 * FT bin gathers in flight
    for (uint32_t i0 = tid; i0 < len; i0 += 512) {
        const uint32_t i1 = i0 + 256;
        const bool v1 = i1 < len;
        const uint64_t r0 = ldg(recs + i0);
        const uint64_t r1 = v1 ? ldg(recs + i1) : r0;
        const uint32_t row0 = rec_row(r0), row1 = rec_row(r1);
        uint32_t b0[FT], b1[FT];
#pragma unroll
        for (int q = 0; q < FT; ++q) {
            b0[q] = ldg(col[q] + row0);
            b1[q] = ldg(col[q] + row1);
        }
        const uint32_t w0 = rec_w(r0), y0 = rec_y(r0);
        const uint32_t w1 = v1 ? rec_w(r1) : 0u, y1 = rec_y(r1);
#pragma unroll
        for (int q = 0; q < FT; ++q) {
            if (q < nf) {
                atomicAdd(&hist[(q * KMAX + y0) * 256 + b0[q]], w0);
                if (v1) atomicAdd(&hist[(q * KMAX + y1) * 256 + b1[q]], w1);
            }
        }
    }
    __syncthreads();
    uint32_t cnode[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) cnode[k] = k < J.K ? F.cls[(size_t)it.node * F.kmax + k] : 0u;
    const uint32_t N = nd.n;
    for (int q = wave; q < nf; q += 4) {
        const Cand fb =
            feature_best<KMAX>(hist + q * KMAX * 256, B, q0 + q, s_feat[q], cnode, N, F.split_rank);
        if (lane == 0) s_fbest[q] = fb;
    }
    __syncthreads();
    if (tid == 0) {
        int bi = 0;  // earliest draw among equal scores: strict comparison
        for (int q = 1; q < nf; ++q)
            if (s_fbest[q].nl != 0 &&
                (s_fbest[bi].nl == 0 || cand_better(s_fbest[q], s_fbest[bi])))
                bi = q;
        s_bi = bi;
        F.cand[(size_t)it.slot * F.max_tiles + it.tile] = s_fbest[bi];
        if (F.alg_bytes)
            atomicAdd((unsigned long long*)&F.alg_bytes[item & 63],
                      (unsigned long long)len * (unsigned long long)(nf + (it.tile == 0 ? 6 : 0)));
    }
    __syncthreads();
    if (wave == 0) {
        // left class counts of the tile's candidate, for the partition step
        const int bi = s_bi;
        const int bt = s_fbest[bi].nl != 0 ? s_fbest[bi].b : -1;
        uint32_t* out = F.cand_cl + ((size_t)it.slot * F.max_tiles + it.tile) * F.kmax;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint4 v = *reinterpret_cast<const uint4*>(hist + (bi * KMAX + k) * 256 + lane * 4);
            const int bl = lane * 4;
            const uint32_t a = (bl <= bt ? v.x : 0u) + (bl + 1 <= bt ? v.y : 0u) +
                               (bl + 2 <= bt ? v.z : 0u) + (bl + 3 <= bt ? v.w : 0u);
            const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(a), 63);
            if (lane == k) out[k] = tot;
        }
    }
    __syncthreads();  // LDS is reused by the next item
    }
}

// Large nodes, phase 2: one workgroup per node.  The node's split is the
// best tile candidate (tiles hold increasing draw positions, so keeping the
// first of equal candidates keeps the earliest draw); a strictly positive
// decrease splits the node and its rows are partitioned stably, left first.
template <int KMAX>
__global__ __launch_bounds__(256) void k_split_finalize(ForestDev F0, int level, uint32_t first,
                                                        uint32_t count) {
    __shared__ Cand s_best;
    __shared__ Cand s_tiles[64];
    __shared__ int s_split, s_bt, s_part;
    __shared__ uint32_t s_wcnt[4];
    __shared__ uint32_t s_runl, s_runr;
    const ForestDev F = level_view(F0, level);
    if (count == 0xFFFFFFFFu) {
        first = 0;
        count = level_slots(F0, level);
    }
    for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
    const uint32_t slot = first + k;
    const uint32_t id = F.slot_node_in[slot];
    const NodeDev nd = F.nodes[id];
    const TreeDev tr = F.trees[nd.tree];
    JobDev& J = F.jobs[tr.job];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t cnode[KMAX];
    uint64_t S = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        cnode[k] = k < J.K ? F.cls[(size_t)id * F.kmax + k] : 0u;
        S += (uint64_t)cnode[k] * cnode[k];
    }
    const uint32_t N = nd.n;
    // the tiles' candidates are loaded in parallel, then ranked in draw order
    // (a strictly better score replaces: the earliest tile keeps a tie)
    int bt = -1;
    for (int t0 = 0; t0 < J.ntiles; t0 += 64) {
        const int nt = min(64, J.ntiles - t0);
        if (tid < nt) s_tiles[tid] = F.cand[(size_t)slot * F.max_tiles + t0 + tid];
        __syncthreads();
        if (tid == 0)
            for (int t = 0; t < nt; ++t)
                if (s_tiles[t].nl != 0 &&
                    (bt < 0 || cand_better(s_tiles[t], s_best)) ) {
                    s_best = s_tiles[t];
                    bt = t0 + t;
                }
        __syncthreads();
    }
    if (tid == 0) {
        s_split = bt >= 0 && cand_positive(s_best, S, N);
        s_bt = bt;
        s_runl = 0;
        s_runr = 0;
        // Rows are partitioned only for a child that is searched next: below
        // the maximum depth with two or more classes (which implies two or
        // more distinct rows); other children are final leaves.
        s_part = 0;
        if (s_split && (int)nd.depth + 1 < J.D) {
            const uint32_t* clt = F.cand_cl + ((size_t)slot * F.max_tiles + bt) * F.kmax;
            int nzl = 0, nzr = 0;
            for (int k = 0; k < KMAX; ++k) {
                const uint32_t l = clt[k];
                nzl += l != 0;
                nzr += cnode[k] != l;
            }
            s_part = nzl >= 2 || nzr >= 2;
        }
    }
    __syncthreads();
    const uint32_t child = F.next_base + 2u * (F.n_small_cur + slot);
    if (!s_split) {  // stays the leaf it was created as
        if (tid == 0) mark_unused_pair(F, child);
        __syncthreads();
        continue;
    }
    const Cand best = s_best;
    const uint8_t* col = ldg(J.colptr + best.f);
    const uint64_t* recs = J.rec[F.parity] + (size_t)tr.tau * J.n + nd.seg;
    uint64_t* rout = J.rec[F.parity ^ 1] + (size_t)tr.tau * J.n + nd.seg;
    // One pass over blocks of 256 x kR rows (thread t owns rows
    // [blk + t kR, blk + t kR + kR)): left rows are written from the front in
    // row order, right rows from the back in reverse row order.  No result
    // depends on the order of a node's rows; each child segment stays
    // monotone in row index, which keeps the next level's gathers local.
    constexpr int kR = 8;
    const uint32_t len = s_part ? nd.len : 0u;  // no partition: both children are leaves
    for (uint32_t blk = 0; blk < len; blk += 256 * kR) {
        const uint32_t i0 = blk + (uint32_t)tid * kR;
        uint64_t r[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) r[u] = i0 + u < len ? ldg(recs + i0 + u) : 0ull;
        int bb[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) bb[u] = i0 + u < len ? (int)ldg(col + rec_row(r[u])) : 0x7FFF;
        uint32_t nlm = 0, nrm = 0;
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            nlm += bb[u] <= best.b;
            nrm += i0 + u < len && bb[u] > best.b;
        }
        // exclusive prefix of (left, right) counts over the block's threads,
        // both packed in one word (a block holds at most 2048 rows)
        const uint32_t mine = nlm | (nrm << 16);
        const uint32_t incl = wave_incl_sum(mine);
        if (lane == 63) s_wcnt[wave] = incl;
        __syncthreads();
        uint32_t pre = incl - mine;
        for (int v = 0; v < wave; ++v) pre += s_wcnt[v];
        const uint32_t blk_tot = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
        uint32_t lrow = s_runl + (pre & 0xFFFFu), rrow = s_runr + (pre >> 16);
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            if (i0 + u >= len) break;
            if (bb[u] <= best.b)
                rout[lrow++] = r[u];
            else
                rout[len - 1 - rrow++] = r[u];
        }
        __syncthreads();
        if (tid == 0) {
            s_runl += blk_tot & 0xFFFFu;
            s_runr += blk_tot >> 16;
        }
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t* clt = F.cand_cl + ((size_t)slot * F.max_tiles + s_bt) * F.kmax;
        uint32_t cl[16], cr[16];
        for (int k = 0; k < 16; ++k) {
            cl[k] = k < KMAX ? clt[k] : 0u;
            cr[k] = (k < KMAX ? cnode[k] : 0u) - cl[k];
        }
        int kinds[2];
        split_node(F, J, tr, id, nd, best, s_runl, cl, cr, cand_gain_fix(best, S, N), child,
                   kinds);
        enqueue_nodes(F, J, child, kinds, 2);
    }
    __syncthreads();  // shared state is reused by the next slot
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
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_split_small<2>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 4: hipLaunchKernelGGL(k_split_small<4>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 8: hipLaunchKernelGGL(k_split_small<8>, grid, dim3(256), 0, st, F, level, first, count); break;
        default: hipLaunchKernelGGL(k_split_small<16>, grid, dim3(256), 0, st, F, level, first, count); break;
    }
}

void launch_hist_tile(const ForestDev& F, int level, uint32_t first, uint32_t count,
                      uint32_t grid_wg, int B, hipStream_t st) {
    if (!count) return;
    const size_t lds = (size_t)32 * 256 * sizeof(uint32_t);  // FT * KMAX * 256 words, FT * KMAX = 32
    const dim3 grid(grid_wg);
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_hist_tile<2>, grid, dim3(256), lds, st, F, level, first, count); break;
        case 4: hipLaunchKernelGGL(k_hist_tile<4>, grid, dim3(256), lds, st, F, level, first, count); break;
        case 8: hipLaunchKernelGGL(k_hist_tile<8>, grid, dim3(256), lds, st, F, level, first, count); break;
        default: hipLaunchKernelGGL(k_hist_tile<16>, grid, dim3(256), lds, st, F, level, first, count); break;
    }
}

void launch_split_finalize(const ForestDev& F, int level, uint32_t first, uint32_t count,
                           uint32_t grid_wg, hipStream_t st) {
    if (!count) return;
    const dim3 grid(grid_wg);
    switch (F.kmax) {
        case 2: hipLaunchKernelGGL(k_split_finalize<2>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 4: hipLaunchKernelGGL(k_split_finalize<4>, grid, dim3(256), 0, st, F, level, first, count); break;
        case 8: hipLaunchKernelGGL(k_split_finalize<8>, grid, dim3(256), 0, st, F, level, first, count); break;
        default: hipLaunchKernelGGL(k_split_finalize<16>, grid, dim3(256), 0, st, F, level, first, count); break;
    }
}

}  // namespace boruta
