// k_prep.hip -- once-per-run and once-per-iteration preparation kernels:
// input validation, quantile binning (per-column bitonic sort + cut table),
// exact binomial decision thresholds, the active/widened column map,
// shadow columns and bootstrap draws.
#include <algorithm>

#include "dev_common.hpp"

namespace boruta {

// ---------------------------------------------------------------------------
// Validation: non-finite X -> flag bit 1, label outside [0, K) -> bit 2.
__global__ void k_validate(const float* X, size_t nx, const int32_t* y, size_t n, int K,
                           uint32_t* flags) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += stride)
        if (!isfinite(X[i])) bad |= 1u;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (y[i] < 0 || y[i] >= K) bad |= 2u;
    if (bad) atomicOr(flags, bad);
}

// Regression inputs: X and the float targets must be finite (flag 1).
__global__ void k_validate_reg(const float* X, size_t nx, const float* y, size_t n,
                               uint32_t* flags) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += stride)
        if (!isfinite(X[i])) bad |= 1u;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (!isfinite(y[i])) bad |= 1u;
    if (bad) atomicOr(flags, bad);
}

// Regression targets (reading of the paper's float-target regressor): the
// exact minimum and maximum of y (one workgroup), from which the host picks
// the scale exponent e (every |y| < 2^e) and the fixed-point shifts.
__global__ __launch_bounds__(1024) void k_target_range(const float* y, size_t n, float* out) {
    __shared__ float s_lo[16], s_hi[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float lo = y[0], hi = y[0];
    for (size_t i = (size_t)tid; i < n; i += 1024) {
        lo = fminf(lo, y[i]);
        hi = fmaxf(hi, y[i]);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, m));
        hi = fmaxf(hi, __shfl_xor(hi, m));
    }
    if (lane == 0) {
        s_lo[wave] = lo;
        s_hi[wave] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int v = 1; v < 16; ++v) {
            lo = fminf(lo, s_lo[v]);
            hi = fmaxf(hi, s_hi[v]);
        }
        lo = fminf(lo, s_lo[0]);
        hi = fmaxf(hi, s_hi[0]);
        out[0] = lo;
        out[1] = hi;
    }
}

// y_fix = rint(y 2^sh): an exact power-of-two scaling in double, rounded to
// the nearest integer (ties to even); |y_fix| < 2^38 for sh = 38 - e.
__global__ void k_target_fix(const float* y, size_t n, int sh, int64_t* out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (int64_t)rint(ldexp((double)y[i], sh));
}

__global__ void k_labels_u8(const int32_t* y, size_t n, uint8_t* out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint8_t)y[i];
}

// ---------------------------------------------------------------------------
// Binning, reading of the binned forest (Sec. 2): per column, the order
// statistics of rank ceil(k n / B) - 1 (k = 1..B-1) are candidate cuts, the
// strictly increasing distinct ones form the cut table U, and x gets the bin
// #{u in U : u < x}.  The order statistics come from a bitonic sort of the
// column's order-preserving 32-bit keys (-0 folded into +0).

__device__ __forceinline__ uint32_t f2key(float v) {
    uint32_t u = __float_as_uint(v == 0.0f ? 0.0f : v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Row-major X[n][p] -> column keys[p][P] (P = power of two >= n, pad = max key).
__global__ void k_to_keys(const float* X, int64_t n, int64_t p, int64_t P, uint32_t* keys) {
    __shared__ float tile[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < n && c < p) ? X[r * p + c] : 0.0f;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < p && r < P) keys[c * P + r] = r < n ? f2key(tile[tx][k]) : 0xFFFFFFFFu;
    }
}

constexpr int kSortTile = 8192;

__device__ __forceinline__ void cmp_swap(uint32_t* a, uint32_t i, uint32_t l, bool asc) {
    const uint32_t x = a[i], y = a[l];
    if ((x > y) == asc) {
        a[i] = y;
        a[l] = x;
    }
}

// Sorts each tile of `tile` keys in LDS (all merge sizes k <= tile), or, with
// kmin > 0, runs only the steps j < tile of merge size kmin.
__global__ __launch_bounds__(1024) void k_sort_tile(uint32_t* keys, int64_t P, int tile,
                                                    int64_t kmin) {
    __shared__ uint32_t s[kSortTile];
    uint32_t* col = keys + (size_t)blockIdx.y * P + (size_t)blockIdx.x * tile;
    const uint32_t gbase = (uint32_t)blockIdx.x * tile;
    for (int i = threadIdx.x; i < tile; i += 1024) s[i] = col[i];
    __syncthreads();
    const int64_t k_lo = kmin > 0 ? kmin : 2, k_hi = kmin > 0 ? kmin : tile;
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (kmin > 0 ? tile : k) >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < tile / 2; t += 1024) {
                const uint32_t i = (uint32_t)((t / j) * 2 * j + (t % j));
                const uint32_t l = i + (uint32_t)j;
                cmp_swap(s, i, l, ((gbase + i) & k) == 0);
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < tile; i += 1024) col[i] = s[i];
}

// One global compare-exchange step (merge size k, distance j >= tile).
__global__ void k_sort_step(uint32_t* keys, int64_t P, int64_t k, int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P / 2) return;
    uint32_t* col = keys + (size_t)blockIdx.y * P;
    const int64_t i = (t / j) * 2 * j + (t % j);
    cmp_swap(col, (uint32_t)i, (uint32_t)(i + j), (i & k) == 0);
}

// Cut table from the sorted keys, then bins of one chunk of rows.
__global__ __launch_bounds__(256) void k_bin(const float* X, int64_t n, int64_t p, int64_t P,
                                             const uint32_t* keys, int B, uint8_t* bins,
                                             int64_t n_pad, int64_t chunk) {
    __shared__ float s_cand[256];
    __shared__ float s_cut[256];
    __shared__ int s_m;
    const int64_t c = blockIdx.y;
    const uint32_t* sk = keys + c * P;
    const int tid = threadIdx.x;
    if (tid >= 1 && tid < B) {
        const int64_t rank = ((int64_t)tid * n + B - 1) / B - 1;
        s_cand[tid] = key2f(sk[rank]);
    }
    __syncthreads();
    if (tid == 0) {
        int m = 0;
        for (int k = 1; k < B; ++k)
            if (m == 0 || s_cand[k] > s_cut[m - 1]) s_cut[m++] = s_cand[k];
        s_m = m;
    }
    __syncthreads();
    const int m = s_m;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = min(r0 + chunk, n_pad);
    uint8_t* out = bins + c * n_pad;
    for (int64_t r = r0 + tid; r < r1; r += 256) {
        if (r >= n) {
            out[r] = 0;
            continue;
        }
        float x = X[r * p + c];
        if (x == 0.0f) x = 0.0f;
        int lo = 0, hi = m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_cut[mid] < x)
                lo = mid + 1;
            else
                hi = mid;
        }
        out[r] = (uint8_t)lo;
    }
}

// ---------------------------------------------------------------------------
// Decision thresholds, reading of test() in Algorithm 1: two one-sided exact
// binomial tails (success probability 1/2), Bonferroni over all p features,
// strict "< alpha".  With alpha = m 2^e exactly, "p P[Bin(t,1/2) <= h] < alpha"
// is the integer test  p L(h) 2^max(0,-s) < m 2^max(0,s),  s = e + t,
// L(h) = sum_{k<=h} C(t,k).  h_rej(t) is the largest h passing it; by the
// symmetry C(t,k) = C(t,t-k) the upper tail gives h_conf(t) = t - h_rej(t).
// s <= -53 makes the right side smaller than 1: no decision at that t.
constexpr int kLimbs = 40;  // 1280 bits: p L(h) 2^52 < 2^(31+1000+52)

struct BigU {
    uint32_t v[kLimbs];
    int len;
};
__device__ void big_set(BigU& a, uint64_t x) {
    for (int i = 0; i < kLimbs; ++i) a.v[i] = 0;
    a.v[0] = (uint32_t)x;
    a.v[1] = (uint32_t)(x >> 32);
    a.len = a.v[1] ? 2 : 1;
}
__device__ void big_mul_small(BigU& a, uint32_t m) {
    uint64_t carry = 0;
    for (int i = 0; i < a.len; ++i) {
        const uint64_t pr = (uint64_t)a.v[i] * m + carry;
        a.v[i] = (uint32_t)pr;
        carry = pr >> 32;
    }
    if (carry && a.len < kLimbs) a.v[a.len++] = (uint32_t)carry;
    while (a.len > 1 && a.v[a.len - 1] == 0) --a.len;
}
__device__ void big_div_small(BigU& a, uint32_t d) {
    uint64_t rem = 0;
    for (int i = a.len - 1; i >= 0; --i) {
        const uint64_t cur = (rem << 32) | a.v[i];
        a.v[i] = (uint32_t)(cur / d);
        rem = cur % d;
    }
    while (a.len > 1 && a.v[a.len - 1] == 0) --a.len;
}
__device__ void big_add(BigU& a, const BigU& b) {
    const int len = a.len > b.len ? a.len : b.len;
    uint64_t carry = 0;
    for (int i = 0; i < len; ++i) {
        const uint64_t s = (uint64_t)a.v[i] + b.v[i] + carry;
        a.v[i] = (uint32_t)s;
        carry = s >> 32;
    }
    a.len = len;
    if (carry && a.len < kLimbs) a.v[a.len++] = (uint32_t)carry;
}
__device__ void big_shl(BigU& a, int s) {
    const int limbs = s >> 5, bits = s & 31;
    for (int i = kLimbs - 1; i >= 0; --i) {
        const int src = i - limbs;
        uint32_t hi = src >= 0 ? a.v[src] : 0u;
        uint32_t lo = src - 1 >= 0 ? a.v[src - 1] : 0u;
        a.v[i] = bits ? (hi << bits) | (lo >> (32 - bits)) : hi;
    }
    a.len = kLimbs;
    while (a.len > 1 && a.v[a.len - 1] == 0) --a.len;
}
__device__ int big_cmp(const BigU& a, const BigU& b) {
    const int len = a.len > b.len ? a.len : b.len;
    for (int i = len - 1; i >= 0; --i)
        if (a.v[i] != b.v[i]) return a.v[i] < b.v[i] ? -1 : 1;
    return 0;
}

__global__ void k_thresholds(int32_t max_iter, int64_t p, uint64_t alpha_m, int32_t alpha_e,
                             int32_t* h_conf, int32_t* h_rej) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (t > max_iter) return;
    const int s = alpha_e + t;
    int hr = -1;
    if (s > -53) {
        BigU rhs, C, L, lhs;
        big_set(rhs, alpha_m);
        if (s > 0) big_shl(rhs, s);
        const int lshift = s < 0 ? -s : 0;
        big_set(C, 1);
        big_set(L, 0);
        for (int h = 0; h <= t; ++h) {
            big_add(L, C);  // L = L(h)
            lhs = L;
            big_mul_small(lhs, (uint32_t)p);
            if (lshift) big_shl(lhs, lshift);
            if (big_cmp(lhs, rhs) >= 0) break;
            hr = h;
            big_mul_small(C, (uint32_t)(t - h));  // C(t, h+1) = C(t, h) (t-h) / (h+1)
            big_div_small(C, (uint32_t)(h + 1));
        }
    }
    h_rej[t] = hr;
    h_conf[t] = hr < 0 ? t + 1 : t - hr;
}

// ---------------------------------------------------------------------------
// Per iteration, one workgroup per job: t += 1, active columns (state >= 0,
// ascending), shadow count (doubled while < 5), widened column map, mtry;
// the importance accumulators are cleared.
__global__ __launch_bounds__(256) void k_active(JobDev* jobs) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_base;
    JobDev& J = jobs[blockIdx.x];
    if (!J.live) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_base = 0;
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int base = 0; base < J.p; base += 256) {
        const int j = base + tid;
        const bool act = j < J.p && J.state[j] >= 0;
        const uint64_t m = __ballot(act);
        if (lane == 0) s_w[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pos = s_base;
        for (int v = 0; v < wave; ++v) pos += s_w[v];
        if (act) J.act[pos + __popcll(m & below)] = j;
        __syncthreads();
        if (tid == 0) s_base += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
    const int p_cur = (int)s_base;
    int n_sha = p_cur;
    while (n_sha > 0 && n_sha < 5) n_sha *= 2;
    const int p_w = p_cur + n_sha;
    // both importances are summed into imp with integer atomics
    for (int c = tid; c < p_w; c += 256) J.imp[c] = 0;
    for (int c = tid; c < p_w; c += 256) {
        if (c < p_cur) {
            J.colptr[c] = J.orig + (size_t)J.act[c] * J.n_pad;
            J.col_src[c] = J.act[c];
        } else {
            J.colptr[c] = J.sha + (size_t)(c - p_cur) * J.n_pad;
            J.col_src[c] = J.act[(c - p_cur) % p_cur];
        }
    }
    if (tid == 0) {
        J.t += 1;
        J.p_cur = p_cur;
        J.n_sha = n_sha;
        J.p_w = p_w;
        int m;
        if (J.mtry_opt > 0) {
            m = J.mtry_opt < p_w ? J.mtry_opt : p_w;
        } else {
            m = (int)sqrt((double)p_w);
            while ((int64_t)m * m > p_w) --m;
            while ((int64_t)(m + 1) * (m + 1) <= p_w) ++m;
            if (m < 1) m = 1;
        }
        J.mtry = m;
    }
}

// Shadow columns (Algorithm 1, "shuffle by rows"): shadow s copies active
// column s mod p_cur through its own keyed permutation of the n rows:
// sha[s][i] = orig[src][pi_s(i)].  One workgroup per (chunk, shadow, job);
// the Feistel round functions are tabulated in LDS first.  Short chunks keep
// many workgroups in flight for the latency-bound cycle walks: chunks of
// 16,384 rows (one table per 8x more rows) made the kernel 50% slower on a
// 100,000-row job.
constexpr int kShadowChunk = 2048;  // rows per workgroup: 256 threads x 4 rows x 2

__global__ __launch_bounds__(256) void k_shadow(JobDev* jobs) {
    extern __shared__ uint16_t tab[];  // rounds x 2^half round-function values
    JobDev& J = jobs[blockIdx.z];
    const int s = blockIdx.y;
    if (!J.live || s >= J.n_sha) return;
    const int64_t r0 = (int64_t)blockIdx.x * kShadowChunk;
    if (r0 >= J.n) return;
    const KeyedPerm P = make_perm(J.seed_lo, J.seed_hi, kShadow, (uint32_t)J.t, (uint32_t)s, 0u,
                                  0u, (uint64_t)J.n);
    const uint32_t entries = P.rounds << P.half;
    for (uint32_t e = threadIdx.x; e < entries; e += 256)
        tab[e] = (uint16_t)perm_round(P, e >> P.half, e & P.mask);
    __syncthreads();
    const uint8_t* src = J.orig + (size_t)J.act[s % J.p_cur] * J.n_pad;
    uint8_t* dst = J.sha + (size_t)s * J.n_pad;
    // four consecutive rows per thread, one 32-bit store (rows are padded to
    // a multiple of 256; pad rows get 0)
    for (int64_t i = r0 + 4 * (int64_t)threadIdx.x; i < r0 + kShadowChunk && i < J.n; i += 1024) {
        uint32_t v = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u < J.n)
                v |= (uint32_t)src[perm_apply_tab(P, tab, (uint32_t)(i + u))] << (8 * u);
        *reinterpret_cast<uint32_t*>(dst + i) = v;
    }
}

// Row-major copy of the widened bins (jobs with rowmaj): rowmaj[i][c] =
// colptr[c][i] for the iteration's p_w widened columns.  Workgroup (row tile,
// column tile, job) moves a 64 x 64 byte tile through LDS: 16-byte column
// reads, 16-byte row writes.
__global__ __launch_bounds__(256) void k_rowmaj(JobDev* jobs) {
    __shared__ uint32_t tile[64][17];  // [column][4-row words], padded
    const JobDev& J = jobs[blockIdx.z];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int c0 = (int)blockIdx.y * 64;
    if (!J.live || !J.rowmaj || r0 >= J.n || c0 >= J.p_w) return;  // the whole workgroup
    const int t = (int)threadIdx.x, g = t & 3;
    {
        const int c = c0 + (t >> 2);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        // columns are n_pad (a multiple of 256) bytes: the 64 rows are in bounds
        if (c < J.p_w) v = *reinterpret_cast<const uint4*>(J.colptr[c] + r0 + 16 * g);
        uint32_t* w = &tile[t >> 2][4 * g];
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    }
    __syncthreads();
    const int r = t >> 2;
    if (r0 + r >= J.n) return;
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t x = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t word = tile[16 * g + 4 * k + u][r >> 2];
            x |= ((word >> (8 * (r & 3))) & 0xFFu) << (8 * u);
        }
        o[k] = x;
    }
    // rm_stride is a multiple of 64: the tile's 64 columns stay in the row
    *reinterpret_cast<uint4*>(J.rowmaj + (size_t)(r0 + r) * J.rm_stride + c0 + 16 * g) =
        make_uint4(o[0], o[1], o[2], o[3]);
}

// Bootstrap draws: draw j of tree tau is floor(u * n / 2^64) with u the
// 64-bit half (j even: words 0-1, odd: words 2-3) of
// Philox(word0(BOOT, 0, t), tau, j / 2, 0); multiplicities by atomics.
// k_boot_draw_lds (n up to kBootLdsRows * kBootLdsChunks): workgroup
// (c, tau) evaluates every draw of tree tau, counts the draws that fall in
// its chunk of `chunk` rows with LDS atomics, then writes the chunk's
// multiplicities, zeros included -- no global atomics.  k_boot_draw (any n):
// one global atomic per draw into multiplicities that start from zero.
constexpr uint32_t kBootLdsRows = 32768;  // longest chunk: 128 KB of counters
constexpr uint32_t kBootLdsChunks = 4;    // each chunk evaluates all n draws

__global__ __launch_bounds__(1024) void k_boot_draw_lds(JobDev* jobs, const TreeDev* trees,
                                                        uint32_t chunk) {
    extern __shared__ uint32_t cnt[];  // [chunk]
    const TreeDev tr = trees[blockIdx.y];
    const JobDev& J = jobs[tr.job];
    const uint32_t n = (uint32_t)J.n;
    const uint32_t r0 = blockIdx.x * chunk;
    if (!J.live || r0 >= n) return;  // the whole workgroup
    const uint32_t rows = min(chunk, n - r0);
    for (uint32_t i = threadIdx.x; i < rows; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    const uint32_t w0 = ctr_word0(kBoot, 0, (uint32_t)J.t);
    const uint32_t pairs = (n + 1u) / 2u;
    for (uint32_t pair = threadIdx.x; pair < pairs; pair += blockDim.x) {
        const Philox4 o = philox4x32_10(w0, (uint32_t)tr.tau, pair, 0u, J.seed_lo, J.seed_hi);
        // rows below r0 wrap to large values and fail the bound
        const uint32_t a = (uint32_t)__umul64hi((uint64_t)o.y << 32 | o.x, n) - r0;
        if (a < rows) atomicAdd(&cnt[a], 1u);
        if (2u * pair + 1u < n) {
            const uint32_t b = (uint32_t)__umul64hi((uint64_t)o.w << 32 | o.z, n) - r0;
            if (b < rows) atomicAdd(&cnt[b], 1u);
        }
    }
    __syncthreads();
    uint32_t* w = J.wbuf + (size_t)tr.tau * n + r0;
    for (uint32_t i = threadIdx.x; i < rows; i += blockDim.x) w[i] = cnt[i];
}

__global__ void k_boot_draw(JobDev* jobs, const TreeDev* trees) {
    const TreeDev tr = trees[blockIdx.y];
    const JobDev& J = jobs[tr.job];
    if (!J.live) return;
    const uint32_t pair = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = (uint32_t)J.n;
    if (2ull * pair >= n) return;
    const Philox4 o =
        philox4x32_10(ctr_word0(kBoot, 0, (uint32_t)J.t), (uint32_t)tr.tau, pair, 0u, J.seed_lo,
                      J.seed_hi);
    uint32_t* w = J.wbuf + (size_t)tr.tau * n;
    const uint64_t u0 = (uint64_t)o.y << 32 | o.x;
    atomicAdd(&w[__umul64hi(u0, n)], 1u);
    if (2ull * pair + 1 < n) {
        const uint64_t u1 = (uint64_t)o.w << 32 | o.z;
        atomicAdd(&w[__umul64hi(u1, n)], 1u);
    }
}

// Grid-stride fill (used instead of memset so that iterations stay capturable).
__global__ void k_fill_u32(uint32_t* p, size_t count, uint32_t v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Host launchers.
void launch_validate(const float* X, size_t nx, const int32_t* y, size_t n, int K,
                     uint32_t* flags, hipStream_t st) {
    const size_t blocks = (nx + 255) / 256;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096)),
                       dim3(256), 0, st, X, nx, y, n, K, flags);
}

void launch_validate_reg(const float* X, size_t nx, const float* y, size_t n, uint32_t* flags,
                         hipStream_t st) {
    const size_t blocks = (nx + 255) / 256;
    hipLaunchKernelGGL(k_validate_reg,
                       dim3((unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096)), dim3(256),
                       0, st, X, nx, y, n, flags);
}

void launch_target_range(const float* y, size_t n, float* out2, hipStream_t st) {
    hipLaunchKernelGGL(k_target_range, dim3(1), dim3(1024), 0, st, y, n, out2);
}

void launch_target_fix(const float* y, size_t n, int sh, int64_t* out, hipStream_t st) {
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_target_fix, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256),
                       0, st, y, n, sh, out);
}

void launch_labels(const int32_t* y, size_t n, uint8_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_labels_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, n,
                       out);
}

// Bins of all p columns of X (device, row-major) into bins[p][n_pad];
// keys is scratch of p * P words.
void launch_binning(const float* X, int64_t n, int64_t p, int B, uint8_t* bins, int64_t n_pad,
                    uint32_t* keys, int64_t P, hipStream_t st) {
    hipLaunchKernelGGL(k_to_keys, dim3((unsigned)((p + 31) / 32), (unsigned)((P + 31) / 32)),
                       dim3(256), 0, st, X, n, p, P, keys);
    const int tile = (int)(P < kSortTile ? P : kSortTile);
    hipLaunchKernelGGL(k_sort_tile, dim3((unsigned)(P / tile), (unsigned)p), dim3(1024), 0, st,
                       keys, P, tile, (int64_t)0);
    for (int64_t k = 2 * (int64_t)tile; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j >= tile; j >>= 1)
            hipLaunchKernelGGL(k_sort_step, dim3((unsigned)((P / 2 + 255) / 256), (unsigned)p),
                               dim3(256), 0, st, keys, P, k, j);
        hipLaunchKernelGGL(k_sort_tile, dim3((unsigned)(P / tile), (unsigned)p), dim3(1024), 0,
                           st, keys, P, tile, k);
    }
    const int64_t chunk = 16384;
    hipLaunchKernelGGL(k_bin, dim3((unsigned)((n_pad + chunk - 1) / chunk), (unsigned)p),
                       dim3(256), 0, st, X, n, p, P, keys, B, bins, n_pad, chunk);
}

void launch_thresholds(int32_t max_iter, int64_t p, uint64_t alpha_m, int32_t alpha_e,
                       int32_t* h_conf, int32_t* h_rej, hipStream_t st) {
    hipLaunchKernelGGL(k_thresholds, dim3((unsigned)((max_iter + 63) / 64)), dim3(64), 0, st,
                       max_iter, p, alpha_m, alpha_e, h_conf, h_rej);
}

void launch_active(JobDev* jobs, int n_jobs, hipStream_t st) {
    hipLaunchKernelGGL(k_active, dim3(n_jobs), dim3(256), 0, st, jobs);
}

void launch_shadow(JobDev* jobs, int n_jobs, int64_t max_n, int max_sha, hipStream_t st) {
    // round-function table of the largest job: the keyed bijection of [0, n)
    // works on 2 * half bits (smallest even >= 2 with 2^bits >= n) with
    // max(6, ceil(24 / half)) rounds
    uint32_t k = 0;
    while ((int64_t(1) << k) < max_n) ++k;
    if (k < 2) k = 2;
    k += k & 1u;
    const uint32_t half = k >> 1, rounds = std::max(6u, (24u + half - 1u) / half);
    const size_t lds = (size_t)(rounds << half) * sizeof(uint16_t);
    hipLaunchKernelGGL(k_shadow,
                       dim3((unsigned)((max_n + kShadowChunk - 1) / kShadowChunk),
                            (unsigned)max_sha, (unsigned)n_jobs),
                       dim3(256), lds, st, jobs);
}

void launch_rowmaj(JobDev* jobs, int n_jobs, int64_t max_n, int max_pw, hipStream_t st) {
    hipLaunchKernelGGL(k_rowmaj,
                       dim3((unsigned)((max_n + 63) / 64), (unsigned)((max_pw + 63) / 64),
                            (unsigned)n_jobs),
                       dim3(256), 0, st, jobs);
}

// Rows per workgroup of k_boot_draw_lds for jobs of at most max_n rows (the
// chunks split max_n evenly, in multiples of 256), or 0 when max_n is beyond
// its reach or its LDS cannot be granted (the global-atomic kernel then runs).
uint32_t prepare_boot_draw(int64_t max_n) {
    if (max_n < 1 || max_n > (int64_t)kBootLdsRows * kBootLdsChunks) return 0;
    const uint32_t nc = (uint32_t)((max_n + kBootLdsRows - 1) / kBootLdsRows);
    const uint32_t chunk = (uint32_t)(((max_n + nc - 1) / nc + 255) / 256 * 256);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        (size_t)lds_max < chunk * sizeof(uint32_t) ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_boot_draw_lds),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(chunk * sizeof(uint32_t))) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return chunk;
}

void launch_boot_draw(JobDev* jobs, const TreeDev* trees, int n_trees, int64_t max_n,
                      uint32_t lds_chunk, hipStream_t st) {
    if (lds_chunk) {
        hipLaunchKernelGGL(k_boot_draw_lds,
                           dim3((unsigned)((max_n + lds_chunk - 1) / lds_chunk),
                                (unsigned)n_trees),
                           dim3(1024), (size_t)lds_chunk * sizeof(uint32_t), st, jobs, trees,
                           lds_chunk);
        return;
    }
    hipLaunchKernelGGL(k_boot_draw,
                       dim3((unsigned)(((max_n + 1) / 2 + 255) / 256), (unsigned)n_trees),
                       dim3(256), 0, st, jobs, trees);
}

void launch_fill_u32(uint32_t* p, size_t count, uint32_t v, hipStream_t st) {
    if (!count) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
}

}  // namespace boruta
