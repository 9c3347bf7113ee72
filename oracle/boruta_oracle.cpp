// boruta_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see boruta_oracle.h).
//
// A plain CPU reference for one Boruta run, written for readability, not
// speed: every quantity is computed the direct way from its definition.
// Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
//
// Paper passages followed (arxiv 2605.09950):
//   * Boruta main loop ............................ Algorithm 1 (Sec. 2)
//   * impurity-decrease importance (TreeImp) ...... Algorithm 2 (Sec. 2.1)
//   * permutation importance (Permut) ............. Sec. 2 (Kursa's accuracy
//     drop) and Sec. 2.2; the out-of-bag accuracy-drop reading is listed
//     with the other readings of the paper in the design notes.
//   * prediction-divergence permutation importance  Algorithm 3 (Sec. 2.2):
//     one shared row permutation, the forest's class probabilities on the
//     full training matrix, KL divergence between unpermuted and permuted
//     predictions (importance mode 2).
//   * options outside Algorithm 1, off by default: a percentile of the
//     shadow importances as the hit threshold, and the rough fix of the
//     features still tentative at the end (both from Kursa's Boruta).
// Where the paper leaves a choice open (binning, split rule, randomness,
// the significance test), the reading implemented here is stated in the
// comment of the function that implements it.
//
// Parity status: every function below is pinned by a CPU test against an
// independent computation (brute force, closed form, library routine or a
// published known-answer vector); none is "parity unpinned".

#include "boruta_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

typedef unsigned __int128 u128;

// Random-stream identifiers placed in the top nibble of counter word 0.
const uint32_t kStreamBoot = 1;     // bootstrap draws, keyed by (t, tree, draw)
const uint32_t kStreamMtry = 2;     // per-node feature draws, keyed by (t, tree, heap id)
const uint32_t kStreamShadow = 3;   // shadow-column shuffles, keyed by (t, shadow)
const uint32_t kStreamOobPerm = 4;  // OOB permutations, keyed by (t, tree, column, replica)
const uint32_t kStreamFlush = 5;    // Algorithm 3's shared row permutation, keyed by t

// ---------------------------------------------------------------------------
// Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11,
// "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of two 32x32
// multiplies with the Weyl-sequence key schedule.
void philox(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)prod1;
        const uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)prod0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Counter word 0: stream (4 bits) | Feistel round (4 bits) | iteration (24 bits).
uint32_t word0(uint32_t stream, uint32_t round, uint32_t t) {
    return (stream << 28) | (round << 24) | (t & 0xFFFFFFu);
}

// A uniformly keyed bijection of [0, m): a balanced Feistel network on the
// smallest even number of bits k >= 2 with 2^k >= m (halves of h = k/2
// bits), max(6, ceil(24/h)) rounds (narrow halves need more rounds to mix),
// round function = word 0 of Philox(counter(stream, round, t, a, b, c_hi | R))
// masked to h bits, and cycle walking until the value lands inside [0, m).
uint64_t keyed_perm(uint64_t seed, uint32_t stream, uint32_t t, uint32_t a, uint32_t b,
                    uint32_t c_hi, uint64_t m, uint64_t x) {
    if (m <= 1) return 0;
    int k = 0;
    while ((uint64_t(1) << k) < m) ++k;
    if (k < 2) k = 2;
    if (k % 2 == 1) ++k;
    const int half = k / 2;
    const uint64_t mask = (uint64_t(1) << half) - 1;
    const uint32_t rounds = (uint32_t)std::max(6, (24 + half - 1) / half);
    do {
        uint64_t left = x >> half, right = x & mask;
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint32_t ctr[4] = {word0(stream, r, t), a, b, c_hi | (uint32_t)right};
            uint32_t o[4];
            philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
            const uint64_t f = o[0] & mask;
            const uint64_t new_left = right;
            right = left ^ f;
            left = new_left;
        }
        x = (left << half) | right;
    } while (x >= m);
    return x;
}

// ---------------------------------------------------------------------------
// Quantile binning (reading of the paper's binned random forest, Sec. 2):
// sort the column, take the order statistics of rank ceil(k n / B) - 1 for
// k = 1..B-1 as candidate cuts, keep the strictly increasing distinct ones,
// and give value x the bin #{cut < x}.
void bin_columns(const float* X, int64_t n, int64_t p, int B, uint8_t* bins, float* cuts_out,
                 int32_t* ncuts_out) {
    std::vector<float> col(n);
    std::vector<float> cuts;
    for (int64_t j = 0; j < p; ++j) {
        for (int64_t i = 0; i < n; ++i) col[i] = X[i * p + j];
        std::sort(col.begin(), col.end());
        cuts.clear();
        for (int64_t k = 1; k < B; ++k) {
            const int64_t rank = (k * n + B - 1) / B - 1;
            const float c = col[rank];
            if (cuts.empty() || c > cuts.back()) cuts.push_back(c);
        }
        for (int64_t i = 0; i < n; ++i) {
            const float x = X[i * p + j];
            bins[j * n + i] =
                (uint8_t)(std::lower_bound(cuts.begin(), cuts.end(), x) - cuts.begin());
        }
        if (cuts_out) {
            for (int k = 0; k < B - 1; ++k)
                cuts_out[j * (B - 1) + k] = k < (int)cuts.size() ? cuts[k] : 0.0f;
        }
        if (ncuts_out) ncuts_out[j] = (int32_t)cuts.size();
    }
}

// Bootstrap: n draws with replacement, draw j = floor(u64_j * n / 2^64) where
// u64_j is half of Philox(counter(BOOT, 0, t, tree, j / 2, 0)).
void bootstrap(uint64_t seed, uint32_t t, uint32_t tree, int64_t n, uint32_t* w) {
    std::fill(w, w + n, 0u);
    for (int64_t j = 0; j < n; ++j) {
        const uint32_t ctr[4] = {word0(kStreamBoot, 0, t), tree, (uint32_t)(j >> 1), 0u};
        uint32_t o[4];
        philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
        const uint64_t u = (j & 1) ? ((uint64_t)o[3] << 32 | o[2]) : ((uint64_t)o[1] << 32 | o[0]);
        const uint64_t idx = (uint64_t)(((u128)u * (u128)n) >> 64);
        w[idx] += 1;
    }
}

// ---------------------------------------------------------------------------
// Split rule (reading of the paper's Gini random forest, Sec. 2.1): for a
// node with weighted class counts c and threshold b, the left child takes
// the rows whose bin is <= b.  With S = sum_k c_k^2 and N = sum_k c_k the
// weighted Gini decrease is  S_L/N_L + S_R/N_R - S/N  (equal to cuML's
// gain x instance_count of Algorithm 2), so the best split maximises
// Q = S_L/N_L + S_R/N_R.  Candidates compare as exact rationals.
struct Cand {
    bool valid = false;
    int q = -1;  // position in the node's feature draw order
    int b = -1;  // threshold bin
    uint64_t nl = 0, sl = 0, nr = 0, sr = 0;
};

// a strictly better than b:  Q_a > Q_b  (cross-multiplied, exact).
bool better(const Cand& a, const Cand& b) {
    const u128 num_a = (u128)a.sl * a.nr + (u128)a.sr * a.nl;
    const u128 num_b = (u128)b.sl * b.nr + (u128)b.sr * b.nl;
    return num_a * ((u128)b.nl * b.nr) > num_b * ((u128)a.nl * a.nr);
}

// Q > S/N (strictly positive decrease).
bool positive_gain(const Cand& c, uint64_t s, uint64_t n) {
    const u128 num = (u128)c.sl * c.nr + (u128)c.sr * c.nl;
    return num * n > (u128)s * c.nl * c.nr;
}

// floor(2^32 * (Q - S/N)).
uint64_t gain_fixed(const Cand& c, uint64_t s, uint64_t n) {
    const u128 num = ((u128)c.sl * c.nr + (u128)c.sr * c.nl) * n - (u128)s * c.nl * c.nr;
    const u128 den = (u128)c.nl * c.nr * n;
    return (uint64_t)((num << 32) / den);
}

// ---------------------------------------------------------------------------
// Minimal unsigned big integer (little-endian 32-bit limbs): the exact
// regression split comparison and the exact binomial test.
struct Big {
    std::vector<uint32_t> v;
    explicit Big(uint64_t x = 0) {
        while (x) {
            v.push_back((uint32_t)x);
            x >>= 32;
        }
    }
    static Big of128(u128 x) {
        Big b((uint64_t)(x >> 64));
        b.shl(64);
        b.add(Big((uint64_t)x));
        return b;
    }
    void trim() {
        while (!v.empty() && v.back() == 0) v.pop_back();
    }
    void add(const Big& o) {
        if (o.v.size() > v.size()) v.resize(o.v.size(), 0);
        uint64_t carry = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            const uint64_t s = (uint64_t)v[i] + (i < o.v.size() ? o.v[i] : 0) + carry;
            v[i] = (uint32_t)s;
            carry = s >> 32;
        }
        if (carry) v.push_back((uint32_t)carry);
    }
    // this -= o, for o <= this
    void sub(const Big& o) {
        int64_t borrow = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            int64_t d = (int64_t)v[i] - (i < o.v.size() ? (int64_t)o.v[i] : 0) - borrow;
            borrow = d < 0 ? 1 : 0;
            if (d < 0) d += (int64_t(1) << 32);
            v[i] = (uint32_t)d;
        }
        trim();
    }
    void mul(uint32_t m) {
        uint64_t carry = 0;
        for (auto& x : v) {
            const uint64_t pr = (uint64_t)x * m + carry;
            x = (uint32_t)pr;
            carry = pr >> 32;
        }
        if (carry) v.push_back((uint32_t)carry);
        trim();
    }
    // this *= m for a 64-bit m: (this * hi) << 32 + this * lo
    void mul64(uint64_t m) {
        Big hi = *this;
        hi.mul((uint32_t)(m >> 32));
        hi.shl(32);
        mul((uint32_t)m);
        add(hi);
        trim();
    }
    void div_exact(uint32_t m) {
        uint64_t rem = 0;
        for (size_t i = v.size(); i-- > 0;) {
            const uint64_t cur = (rem << 32) | v[i];
            v[i] = (uint32_t)(cur / m);
            rem = cur % m;
        }
        trim();
    }
    void shl(int s) {
        const int limbs = s / 32, bits = s % 32;
        if (bits) {
            uint32_t carry = 0;
            for (auto& x : v) {
                const uint32_t nx = (x << bits) | carry;
                carry = x >> (32 - bits);
                x = nx;
            }
            if (carry) v.push_back(carry);
        }
        v.insert(v.begin(), (size_t)limbs, 0u);
        trim();
    }
    int bits() const {
        if (v.empty()) return 0;
        int b = 32 * (int)(v.size() - 1);
        uint32_t top = v.back();
        while (top) {
            ++b;
            top >>= 1;
        }
        return b;
    }
    bool bit(int i) const { return (size_t)(i / 32) < v.size() && ((v[i / 32] >> (i % 32)) & 1u); }
    static int cmp(Big a, Big b) {
        a.trim();
        b.trim();
        if (a.v.size() != b.v.size()) return a.v.size() < b.v.size() ? -1 : 1;
        for (size_t i = a.v.size(); i-- > 0;)
            if (a.v[i] != b.v[i]) return a.v[i] < b.v[i] ? -1 : 1;
        return 0;
    }
    // floor(a / d), d > 0, by binary long division (bit by bit from the top)
    static Big div(const Big& a, const Big& d) {
        Big q, r;
        for (int i = a.bits() - 1; i >= 0; --i) {
            r.shl(1);
            if (a.bit(i)) r.add(Big(1));
            q.shl(1);
            if (cmp(r, d) >= 0) {
                r.sub(d);
                q.add(Big(1));
            }
        }
        return q;
    }
    uint64_t low64() const {
        return (v.size() > 0 ? v[0] : 0) | ((uint64_t)(v.size() > 1 ? v[1] : 0) << 32);
    }
};

// ---------------------------------------------------------------------------
// Regression forest (reading of the paper's regression experiments, Sec. 3,
// which run Boruta on a random-forest regressor with squared-error loss,
// Sec. 2.2).
//
// Targets.  Each float32 target y is held exactly as the integer
// y_fix = rint(y * 2^(38 - e)), with e the smallest integer such that every
// |y| < 2^e (e = 0 for an all-zero target): a power-of-two scaling, exact for
// every target with |y| >= 2^(e - 15) (the 15 binades below 2^e), and within
// half a unit of 2^(e - 38) below that; |y_fix| < 2^38.
//
// Split rule.  A node with bootstrap weights w has W = sum w and
// T = sum w y_fix; the split that minimises the children's weighted squared
// error maximises Q = T_L^2/W_L + T_R^2/W_R (compared as exact rationals,
// with big integers), ties as for classification, and splits only when the
// decrease D = Q - T^2/W is strictly positive.  D equals
// (T_L W - T W_L)^2 / (W_L W_R W).
//
// Fixed point.  With R = max y_fix - min y_fix and n rows, a tree's summed
// decrease is at most n R^2 / 4; Algorithm 2 accumulates
// floor(D / 2^s_gain), s_gain = max(0, bits(n) + 2 bits(R) - 64), so a
// tree's sum stays below 2^62.  A leaf predicts floor(T / W).  The
// permutation importance scores a row by floor((y_fix - pred)^2 / 2^s_perm),
// s_perm = max(0, bits(n_trees n_perm n) + 2 bits(R + 1) - 63), so the summed
// increases stay within 64 bits; Algorithm 3 scores a row by
// floor(Dsum^2 / (n_trees^2 2^s_kl)), Dsum the change of the row's summed
// leaf predictions, s_kl = max(0, bits(n) + 2 bits(R + 1) - 63).  The
// reported importances are in squared target units.
int bit_length(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

struct RegScale {
    int e = 0;          // targets scaled by 2^(38 - e)
    int64_t range = 0;  // max y_fix - min y_fix
    int s_gain = 0, s_perm = 0, s_kl = 0;
};

void fix_targets(const float* y, int64_t n, int64_t* out, int* e_out) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs((double)y[i]));
    int e = 0;
    if (m > 0.0) std::frexp(m, &e);  // m = f 2^e with f in [1/2, 1): m < 2^e
    for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)std::rint(std::ldexp((double)y[i], 38 - e));
    *e_out = e;
}

RegScale reg_scale(const int64_t* yfix, int64_t n, int e, int n_trees, int n_perm) {
    RegScale s;
    s.e = e;
    int64_t lo = yfix[0], hi = yfix[0];
    for (int64_t i = 1; i < n; ++i) {
        lo = std::min(lo, yfix[i]);
        hi = std::max(hi, yfix[i]);
    }
    s.range = hi - lo;
    const int br = bit_length((uint64_t)s.range), br1 = bit_length((uint64_t)s.range + 1);
    s.s_gain = std::max(0, bit_length((uint64_t)n) + 2 * br - 64);
    s.s_perm = std::max(0, bit_length((uint64_t)n_trees * (uint64_t)n_perm * (uint64_t)n) +
                               2 * br1 - 63);
    s.s_kl = std::max(0, bit_length((uint64_t)n) + 2 * br1 - 63);
    return s;
}

// Regression split candidate: left/right weights and weighted target sums.
struct RegCand {
    bool valid = false;
    int q = -1, b = -1;
    uint64_t wl = 0, wr = 0;
    int64_t tl = 0, tr = 0;
};

Big sq_big(int64_t t) {
    const uint64_t a = (uint64_t)(t < 0 ? -t : t);
    return Big::of128((u128)a * a);
}

// Q_a > Q_b exactly: (TLa^2 WRa + TRa^2 WLa) WLb WRb > (TLb^2 WRb + TRb^2 WLb) WLa WRa.
bool better_reg(const RegCand& a, const RegCand& b) {
    Big lhs = sq_big(a.tl), t2 = sq_big(a.tr);
    lhs.mul64(a.wr);
    t2.mul64(a.wl);
    lhs.add(t2);
    lhs.mul64(b.wl);
    lhs.mul64(b.wr);
    Big rhs = sq_big(b.tl), u2 = sq_big(b.tr);
    rhs.mul64(b.wr);
    u2.mul64(b.wl);
    rhs.add(u2);
    rhs.mul64(a.wl);
    rhs.mul64(a.wr);
    return Big::cmp(lhs, rhs) > 0;
}

// |T_L W - T W_L|: the decrease is its square over W_L W_R W, positive iff it
// is nonzero.
u128 reg_gap(const RegCand& c) {
    const __int128 W = (__int128)(c.wl + c.wr), T = (__int128)c.tl + c.tr;
    const __int128 g = (__int128)c.tl * W - T * (__int128)c.wl;
    return (u128)(g < 0 ? -g : g);
}

// floor(D / 2^s) = floor(gap^2 / (W_L W_R W 2^s)).
uint64_t gain_fixed_reg(const RegCand& c, int s) {
    const u128 g = reg_gap(c);
    Big num = Big::of128(g), hi = Big::of128(g);  // g^2 = g lo + (g hi) 2^64
    num.mul64((uint64_t)g);
    hi.mul64((uint64_t)(g >> 64));
    hi.shl(64);
    num.add(hi);
    Big den = Big::of128((u128)c.wl * c.wr);
    den.mul64(c.wl + c.wr);
    den.shl(s);
    return Big::div(num, den).low64();
}

// floor(T / W) toward minus infinity.
int64_t floor_div(int64_t t, uint64_t w) {
    const int64_t q = t / (int64_t)w;
    return (q * (int64_t)w != t && t < 0) ? q - 1 : q;
}

struct Data {
    int64_t n = 0;
    int64_t p_w = 0;
    std::vector<const uint8_t*> col;  // [p_w] column base pointers, each [n]
    const int32_t* y = nullptr;  // class labels (classification)
    int K = 2;
    int B = 256;
    bool reg = false;
    const int64_t* yfix = nullptr;  // regression: fixed-point targets
    RegScale rs;                    // regression: scale and fixed-point shifts
};

// Regression form of best_split: per bin the weight and the weighted target
// sum; the first best in (draw position, threshold) order by the exact rule.
RegCand best_split_reg(const Data& d, const std::vector<uint32_t>& rows, const uint32_t* w,
                       const std::vector<int32_t>& feats, uint64_t W, int64_t T) {
    std::vector<uint64_t> hw((size_t)d.B);
    std::vector<int64_t> ht((size_t)d.B);
    RegCand best;
    for (size_t q = 0; q < feats.size(); ++q) {
        const uint8_t* col = d.col[feats[q]];
        std::fill(hw.begin(), hw.end(), 0);
        std::fill(ht.begin(), ht.end(), 0);
        for (uint32_t i : rows) {
            hw[col[i]] += w[i];
            ht[col[i]] += (int64_t)w[i] * d.yfix[i];
        }
        uint64_t lw = 0;
        int64_t lt = 0;
        for (int b = 0; b + 1 < d.B; ++b) {
            lw += hw[(size_t)b];
            lt += ht[(size_t)b];
            RegCand c;
            c.valid = true;
            c.q = (int)q;
            c.b = b;
            c.wl = lw;
            c.wr = W - lw;
            c.tl = lt;
            c.tr = T - lt;
            if (c.wl == 0 || c.wr == 0) continue;
            if (!best.valid || better_reg(c, best)) best = c;
        }
    }
    return best;
}

// Exhaustive search over the node's drawn features and every threshold
// b = 0..B-2, keeping the first best in (draw position, threshold) order.
Cand best_split(const Data& d, const std::vector<uint32_t>& rows, const uint32_t* w,
                const std::vector<int32_t>& feats, const std::vector<uint64_t>& counts) {
    std::vector<uint64_t> hist((size_t)d.B * d.K);
    std::vector<uint64_t> left(d.K);
    Cand best;
    for (size_t q = 0; q < feats.size(); ++q) {
        const uint8_t* col = d.col[feats[q]];
        std::fill(hist.begin(), hist.end(), 0);
        for (uint32_t i : rows) hist[(size_t)col[i] * d.K + d.y[i]] += w[i];
        std::fill(left.begin(), left.end(), 0);
        for (int b = 0; b + 1 < d.B; ++b) {
            for (int k = 0; k < d.K; ++k) left[k] += hist[(size_t)b * d.K + k];
            Cand c;
            c.valid = true;
            c.q = (int)q;
            c.b = b;
            for (int k = 0; k < d.K; ++k) {
                const uint64_t r = counts[k] - left[k];
                c.nl += left[k];
                c.sl += left[k] * left[k];
                c.nr += r;
                c.sr += r * r;
            }
            if (c.nl == 0 || c.nr == 0) continue;
            if (!best.valid || better(c, best)) best = c;
        }
    }
    return best;
}

struct TNode {
    int64_t heap = 1;
    int depth = 0;
    int32_t feat = -1;  // -1: leaf
    int32_t thr = 0;
    int64_t leaf_class = 0;  // regression: the prediction floor(T / W)
    uint64_t n = 0;          // weighted rows (regression: W)
    int64_t tsum = 0;        // regression: T
    uint64_t gain = 0;  // floor(2^32 * Gini decrease), split nodes only
    int32_t left = -1, right = -1;
    std::vector<uint64_t> counts;  // weighted in-bag class counts
};

struct TreeCtx {
    const Data* d;
    const uint32_t* w;
    int D;
    int mtry;
    uint64_t seed;
    uint32_t t;
    uint32_t tree;
    std::vector<TNode> nodes;
};

// Recursive growth: a node is a leaf at depth D or when no valid candidate
// gives a strictly positive decrease; a leaf predicts the class with the
// largest weighted count (smallest class index on ties).
int32_t grow(TreeCtx& c, const std::vector<uint32_t>& rows, int depth, int64_t heap) {
    const Data& d = *c.d;
    const int32_t idx = (int32_t)c.nodes.size();
    c.nodes.emplace_back();
    std::vector<uint64_t> counts(d.K, 0);
    uint64_t n = 0, s = 0;
    int64_t T = 0;
    if (d.reg) {
        for (uint32_t i : rows) {
            n += c.w[i];
            T += (int64_t)c.w[i] * d.yfix[i];
        }
        c.nodes[idx].tsum = T;
    } else {
        for (uint32_t i : rows) counts[d.y[i]] += c.w[i];
        for (uint64_t v : counts) {
            n += v;
            s += v * v;
        }
    }
    c.nodes[idx].n = n;
    c.nodes[idx].heap = heap;
    c.nodes[idx].depth = depth;
    c.nodes[idx].counts = counts;

    std::vector<int32_t> feats;
    if (depth < c.D)
        for (int q = 0; q < c.mtry; ++q)
            feats.push_back((int32_t)keyed_perm(c.seed, kStreamMtry, c.t, c.tree, (uint32_t)heap,
                                                0u, (uint64_t)d.p_w, (uint64_t)q));
    // the chosen split: feature, threshold, decrease in fixed point
    bool split = false;
    int32_t f = -1, thr = 0;
    uint64_t gain = 0;
    if (d.reg) {
        RegCand best;
        if (!feats.empty()) best = best_split_reg(d, rows, c.w, feats, n, T);
        if (best.valid && reg_gap(best) != 0) {
            split = true;
            f = feats[best.q];
            thr = best.b;
            gain = gain_fixed_reg(best, d.rs.s_gain);
        }
    } else {
        Cand best;
        if (!feats.empty()) best = best_split(d, rows, c.w, feats, counts);
        if (best.valid && positive_gain(best, s, n)) {
            split = true;
            f = feats[best.q];
            thr = best.b;
            gain = gain_fixed(best, s, n);
        }
    }
    if (split) {
        std::vector<uint32_t> lrows, rrows;
        for (uint32_t i : rows) (d.col[f][i] <= thr ? lrows : rrows).push_back(i);
        c.nodes[idx].feat = f;
        c.nodes[idx].thr = thr;
        c.nodes[idx].gain = gain;
        const int32_t l = grow(c, lrows, depth + 1, 2 * heap);
        const int32_t r = grow(c, rrows, depth + 1, 2 * heap + 1);
        c.nodes[idx].left = l;
        c.nodes[idx].right = r;
    } else if (d.reg) {
        c.nodes[idx].leaf_class = floor_div(T, n);
    } else {
        int arg = 0;
        for (int k = 1; k < d.K; ++k)
            if (counts[k] > counts[arg]) arg = k;
        c.nodes[idx].leaf_class = arg;
    }
    return idx;
}

// Prediction of one row, optionally with column sub_f's bin replaced by sub_b.
int predict(const std::vector<TNode>& nodes, const Data& d, uint32_t row, int32_t sub_f,
            int sub_b) {
    int32_t i = 0;
    while (nodes[i].feat >= 0) {
        const int32_t f = nodes[i].feat;
        const int b = (f == sub_f) ? sub_b : d.col[f][row];
        i = (b <= nodes[i].thr) ? nodes[i].left : nodes[i].right;
    }
    return nodes[i].leaf_class;
}

// Leaf reached by a row, optionally with column sub_f's bin replaced by sub_b.
int32_t predict_leaf(const std::vector<TNode>& nodes, const Data& d, uint32_t row, int32_t sub_f,
                     int sub_b) {
    int32_t i = 0;
    while (nodes[i].feat >= 0) {
        const int32_t f = nodes[i].feat;
        const int b = (f == sub_f) ? sub_b : d.col[f][row];
        i = (b <= nodes[i].thr) ? nodes[i].left : nodes[i].right;
    }
    return i;
}

// Regression: a row's squared error against its leaf's prediction, shifted
// right by s_perm bits (floor).
int64_t sq_error_fix(const TNode& leaf, int64_t yfix, int s_perm) {
    const __int128 e = (__int128)yfix - leaf.leaf_class;
    const u128 sq = (u128)(e * e);
    return (int64_t)(sq >> s_perm);
}

struct TreeResult {
    std::vector<TNode> nodes;
    int64_t n_inbag = 0, n_oob = 0, oob_correct = 0;
    std::vector<uint64_t> gain_sum;  // [p_w] TreeImp: per-feature sum of fixed-point gains
    std::vector<int64_t> drop;       // [p_w] Permut: sum over replicas/rows of correct drops
};

struct IterParams {
    int D, mtry, mode, R;
    uint64_t seed;
    uint32_t t;
    bool naive;
};

// One tree of iteration t: bootstrap, growth, and the importance terms.
void run_tree(const Data& d, const IterParams& ip, uint32_t tree, TreeResult& out) {
    std::vector<uint32_t> w(d.n);
    bootstrap(ip.seed, ip.t, tree, d.n, w.data());
    std::vector<uint32_t> inbag, oob;
    for (int64_t i = 0; i < d.n; ++i) (w[i] > 0 ? inbag : oob).push_back((uint32_t)i);
    TreeCtx c{&d, w.data(), ip.D, ip.mtry, ip.seed, ip.t, tree, {}};
    grow(c, inbag, 0, 1);
    out.nodes = std::move(c.nodes);
    out.n_inbag = (int64_t)inbag.size();
    out.n_oob = (int64_t)oob.size();
    if (ip.mode == 0) {
        out.gain_sum.assign(d.p_w, 0);
        for (const TNode& nd : out.nodes)
            if (nd.feat >= 0) out.gain_sum[nd.feat] += nd.gain;
        return;
    }
    if (ip.mode == 2) return;  // scored over the whole forest (forest_divergence)
    // Out-of-bag accuracy drop under permutation of one column among the
    // tree's OOB rows (Kursa's importance): rows o_0 < o_1 < ... of the OOB
    // set; replica r of column f moves the bin of o_pi(j) into row o_j, with
    // pi the keyed bijection of [0, m) for (t, tree, f, r).
    // For a regression forest the score of a row is the negated squared error
    // against its leaf's prediction (sq_error_fix, in 2^s_perm units), so the
    // drop is the increase of the squared error.
    const uint64_t m = oob.size();
    std::vector<int64_t> base(m);
    for (uint64_t j = 0; j < m; ++j) {
        if (d.reg) {
            base[j] = -sq_error_fix(out.nodes[predict_leaf(out.nodes, d, oob[j], -1, 0)],
                                    d.yfix[oob[j]], d.rs.s_perm);
        } else {
            base[j] = predict(out.nodes, d, oob[j], -1, 0) == d.y[oob[j]];
            out.oob_correct += base[j];
        }
    }
    out.drop.assign(d.p_w, 0);
    auto permuted_correct = [&](int32_t f, int r, uint64_t j) -> int64_t {
        const uint64_t src = keyed_perm(ip.seed, kStreamOobPerm, ip.t, tree, (uint32_t)f,
                                        (uint32_t)r << 16, m, j);
        const int sb = d.col[f][oob[src]];
        if (d.reg)
            return -sq_error_fix(out.nodes[predict_leaf(out.nodes, d, oob[j], f, sb)],
                                 d.yfix[oob[j]], d.rs.s_perm);
        return (int64_t)(predict(out.nodes, d, oob[j], f, sb) == d.y[oob[j]]);
    };
    if (ip.naive) {
        for (int32_t f = 0; f < d.p_w; ++f)
            for (int r = 0; r < ip.R; ++r)
                for (uint64_t j = 0; j < m; ++j) out.drop[f] += base[j] - permuted_correct(f, r, j);
        return;
    }
    // Only columns tested on the row's own path can change its prediction.
    std::vector<int32_t> path;
    for (uint64_t j = 0; j < m; ++j) {
        path.clear();
        int32_t i = 0;
        while (out.nodes[i].feat >= 0) {
            const int32_t f = out.nodes[i].feat;
            if (std::find(path.begin(), path.end(), f) == path.end()) path.push_back(f);
            i = (d.col[f][oob[j]] <= out.nodes[i].thr) ? out.nodes[i].left : out.nodes[i].right;
        }
        for (int32_t f : path)
            for (int r = 0; r < ip.R; ++r) out.drop[f] += base[j] - permuted_correct(f, r, j);
    }
}

// ---------------------------------------------------------------------------
// Algorithm 3 (importance mode 2), with these readings:
//   * the forest's predicted class distribution for a row is the mean over
//     trees of the class frequencies of the leaf the row reaches (weighted
//     in-bag counts), each frequency held as floor(2^32 c_k / N) and summed
//     over the trees exactly;
//   * one row permutation pi per iteration (keyed by t) serves every column:
//     the permuted matrix gives row r the bin of row pi(r) in the column;
//   * the loss is the KL divergence KL(P || Q) of the unpermuted prediction
//     P from the permuted one Q, in bits, with 32 fractional bits, summed
//     over all n rows; a class that P gives positive probability and Q none
//     is given one fixed-point unit in Q (so identical predictions give 0).

// floor-ish 2^32 * log2(x), x in [1, 2^62): the integer part from the bit
// length, then 32 fraction digits by repeated squaring of the mantissa
// (held in [1, 2) with 62 fractional bits, truncated after each squaring).
uint64_t log2_fix32(uint64_t x) {
    int e = 63;
    while (!(x >> e)) --e;
    uint64_t m = x << (62 - e);
    uint64_t frac = 0;
    for (int i = 0; i < 32; ++i) {
        m = (uint64_t)(((u128)m * m) >> 62);
        frac <<= 1;
        if (m >> 63) {
            frac |= 1;
            m >>= 1;
        }
    }
    return ((uint64_t)e << 32) | frac;
}

// KL(P || Q) in bits with 32 fractional bits, P = S / sum S and
// Q = S~ / sum S~ with S~_k = Sq_k, raised to 1 where Sq_k = 0 < S_k:
//   sum over S_k > 0 of (S_k / sum S) (log2 S_k - log2 S~_k) + log2 sum S~ - log2 sum S,
// the first term floored as a whole.
int64_t kl_fix32(const uint64_t* S, const uint64_t* Sq, int K) {
    uint64_t sp = 0, sq = 0;
    __int128 v = 0;
    for (int k = 0; k < K; ++k) {
        const uint64_t q = (Sq[k] == 0 && S[k] != 0) ? 1 : Sq[k];
        sp += S[k];
        sq += q;
        if (S[k])
            v += (__int128)S[k] * ((__int128)log2_fix32(S[k]) - (__int128)log2_fix32(q));
    }
    __int128 first = v / (__int128)sp;
    if (v < 0 && first * (__int128)sp != v) first -= 1;  // floor
    return (int64_t)first + (int64_t)log2_fix32(sq) - (int64_t)log2_fix32(sp);
}

// Leaf reached by a row, with column sub_f's bin replaced by sub_b.
int32_t leaf_of_row(const std::vector<TNode>& nodes, const Data& d, uint32_t row, int32_t sub_f,
                    int sub_b) {
    int32_t i = 0;
    while (nodes[i].feat >= 0) {
        const int32_t f = nodes[i].feat;
        const int b = (f == sub_f) ? sub_b : d.col[f][row];
        i = (b <= nodes[i].thr) ? nodes[i].left : nodes[i].right;
    }
    return i;
}

// Summed fixed-point class frequencies of the leaves row `row` reaches.
void forest_predict(const std::vector<std::vector<TNode>*>& forest, const Data& d, uint32_t row,
                    int32_t sub_f, int sub_b, uint64_t* S) {
    for (int k = 0; k < d.K; ++k) S[k] = 0;
    for (const std::vector<TNode>* tree : forest) {
        const TNode& leaf = (*tree)[leaf_of_row(*tree, d, row, sub_f, sub_b)];
        for (int k = 0; k < d.K; ++k) S[k] += (uint64_t)(((u128)leaf.counts[k] << 32) / leaf.n);
    }
}

// imp[f] = sum over rows of the fixed-point divergence for column f: for
// each column, the predictions of the matrix with that column permuted
// against those of the unpermuted matrix (Algorithm 3, one predict call
// per column).
// Regression form (reading): the forest's prediction of a row is the mean
// over trees of its leaves' predictions; with S the sum over trees of the
// leaves' floor(T / W) and Dsum = S(permuted) - S(unpermuted), a row's loss
// is floor(Dsum^2 / (n_trees^2 2^s_kl)), the squared difference of the two
// mean predictions in 2^s_kl units of squared fixed-point target units.
int64_t forest_pred_sum(const std::vector<std::vector<TNode>*>& forest, const Data& d,
                        uint32_t row, int32_t sub_f, int sub_b) {
    int64_t s = 0;
    for (const std::vector<TNode>* tree : forest)
        s += (*tree)[leaf_of_row(*tree, d, row, sub_f, sub_b)].leaf_class;
    return s;
}

void forest_divergence(const std::vector<std::vector<TNode>*>& forest, const Data& d,
                       uint64_t seed, uint32_t t, int n_threads, int64_t* imp,
                       const std::vector<int32_t>& only) {
    const int K = d.K;
    std::vector<uint64_t> base((size_t)d.n * K);
    std::vector<uint32_t> pi((size_t)d.n);
    for (int64_t r = 0; r < d.n; ++r) {
        if (!d.reg) forest_predict(forest, d, (uint32_t)r, -1, 0, &base[(size_t)r * K]);
        pi[r] = (uint32_t)keyed_perm(seed, kStreamFlush, t, 0u, 0u, 0u, (uint64_t)d.n, (uint64_t)r);
    }
    // the columns to score: all, or (checks at full size) the listed ones
    std::vector<int32_t> cols;
    for (int32_t f = 0; f < d.p_w; ++f)
        if (only.empty() || std::find(only.begin(), only.end(), f) != only.end()) cols.push_back(f);
    if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    const int64_t nc = (int64_t)cols.size();
    std::vector<std::thread> pool;
    for (int w = 0; w < std::min<int64_t>(n_threads, nc); ++w)
        pool.emplace_back([&, w] {
            std::vector<uint64_t> q(K);
            for (int64_t ci = w; ci < nc; ci += n_threads) {
                const int32_t f = cols[ci];
                int64_t acc = 0;
                for (int64_t r = 0; r < d.n; ++r) {
                    if (d.reg) {
                        const int64_t diff =
                            forest_pred_sum(forest, d, (uint32_t)r, (int32_t)f, d.col[f][pi[r]]) -
                            forest_pred_sum(forest, d, (uint32_t)r, -1, 0);
                        const u128 a = (u128)(diff < 0 ? -diff : diff);
                        const u128 T = forest.size();
                        acc += (int64_t)((a * a / (T * T)) >> d.rs.s_kl);
                        continue;
                    }
                    forest_predict(forest, d, (uint32_t)r, (int32_t)f, d.col[f][pi[r]], q.data());
                    acc += kl_fix32(&base[(size_t)r * K], q.data(), K);
                }
                imp[f] = acc;
            }
        });
    for (auto& th : pool) th.join();
}

// Reading of the unspecified test() of Algorithm 1: two one-sided exact
// binomial tails with success probability 1/2 after t trials, Bonferroni
// corrected over all p original features, strict comparison with alpha:
//   confirm iff p * P[Bin(t,1/2) >= h] < alpha,
//   reject  iff p * P[Bin(t,1/2) <= h] < alpha.
// With alpha = m * 2^e exactly (m integer), P = U / 2^t, both become integer
// comparisons  p * U < m * 2^(e+t).
int binom_decide(int h, int t, int64_t p, double alpha) {
    std::vector<Big> row;
    Big c(1);
    for (int k = 0; k <= t; ++k) {
        row.push_back(c);
        c.mul((uint32_t)(t - k));
        c.div_exact((uint32_t)(k + 1));
    }
    Big upper(0), lower(0);
    for (int k = 0; k <= t; ++k) {
        if (k >= h) upper.add(row[k]);
        if (k <= h) lower.add(row[k]);
    }
    int ex = 0;
    const double fr = std::frexp(alpha, &ex);
    const uint64_t mant = (uint64_t)std::ldexp(fr, 53);
    const int shift = ex - 53 + t;
    auto below_alpha = [&](Big tail) {
        tail.mul((uint32_t)p);
        Big rhs(mant);
        if (shift >= 0)
            rhs.shl(shift);
        else
            tail.shl(-shift);
        return Big::cmp(tail, rhs) < 0;
    };
    if (below_alpha(upper)) return 1;
    if (below_alpha(lower)) return -1;
    return 0;
}

// ---------------------------------------------------------------------------
struct Run {
    int64_t n, p;
    int K, T, D, mtry_opt, mode, B, R;
    double alpha;
    uint64_t seed;
    const int32_t* y;
    std::vector<uint8_t> orig;  // [p][n]
    int n_threads;
    bool naive;
    std::vector<int32_t> kl_cols;  // mode 2: score only these columns (empty: all)
    int perc = 100;                // hit threshold: percentile of the shadow importances
    bool reg = false;              // regression forest
    std::vector<int64_t> yfix;     // regression: fixed-point targets
    std::vector<int32_t> yzero;    // regression: placeholder labels (all 0)
    RegScale rs;
};

// Hit threshold of an iteration: the perc-th percentile of the m shadow
// importances by the nearest-rank rule, i.e. the ceil(perc m / 100)-th
// smallest.  perc = 100 gives the maximum that Algorithm 1 compares against.
int64_t shadow_threshold(const int64_t* sha, int m, int perc) {
    std::vector<int64_t> v(sha, sha + m);
    std::sort(v.begin(), v.end());
    const int64_t rank = ((int64_t)perc * m + 99) / 100;  // 1-based, >= 1 for perc >= 1
    return v[(size_t)(rank - 1)];
}

// Median of a list of doubles; an even count takes the mean of the two middle
// values.
double median_of(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t k = v.size();
    return k % 2 ? v[k / 2] : (v[k / 2 - 1] + v[k / 2]) / 2.0;
}

// Rough fix of the features still tentative after the last iteration (an
// extension of Kursa's Boruta, not part of Algorithm 1): a tentative feature
// is confirmed when the median of its history importances exceeds the median
// of the per-iteration shadow thresholds, and rejected otherwise.  A
// tentative feature was active in every iteration, so its history has no NaN.
void rough_fix(int8_t* state, const double* hist, const double* smax, int64_t p, int n_iter) {
    if (n_iter < 1) return;
    const double ms = median_of(std::vector<double>(smax, smax + n_iter));
    for (int64_t j = 0; j < p; ++j) {
        if (state[j] != 0) continue;
        std::vector<double> col((size_t)n_iter);
        for (int t = 0; t < n_iter; ++t) col[(size_t)t] = hist[(size_t)t * p + j];
        state[j] = median_of(col) > ms ? 1 : -1;
    }
}

// Labels must lie in [0, y_hi): the classes, or the quantised levels of a
// regression target.
int validate(const float* X, const int32_t* y, int64_t n, int64_t p, int K, int T, int D,
             int mtry, int mode, int max_iter, double alpha, int B, int R, int y_hi) {
    if (!X || !y) return -1;
    if (n < 2 || n > (int64_t(1) << 24) || p < 1 || p > (int64_t(1) << 30)) return -1;
    if (K < 2 || K > 16 || T < 1 || T > 65535 || D < 1 || D > 30 || mtry < 0) return -1;
    if (mode < 0 || mode > 2) return -1;
    if (max_iter < 1 || max_iter > 1000) return -1;
    if (!(alpha > 0.0 && alpha < 0.5)) return -1;
    if (B < 2 || B > 256 || R < 1 || R > 65535) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (y[i] < 0 || y[i] >= y_hi) return -1;
    for (int64_t i = 0; i < n * p; ++i)
        if (!std::isfinite(X[i])) return -2;
    return 0;
}

int64_t isqrt(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

template <class F>
void parallel_for(int n_threads, int count, F fn) {
    if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    n_threads = std::min(n_threads, count);
    if (n_threads <= 1) {
        for (int i = 0; i < count; ++i) fn(i);
        return;
    }
    std::vector<std::thread> pool;
    for (int w = 0; w < n_threads; ++w)
        pool.emplace_back([&, w] {
            for (int i = w; i < count; i += n_threads) fn(i);
        });
    for (auto& th : pool) th.join();
}

// One iteration of Algorithm 1 (full = importances, hits and decision too).
void iteration(const Run& run, int t, int8_t* state, int32_t* hits,
               const std::vector<int32_t>& trees, bool full, double* imp_row,
               double* shadow_max, oracle_trace_fn trace, void* user) {
    const int64_t n = run.n, p = run.p;
    // Active columns X[:, state >= 0] in ascending order, then shadow copies
    // (doubled until there are at least five), each shuffled by its own
    // keyed permutation of the rows.
    std::vector<int32_t> active;
    for (int64_t j = 0; j < p; ++j)
        if (state[j] >= 0) active.push_back((int32_t)j);
    const int p_cur = (int)active.size();
    if (p_cur == 0) return;
    int n_sha = p_cur;
    while (n_sha < 5) n_sha *= 2;
    std::vector<uint8_t> shadow((size_t)n_sha * n);
    Data d;
    d.n = n;
    d.p_w = p_cur + n_sha;
    d.y = run.y;
    d.K = run.K;
    d.B = run.B;
    d.reg = run.reg;
    d.yfix = run.yfix.data();
    d.rs = run.rs;
    std::vector<int32_t> col_src(d.p_w);
    for (int c = 0; c < p_cur; ++c) {
        d.col.push_back(run.orig.data() + (size_t)active[c] * n);
        col_src[c] = active[c];
    }
    for (int s = 0; s < n_sha; ++s) {
        const int32_t src = active[s % p_cur];
        const uint8_t* from = run.orig.data() + (size_t)src * n;
        uint8_t* to = shadow.data() + (size_t)s * n;
        for (int64_t i = 0; i < n; ++i)
            to[i] = from[keyed_perm(run.seed, kStreamShadow, (uint32_t)t, (uint32_t)s, 0u, 0u,
                                    (uint64_t)n, (uint64_t)i)];
        d.col.push_back(to);
        col_src[p_cur + s] = src;
    }
    IterParams ip;
    ip.D = run.D;
    ip.mtry = run.mtry_opt > 0 ? (int)std::min<int64_t>(run.mtry_opt, d.p_w)
                               : (int)std::max<int64_t>(1, isqrt(d.p_w));
    ip.mode = run.mode;
    ip.R = run.R;
    ip.seed = run.seed;
    ip.t = (uint32_t)t;
    ip.naive = run.naive;

    std::vector<TreeResult> res(trees.size());
    parallel_for(run.n_threads, (int)trees.size(),
                 [&](int i) { run_tree(d, ip, (uint32_t)trees[i], res[i]); });

    std::vector<int64_t> imp(d.p_w, 0);
    if (full) {
        double denom = 0.0;
        int scale_exp = 0;  // reported value = ldexp(v / denom, scale_exp)
        if (run.mode == 0) {
            // Algorithm 2: per-tree normalisation of the accumulated decreases
            // (a tree without any split contributes zeros), mean over trees,
            // renormalisation.  Fixed point: floor(2^44 * G_f / sum_g G_g) per
            // tree, summed over trees; the 1/T of the mean cancels in the
            // final renormalisation.
            for (const TreeResult& r : res) {
                u128 tot = 0;
                for (uint64_t g : r.gain_sum) tot += g;
                if (tot == 0) continue;
                for (int64_t f = 0; f < d.p_w; ++f)
                    imp[f] += (int64_t)(((u128)r.gain_sum[f] << 44) / tot);
            }
            int64_t s = 0;
            for (int64_t v : imp) s += v;
            denom = (double)s;
        } else if (run.mode == 2) {
            // Algorithm 3 over the whole forest of the iteration; reported as
            // the mean divergence per row in bits
            std::vector<std::vector<TNode>*> forest;
            for (TreeResult& r : res) forest.push_back(&r.nodes);
            forest_divergence(forest, d, run.seed, (uint32_t)t, run.n_threads, imp.data(),
                              run.kl_cols);
            // mean divergence per row in bits (regression: mean squared
            // difference of the predictions in squared target units)
            denom = (double)d.n * (run.reg ? 1.0 : 4294967296.0);
            if (run.reg) scale_exp = run.rs.s_kl - 2 * (38 - run.rs.e);
        } else {
            int64_t oob_total = 0;
            for (const TreeResult& r : res) {
                oob_total += r.n_oob;
                for (int64_t f = 0; f < d.p_w; ++f) imp[f] += r.drop[f];
            }
            denom = (double)((int64_t)run.R * oob_total);
            // regression: squared errors in squared target units
            if (run.reg) scale_exp = run.rs.s_perm - 2 * (38 - run.rs.e);
        }
        auto report = [&](int64_t v) {
            return denom > 0.0 ? std::ldexp((double)v / denom, scale_exp) : 0.0;
        };
        // Hit: strictly above the best shadow (Algorithm 1), or above the
        // shadows' perc-th percentile when that option is set.
        const int64_t best_shadow = shadow_threshold(&imp[p_cur], n_sha, run.perc);
        if (imp_row) {
            for (int64_t j = 0; j < p; ++j) imp_row[j] = std::nan("");
            for (int c = 0; c < p_cur; ++c) imp_row[active[c]] = report(imp[c]);
        }
        if (shadow_max) *shadow_max = report(best_shadow);
        for (int c = 0; c < p_cur; ++c)
            if (imp[c] > best_shadow) hits[active[c]] += 1;
        for (int64_t j = 0; j < p; ++j)
            if (state[j] == 0) state[j] = (int8_t)binom_decide(hits[j], t, p, run.alpha);
    }

    if (trace) {
        std::vector<int64_t> stats, nodes;
        for (size_t i = 0; i < res.size(); ++i) {
            const TreeResult& r = res[i];
            stats.insert(stats.end(), {(int64_t)trees[i], r.n_inbag, r.n_oob, r.oob_correct,
                                       (int64_t)r.nodes.size()});
            std::vector<const TNode*> sorted;
            for (const TNode& nd : r.nodes) sorted.push_back(&nd);
            std::sort(sorted.begin(), sorted.end(),
                      [](const TNode* a, const TNode* b) { return a->heap < b->heap; });
            for (const TNode* nd : sorted)
                nodes.insert(nodes.end(),
                             {(int64_t)trees[i], nd->heap, (int64_t)nd->feat,
                              (int64_t)(nd->feat >= 0 ? nd->thr : nd->leaf_class),
                              (int64_t)nd->n, (int64_t)nd->gain});
        }
        oracle_iter_trace tr;
        tr.t = t;
        tr.p_cur = p_cur;
        tr.n_sha = n_sha;
        tr.p_w = (int32_t)d.p_w;
        tr.mtry = ip.mtry;
        tr.n_trees = (int32_t)trees.size();
        tr.col_src = col_src.data();
        tr.imp_int = imp.data();
        tr.hits = hits;
        tr.state = state;
        tr.tree_stats = stats.data();
        tr.n_nodes = (int64_t)(nodes.size() / 6);
        tr.nodes = nodes.data();
        trace(user, &tr);
    }
}

int setup(Run& run, const float* X, const int32_t* y, int64_t n, int64_t p, int K, int T, int D,
          int mtry, int mode, int max_iter, double alpha, uint64_t seed, int B, int R,
          int n_threads, int naive, int y_hi = 0) {
    const int rc =
        validate(X, y, n, p, K, T, D, mtry, mode, max_iter, alpha, B, R, y_hi ? y_hi : K);
    if (rc) return rc;
    run.n = n;
    run.p = p;
    run.K = K;
    run.T = T;
    run.D = D;
    run.mtry_opt = mtry;
    run.mode = mode;
    run.B = B;
    run.R = R;
    run.alpha = alpha;
    run.seed = seed;
    run.y = y;
    run.n_threads = n_threads;
    run.naive = naive != 0;
    run.orig.resize((size_t)n * p);
    bin_columns(X, n, p, B, run.orig.data(), nullptr, nullptr);
    return 0;
}

// The Boruta loop over a prepared run (defined below the exported functions).
int fit_run(Run& run, int n_trees, int max_iter, int rough, int8_t* decision_out,
            double* imp_history_out, int32_t* hits_out, double* shadow_max_out,
            int32_t* n_iter_out, oracle_trace_fn trace, void* trace_user);

}  // namespace

extern "C" {

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox(ctr, key[0], key[1], out);
}

uint64_t oracle_keyed_perm(uint64_t seed, uint32_t stream, uint32_t t, uint32_t a, uint32_t b,
                           uint32_t c_hi, uint64_t m, uint64_t x) {
    return keyed_perm(seed, stream, t, a, b, c_hi, m, x);
}

int oracle_bin(const float* X, int64_t n, int64_t p, int32_t n_bins, uint8_t* bins_out,
               float* cuts_out, int32_t* ncuts_out) {
    if (!X || !bins_out || n < 1 || p < 1 || n_bins < 2 || n_bins > 256) return -1;
    for (int64_t i = 0; i < n * p; ++i)
        if (!std::isfinite(X[i])) return -2;
    bin_columns(X, n, p, n_bins, bins_out, cuts_out, ncuts_out);
    return 0;
}

uint64_t oracle_log2_fix32(uint64_t x) { return x ? log2_fix32(x) : 0; }

int64_t oracle_kl_fix32(const uint64_t* S, const uint64_t* Sq, int32_t K) {
    return kl_fix32(S, Sq, K);
}

void oracle_bootstrap(uint64_t seed, uint32_t t, uint32_t tree, int64_t n, uint32_t* w_out) {
    bootstrap(seed, t, tree, n, w_out);
}

int oracle_best_split(const uint8_t* bins, int64_t n, const int32_t* y, const uint32_t* w,
                      const uint32_t* rows, int64_t n_rows, const int32_t* feats, int32_t n_feats,
                      int32_t n_classes, int32_t n_bins, uint64_t out[8]) {
    if (!bins || !y || !w || !rows || !feats || n_feats < 1 || n_classes < 1 || n_bins < 2)
        return -1;
    Data d;
    d.n = n;
    d.y = y;
    d.K = n_classes;
    d.B = n_bins;
    int32_t maxf = 0;
    for (int q = 0; q < n_feats; ++q) maxf = std::max(maxf, feats[q]);
    d.p_w = maxf + 1;
    for (int64_t f = 0; f < d.p_w; ++f) d.col.push_back(bins + f * n);
    std::vector<uint32_t> rv(rows, rows + n_rows);
    std::vector<int32_t> fv(feats, feats + n_feats);
    std::vector<uint64_t> counts(n_classes, 0);
    for (uint32_t i : rv) counts[y[i]] += w[i];
    uint64_t N = 0, S = 0;
    for (uint64_t c : counts) {
        N += c;
        S += c * c;
    }
    const Cand c = best_split(d, rv, w, fv, counts);
    const bool found = c.valid && positive_gain(c, S, N);
    out[0] = found;
    out[1] = (uint64_t)c.q;
    out[2] = (uint64_t)c.b;
    out[3] = c.nl;
    out[4] = c.sl;
    out[5] = c.nr;
    out[6] = c.sr;
    out[7] = found ? gain_fixed(c, S, N) : 0;
    return 0;
}

int64_t oracle_grow_tree(const uint8_t* bins, int64_t n, int64_t p_w, const int32_t* y,
                         const uint32_t* w, int32_t n_classes, int32_t n_bins, int32_t max_depth,
                         int32_t mtry, uint64_t seed, uint32_t t, uint32_t tree, int64_t* nodes_out,
                         int64_t max_nodes, uint64_t* gain_sum_out) {
    if (!bins || !y || !w || n < 1 || p_w < 1 || mtry < 1 || mtry > p_w || max_depth < 1)
        return -1;
    Data d;
    d.n = n;
    d.p_w = p_w;
    d.y = y;
    d.K = n_classes;
    d.B = n_bins;
    for (int64_t f = 0; f < p_w; ++f) d.col.push_back(bins + f * n);
    std::vector<uint32_t> inbag;
    for (int64_t i = 0; i < n; ++i)
        if (w[i] > 0) inbag.push_back((uint32_t)i);
    TreeCtx c{&d, w, max_depth, mtry, seed, t, tree, {}};
    grow(c, inbag, 0, 1);
    std::vector<const TNode*> sorted;
    for (const TNode& nd : c.nodes) sorted.push_back(&nd);
    std::sort(sorted.begin(), sorted.end(),
              [](const TNode* a, const TNode* b) { return a->heap < b->heap; });
    const int64_t cnt = (int64_t)sorted.size();
    for (int64_t i = 0; i < cnt && i < max_nodes && nodes_out; ++i) {
        const TNode* nd = sorted[i];
        int64_t* o = nodes_out + 6 * i;
        o[0] = tree;
        o[1] = nd->heap;
        o[2] = nd->feat;
        o[3] = nd->feat >= 0 ? nd->thr : nd->leaf_class;
        o[4] = (int64_t)nd->n;
        o[5] = (int64_t)nd->gain;
    }
    if (gain_sum_out) {
        std::fill(gain_sum_out, gain_sum_out + p_w, 0);
        for (const TNode& nd : c.nodes)
            if (nd.feat >= 0) gain_sum_out[nd.feat] += nd.gain;
    }
    return cnt;
}

int oracle_binom_decide(int32_t hits, int32_t t, int64_t p, double alpha) {
    if (t < 1 || hits < 0 || hits > t || p < 1 || p > 0xFFFFFFFFll || !(alpha > 0 && alpha < 0.5))
        return 0;
    return binom_decide(hits, t, p, alpha);
}

int oracle_boruta_fit(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                      int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                      int32_t max_iter, double alpha, uint64_t seed, int32_t n_bins,
                      int32_t n_perm, int32_t n_threads, int32_t permut_naive,
                      int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                      double* shadow_max_out, int32_t* n_iter_out, oracle_trace_fn trace,
                      void* trace_user) {
    return oracle_boruta_fit_ext(X, y, n, p, n_classes, n_trees, max_depth, mtry,
                                 importance_mode, max_iter, alpha, seed, n_bins, n_perm,
                                 n_threads, permut_naive, 100, 0, decision_out, imp_history_out,
                                 hits_out, shadow_max_out, n_iter_out, trace, trace_user);
}

int oracle_boruta_fit_ext(const float* X, const int32_t* y, int64_t n, int64_t p,
                          int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                          int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                          int32_t n_bins, int32_t n_perm, int32_t n_threads,
                          int32_t permut_naive, int32_t perc, int32_t rough,
                          int8_t* decision_out, double* imp_history_out, int32_t* hits_out,
                          double* shadow_max_out, int32_t* n_iter_out, oracle_trace_fn trace,
                          void* trace_user) {
    if (!decision_out || !imp_history_out || !n_iter_out) return -1;
    if (perc < 1 || perc > 100 || (rough != 0 && rough != 1)) return -1;
    Run run;
    const int rc = setup(run, X, y, n, p, n_classes, n_trees, max_depth, mtry, importance_mode,
                         max_iter, alpha, seed, n_bins, n_perm, n_threads, permut_naive);
    if (rc) return rc;
    run.perc = perc;
    return fit_run(run, n_trees, max_iter, rough, decision_out, imp_history_out, hits_out,
                   shadow_max_out, n_iter_out, trace, trace_user);
}

int oracle_boruta_fit_reg(const float* X, const float* y, int64_t n, int64_t p,
                          int32_t n_trees, int32_t max_depth, int32_t mtry,
                          int32_t importance_mode, int32_t max_iter, double alpha, uint64_t seed,
                          int32_t n_bins, int32_t n_perm, int32_t n_threads,
                          int32_t permut_naive, int8_t* decision_out, double* imp_history_out,
                          int32_t* hits_out, double* shadow_max_out, int32_t* n_iter_out,
                          oracle_trace_fn trace, void* trace_user) {
    if (!decision_out || !imp_history_out || !n_iter_out || !y) return -1;
    if (n < 2 || importance_mode < 0 || importance_mode > 2) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(y[i])) return -2;
    Run run;
    run.reg = true;
    run.yfix.resize((size_t)n);
    int e = 0;
    fix_targets(y, n, run.yfix.data(), &e);
    run.yzero.assign((size_t)n, 0);
    const int rc = setup(run, X, run.yzero.data(), n, p, 2, n_trees, max_depth, mtry,
                         importance_mode, max_iter, alpha, seed, n_bins, n_perm, n_threads,
                         permut_naive);
    if (rc) return rc;
    run.rs = reg_scale(run.yfix.data(), n, e, n_trees, n_perm);
    return fit_run(run, n_trees, max_iter, 0, decision_out, imp_history_out, hits_out,
                   shadow_max_out, n_iter_out, trace, trace_user);
}

// The fixed-point targets and the scale exponent e (see fix_targets); shifts
// out[0..3] = (s_gain, s_perm, s_kl, range) for n_trees trees and n_perm
// replicas.
int32_t oracle_fix_targets(const float* y, int64_t n, int32_t n_trees, int32_t n_perm,
                           int64_t* yfix_out, int64_t* shifts_out) {
    int e = 0;
    fix_targets(y, n, yfix_out, &e);
    const RegScale rs = reg_scale(yfix_out, n, e, n_trees, n_perm);
    if (shifts_out) {
        shifts_out[0] = rs.s_gain;
        shifts_out[1] = rs.s_perm;
        shifts_out[2] = rs.s_kl;
        shifts_out[3] = rs.range;
    }
    return e;
}

// Best regression split of one node: out = (found, q, b, W_L, W_R, T_L, T_R,
// floor(D / 2^s_gain)).
int oracle_best_split_reg(const uint8_t* bins, int64_t n, const int64_t* yfix, const uint32_t* w,
                          const uint32_t* rows, int64_t n_rows, const int32_t* feats,
                          int32_t n_feats, int32_t n_bins, int32_t s_gain, int64_t out[8]) {
    if (!bins || !yfix || !w || !rows || !feats || n_feats < 1 || n_bins < 2) return -1;
    Data d;
    d.n = n;
    d.B = n_bins;
    d.reg = true;
    d.yfix = yfix;
    int32_t maxf = 0;
    for (int q = 0; q < n_feats; ++q) maxf = std::max(maxf, feats[q]);
    d.p_w = maxf + 1;
    for (int64_t f = 0; f < d.p_w; ++f) d.col.push_back(bins + f * n);
    std::vector<uint32_t> rv(rows, rows + n_rows);
    std::vector<int32_t> fv(feats, feats + n_feats);
    uint64_t W = 0;
    int64_t T = 0;
    for (uint32_t i : rv) {
        W += w[i];
        T += (int64_t)w[i] * yfix[i];
    }
    const RegCand c = best_split_reg(d, rv, w, fv, W, T);
    const bool found = c.valid && reg_gap(c) != 0;
    out[0] = found;
    out[1] = c.q;
    out[2] = c.b;
    out[3] = (int64_t)c.wl;
    out[4] = (int64_t)c.wr;
    out[5] = c.tl;
    out[6] = c.tr;
    out[7] = found ? (int64_t)gain_fixed_reg(c, s_gain) : 0;
    return 0;
}

}  // extern "C"

namespace {

int fit_run(Run& run, int n_trees, int max_iter, int rough, int8_t* decision_out,
            double* imp_history_out, int32_t* hits_out, double* shadow_max_out,
            int32_t* n_iter_out, oracle_trace_fn trace, void* trace_user) {
    const int64_t p = run.p;
    std::vector<double> smax_all((size_t)max_iter, 0.0);
    std::vector<int8_t> state(p, 0);
    std::vector<int32_t> hits(p, 0);
    std::vector<int32_t> all_trees(n_trees);
    for (int i = 0; i < n_trees; ++i) all_trees[i] = i;
    int t = 0;
    auto undecided = [&] {
        for (int8_t s : state)
            if (s == 0) return true;
        return false;
    };
    while (t < max_iter && undecided()) {
        ++t;
        double smax = 0.0;
        iteration(run, t, state.data(), hits.data(), all_trees, true,
                  imp_history_out + (size_t)(t - 1) * p, &smax, trace, trace_user);
        if (shadow_max_out) shadow_max_out[t - 1] = smax;
        smax_all[(size_t)(t - 1)] = smax;
    }
    if (rough) rough_fix(state.data(), imp_history_out, smax_all.data(), p, t);
    std::copy(state.begin(), state.end(), decision_out);
    if (hits_out) std::copy(hits.begin(), hits.end(), hits_out);
    *n_iter_out = t;
    return 0;
}

}  // namespace

extern "C" {

// Final ranking of Algorithm 1: confirmed features rank 1, undecided ones 2,
// rejected ones by descending historical importance from 3 on.  Reading: a
// rejected feature's historical importance is the mean of its finite history
// entries (the iterations in which it was active), summed in iteration order;
// its rank is 3 plus the number of rejected features with a strictly larger
// mean (equal means share a rank).
void oracle_rank(const int8_t* decision, const double* imp_history, int64_t p, int32_t n_iter,
                 int32_t* rank_out) {
    std::vector<double> mean(p, 0.0);
    for (int64_t j = 0; j < p; ++j) {
        if (decision[j] != -1) continue;
        double s = 0.0;
        int c = 0;
        for (int32_t t = 0; t < n_iter; ++t) {
            const double v = imp_history[(size_t)t * p + j];
            if (std::isnan(v)) continue;
            s += v;
            ++c;
        }
        mean[j] = c ? s / c : 0.0;
    }
    for (int64_t j = 0; j < p; ++j) {
        if (decision[j] == 1) {
            rank_out[j] = 1;
        } else if (decision[j] == 0) {
            rank_out[j] = 2;
        } else {
            int32_t above = 0;
            for (int64_t g = 0; g < p; ++g)
                if (decision[g] == -1 && mean[g] > mean[j]) ++above;
            rank_out[j] = 3 + above;
        }
    }
}

// The paper's multi-seed protocol (Sec. 3: runs with different seeds, the
// median importance as the basis of the selection).  Reading: per run, a
// feature's importance is the mean of its finite history entries (summed in
// iteration order); the median over runs (the mean of the two middle values
// for an even count); the selection is the lower median of the runs'
// decisions (confirmed in more than half of the runs -> confirmed; rejected
// in at least half -> rejected; else tentative).
int64_t oracle_shadow_threshold(const int64_t* sha, int32_t m, int32_t perc) {
    return shadow_threshold(sha, m, perc);
}

void oracle_rough_fix(int8_t* decision, const double* imp_history, const double* shadow_max,
                      int64_t p, int32_t n_iter) {
    rough_fix(decision, imp_history, shadow_max, p, n_iter);
}

void oracle_seed_median(const int8_t* decisions, const double* histories, const int32_t* n_iters,
                        int64_t p, int32_t max_iter, int32_t n_runs, double* median_out,
                        int8_t* decision_out) {
    std::vector<double> v(n_runs);
    std::vector<int8_t> dv(n_runs);
    for (int64_t j = 0; j < p; ++j) {
        for (int32_t r = 0; r < n_runs; ++r) {
            const double* h = histories + (size_t)r * max_iter * p;
            double sum = 0.0;
            int c = 0;
            for (int32_t t = 0; t < n_iters[r]; ++t) {
                const double x = h[(size_t)t * p + j];
                if (std::isnan(x)) continue;
                sum += x;
                ++c;
            }
            v[r] = c ? sum / c : 0.0;
            dv[r] = decisions[(size_t)r * p + j];
        }
        std::sort(v.begin(), v.end());
        std::sort(dv.begin(), dv.end());
        median_out[j] = n_runs % 2 ? v[n_runs / 2] : (v[n_runs / 2 - 1] + v[n_runs / 2]) / 2.0;
        decision_out[j] = dv[(n_runs - 1) / 2];
    }
}

int oracle_boruta_step(const float* X, const int32_t* y, int64_t n, int64_t p, int32_t n_classes,
                       int32_t n_trees, int32_t max_depth, int32_t mtry, int32_t importance_mode,
                       double alpha, uint64_t seed, int32_t n_bins, int32_t n_perm, int32_t t,
                       int8_t* state, int32_t* hits, const int32_t* tree_subset, int32_t n_subset,
                       int32_t n_threads, int32_t permut_naive, double* imp_row_out,
                       double* shadow_max_out, oracle_trace_fn trace, void* trace_user) {
    return oracle_boruta_step_cols(X, y, n, p, n_classes, n_trees, max_depth, mtry,
                                   importance_mode, alpha, seed, n_bins, n_perm, t, state, hits,
                                   tree_subset, n_subset, nullptr, 0, n_threads, permut_naive,
                                   imp_row_out, shadow_max_out, trace, trace_user);
}

int oracle_boruta_step_cols(const float* X, const int32_t* y, int64_t n, int64_t p,
                            int32_t n_classes, int32_t n_trees, int32_t max_depth, int32_t mtry,
                            int32_t importance_mode, double alpha, uint64_t seed, int32_t n_bins,
                            int32_t n_perm, int32_t t, int8_t* state, int32_t* hits,
                            const int32_t* tree_subset, int32_t n_subset, const int32_t* kl_cols,
                            int32_t n_kl_cols, int32_t n_threads, int32_t permut_naive,
                            double* imp_row_out, double* shadow_max_out, oracle_trace_fn trace,
                            void* trace_user) {
    if (!state || !hits || t < 1 || t > 1000) return -1;
    Run run;
    const int rc = setup(run, X, y, n, p, n_classes, n_trees, max_depth, mtry, importance_mode,
                         1000, alpha, seed, n_bins, n_perm, n_threads, permut_naive);
    if (rc) return rc;
    if (kl_cols) run.kl_cols.assign(kl_cols, kl_cols + n_kl_cols);
    std::vector<int32_t> trees;
    if (tree_subset) {
        for (int i = 0; i < n_subset; ++i) {
            if (tree_subset[i] < 0 || tree_subset[i] >= n_trees) return -1;
            trees.push_back(tree_subset[i]);
        }
    } else {
        for (int i = 0; i < n_trees; ++i) trees.push_back(i);
    }
    iteration(run, t, state, hits, trees, tree_subset == nullptr, imp_row_out, shadow_max_out,
              trace, trace_user);
    return 0;
}

}  // extern "C"
