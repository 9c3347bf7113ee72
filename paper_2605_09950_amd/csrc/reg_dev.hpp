// reg_dev.hpp -- exact arithmetic of the regression forest on the device.
//
// Reading of the paper's regression experiments (a random-forest regressor
// with squared-error loss, Sec. 2.2 and Sec. 3): targets are held as the
// integers y_fix = rint(y 2^(38 - e)) (|y_fix| < 2^38); a node has bootstrap
// weight W = sum w and weighted target sum T = sum w y_fix.  A threshold
// leaves (W_L, T_L) on the left and (W_R, T_R) on the right; the squared-
// error decrease is D = g^2 / (W_L W_R W) with the gap g = T_L W_R - T_R W_L,
// so within one node candidates order by g^2 / (W_L W_R).  A split needs
// g != 0.  Algorithm 2 accumulates floor(D / 2^s_gain); a leaf predicts
// floor(T / W).
//
// A regression candidate reuses Cand: nl = W_L, nr = W_R, sl = T_L and
// sr = T_R (two's complement).
#pragma once

#include "dev_common.hpp"

namespace boruta {

struct U256 {
    uint64_t w[4];  // little-endian 64-bit limbs
};

// Full product of two values below 2^128.
__device__ __forceinline__ U256 mul128_full(u128 a, u128 b) {
    const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
    const uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0,
               p11 = (u128)a1 * b1;
    U256 r;
    r.w[0] = (uint64_t)p00;
    const u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    r.w[1] = (uint64_t)mid;
    const u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
    r.w[2] = (uint64_t)hi;
    r.w[3] = (uint64_t)(hi >> 64) + (uint64_t)(p11 >> 64);
    return r;
}

// a * m, for products below 2^256.
__device__ __forceinline__ U256 mul256_64(const U256& a, uint64_t m) {
    U256 r;
    u128 carry = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const u128 t = (u128)a.w[i] * m + carry;
        r.w[i] = (uint64_t)t;
        carry = t >> 64;
    }
    return r;
}

__device__ __forceinline__ int cmp256(const U256& a, const U256& b) {
#pragma unroll
    for (int i = 3; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

__device__ __forceinline__ U256 sub256(const U256& a, const U256& b) {
    U256 r;
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t d = a.w[i] - b.w[i];
        const uint64_t b1 = a.w[i] < b.w[i];
        r.w[i] = d - borrow;
        borrow = b1 | (d < borrow);
    }
    return r;
}

// d << s as 256 bits, for d < 2^128 and s < 128.
__device__ __forceinline__ U256 shl128(u128 d, int s) {
    U256 r;
    const uint64_t lo = (uint64_t)d, hi = (uint64_t)(d >> 64);
    const int limb = s >> 6, bits = s & 63;
    uint64_t v[3];
    v[0] = lo << bits;
    v[1] = bits ? (hi << bits) | (lo >> (64 - bits)) : hi;
    v[2] = bits ? hi >> (64 - bits) : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = i - limb;
        r.w[i] = (k >= 0 && k < 3) ? v[k] : 0;
    }
    return r;
}

// floor(num / den) for a quotient below 2^64 (restoring division, one
// quotient bit per step).
__device__ inline uint64_t udiv256_128(U256 num, u128 den) {
    uint64_t q = 0;
    for (int i = 63; i >= 0; --i) {
        const U256 d = shl128(den, i);
        if (cmp256(num, d) >= 0) {
            num = sub256(num, d);
            q |= 1ull << i;
        }
    }
    return q;
}

__device__ __forceinline__ int64_t reg_tl(const Cand& c) { return (int64_t)c.sl; }
__device__ __forceinline__ int64_t reg_tr(const Cand& c) { return (int64_t)c.sr; }

// |g| = |T_L W_R - T_R W_L| (< 2^87).
__device__ __forceinline__ u128 reg_gap(const Cand& c) {
    const __int128 g = (__int128)reg_tl(c) * (int64_t)c.nr - (__int128)reg_tr(c) * (int64_t)c.nl;
    return (u128)(g < 0 ? -g : g);
}

// D_a > D_b exactly for candidates of one node: g_a^2 W_Lb W_Rb > g_b^2 W_La W_Ra
// (products below 2^221).
__device__ inline bool reg_better(const Cand& a, const Cand& b) {
    const u128 ga = reg_gap(a), gb = reg_gap(b);
    const U256 lhs = mul256_64(mul128_full(ga, ga), (uint64_t)b.nl * b.nr);
    const U256 rhs = mul256_64(mul128_full(gb, gb), (uint64_t)a.nl * a.nr);
    return cmp256(lhs, rhs) > 0;
}

// FP64 ranking score g^2 / (W_L W_R): relative error at most 5 units of
// 2^-53 (two roundings converting g, one squaring, one division; W_L W_R <
// 2^48 is exact).
__device__ __forceinline__ double reg_q64(const Cand& c) {
    const double g = u128_to_double(reg_gap(c));
    return g * g / (double)((uint64_t)c.nl * c.nr);
}

// Margin of the FP64 ranking: the exact best scores at least (1 - 10 u) of the
// FP64 maximum, far above (1 - 2^-40).
__device__ __forceinline__ double fp64_floor(double qmax) { return qmax * (1.0 - 0x1.0p-40); }

__device__ __forceinline__ double u256_to_double(const U256& a) {
    return (((double)a.w[3] * 18446744073709551616.0 + (double)a.w[2]) * 18446744073709551616.0 +
            (double)a.w[1]) * 18446744073709551616.0 + (double)a.w[0];
}

// floor(num / den) for a quotient below 2^63: an FP64 estimate (relative
// error a few units of 2^-53), one FP64 correction from the exact 256-bit
// remainder, then at most a few exact +-1 steps; should those not settle the
// quotient, the restoring division gives it.
__device__ inline uint64_t udiv256_128_est(const U256& num, u128 den) {
    const double dd = u128_to_double(den);
    double qd = u256_to_double(num) / dd;
    qd = qd < 9.2e18 ? qd : 9.2e18;
    uint64_t q = (uint64_t)qd;
    U256 prod = mul128_full((u128)q, den);
    const bool over = cmp256(prod, num) > 0;
    const U256 diff = over ? sub256(prod, num) : sub256(num, prod);
    const uint64_t c = (uint64_t)(u256_to_double(diff) / dd);
    q = over ? q - (c < q ? c : q) : q + c;
    prod = mul128_full((u128)q, den);
    for (int step = 0; step < 4; ++step) {
        if (cmp256(prod, num) > 0) {  // q too large
            --q;
            prod = sub256(prod, shl128(den, 0));
            continue;
        }
        const U256 next = mul128_full((u128)q + 1, den);
        if (cmp256(next, num) <= 0) {  // q too small
            ++q;
            prod = next;
            continue;
        }
        return q;
    }
    return udiv256_128(num, den);
}

// floor(D / 2^s) = floor(g^2 / (W_L W_R W 2^s)); W_L W_R W 2^s < 2^128 and the
// quotient < 2^63 for the shifts the engine chooses.
__device__ inline uint64_t reg_gain_fix(const Cand& c, int s) {
    const u128 g = reg_gap(c);
    const u128 den = ((u128)((uint64_t)c.nl * c.nr) * (c.nl + c.nr)) << s;
    return udiv256_128_est(mul128_full(g, g), den);
}

// floor(T / W), toward minus infinity.
__device__ __forceinline__ int64_t reg_pred(int64_t T, uint32_t W) {
    const int64_t q = T / (int64_t)W;
    return (q * (int64_t)W != T && T < 0) ? q - 1 : q;
}

// Order of one feature's candidates: larger D, then the smaller threshold;
// invalid ones (nl == 0) last.
__device__ __forceinline__ bool reg_wins_same_feature(const Cand& a, const Cand& b) {
    if (b.nl == 0) return a.nl != 0 || a.b < b.b;
    if (a.nl == 0) return false;
    if (reg_better(a, b)) return true;
    if (reg_better(b, a)) return false;
    return a.b < b.b;
}

// Total order over a node's candidates: larger D, then the earlier draw
// position, then the smaller threshold.
__device__ __forceinline__ bool reg_wins_total(const Cand& a, const Cand& b) {
    if (b.nl == 0) return a.nl != 0;
    if (a.nl == 0) return false;
    if (reg_better(a, b)) return true;
    if (reg_better(b, a)) return false;
    return a.q < b.q || (a.q == b.q && a.b < b.b);
}

}  // namespace boruta
