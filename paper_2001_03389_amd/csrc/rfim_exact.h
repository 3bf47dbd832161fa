// Exact integer arithmetic for the sigma-cut decisions (device side).
//
// The outlier test of Section IV, |x - mu| > k*sigma with the population
// standard deviation, is evaluated without rounding: for a row of n samples
// with S1 = sum x and S2 = sum x^2 it reads (n*x - S1)^2 > k^2 * (n*S2 - S1^2),
// and for a time sample's C mean-corrected channels Z_c = B*x_c - S_b (whose
// sum is exactly zero) it reads C*Z_c^2 > k^2 * sum Z^2.  k is the exact binary
// value of the caller's double, k = mk * 2^ek with mk odd.  FP64 is used only to
// estimate where the cut falls; the exact test then settles the boundary.
#pragma once

#include "rfim_internal.h"

namespace rfim {

typedef unsigned __int128 u128;
typedef __int128 i128;

// 512-bit unsigned integer, little-endian 64-bit limbs.
struct U512 {
    uint64_t w[8];
};

__device__ inline U512 u512_from(u128 v) {
    U512 r;
#pragma unroll
    for (int i = 0; i < 8; i++) r.w[i] = 0;
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)(v >> 64);
    return r;
}

// a * b for operands below 2^128 (result below 2^256 fits easily)
__device__ inline U512 u512_mul128(u128 a, u128 b) {
    uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
    uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
    U512 r = u512_from(0);
    r.w[0] = (uint64_t)p00;
    u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    r.w[1] = (uint64_t)mid;
    u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
    r.w[2] = (uint64_t)hi;
    r.w[3] = (uint64_t)((hi >> 64) + (p11 >> 64));
    return r;
}

// a * 2^s, 0 <= s < 512 (bits shifted past 2^512 are lost; callers keep
// values far below that).  Constant limb indices only, so it stays in registers.
__device__ inline U512 u512_shl(U512 a, int s) {
    for (int ws = s >> 6; ws > 0; ws--) {
#pragma unroll
        for (int i = 7; i > 0; i--) a.w[i] = a.w[i - 1];
        a.w[0] = 0;
    }
    const int bs = s & 63;
    if (bs) {
#pragma unroll
        for (int i = 7; i > 0; i--) a.w[i] = (a.w[i] << bs) | (a.w[i - 1] >> (64 - bs));
        a.w[0] <<= bs;
    }
    return a;
}

__device__ inline int u512_cmp(const U512& a, const U512& b) {
#pragma unroll
    for (int i = 7; i >= 0; i--)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

__device__ inline int bitlen_u128(u128 v) {
    uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    if (hi) return 128 - __clzll((long long)hi);
    return lo ? 64 - __clzll((long long)lo) : 0;
}

// A <= k^2 * V in 512-bit integers (the general case)
__device__ inline bool le_k2_wide(u128 A, u128 V, const KExact& kx) {
    u128 mk2 = ((u128)kx.mk2_hi << 64) | kx.mk2_lo;
    U512 rhs = u512_mul128(mk2, V);
    U512 lhs = u512_from(A);
    if (kx.ek >= 0)
        rhs = u512_shl(rhs, 2 * kx.ek);
    else
        lhs = u512_shl(lhs, -2 * kx.ek);
    return u512_cmp(lhs, rhs) <= 0;
}

// A <= k^2 * V, exactly.  A and V below 2^128; k as described by kx.  The
// comparison runs in 128-bit integers when both sides provably fit, else in
// 512-bit integers.
__device__ inline bool le_k2(u128 A, u128 V, const KExact& kx) {
    if (kx.mode == 1) return A == 0;   // k^2 * V < 1 for every V < 2^128
    if (kx.mode == 2) return true;     // no outlier can exist (Samuelson)
    u128 mk2 = ((u128)kx.mk2_hi << 64) | kx.mk2_lo;
    const int lv = bitlen_u128(V);
    if (kx.ek >= 0) {
        const int s = 2 * kx.ek;
        if (kx.mk2_bits + lv + s <= 127) return A <= ((mk2 * V) << s);
    } else {
        const int s = -2 * kx.ek;
        if (bitlen_u128(A) + s <= 127 && kx.mk2_bits + lv <= 127) return (A << s) <= mk2 * V;
    }
    return le_k2_wide(A, V, kx);
}

// A <= k^2 * V when both sides fit 64 bits (the usual case for small k
// mantissas); otherwise the 128/512-bit comparison.
__device__ inline bool le_k2_small(uint64_t A, uint64_t V, const KExact& kx) {
    if (kx.mode == 0 && kx.mk2_hi == 0) {
        const int la = A ? 64 - __clzll((long long)A) : 0;
        const int lv = V ? 64 - __clzll((long long)V) : 0;
        if (kx.ek <= 0) {
            const int s = -2 * kx.ek;
            if (la + s <= 63 && kx.mk2_bits + lv <= 63) return (A << s) <= kx.mk2_lo * V;
        } else {
            const int s = 2 * kx.ek;
            if (kx.mk2_bits + lv + s <= 63) return A <= ((kx.mk2_lo * V) << s);
        }
    }
    return le_k2((u128)A, (u128)V, kx);
}

// num / den rounded to nearest, ties to even (den > 0, den < 2^62)
__device__ inline uint64_t rn_div_u64(uint64_t num, uint64_t den) {
    uint64_t q = num / den, r = num - q * den;
    if (2 * r > den || (2 * r == den && (q & 1))) q++;
    return q;
}

__device__ inline int64_t floor_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q--;
    return q;
}

__device__ inline int64_t ceil_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a > 0)) q++;
    return q;
}

// FD cut of one time sample: the largest z in [0, zcap] with C*z^2 <= k^2 SZ2;
// channel c is an outlier exactly when |Z_c| > z (Z_c is an integer, |Z_c| <= zcap).
__device__ inline uint64_t fd_zthr(u128 SZ2, int64_t C, const KExact& kx, uint64_t zcap) {
    auto ok = [&](uint64_t z) -> bool { return le_k2((u128)C * ((u128)z * z), SZ2, kx); };
    double e = kx.mode == 0 ? floor(kx.k * sqrt((double)SZ2 / (double)C))
                            : (kx.mode == 2 ? (double)zcap : 0.0);
    uint64_t z = e >= (double)zcap ? zcap : (e < 0.0 ? 0 : (uint64_t)e);
    while (z < zcap && ok(z + 1)) z++;
    while (z > 0 && !ok(z)) z--;
    return z;
}

// fd_zthr for sums that fit 64 bits: the largest z in [0, zcap] with
// C*z^2 <= k^2 * SZ2 (zcap < 2^24, C < 2^31)
__device__ inline uint32_t fd_zthr_small(uint64_t SZ2, uint32_t C, const KExact& kx, uint32_t zcap) {
    auto ok = [&](uint32_t z) -> bool { return le_k2_small((uint64_t)C * ((uint64_t)z * z), SZ2, kx); };
    double e = kx.mode == 0 ? floor(kx.k * sqrt((double)SZ2 / (double)C)) : (kx.mode == 2 ? (double)zcap : 0.0);
    uint32_t z = e >= (double)zcap ? zcap : (e < 0.0 ? 0u : (uint32_t)e);
    while (z < zcap && ok(z + 1)) z++;
    while (z > 0 && !ok(z)) z--;
    return z;
}

}  // namespace rfim
