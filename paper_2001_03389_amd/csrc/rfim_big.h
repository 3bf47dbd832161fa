// Wide integers for the float32 fallback kernels (device side).
//
// A float32 value is an integer number of units 2^-149 (at most 2^277) and its
// square an integer number of units 2^-298 (at most 2^554).  Row and column
// sums, D = n*S2 - S1^2 and both sides of the squared outlier test of
// Section IV stay below 2^896 for n, C < 2^24, so every quantity fits Big.
// These routines serve rows and columns with values spread over more than the
// fast window; they favour simplicity over speed.
#pragma once

#include "rfim_f32_exact.h"

namespace rfim {

constexpr int kBigL = 28;   // 32-bit limbs

struct Big {
    uint32_t d[kBigL];   // magnitude, little-endian
    int neg;             // sign (never set for zero)
};

__device__ inline void big_zero(Big& a) {
    for (int i = 0; i < kBigL; i++) a.d[i] = 0;
    a.neg = 0;
}

__device__ inline bool big_is_zero(const Big& a) {
    for (int i = 0; i < kBigL; i++)
        if (a.d[i]) return false;
    return true;
}

__device__ inline void big_set_u64(Big& a, uint64_t v) {
    big_zero(a);
    a.d[0] = (uint32_t)v;
    a.d[1] = (uint32_t)(v >> 32);
}

__device__ inline int big_bitlen(const Big& a) {
    for (int i = kBigL - 1; i >= 0; i--)
        if (a.d[i]) return 32 * i + 32 - __clz((int)a.d[i]);
    return 0;
}

__device__ inline int mag_cmp(const Big& a, const Big& b) {
    for (int i = kBigL - 1; i >= 0; i--)
        if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
    return 0;
}

// |r| = |a| + |b|
__device__ inline void mag_add(Big& r, const Big& a, const Big& b) {
    uint64_t c = 0;
    for (int i = 0; i < kBigL; i++) {
        c += (uint64_t)a.d[i] + b.d[i];
        r.d[i] = (uint32_t)c;
        c >>= 32;
    }
}

// |r| = |a| - |b|, |a| >= |b|
__device__ inline void mag_sub(Big& r, const Big& a, const Big& b) {
    int64_t br = 0;
    for (int i = 0; i < kBigL; i++) {
        int64_t s = (int64_t)a.d[i] - b.d[i] - br;
        br = s < 0;
        r.d[i] = (uint32_t)(s + (br ? ((int64_t)1 << 32) : 0));
    }
}

__device__ inline void big_fix_sign(Big& r) {
    if (big_is_zero(r)) r.neg = 0;
}

// r = a + b (signed); r may alias a or b
__device__ inline void big_add(Big& r, const Big& a, const Big& b) {
    const int an = a.neg, bn = b.neg;
    if (an == bn) {
        mag_add(r, a, b);
        r.neg = an;
    } else if (mag_cmp(a, b) >= 0) {
        mag_sub(r, a, b);
        r.neg = an;
    } else {
        mag_sub(r, b, a);
        r.neg = bn;
    }
    big_fix_sign(r);
}

__device__ inline void big_sub(Big& r, const Big& a, const Big& b) {
    Big nb = b;
    nb.neg = big_is_zero(b) ? 0 : !b.neg;
    big_add(r, a, nb);
}

// r = a * b (signed, truncated to kBigL limbs; callers stay in range)
__device__ inline void big_mul(Big& r, const Big& a, const Big& b) {
    int la = kBigL, lb = kBigL;
    while (la > 0 && a.d[la - 1] == 0) la--;
    while (lb > 0 && b.d[lb - 1] == 0) lb--;
    Big t;
    big_zero(t);
    for (int i = 0; i < la; i++) {
        uint64_t c = 0;
        const uint64_t ai = a.d[i];
        for (int j = 0; j < lb && i + j < kBigL; j++) {
            c += ai * b.d[j] + t.d[i + j];
            t.d[i + j] = (uint32_t)c;
            c >>= 32;
        }
        for (int k = i + lb; c && k < kBigL; k++) {
            c += t.d[k];
            t.d[k] = (uint32_t)c;
            c >>= 32;
        }
    }
    t.neg = a.neg ^ b.neg;
    big_fix_sign(t);
    r = t;
}

__device__ inline void big_mul_u64(Big& r, const Big& a, uint64_t m) {
    Big b;
    big_set_u64(b, m);
    big_mul(r, a, b);
}

// r = a * 2^s (magnitude shift, sign kept)
__device__ inline void big_shl(Big& r, const Big& a, int s) {
    Big t;
    big_zero(t);
    const int ws = s >> 5, bs = s & 31;
    for (int i = kBigL - 1; i >= ws; i--) {
        uint32_t v = a.d[i - ws] << bs;
        if (bs && i - ws - 1 >= 0) v |= a.d[i - ws - 1] >> (32 - bs);
        t.d[i] = v;
    }
    t.neg = a.neg;
    big_fix_sign(t);
    r = t;
}

// magnitude >> s, and whether any bit shifted out was set
__device__ inline uint64_t big_shr_low64(const Big& a, int s, bool* sticky) {
    bool st = false;
    const int ws = s >> 5, bs = s & 31;
    for (int i = 0; i < ws && i < kBigL; i++) st |= a.d[i] != 0;
    if (bs && ws < kBigL) st |= (a.d[ws] & ((1u << bs) - 1)) != 0;
    uint64_t r = 0;
    for (int k = 0; k < 2; k++) {   // bits [s, s + 64)
        const int i = ws + k;
        if (i >= kBigL) break;
        uint64_t v = (uint64_t)a.d[i] >> bs;
        if (bs && i + 1 < kBigL) v |= ((uint64_t)a.d[i + 1] << (32 - bs)) & 0xFFFFFFFFull;
        r |= v << (32 * k);
    }
    *sticky = st;
    return r;
}

// value as a double (correct to about 2^-60 relative): estimates only
__device__ inline double big_to_double(const Big& a) {
    const int bl = big_bitlen(a);
    if (bl == 0) return 0.0;
    const int s = bl > 64 ? bl - 64 : 0;
    bool st;
    const uint64_t top = big_shr_low64(a, s, &st);
    const double v = ldexp((double)top, s);
    return a.neg ? -v : v;
}

// float32 value (finite) in units of 2^-149
__device__ inline void big_from_f32(Big& a, uint32_t bits) {
    big_zero(a);
    const uint32_t e = (bits >> 23) & 0xFFu;
    const uint64_t m = (bits & 0x7FFFFFu) | (e ? 0x800000u : 0u);
    if (m == 0) return;
    const int off = (e ? (int)e : 1) - 1;
    const uint64_t v = m << (off & 31);
    const int li = off >> 5;
    a.d[li] = (uint32_t)v;
    if (li + 1 < kBigL) a.d[li + 1] = (uint32_t)(v >> 32);
    a.neg = (int)(bits >> 31);
}

// num * 2^-149 / den rounded to float32 in `mode`
__device__ inline float big_round_ratio_f32(const Big& num, uint32_t den, int mode) {
    if (big_is_zero(num)) return 0.0f;
    const bool neg = num.neg;
    const int bl = big_bitlen(num), bn = bitlen_u64(den);
    const int g = 27 + bn - bl;
    uint64_t NN;
    bool sticky = false;
    if (g >= 0) {
        bool st;
        NN = big_shr_low64(num, 0, &st) << g;   // bl <= 27 + bn <= 59 bits
    } else {
        NN = big_shr_low64(num, -g, &sticky);
    }
    const uint64_t q = NN / den;
    sticky |= (NN - q * den) != 0;
    const int e = -149;
    const int bq = bitlen_u64(q) - 1;
    const int E = bq + e - g;
    const int sp = (E > -126 ? E : -126) - 23;
    const int drop = sp - (e - g);
    const uint64_t qr = round_drop(q, drop, sticky, mode, neg);
    const float f = f32_from_scaled(qr, sp);
    return neg ? -f : f;
}

// Per-thread accumulators of float32 values in units of 2^-149: u64 "limb
// counters", each collecting 32-bit chunks of bits [32 i, 32 i + 32), so no
// carry is propagated per sample.  kAccS limbs for values, kAccQ for squares.
constexpr int kAccS = 10;   // 277-bit values, chunks up to limb 9
constexpr int kAccQ = 19;   // 554-bit squares, chunks up to limb 18

__device__ inline void acc_add_f32(uint64_t* pos, uint64_t* negv, uint64_t* sq, uint32_t bits) {
    const uint32_t e = (bits >> 23) & 0xFFu;
    const uint64_t m = (bits & 0x7FFFFFu) | (e ? 0x800000u : 0u);
    if (m == 0) return;
    const int off = (e ? (int)e : 1) - 1;
    uint64_t* s = (bits >> 31) ? negv : pos;
    const uint64_t v = m << (off & 31);
    s[off >> 5] += (uint32_t)v;
    s[(off >> 5) + 1] += v >> 32;
    const int off2 = 2 * off;
    const uint64_t m2 = m * m;   // < 2^48
    const int li = off2 >> 5, sh = off2 & 31;
    const uint64_t lo = m2 << sh;                         // bits [0, 64) of m2 << sh
    const uint64_t hi = sh ? (m2 >> (64 - sh)) : 0;      // bits [64, 80)
    sq[li] += (uint32_t)lo;
    sq[li + 1] += lo >> 32;
    sq[li + 2] += hi;
}

// counters (u64 per 32-bit limb, each below 2^63) to a Big magnitude
__device__ inline void big_from_counters(Big& r, const uint64_t* cnt, int n) {
    big_zero(r);
    u128 c = 0;
    for (int i = 0; i < kBigL; i++) {
        if (i < n) c += cnt[i];
        r.d[i] = (uint32_t)c;
        c >>= 32;
    }
}

// M * (n*a - S)^2 <= k^2 * R, with a = v * 2^149 (k != 0, mode != 2)
__device__ inline bool big_pass(uint32_t vbits, const Big& S, uint32_t n, uint32_t M, const Big& R,
                                const KExact& kx) {
    Big a, t;
    big_from_f32(a, vbits);
    big_mul_u64(t, a, n);
    big_sub(t, t, S);
    if (kx.k == 0.0) return big_is_zero(t);
    if (big_is_zero(t)) return true;
    Big lhs, rhs, mk2;
    big_mul(lhs, t, t);
    big_mul_u64(lhs, lhs, M);
    big_zero(mk2);
    mk2.d[0] = (uint32_t)kx.mk2_lo;
    mk2.d[1] = (uint32_t)(kx.mk2_lo >> 32);
    mk2.d[2] = (uint32_t)kx.mk2_hi;
    mk2.d[3] = (uint32_t)(kx.mk2_hi >> 32);
    big_mul(rhs, mk2, R);
    if (big_is_zero(rhs)) return false;
    // compare lhs * 2^ls <= rhs * 2^rs
    const int ls = kx.ek < 0 ? -2 * kx.ek : 0, rs = kx.ek > 0 ? 2 * kx.ek : 0;
    const int lb = big_bitlen(lhs) + ls, rb = big_bitlen(rhs) + rs;
    if (lb > rb) return false;
    if (lb < rb) return true;
    if (ls) big_shl(lhs, lhs, ls);
    if (rs) big_shl(rhs, rhs, rs);
    return mag_cmp(lhs, rhs) <= 0;
}

// Cut thresholds of one row (TD: M = 1, R = D, n = T, S = S1) or one bin (FD:
// M = C, R = sum of Z^2 over the time sample, n = B, S = S_b): the float32 values
// that pass are exactly those in [*lo, *hi] (empty when *lo > *hi).  The
// passing set is an interval around S/n; its ends are located from an FP64
// estimate and settled with the exact test.
__device__ inline void big_thresholds(const Big& S, uint32_t n, uint32_t M, const Big& R, const KExact& kx,
                                      float* lo, float* hi) {
    const float inf = __builtin_inff();
    if (kx.mode == 2) {
        *lo = -inf;
        *hi = inf;
        return;
    }
    const float c = big_round_ratio_f32(S, n, kRN);
    const uint32_t kc = f32_key(f32_bits(c));
    auto pass = [&](uint32_t key) { return big_pass(key_f32(key), S, n, M, R, kx); };
    if (!pass(kc)) {
        *lo = inf;
        *hi = -inf;
        return;
    }
    const double mu = ldexp(big_to_double(S), -149) / n;
    const double hw = kx.k * sqrt(big_to_double(R) / (double)M) / n * 0x1p-149;
    const uint32_t kmax = f32_key(0x7F7FFFFFu), kmin = f32_key(0xFF7FFFFFu);
    // upper end: largest passing key in [kc, kmax]
    {
        uint32_t good = kc, bad = 0;   // bad == 0: none known
        float e = (float)(mu + hw);
        uint32_t ke = (e == e) ? f32_key(f32_bits(e)) : kmax;
        if (e >= 3.0e38f) ke = kmax;
        if (ke > good) {
            if (pass(ke)) good = ke; else bad = ke;
        }
        if (bad == 0) {   // gallop up from good
            uint64_t step = 1;
            while (true) {
                if (good == kmax) break;
                const uint32_t nk = (uint64_t)(kmax - good) < step ? kmax : (uint32_t)(good + step);
                if (pass(nk)) {
                    good = nk;
                    step <<= 1;
                } else {
                    bad = nk;
                    break;
                }
            }
        } else {          // gallop down from bad towards good
            uint64_t step = 1;
            while (bad - good > 1) {
                const uint32_t nk = (uint64_t)(bad - good) <= step ? good : (uint32_t)(bad - step);
                if (nk == good) break;
                if (pass(nk)) {
                    good = nk;
                    break;
                }
                bad = nk;
                step <<= 1;
            }
        }
        while (bad != 0 && bad - good > 1) {
            const uint32_t mid = good + (bad - good) / 2;
            if (pass(mid)) good = mid; else bad = mid;
        }
        *hi = (bad == 0 && good == kmax) ? inf : __uint_as_float(key_f32(good));
    }
    // lower end: smallest passing key in [kmin, kc]
    {
        uint32_t good = kc, bad = 0xFFFFFFFFu;   // none known
        float e = (float)(mu - hw);
        uint32_t ke = (e == e) ? f32_key(f32_bits(e)) : kmin;
        if (e <= -3.0e38f) ke = kmin;
        if (ke < good) {
            if (pass(ke)) good = ke; else bad = ke;
        }
        if (bad == 0xFFFFFFFFu) {
            uint64_t step = 1;
            while (true) {
                if (good == kmin) break;
                const uint32_t nk = (uint64_t)(good - kmin) < step ? kmin : (uint32_t)(good - step);
                if (pass(nk)) {
                    good = nk;
                    step <<= 1;
                } else {
                    bad = nk;
                    break;
                }
            }
        } else {
            uint64_t step = 1;
            while (good - bad > 1) {
                const uint32_t nk = (uint64_t)(good - bad) <= step ? good : (uint32_t)(bad + step);
                if (nk == good) break;
                if (pass(nk)) {
                    good = nk;
                    break;
                }
                bad = nk;
                step <<= 1;
            }
        }
        while (bad != 0xFFFFFFFFu && good - bad > 1) {
            const uint32_t mid = bad + (good - bad) / 2;
            if (pass(mid)) good = mid; else bad = mid;
        }
        *lo = (bad == 0xFFFFFFFFu && good == kmin) ? -inf : __uint_as_float(key_f32(good));
    }
}

}  // namespace rfim
