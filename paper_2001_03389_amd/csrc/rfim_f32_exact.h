// Exact arithmetic for float32 beams (device side).
//
// A float32 value is m * 2^(E - 150) with m < 2^24 an integer and E = max(e, 1)
// for the biased exponent e, so every float32 is an integer multiple of a
// power of two.  The sigma-cut statistics of Section IV (sums and sums of
// squares over a row or a time sample) are kept exactly in that fixed point:
//
//  * Window fast path.  For a row (or column) whose largest biased exponent is
//    EM, the unit u = 2^(EM - 174) makes every value with E >= EM - 24 an
//    integer a = x/u with |a| < 2^48.  Such integers are exact in FP64, as are
//    sums of up to 32 of them (below 2^53) and their squares (48 significant
//    bits).  A square d = a^2 < 2^96 is split exactly into a multiple of 2^48
//    and a remainder of at most 2^47, so 32 squares also sum exactly in two
//    FP64 accumulators.  Partial sums then move to int64 / 128-bit integers.
//  * Samples below the window (tiny but non-zero) send the row or column to
//    the wide path: big integers in units of 2^-149 (values) and 2^-298
//    (squares), which hold every float32 sum exactly.
//
// Cuts are turned into float32 thresholds.  With z the largest integer that
// passes the exact test (|n*a - S| <= z), a window value x is kept iff
// Lo <= x <= H where H = RD((S + z)*u/n) and Lo = RU((S - z)*u/n), rounded to
// float32 toward -inf / +inf.  That is exact because every value the cut is
// applied to (the data and the replacement values) is an integer in units of u;
// the kernels check that replacement values are.
#pragma once

#include "rfim_exact.h"

namespace rfim {

enum RoundMode { kRN = 0, kRD = 1, kRU = 2 };

__device__ inline int bitlen_u64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

__device__ inline uint32_t f32_bits(float f) { return __float_as_uint(f); }

// IEEE totalOrder as an unsigned key (-0 < +0), and back
__device__ inline uint32_t f32_key(uint32_t b) {
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ inline uint32_t key_f32(uint32_t k) {
    return k ^ ((uint32_t)((int32_t)~k >> 31) | 0x80000000u);
}

// biased exponent with subnormals and zero counted as 1
__device__ inline int f32_E(uint32_t b) {
    const int e = (int)((b >> 23) & 0xFFu);
    return e > 0 ? e : 1;
}

// q * 2^sp as a float (q < 2^25 and q * 2^sp a float32 or just past FLT_MAX)
__device__ inline float f32_from_scaled(uint64_t q, int sp) {
    return (float)ldexp((double)q, sp);
}

// Rounds q + frac (frac in [0,1), nonzero iff sticky) to a multiple of 2^drop
// (drop >= 1) in the given mode; neg is the sign of the represented value.
__device__ inline uint64_t round_drop(uint64_t q, int drop, bool sticky, int mode, bool neg) {
    if (drop > 63) drop = 63;
    const uint64_t qr = q >> drop;
    const uint64_t low = q & ((1ull << drop) - 1);
    bool up;
    if (mode == kRN) {
        const uint64_t half = 1ull << (drop - 1);
        up = low > half || (low == half && (sticky || (qr & 1)));
    } else {
        const bool away = (mode == kRU) != neg;   // magnitude rounds up
        up = away && (low != 0 || sticky);
    }
    return qr + (up ? 1 : 0);
}

// num * 2^e / den rounded to float32 in `mode` (den >= 1).  Exact: the quotient
// is formed to 27+ significant bits with a sticky bit, then rounded once.
__device__ inline float f32_round_ratio(i128 num, uint32_t den, int e, int mode) {
    if (num == 0) return 0.0f;
    if ((den & (den - 1)) == 0) {   // a power of two: fold it into the exponent
        e -= __ffs((int)den) - 1;
        den = 1;
    }
    const bool neg = num < 0;
    const u128 N = neg ? (u128)(-num) : (u128)num;
    const int bl = bitlen_u128(N), bn = bitlen_u64(den);
    const int g = 27 + bn - bl;  // N * 2^g / den lies in (2^26, 2^28)
    uint64_t NN;
    bool sticky = false;
    if (g >= 0) {
        NN = (uint64_t)(N << g);
    } else {
        const int s = -g;
        NN = (uint64_t)(N >> s);
        sticky = (N & ((((u128)1) << s) - 1)) != 0;
    }
    uint64_t q = NN;
    if (den != 1) {
        q = NN / den;
        sticky |= (NN - q * den) != 0;
    }
    const int bq = bitlen_u64(q) - 1;
    const int E = bq + e - g;                    // exponent of the value (unbiased)
    const int sp = (E > -126 ? E : -126) - 23;  // float32 spacing there
    const int drop = sp - (e - g);               // >= bq - 23 >= 3
    const uint64_t qr = round_drop(q, drop, sticky, mode, neg);
    const float f = f32_from_scaled(qr, sp);
    return neg ? -f : f;
}


// U512 helpers for the window decisions -------------------------------------


// k^2 * V as U512 together with a left shift to apply to the other side when
// ek < 0; returns the shift for the left-hand side.
__device__ inline int k2_times(const KExact& kx, u128 V, U512* rhs) {
    const u128 mk2 = ((u128)kx.mk2_hi << 64) | kx.mk2_lo;
    *rhs = u512_mul128(mk2, V);
    if (kx.ek >= 0) {
        *rhs = u512_shl(*rhs, 2 * kx.ek);
        return 0;
    }
    return -2 * kx.ek;
}

// a - b for a >= b
__device__ inline U512 u512_sub(const U512& a, const U512& b) {
    U512 r;
    uint64_t br = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint64_t x = a.w[i], y = b.w[i];
        const uint64_t d = x - y - br;
        br = (x < y || (x == y && br)) ? 1 : 0;
        r.w[i] = d;
    }
    return r;
}

__device__ inline double u512_to_double(const U512& a) {
    double v = 0.0;
#pragma unroll
    for (int i = 7; i >= 0; i--) v = v * 0x1p64 + (double)a.w[i];
    return v;
}

// M * z^2 for M, z below 2^128 with M * z^2 below 2^384
__device__ inline U512 mz2(u128 M, u128 z) {
    U512 z2 = u512_mul128(z, z);
    // (z^2) * M: z^2 < 2^256 as four limbs times M < 2^128
    U512 lhs = u512_from(0);
    const uint64_t m0 = (uint64_t)M, m1 = (uint64_t)(M >> 64);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const u128 p0 = (u128)z2.w[i] * m0;
        const u128 p1 = (u128)z2.w[i] * m1;
        // add p0 at limb i, p1 at limb i+1
        u128 acc = (u128)lhs.w[i] + (uint64_t)p0;
        lhs.w[i] = (uint64_t)acc;
        acc = (acc >> 64) + (u128)lhs.w[i + 1] + (uint64_t)(p0 >> 64) + (uint64_t)p1;
        lhs.w[i + 1] = (uint64_t)acc;
        acc = (acc >> 64) + (u128)lhs.w[i + 2] + (uint64_t)(p1 >> 64);
        lhs.w[i + 2] = (uint64_t)acc;
        lhs.w[i + 3] += (uint64_t)(acc >> 64);
    }
    return lhs;
}

// M * z^2 <= k^2 * R for mode-0 k, with rhs = k^2 R * 2^lsh
__device__ inline bool mz2_le_k2r(u128 M, u128 z, const U512& rhs, int lsh) {
    U512 lhs = mz2(M, z);
    if (lsh) lhs = u512_shl(lhs, lsh);
    return u512_cmp(lhs, rhs) <= 0;
}

__device__ inline double u128_to_double(u128 v) {
    return ldexp((double)(uint64_t)(v >> 64), 64) + (double)(uint64_t)v;
}

// One Newton step on an estimate z0 of the root of M z^2 = k^2 R, from the
// exact residual k^2 R - M z0^2 (rhs = k^2 R * 2^lsh): the FP64 estimate of a
// root near 2^64 is only good to about 2^11, the corrected one to a unit or
// two, which leaves the exact search a step or two.  Any z0 is acceptable
// input and any result is acceptable output: the exact search decides.
__device__ inline u128 zrefine(u128 M, u128 z0, const U512& rhs, int lsh, u128 zcap) {
    if (z0 == 0 || z0 >= zcap) return z0;
    U512 lhs = mz2(M, z0);
    if (lsh) lhs = u512_shl(lhs, lsh);
    const int c = u512_cmp(lhs, rhs);
    if (c == 0) return z0;
    const U512 d = c > 0 ? u512_sub(lhs, rhs) : u512_sub(rhs, lhs);
    const double delta = ldexp(u512_to_double(d), -lsh) / (2.0 * u128_to_double(M) * u128_to_double(z0));
    if (!(delta < 0x1p100)) return z0;
    const double fl = floor(delta);
    const u128 dz = ((u128)(uint64_t)ldexp(fl, -64) << 64) | (uint64_t)(fl - ldexp(floor(ldexp(fl, -64)), 64));
    if (c > 0) return dz >= z0 ? 0 : z0 - dz;   // z0 too large
    return zcap - z0 <= dz ? zcap : z0 + dz;    // z0 too small
}

// Largest z in [0, zcap] with M * z^2 <= k^2 * R (M >= 1).  The FP64 estimate
// k*sqrt(R/M) is confirmed or corrected with the exact test; galloping plus
// bisection bound the work when the estimate is far off.
__device__ inline u128 zmax_k2(u128 M, u128 R, const KExact& kx, u128 zcap) {
    if (kx.mode == 1) return 0;   // k^2 * R < 1 <= M * 1
    if (kx.mode == 2) return zcap;
    U512 rhs;
    const int lsh = k2_times(kx, R, &rhs);
    auto ok = [&](u128 z) { return mz2_le_k2r(M, z, rhs, lsh); };
    const double est = kx.k * sqrt((double)R / (double)M);
    u128 z;
    if (!(est < (double)zcap)) {
        z = zcap;
    } else {
        const double fl = floor(est);
        const uint64_t hi = (uint64_t)ldexp(fl, -64);
        const uint64_t lo = (uint64_t)(fl - ldexp((double)hi, 64));
        z = ((u128)hi << 64) | lo;
        if (est >= 0x1p50) z = zrefine(M, z, rhs, lsh, zcap);   // below 2^50 the estimate is within a unit
    }
    if (ok(z)) {
        // gallop up, then bisect in (z, z + step]
        u128 step = 1;
        while (z < zcap) {
            const u128 nz = zcap - z < step ? zcap : z + step;
            if (!ok(nz)) {
                u128 lo = z, hi = nz;   // ok(lo), !ok(hi)
                while (hi - lo > 1) {
                    const u128 mid = lo + (hi - lo) / 2;
                    if (ok(mid)) lo = mid; else hi = mid;
                }
                return lo;
            }
            z = nz;
            step <<= 1;
        }
        return z;
    }
    // gallop down: z fails, 0 always passes
    u128 step = 1, hi = z;
    while (true) {
        const u128 nz = hi < step ? 0 : hi - step;
        if (nz == 0 || ok(nz)) {
            u128 lo = nz;   // ok(lo) (0 passes), !ok(hi)
            while (hi - lo > 1) {
                const u128 mid = lo + (hi - lo) / 2;
                if (ok(mid)) lo = mid; else hi = mid;
            }
            return lo;
        }
        hi = nz;
        step <<= 1;
    }
}

// ---- FP64 evaluation of the cut with a certified rounding ------------------
// A window value x (an integer a in units u = 2^e) is kept iff
// |den*a - S| <= zr with zr = k*sqrt(R/M) the real cut radius, i.e. iff
// RU((S - zr)*u/den) <= x <= RD((S + zr)*u/den): for x on the u grid the
// comparison with the real bound and with the largest integer below it agree.
// These bounds (and the mean's rounding) are evaluated in FP64 with an error
// bound; when both ends of the error interval round to the same float32, that
// float32 is the exact rounding, otherwise the caller takes the exact integer
// path.  With the 2^-44 relative margin below, an FP64 evaluation is about
// 2^-21 likely to miss certification, so the exact path becomes rare.

// nearest float32 at or below / at or above d (RN conversion, then one step
// back when it landed on the wrong side; +-inf beyond the float32 range)
__device__ inline float f32_step_down(float f) {
    const uint32_t b = __float_as_uint(f);
    if (f == 0.0f) return __uint_as_float(0x80000001u);
    return __uint_as_float(f > 0.0f ? b - 1u : b + 1u);
}
__device__ inline float f32_step_up(float f) {
    const uint32_t b = __float_as_uint(f);
    if (f == 0.0f) return __uint_as_float(0x00000001u);
    return __uint_as_float(f > 0.0f ? b + 1u : b - 1u);
}
__device__ inline float f32_rd(double d) {
    const float f = (float)d;
    return (double)f > d ? f32_step_down(f) : f;
}
__device__ inline float f32_ru(double d) {
    const float f = (float)d;
    return (double)f < d ? f32_step_up(f) : f;
}

// rounding in `mode` of a real known to lie in [t - E, t + E], when both ends
// round to the same float32 (bit for bit)
__device__ inline bool f32_round_cert(double t, double E, int mode, float* out) {
    const double a = t - E, b = t + E;
    float fa, fb;
    if (mode == kRD) {
        fa = f32_rd(a);
        fb = f32_rd(b);
    } else if (mode == kRU) {
        fa = f32_ru(a);
        fb = f32_ru(b);
    } else {
        fa = (float)a;
        fb = (float)b;
    }
    *out = fa;
    return __float_as_uint(fa) == __float_as_uint(fb);
}

__device__ inline double i128_to_double(i128 v) {
    const double m = u128_to_double(v < 0 ? (u128)(-v) : (u128)v);
    return v < 0 ? -m : m;
}

// Cut interval [Lo, H] (kRU / kRD roundings of (S -+ zr) * 2^e / den) from
// Sd = S and zr = k*sqrt(R/M) in FP64 (each within a relative 2^-49 of the
// real value); false when either end is not certified.
__device__ inline bool f32_cut_fast(double Sd, double zr, double den, int e, float* H, float* Lo) {
    const double E = ldexp((fabs(Sd) + zr) / den, e) * 0x1p-44;
    const double th = ldexp((Sd + zr) / den, e), tl = ldexp((Sd - zr) / den, e);
    return f32_round_cert(th, E, kRD, H) && f32_round_cert(tl, E, kRU, Lo);
}

// RN(S * 2^e / den) to float32 from Sd = S in FP64
__device__ inline bool f32_mean_fast(double Sd, double den, int e, float* r) {
    const double E = ldexp(fabs(Sd) / den, e) * 0x1p-44;
    return f32_round_cert(ldexp(Sd / den, e), E, kRN, r);
}

// ---- wider statistics (two windows) ----------------------------------------
// A row or time sample whose values reach more than 24 exponents below its
// largest value keeps a second window 24 exponents lower (unit u1 = u / 2^24);
// combined sums are S = S0 * 2^24 + S1 and Q = Q0 * 2^48 + Q1 in units of u1
// and u1^2, which need more than 128 bits for Q and D.

__device__ inline U512 u512_add(const U512& a, const U512& b) {
    U512 r;
    u128 c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (u128)a.w[i] + b.w[i];
        r.w[i] = (uint64_t)c;
        c >>= 64;
    }
    return r;
}

// a * m, truncated to 512 bits (callers keep the product below 2^512)
__device__ inline U512 u512_mul_u128(const U512& a, u128 m) {
    const uint64_t m0 = (uint64_t)m, m1 = (uint64_t)(m >> 64);
    U512 r = u512_from(0);
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const u128 p0 = (u128)a.w[i] * m0;
        u128 acc = (u128)r.w[i] + (uint64_t)p0;
        r.w[i] = (uint64_t)acc;
        if (i + 1 < 8) {
            const u128 p1 = (u128)a.w[i] * m1;
            acc = (acc >> 64) + (u128)r.w[i + 1] + (uint64_t)(p0 >> 64) + (uint64_t)p1;
            r.w[i + 1] = (uint64_t)acc;
            if (i + 2 < 8) {
                acc = (acc >> 64) + (u128)r.w[i + 2] + (uint64_t)(p1 >> 64);
                r.w[i + 2] = (uint64_t)acc;
                if (i + 3 < 8) r.w[i + 3] += (uint64_t)(acc >> 64);
            }
        }
    }
    return r;
}


// Q0 * 2^48 + Q1 (Q0, Q1 below 2^128)
__device__ inline U512 q_combine(u128 Q0, u128 Q1) {
    U512 a = u512_shl(u512_from(Q0), 48);
    return u512_add(a, u512_from(Q1));
}

// n * Q - S^2 (>= 0 by Cauchy-Schwarz) for the combined window sums
__device__ inline U512 d_combine(uint64_t n, const U512& Q, i128 S) {
    const u128 Sa = S < 0 ? (u128)(-S) : (u128)S;
    return u512_sub(u512_mul_u128(Q, (u128)n), u512_mul128(Sa, Sa));
}

// Largest z in [0, zcap] with M * z^2 <= k^2 * R (R below 2^330, M below 2^32,
// zcap below 2^100).
__device__ inline u128 zmax_k2w(u128 M, const U512& R, const KExact& kx, u128 zcap) {
    if (kx.mode == 2) return zcap;
    if (kx.k == 0.0) return 0;
    const u128 mk2 = ((u128)kx.mk2_hi << 64) | kx.mk2_lo;
    U512 rhs = u512_mul_u128(R, mk2);
    int lsh = 0;
    if (kx.ek >= 0) rhs = u512_shl(rhs, 2 * kx.ek);
    else lsh = -2 * kx.ek;
    int rb = 0;   // bit length of k^2 R (scaled)
    for (int i = 7; i >= 0; i--)
        if (rhs.w[i]) {
            rb = 64 * i + 64 - __clzll((long long)rhs.w[i]);
            break;
        }
    auto ok = [&](u128 z) -> bool {
        if (z == 0) return true;
        // bit lengths settle most comparisons (and keep the exact one in range)
        const int lo_bits = (bitlen_u128(M) - 1) + 2 * (bitlen_u128(z) - 1) + lsh;   // lhs >= 2^lo_bits
        const int hi_bits = bitlen_u128(M) + 2 * bitlen_u128(z) + lsh;               // lhs < 2^hi_bits
        if (lo_bits >= rb) return false;
        if (hi_bits <= rb - 1) return true;
        return mz2_le_k2r(M, z, rhs, lsh);
    };
    const double est = kx.k * sqrt(u512_to_double(R) / (double)M);
    u128 z;
    if (!(est < (double)zcap)) {
        z = zcap;
    } else {
        const double fl = floor(est);
        const uint64_t hi = (uint64_t)ldexp(fl, -64);
        const uint64_t lo = (uint64_t)(fl - ldexp((double)hi, 64));
        // rb past 384 bits would take M z^2 out of mz2's range: keep the estimate
        z = ((u128)hi << 64) | lo;
        if (est >= 0x1p50 && rb < 380) z = zrefine(M, z, rhs, lsh, zcap);
    }
    if (ok(z)) {
        u128 step = 1;
        while (z < zcap) {
            const u128 nz = zcap - z < step ? zcap : z + step;
            if (!ok(nz)) {
                u128 lo = z, hi = nz;
                while (hi - lo > 1) {
                    const u128 mid = lo + (hi - lo) / 2;
                    if (ok(mid)) lo = mid; else hi = mid;
                }
                return lo;
            }
            z = nz;
            step <<= 1;
        }
        return z;
    }
    u128 step = 1, hi = z;
    while (true) {
        const u128 nz = hi < step ? 0 : hi - step;
        if (nz == 0 || ok(nz)) {
            u128 lo = nz;
            while (hi - lo > 1) {
                const u128 mid = lo + (hi - lo) / 2;
                if (ok(mid)) lo = mid; else hi = mid;
            }
            return lo;
        }
        hi = nz;
        step <<= 1;
    }
}

// Split of an exact square d = a^2 < 2^96 (an integer held in FP64) into a
// multiple of 2^48 and a remainder of magnitude at most 2^47.
__device__ inline void split_sq(double d, double* hi, double* lo) {
    const double C = 0x1p100;   // spacing of FP64 at 2^100 is 2^48
    const double h = (d + C) - C;
    *hi = h;
    *lo = d - h;
}

// Exact window statistics of up to 32 values held in FP64 as integers a:
// sum a (|.| < 2^53) and the split sum of squares.
struct WinAcc {
    double s, qh, ql;
};

__device__ inline void winacc_add(WinAcc& w, double a) {
    w.s += a;
    const double d = a * a;
    double h, l;
    split_sq(d, &h, &l);
    w.qh += h;
    w.ql += l;
}

// sum of squares of a flushed accumulator as an integer: qh is a multiple of
// 2^48 below 2^102, ql an integer of magnitude below 2^53
__device__ inline u128 winacc_q(const WinAcc& w) {
    const uint64_t h = (uint64_t)ldexp(w.qh, -48);
    const int64_t l = (int64_t)w.ql;
    return ((u128)h << 48) + (u128)(i128)l;
}

}  // namespace rfim
