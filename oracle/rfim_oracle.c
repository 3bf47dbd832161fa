/*
 * rfim_oracle.c -- reference implementation of the time- and frequency-domain
 * sigma cuts (RFIm, arXiv:2001.03389, Section IV), used ONLY as test
 * infrastructure: the tests, the smoke check and the CPU-baseline leg of the
 * benchmark call it; the product library never links or calls it.
 *
 * Plain, slow, single-threaded and exact.  Every step reads the data as it was
 * when the step started, steps run in list order, beams are independent.
 *
 *   TD step (Section IV, Fig. 2): for each channel (row) of n samples x_i,
 *     mu = S1/n, sigma^2 = D/n^2 with S1 = sum x, S2 = sum x^2, D = n*S2 - S1^2
 *     (population standard deviation); sample i is an outlier when
 *     |x_i - mu| > k*sigma, i.e. (n*x_i - S1)^2 > k^2 * D (the comparison is
 *     symmetric, Fig. 2 caption; strict '>', Section IV).  Outliers become the
 *     row's replacement value (mean rounded to the data type, or lower median).
 *
 *   FD step (Section IV, Fig. 3): for each time sample (column) of C channels,
 *     channels are grouped into bins of B consecutive channels; the bin mean
 *     m_b = S_b/B is subtracted from each channel (mean-corrected sample
 *     y_c = x_c - m_b).  The same outlier test as TD is applied to y over all C
 *     channels.  The ORIGINAL value of an outlier channel is replaced by its
 *     bin's replacement value (mean of the bin rounded to the data type, or the
 *     bin's lower median).  Here the test is run on Z_c = B*y_c = B*x_c - S_b,
 *     which is the same test (scaling by B cancels on both sides).
 *
 *   Masked TD step (a reading of the iterated cut, Sections IV and V-A): the
 *     same test, but a run of consecutive masked TD steps keeps a per-sample
 *     mask of what it has replaced, and each step's statistics, cut and
 *     replacement value use only the unmasked samples of the row.
 *
 *   Replacement (Section IV, strategy parameter): "mean" = the statistics'
 *     mean rounded to nearest, ties to even (uint8: to an integer, float32:
 *     to the nearest float32); "median" = element of rank floor((n-1)/2) in
 *     ascending order (float32: IEEE totalOrder, so -0 < +0).
 *
 * Exactness: uint8 values are integers; a float32 value is an integer multiple
 * of 2^-149, so every sum below is an exact integer in units of 2^-149 (values)
 * or 2^-298 (squares).  k is taken as the exact binary value of the double,
 * k = mk * 2^ek.  All comparisons are done on arbitrary-precision integers.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Test-only switch: a non-zero value plants one known mistake so that the
 * tests can show their pins catch it.  The default build plants nothing. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* ------------------------------------------------------------------------ */
/* Arbitrary-precision signed integers: sign + magnitude, 32-bit limbs.      */
/* ------------------------------------------------------------------------ */
#define BI_L 160 /* 5120 bits: enough for every double k and float32 input */

typedef struct {
    int neg;          /* 1 if negative (never set for zero) */
    int n;            /* limbs in use, no leading zero limbs */
    uint32_t d[BI_L]; /* little-endian limbs */
} bi;

static void bi_die(const char* why) {
    fprintf(stderr, "rfim oracle: bigint overflow (%s)\n", why);
    abort();
}

static void bi_trim(bi* a) {
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) a->neg = 0;
}

static void bi_set_u64(bi* a, uint64_t v) {
    a->neg = 0;
    a->n = 0;
    while (v) {
        a->d[a->n++] = (uint32_t)v;
        v >>= 32;
    }
}

static void bi_set_i64(bi* a, int64_t v) {
    uint64_t m = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
    bi_set_u64(a, m);
    a->neg = (v < 0) && a->n > 0;
}

static void bi_copy(bi* r, const bi* a) {
    r->neg = a->neg;
    r->n = a->n;
    memcpy(r->d, a->d, sizeof(uint32_t) * (size_t)a->n);
}


static int mag_cmp(const bi* a, const bi* b) {
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; i--)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* |r| = |a| + |b| (sign left to caller) */
static void mag_add(bi* r, const bi* a, const bi* b) {
    int n = a->n > b->n ? a->n : b->n;
    uint64_t c = 0;
    bi t;
    for (int i = 0; i < n; i++) {
        uint64_t s = c + (i < a->n ? a->d[i] : 0) + (i < b->n ? b->d[i] : 0);
        t.d[i] = (uint32_t)s;
        c = s >> 32;
    }
    if (c) {
        if (n >= BI_L) bi_die("add");
        t.d[n++] = (uint32_t)c;
    }
    t.n = n;
    t.neg = 0;
    bi_copy(r, &t);
}

/* |r| = |a| - |b|, requires |a| >= |b| */
static void mag_sub(bi* r, const bi* a, const bi* b) {
    int64_t br = 0;
    bi t;
    for (int i = 0; i < a->n; i++) {
        int64_t s = (int64_t)a->d[i] - (i < b->n ? b->d[i] : 0) - br;
        br = s < 0;
        t.d[i] = (uint32_t)(s + (br ? ((int64_t)1 << 32) : 0));
    }
    t.n = a->n;
    t.neg = 0;
    bi_trim(&t);
    bi_copy(r, &t);
}

static void bi_add(bi* r, const bi* a, const bi* b) {
    int an = a->neg, bn = b->neg;
    if (an == bn) {
        mag_add(r, a, b);
        r->neg = an;
    } else if (mag_cmp(a, b) >= 0) {
        mag_sub(r, a, b);
        r->neg = an;
    } else {
        mag_sub(r, b, a);
        r->neg = bn;
    }
    bi_trim(r);
}

static void bi_sub(bi* r, const bi* a, const bi* b) {
    bi nb;
    bi_copy(&nb, b);
    if (nb.n) nb.neg = !nb.neg;
    bi_add(r, a, &nb);
}

static void bi_mul(bi* r, const bi* a, const bi* b) {
    bi t;
    if (a->n == 0 || b->n == 0) {
        r->n = 0;
        r->neg = 0;
        return;
    }
    int n = a->n + b->n;
    if (n > BI_L) bi_die("mul");
    memset(t.d, 0, sizeof(uint32_t) * (size_t)n);
    for (int i = 0; i < a->n; i++) {
        uint64_t c = 0;
        for (int j = 0; j < b->n; j++) {
            uint64_t s = (uint64_t)a->d[i] * b->d[j] + t.d[i + j] + c;
            t.d[i + j] = (uint32_t)s;
            c = s >> 32;
        }
        t.d[i + b->n] = (uint32_t)c;
    }
    t.n = n;
    t.neg = a->neg ^ b->neg;
    bi_trim(&t);
    bi_copy(r, &t);
}

static void bi_mul_i64(bi* r, const bi* a, int64_t m) {
    bi bm;
    bi_set_i64(&bm, m);
    bi_mul(r, a, &bm);
}

/* r = a * 2^s, s >= 0 */
static void bi_shl(bi* r, const bi* a, int s) {
    if (a->n == 0) {
        r->n = 0;
        r->neg = 0;
        return;
    }
    int w = s / 32, b = s % 32;
    int n = a->n + w + 1;
    if (n > BI_L) bi_die("shl");
    bi t;
    memset(t.d, 0, sizeof(uint32_t) * (size_t)n);
    for (int i = 0; i < a->n; i++) {
        uint64_t v = (uint64_t)a->d[i] << b;
        t.d[i + w] |= (uint32_t)v;
        t.d[i + w + 1] |= (uint32_t)(v >> 32);
    }
    t.n = n;
    t.neg = a->neg;
    bi_trim(&t);
    bi_copy(r, &t);
}

/* r = floor(|a| / 2^s) with the sign of a dropped (used on non-negatives only) */
static void bi_shr_mag(bi* r, const bi* a, int s) {
    int w = s / 32, b = s % 32;
    if (w >= a->n) {
        r->n = 0;
        r->neg = 0;
        return;
    }
    bi t;
    int n = a->n - w;
    for (int i = 0; i < n; i++) {
        uint64_t lo = a->d[i + w];
        uint64_t hi = (i + w + 1 < a->n) ? a->d[i + w + 1] : 0;
        t.d[i] = (uint32_t)(((hi << 32) | lo) >> b);
    }
    t.n = n;
    t.neg = 0;
    bi_trim(&t);
    bi_copy(r, &t);
}

/* signed comparison: -1, 0, 1 */
static int bi_cmp(const bi* a, const bi* b) {
    if (a->neg != b->neg) return a->neg ? -1 : 1;
    int m = mag_cmp(a, b);
    return a->neg ? -m : m;
}

/* q = floor(|a| / d), *rem = |a| mod d, for d in [1, 2^32) */
static void bi_divmod_u32(bi* q, uint32_t* rem, const bi* a, uint32_t d) {
    bi t;
    uint64_t r = 0;
    for (int i = a->n - 1; i >= 0; i--) {
        uint64_t cur = (r << 32) | a->d[i];
        t.d[i] = (uint32_t)(cur / d);
        r = cur % d;
    }
    t.n = a->n;
    t.neg = 0;
    bi_trim(&t);
    bi_copy(q, &t);
    *rem = (uint32_t)r;
}

static int bi_bitlen(const bi* a) {
    if (a->n == 0) return 0;
    uint32_t top = a->d[a->n - 1];
    int b = 0;
    while (top) {
        b++;
        top >>= 1;
    }
    return 32 * (a->n - 1) + b;
}

static uint64_t bi_low_u64(const bi* a) {
    uint64_t v = 0;
    if (a->n > 0) v |= a->d[0];
    if (a->n > 1) v |= (uint64_t)a->d[1] << 32;
    return v;
}

/* ------------------------------------------------------------------------ */
/* The threshold k as an exact binary fraction k = mk * 2^ek.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    bi mk2; /* mk^2 */
    int ek;
} kexact;

static void k_split(kexact* kx, double k) {
    int e = 0;
    double f = frexp(k, &e); /* k = f * 2^e, f in [0.5, 1) */
    int64_t mk = (int64_t)ldexp(f, 53);
    int ek = e - 53;
    if (mk == 0) ek = 0;
    while (mk != 0 && (mk & 1) == 0) {
        mk >>= 1;
        ek++;
    }
    bi m;
    bi_set_i64(&m, mk);
    bi_mul(&kx->mk2, &m, &m);
    kx->ek = ek;
}

/* The two sides of "A > k^2 * V" brought to integers: rhs = mk^2 * V (times
 * 2^(2ek) when ek >= 0); the left side is A (times 2^(-2ek) when ek < 0). */
static void k2_times(bi* rhs, const bi* V, const kexact* kx) {
    bi_mul(rhs, V, &kx->mk2);
    if (kx->ek >= 0) bi_shl(rhs, rhs, 2 * kx->ek);
}

static int lhs_exceeds(const bi* A, const bi* rhs, const kexact* kx) {
    bi lhs;
    if (kx->ek >= 0)
        bi_copy(&lhs, A);
    else
        bi_shl(&lhs, A, -2 * kx->ek);
#if ORACLE_MUTANT == 1 /* planted: '>=' instead of '>' */
    return bi_cmp(&lhs, rhs) >= 0;
#else
    return bi_cmp(&lhs, rhs) > 0;
#endif
}

/* ------------------------------------------------------------------------ */
/* Element values as exact integers.                                         */
/* ------------------------------------------------------------------------ */
#define DT_U8 0
#define DT_F32 1
#define F32_SHIFT 149 /* a float32 is an integer multiple of 2^-149 */

/* value of element as an integer: uint8 in units of 1, float32 in 2^-149 */
static void value_int(bi* r, int dtype, const void* base, int64_t idx) {
    if (dtype == DT_U8) {
        bi_set_u64(r, ((const uint8_t*)base)[idx]);
        return;
    }
    float x = ((const float*)base)[idx];
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t e = (u >> 23) & 0xffu, m = u & 0x7fffffu;
    if (e == 0xffu) {
        fprintf(stderr, "rfim oracle: non-finite float32 input\n");
        abort();
    }
    uint64_t M = e ? (m | 0x800000u) : m;
    int sh = e ? (int)e - 1 : 0; /* x * 2^149 = M * 2^sh */
    bi_set_u64(r, M);
    bi_shl(r, r, sh);
    if ((u >> 31) && r->n) r->neg = 1;
}

/* Round the non-negative-denominator rational num/den (num in value units) to
 * the data type, nearest with ties to even, and store it at out[idx]. */
static void store_rounded(int dtype, void* out, int64_t idx, const bi* num, uint32_t den) {
    int neg = num->neg;
    bi N;
    bi_copy(&N, num);
    N.neg = 0;
    if (dtype == DT_U8) {
        bi q;
        uint32_t rem;
        bi_divmod_u32(&q, &rem, &N, den);
        uint64_t qv = bi_low_u64(&q);
        uint64_t twice = 2 * (uint64_t)rem;
#if ORACLE_MUTANT == 3 /* planted: ties round up */
        if (twice >= den) qv++;
#else
        if (twice > den || (twice == den && (qv & 1))) qv++;
#endif
        if (neg || qv > 255) {
            fprintf(stderr, "rfim oracle: uint8 mean out of range\n");
            abort();
        }
        ((uint8_t*)out)[idx] = (uint8_t)qv;
        return;
    }
    /* float32: value = N / den in units of 2^-149.  The float32 grid spacing
     * there is 2^sh units with sh = max(0, floor(log2(N/den)) - 23). */
    bi fl;
    uint32_t rem0;
    bi_divmod_u32(&fl, &rem0, &N, den);
    int b = bi_bitlen(&fl) - 1; /* floor(log2(N/den)) when N/den >= 1 */
    int sh = b - 23 > 0 ? b - 23 : 0;
    bi ns, q;
    uint32_t rem;
    bi_shr_mag(&ns, &N, sh);
    bi_divmod_u32(&q, &rem, &ns, den); /* q = floor(N / (den * 2^sh)) */
    /* exact remainder R = N - q*den*2^sh, compare 2R with den*2^sh */
    bi qd, R, twoR, step;
    bi_mul_i64(&qd, &q, (int64_t)den);
    bi_shl(&qd, &qd, sh);
    bi_sub(&R, &N, &qd);
    bi_shl(&twoR, &R, 1);
    bi_set_u64(&step, den);
    bi_shl(&step, &step, sh);
    int c = bi_cmp(&twoR, &step);
    uint64_t qv = bi_low_u64(&q); /* q < 2^25 */
    if (c > 0 || (c == 0 && (qv & 1))) qv++;
    double v = ldexp((double)qv, sh - F32_SHIFT);
    float f = (float)v; /* exact: qv * 2^sh is a float32 by construction */
    if (neg) f = -f;
    ((float*)out)[idx] = f;
}

static uint32_t f32_total_order_key(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

static int cmp_u8(const void* a, const void* b) {
    return (int)*(const uint8_t*)a - (int)*(const uint8_t*)b;
}

static int cmp_f32_total(const void* a, const void* b) {
    uint32_t ka = f32_total_order_key(*(const float*)a), kb = f32_total_order_key(*(const float*)b);
    return ka < kb ? -1 : (ka > kb);
}

/* lower median (rank floor((n-1)/2)) of n elements spaced `step` apart */
static void lower_median(int dtype, const void* base, int64_t first, int64_t step, int64_t n,
                         void* out, int64_t out_idx) {
    size_t es = dtype == DT_U8 ? 1 : 4;
    unsigned char* tmp = (unsigned char*)malloc((size_t)n * es);
    if (!tmp) abort();
    for (int64_t i = 0; i < n; i++)
        memcpy(tmp + i * es, (const unsigned char*)base + (first + i * step) * es, es);
    qsort(tmp, (size_t)n, es, dtype == DT_U8 ? cmp_u8 : cmp_f32_total);
#if ORACLE_MUTANT == 4 /* planted: upper median */
    memcpy((unsigned char*)out + out_idx * es, tmp + (n / 2) * es, es);
#else
    memcpy((unsigned char*)out + out_idx * es, tmp + ((n - 1) / 2) * es, es);
#endif
    free(tmp);
}

static void copy_elem(int dtype, void* dst, int64_t di, const void* src, int64_t si) {
    size_t es = dtype == DT_U8 ? 1 : 4;
    memcpy((unsigned char*)dst + di * es, (const unsigned char*)src + si * es, es);
}

/* ------------------------------------------------------------------------ */
/* The sigma test on a vector v[0..n) of exact integers:                     */
/* flag_i <=> (n*v_i - S1)^2 > k^2 * (n*S2 - S1^2).                          */
/* ------------------------------------------------------------------------ */
static void sigma_test(const bi* v, int64_t n, const kexact* kx, uint8_t* flagged, bi* S1_out) {
    bi S1, S2, sq, D, t;
    S1.n = S1.neg = 0;
    S2.n = S2.neg = 0;
    for (int64_t i = 0; i < n; i++) {
        bi_add(&S1, &S1, &v[i]);
        bi_mul(&sq, &v[i], &v[i]);
        bi_add(&S2, &S2, &sq);
    }
    bi_mul_i64(&D, &S2, n);
    bi_mul(&t, &S1, &S1);
    bi_sub(&D, &D, &t); /* D = n*S2 - S1^2 >= 0 */
    bi rhs;
    k2_times(&rhs, &D, kx);
    for (int64_t i = 0; i < n; i++) {
        bi dev, A;
        bi_mul_i64(&dev, &v[i], n);
        bi_sub(&dev, &dev, &S1);
        bi_mul(&A, &dev, &dev);
#if ORACLE_MUTANT == 2 /* planted: sample standard deviation (n - 1) */
        bi_mul_i64(&A, &A, n - 1);
        if (i == 0) bi_mul_i64(&rhs, &rhs, n);
#endif
        flagged[i] = (uint8_t)lhs_exceeds(&A, &rhs, kx);
    }
    if (S1_out) bi_copy(S1_out, &S1);
}

/* ------------------------------------------------------------------------ */
/* Public API                                                                */
/* ------------------------------------------------------------------------ */
#define OR_TD 0
#define OR_FD 1
#define OR_TD_MASKED 2
#define OR_MEAN 0
#define OR_MEDIAN 1

typedef struct {
    int32_t domain;  /* OR_TD / OR_FD / OR_TD_MASKED */
    int32_t replace; /* OR_MEAN / OR_MEDIAN */
    double k;
    int64_t bin_size; /* FD: channels per bin; 0 = all channels */
} or_step;

static int valid_k(double k) { return isfinite(k) && k >= 0.0; }

/* One TD step on one beam, in place.  data is [C][stride]; flags (nullable)
 * gets bit `bit` set where a sample is replaced. */
int oracle_td_step(int dtype, void* data, int64_t C, int64_t T, int64_t stride, double k,
                   int replace, uint8_t* flags, int bit) {
    if (C < 1 || T < 1 || stride < T || !valid_k(k) || T >= ((int64_t)1 << 32)) return -1;
    kexact kx;
    k_split(&kx, k);
    bi* v = (bi*)malloc(sizeof(bi) * (size_t)T);
    uint8_t* fl = (uint8_t*)malloc((size_t)T);
    unsigned char rbuf[4];
    if (!v || !fl) abort();
    for (int64_t c = 0; c < C; c++) {
        int64_t base = c * stride;
        for (int64_t t = 0; t < T; t++) value_int(&v[t], dtype, data, base + t);
        bi S1;
        sigma_test(v, T, &kx, fl, &S1);
        if (replace == OR_MEAN)
            store_rounded(dtype, rbuf, 0, &S1, (uint32_t)T);
        else
            lower_median(dtype, data, base, 1, T, rbuf, 0);
        for (int64_t t = 0; t < T; t++) {
#if ORACLE_MUTANT == 8 /* planted: the last sample of a row is never tested */
            if (t == T - 1) continue;
#endif
            if (!fl[t]) continue;
            copy_elem(dtype, data, base + t, rbuf, 0);
            if (flags) flags[base + t] |= (uint8_t)(1u << bit);
        }
    }
    free(v);
    free(fl);
    return 0;
}

/* One masked TD step on one beam, in place (a reading of the iterated TD
 * cut of Sections IV and V-A in which a sample that was cut is set aside):
 * mask is [C][T], 1 where an earlier step of the same run of masked TD steps
 * replaced the sample.  Per row, the statistics, the cut and the replacement
 * value (mean of the unmasked samples rounded to the data type, or their lower
 * median) use only the m unmasked samples; the cut samples are replaced, get
 * flag bit `bit` and join the mask.  A row with no unmasked sample is left as
 * it is. */
int oracle_td_step_masked(int dtype, void* data, int64_t C, int64_t T, int64_t stride, double k,
                          int replace, uint8_t* flags, int bit, uint8_t* mask) {
    if (C < 1 || T < 1 || stride < T || !valid_k(k) || T >= ((int64_t)1 << 32) || !mask) return -1;
    kexact kx;
    k_split(&kx, k);
    size_t es = dtype == DT_U8 ? 1 : 4;
    bi* v = (bi*)malloc(sizeof(bi) * (size_t)T);
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)T);
    unsigned char* kept = (unsigned char*)malloc((size_t)T * es);
    uint8_t* fl = (uint8_t*)malloc((size_t)T);
    unsigned char rbuf[4];
    if (!v || !idx || !kept || !fl) abort();
    for (int64_t c = 0; c < C; c++) {
        int64_t base = c * stride, m = 0;
        for (int64_t t = 0; t < T; t++) {
#if ORACLE_MUTANT != 9 /* planted: set-aside samples stay in the statistics */
            if (mask[c * T + t]) continue;
#endif
            idx[m] = t;
            value_int(&v[m], dtype, data, base + t);
            copy_elem(dtype, kept, m, data, base + t);
            m++;
        }
        if (m == 0) continue;
        bi S1;
        sigma_test(v, m, &kx, fl, &S1);
        if (replace == OR_MEAN)
            store_rounded(dtype, rbuf, 0, &S1, (uint32_t)m);
        else
            lower_median(dtype, kept, 0, 1, m, rbuf, 0);
        for (int64_t i = 0; i < m; i++) {
            if (!fl[i]) continue;
            copy_elem(dtype, data, base + idx[i], rbuf, 0);
            mask[c * T + idx[i]] = 1;
            if (flags) flags[base + idx[i]] |= (uint8_t)(1u << bit);
        }
    }
    free(v);
    free(idx);
    free(kept);
    free(fl);
    return 0;
}

/* One FD step on one beam, in place. */
int oracle_fd_step(int dtype, void* data, int64_t C, int64_t T, int64_t stride, double k,
                   int64_t bin_size, int replace, uint8_t* flags, int bit) {
    if (C < 1 || T < 1 || stride < T || !valid_k(k)) return -1;
    int64_t B = bin_size == 0 ? C : bin_size;
    if (B < 1 || C % B != 0 || B >= ((int64_t)1 << 32)) return -1;
    int64_t nb = C / B;
    kexact kx;
    k_split(&kx, k);
    bi* x = (bi*)malloc(sizeof(bi) * (size_t)C);
    bi* z = (bi*)malloc(sizeof(bi) * (size_t)C);
    bi* Sb = (bi*)malloc(sizeof(bi) * (size_t)nb);
    uint8_t* fl = (uint8_t*)malloc((size_t)C);
    unsigned char* rep = (unsigned char*)malloc((size_t)nb * 4);
    if (!x || !z || !Sb || !fl || !rep) abort();
    for (int64_t t = 0; t < T; t++) {
        for (int64_t c = 0; c < C; c++) value_int(&x[c], dtype, data, c * stride + t);
        for (int64_t b = 0; b < nb; b++) { /* bin sums and replacement values */
            Sb[b].n = Sb[b].neg = 0;
            for (int64_t c = b * B; c < (b + 1) * B; c++) bi_add(&Sb[b], &Sb[b], &x[c]);
            if (replace == OR_MEAN)
                store_rounded(dtype, rep, b, &Sb[b], (uint32_t)B);
            else
                lower_median(dtype, data, b * B * stride + t, stride, B, rep, b);
        }
        for (int64_t c = 0; c < C; c++) { /* Z_c = B * (x_c - S_b / B) */
            bi_mul_i64(&z[c], &x[c], B);
#if ORACLE_MUTANT == 5 /* planted: corrected with the neighbouring bin's mean */
            bi_sub(&z[c], &z[c], &Sb[(c / B + 1) % nb]);
#else
            bi_sub(&z[c], &z[c], &Sb[c / B]);
#endif
        }
#if ORACLE_MUTANT == 6 /* planted: statistics of the raw column, not the corrected one */
        sigma_test(x, C, &kx, fl, NULL);
#else
        sigma_test(z, C, &kx, fl, NULL);
#endif
        for (int64_t c = 0; c < C; c++) {
            if (!fl[c]) continue;
#if ORACLE_MUTANT == 7 /* planted: replaced with the first bin's value */
            copy_elem(dtype, data, c * stride + t, rep, 0);
#else
            copy_elem(dtype, data, c * stride + t, rep, c / B);
#endif
            if (flags) flags[c * stride + t] |= (uint8_t)(1u << bit);
        }
    }
    free(x);
    free(z);
    free(Sb);
    free(fl);
    free(rep);
    return 0;
}

/* Whole step list on one beam: out = steps(in).  in/out are [C][stride];
 * in == out is allowed.  flags (nullable, [C][stride]) receives bit j for step
 * j (only the first 8 steps are recorded). */
int oracle_pipeline(int dtype, const void* in, void* out, int64_t C, int64_t T, int64_t stride,
                    const or_step* steps, int nsteps, uint8_t* flags) {
    if (C < 1 || T < 1 || stride < T || nsteps < 0) return -1;
    if (flags && nsteps > 8) return -1;
    size_t es = dtype == DT_U8 ? 1 : 4;
    if (dtype != DT_U8 && dtype != DT_F32) return -1;
    for (int s = 0; s < nsteps; s++) {
        if (!valid_k(steps[s].k)) return -1;
        if (steps[s].domain == OR_FD) {
            int64_t B = steps[s].bin_size == 0 ? C : steps[s].bin_size;
            if (B < 1 || C % B != 0) return -1;
        } else if (steps[s].domain != OR_TD && steps[s].domain != OR_TD_MASKED) {
            return -1;
        }
    }
    /* the mask of a run of consecutive masked TD steps (cleared when a run starts) */
    uint8_t* mask = NULL;
    for (int s = 0; s < nsteps; s++)
        if (steps[s].domain == OR_TD_MASKED && !mask) {
            mask = (uint8_t*)malloc((size_t)(C * T));
            if (!mask) abort();
        }
    if (in != out)
        for (int64_t c = 0; c < C; c++)
            memcpy((unsigned char*)out + c * stride * es, (const unsigned char*)in + c * stride * es,
                   (size_t)T * es);
    if (flags)
        for (int64_t c = 0; c < C; c++) memset(flags + c * stride, 0, (size_t)T);
    int rc = 0;
    for (int s = 0; s < nsteps && !rc; s++) {
        const or_step* st = &steps[s];
        if (st->domain == OR_TD_MASKED) {
#if ORACLE_MUTANT == 10 /* planted: the mask is cleared only once, not at every run */
            if (s == 0 || (steps[s - 1].domain != OR_TD_MASKED && 0))
#else
            if (s == 0 || steps[s - 1].domain != OR_TD_MASKED)
#endif
                memset(mask, 0, (size_t)(C * T));
            rc = oracle_td_step_masked(dtype, out, C, T, stride, st->k, st->replace, flags, s, mask);
        } else if (st->domain == OR_TD) {
            rc = oracle_td_step(dtype, out, C, T, stride, st->k, st->replace, flags, s);
        } else {
            rc = oracle_fd_step(dtype, out, C, T, stride, st->k, st->bin_size, st->replace, flags, s);
        }
    }
    free(mask);
    return rc;
}

/* Helpers exposed for the pins. */

/* exact mean of n float32 values rounded to the nearest float32 (ties to
 * even): the TD mean replacement value of a row */
float oracle_mean_f32(const float* x, int64_t n) {
    bi S, v;
    S.n = S.neg = 0;
    for (int64_t i = 0; i < n; i++) {
        value_int(&v, DT_F32, x, i);
        bi_add(&S, &S, &v);
    }
    float out;
    store_rounded(DT_F32, &out, 0, &S, (uint32_t)n);
    return out;
}

/* exact mean of n uint8 values rounded to an integer, ties to even */
uint8_t oracle_mean_u8(const uint8_t* x, int64_t n) {
    bi S, v;
    S.n = S.neg = 0;
    for (int64_t i = 0; i < n; i++) {
        value_int(&v, DT_U8, x, i);
        bi_add(&S, &S, &v);
    }
    uint8_t out;
    store_rounded(DT_U8, &out, 0, &S, (uint32_t)n);
    return out;
}
