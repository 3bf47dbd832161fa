/*
 * dedisp_oracle.c -- reference implementation of incoherent dedispersion and
 * the detection signal-to-noise ratio (RFIm, arXiv:2001.03389: the search
 * stage that follows RFI mitigation, Section I and Eq. 2; the dedispersed
 * pulse of Section V-A, Fig. 6), used ONLY as test infrastructure: the tests,
 * the smoke check and the CPU-baseline leg of the benchmark call it; the
 * product library never links or calls it.
 *
 * Plain, slow and single-threaded:
 *
 *   Delay (Eq. 2): a signal at frequency f arrives later than at the reference
 *     frequency f_ref by k_DM * DM * (f^-2 - f_ref^-2) seconds, k_DM = 4.15e3
 *     MHz^2 pc^-1 cm^3 s.  Channel c (0 = lowest) is centred at
 *     f_c = f_low + (c + 1/2) * bw; the reference is the top channel's centre.
 *     In samples: the delay divided by the sampling time, rounded to the
 *     nearest integer (ties to even).
 *
 *   Dedispersed series of trial DM d: D_d[t] = sum over channels c, in
 *     ascending order, of x[c][t + delay_d[c]], for t in [0, n), n = nsamp minus
 *     the largest delay of every trial.  uint8 input: exact integer sums;
 *     float32 input: the values converted to double and added in channel order.
 *
 *   Statistics of one series of n values: mean m = S1/n, population standard
 *     deviation s = sqrt(S2/n - m^2), peak = the largest value and its first
 *     index, SNR = (peak - m) / s (0 when s = 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_K_DM 4.15e3

/* delays[d * nchan + c] in samples; returns 0, or -1 for invalid arguments */
int oracle_dedisp_delays(int64_t nchan, double f_low_mhz, double chan_bw_mhz, double tsamp_s, const double* dms,
                         int32_t ndm, int32_t* delays) {
    if (nchan < 1 || ndm < 1 || !(chan_bw_mhz > 0.0) || !(f_low_mhz > 0.0) || !(tsamp_s > 0.0)) return -1;
    const double f_ref = f_low_mhz + ((double)(nchan - 1) + 0.5) * chan_bw_mhz;
    for (int32_t d = 0; d < ndm; d++) {
        if (!(dms[d] >= 0.0)) return -1;
        for (int64_t c = 0; c < nchan; c++) {
            const double f = f_low_mhz + ((double)c + 0.5) * chan_bw_mhz;
            const double seconds = ORACLE_K_DM * dms[d] * (1.0 / (f * f) - 1.0 / (f_ref * f_ref));
            const double samples = nearbyint(seconds / tsamp_s);
            if (samples < 0.0 || samples > 2147483647.0) return -1;
            delays[d * nchan + c] = (int32_t)samples;
        }
    }
    return 0;
}

/* series: int64 [ndm][nout] (dtype 0, uint8 input) or double (dtype 1,
 * float32 input); x is [nchan][stride] */
int oracle_dedisperse(int dtype, const void* x, int64_t nchan, int64_t nsamp, int64_t stride, const int32_t* delays,
                      int32_t ndm, int64_t nout, void* series) {
    if (nout < 1) return -1;
    for (int32_t d = 0; d < ndm; d++) {
        for (int64_t c = 0; c < nchan; c++)
            if ((int64_t)delays[d * nchan + c] + nout > nsamp) return -1;
        for (int64_t t = 0; t < nout; t++) {
            if (dtype == 0) {
                const uint8_t* xb = (const uint8_t*)x;
                int64_t s = 0;
                for (int64_t c = 0; c < nchan; c++) s += xb[c * stride + t + delays[d * nchan + c]];
                ((int64_t*)series)[(int64_t)d * nout + t] = s;
            } else {
                const float* xf = (const float*)x;
                double s = 0.0;
                for (int64_t c = 0; c < nchan; c++) s += (double)xf[c * stride + t + delays[d * nchan + c]];
                ((double*)series)[(int64_t)d * nout + t] = s;
            }
        }
    }
    return 0;
}

/* per series: snr, peak, peak index, mean, standard deviation.  uint8 series
 * (int64 values) use exact integer sums; float32 series long double sums. */
int oracle_series_stats(int dtype, const void* series, int32_t ndm, int64_t nout, double* snr, double* peak,
                        int64_t* peak_t, double* mean, double* stdev) {
    if (nout < 1) return -1;
    for (int32_t d = 0; d < ndm; d++) {
        long double m, var, pk;
        int64_t at = 0;
        if (dtype == 0) {
            const int64_t* s = (const int64_t*)series + (int64_t)d * nout;
            __int128 s1 = 0, s2 = 0;
            int64_t best = s[0];
            for (int64_t t = 0; t < nout; t++) {
                s1 += s[t];
                s2 += (__int128)s[t] * s[t];
                if (s[t] > best) {
                    best = s[t];
                    at = t;
                }
            }
            /* n^2 * var = n * S2 - S1^2, exact */
            const __int128 dn = (__int128)nout * s2 - s1 * s1;
            m = (long double)s1 / (long double)nout;
            var = (long double)dn / ((long double)nout * (long double)nout);
            pk = (long double)best;
        } else {
            const double* s = (const double*)series + (int64_t)d * nout;
            long double s1 = 0.0L;
            double best = s[0];
            for (int64_t t = 0; t < nout; t++) {
                s1 += s[t];
                if (s[t] > best) {
                    best = s[t];
                    at = t;
                }
            }
            m = s1 / (long double)nout;
            long double ss = 0.0L;
            for (int64_t t = 0; t < nout; t++) ss += ((long double)s[t] - m) * ((long double)s[t] - m);
            var = ss / (long double)nout;
            pk = (long double)best;
        }
        const long double sd = var > 0.0L ? sqrtl(var) : 0.0L;
        snr[d] = sd > 0.0L ? (double)((pk - m) / sd) : 0.0;
        peak[d] = (double)pk;
        peak_t[d] = at;
        mean[d] = (double)m;
        stdev[d] = (double)sd;
    }
    return 0;
}
