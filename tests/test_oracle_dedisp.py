"""Pins of the oracle's dedispersion and detection statistics (Eq. 2; the
dedispersed pulse of Section V-A, Fig. 6), CPU only: exact rational delays,
an independent numpy form of the sum, closed forms and invariants."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

F_LOW, TSAMP = 1220.0, 81.92e-6


def exact_delays(nchan, f_low, bw, tsamp, dms):
    """Eq. 2 evaluated in exact rationals from the binary values of the inputs:
    k_DM * DM * (f_c^-2 - f_top^-2) / tsamp, f_c = f_low + (c + 1/2) bw,
    rounded to the nearest integer, ties to even.  Also returns the distance of
    each exact value from the nearest rounding tie."""
    kdm = Fraction(4150)
    fl, b, ts = Fraction(f_low), Fraction(bw), Fraction(tsamp)
    ftop = fl + (Fraction(nchan - 1) + Fraction(1, 2)) * b
    out = np.zeros((len(dms), nchan), dtype=np.int64)
    tie = np.zeros((len(dms), nchan))
    for d, dm in enumerate(dms):
        for c in range(nchan):
            f = fl + (Fraction(c) + Fraction(1, 2)) * b
            v = kdm * Fraction(dm) * (1 / (f * f) - 1 / (ftop * ftop)) / ts
            out[d, c] = round(v)          # Fraction rounds half to even
            tie[d, c] = abs(float(v - int(v)) - 0.5)
    return out, tie


@pytest.mark.parametrize("nchan,bw", [(64, 300.0 / 64), (96, 300.0 / 96), (17, 1.5)])
def test_delays_match_exact_rationals(nchan, bw):
    dms = [0.0, 0.5, 12.25, 100.0, 499.75, 500.0, 1000.0]
    got = oracle.dedisp_delays(nchan, F_LOW, bw, TSAMP, dms)
    want, tie = exact_delays(nchan, F_LOW, bw, TSAMP, dms)
    ok = tie > 1e-9          # FP64 evaluation can only differ next to a rounding tie
    assert ok.mean() > 0.99
    np.testing.assert_array_equal(got[ok], want[ok])


def test_delay_of_the_band_at_dm500():
    """1536 channels over 1220-1520 MHz at 81.92 us: the lowest channel centre
    (1220.09765625 MHz) trails the highest (1519.90234375 MHz) by
    4150 * 500 * (f_lo^-2 - f_hi^-2) = 0.49568... s = 6050.8 samples -> 6051;
    the top channel has no delay and delays fall with frequency."""
    d = oracle.dedisp_delays(1536, F_LOW, 300.0 / 1536, TSAMP, [500.0])[0]
    assert d[0] == 6051 and d[-1] == 0
    assert np.all(np.diff(d) <= 0)
    assert oracle.dedisp_delays(1536, F_LOW, 300.0 / 1536, TSAMP, [0.0]).max() == 0


def numpy_dedisperse(x, delays, nout):
    """Different form: one vectorised shifted row slice added per channel."""
    acc = np.zeros((delays.shape[0], nout), dtype=np.int64 if x.dtype == np.uint8 else np.float64)
    for d in range(delays.shape[0]):
        for c in range(x.shape[0]):
            acc[d] += x[c, delays[d, c]:delays[d, c] + nout].astype(acc.dtype)
    return acc


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_dedisperse_matches_numpy_form(dtype):
    rng = np.random.default_rng(5)
    C, T = 48, 900
    x = (rng.integers(0, 256, size=(C, T), dtype=np.uint8) if dtype == "u8"
         else rng.standard_normal((C, T)).astype(np.float32))
    dms = [0.0, 7.0, 30.0, 61.5]
    dl = oracle.dedisp_delays(C, F_LOW, 300.0 / C, TSAMP, dms)
    got = oracle.dedisperse(x, dl)
    nout = T - dl.max()
    assert got.shape == (4, nout)
    want = numpy_dedisperse(x, dl, nout)
    np.testing.assert_array_equal(got, want)      # same channel order: exact for float32 too


def test_dedisperse_zero_dm_is_column_sum_and_respects_nsamp():
    rng = np.random.default_rng(6)
    x = rng.integers(0, 256, size=(32, 600), dtype=np.uint8)
    dl = oracle.dedisp_delays(32, F_LOW, 300.0 / 32, TSAMP, [0.0])
    s = oracle.dedisperse(x, dl, nsamp=550)
    np.testing.assert_array_equal(s[0], x[:, :550].astype(np.int64).sum(axis=0))


def test_dispersed_pulse_collects_into_one_sample():
    """A one-sample pulse of height h along the Eq. 2 track of DM 300 (zero
    background) dedisperses to C*h at its arrival time at that DM, and to a
    smaller peak at other trial DMs; its SNR at the true DM is sqrt(n-1)."""
    C, T, h, t_arr = 64, 5000, 3, 700
    dms = [250.0, 300.0, 350.0]
    dl = oracle.dedisp_delays(C, F_LOW, 300.0 / C, TSAMP, dms)
    x = np.zeros((C, T), dtype=np.uint8)
    x[np.arange(C), t_arr + dl[1]] = h
    s = oracle.dedisperse(x, dl)
    n = s.shape[1]
    assert s[1, t_arr] == C * h and s[1].sum() == C * h
    assert s[0].max() < C * h and s[2].max() < C * h
    st = oracle.series_stats(s)
    assert st["peak_t"][1] == t_arr and st["peak"][1] == C * h
    assert st["snr"][1] == pytest.approx(np.sqrt(n - 1), rel=1e-12)


def test_series_stats_closed_forms_and_invariants():
    n, h = 1000, 37
    s = np.zeros((1, n), dtype=np.int64)
    s[0, 123] = h
    st = oracle.series_stats(s)
    assert st["mean"][0] == pytest.approx(h / n, rel=1e-15)
    assert st["std"][0] == pytest.approx(h * np.sqrt(n - 1) / n, rel=1e-14)
    assert st["snr"][0] == pytest.approx(np.sqrt(n - 1), rel=1e-14)
    # first index of a repeated peak; a constant series has SNR 0
    s2 = np.array([[1, 5, 2, 5, 5, 0]], dtype=np.int64)
    st2 = oracle.series_stats(s2)
    assert st2["peak_t"][0] == 1 and st2["peak"][0] == 5
    assert oracle.series_stats(np.full((1, 50), 9, dtype=np.int64))["snr"][0] == 0.0
    # SNR is invariant under shift and positive scale; float32 series agree
    rng = np.random.default_rng(8)
    v = rng.integers(0, 10000, size=(3, 777)).astype(np.int64)
    a = oracle.series_stats(v)
    b = oracle.series_stats(3 * v + 12345)
    c = oracle.series_stats(v.astype(np.float64))
    np.testing.assert_allclose(a["snr"], b["snr"], rtol=1e-12)
    np.testing.assert_allclose(a["snr"], c["snr"], rtol=1e-12)
    np.testing.assert_array_equal(a["peak_t"], c["peak_t"])
    # against numpy's own mean / population std
    np.testing.assert_allclose(a["std"], v.std(axis=1), rtol=1e-12)
    np.testing.assert_allclose(a["snr"], (v.max(axis=1) - v.mean(axis=1)) / v.std(axis=1), rtol=1e-12)


def test_mitigation_keeps_the_dm500_pulse_detectable():
    """On the 1536 x 12500 uint8 beam, TD 3.25 + FD 2.75 mitigation keeps the
    injected DM-500 pulse well above SNR 8 at DM 500 (Section V-A)."""
    x = synth.make_beam(synth.BeamSpec("u8", 1536, 12500, 1, 0))
    out, _ = oracle.pipeline(x, list(synth.STEPS_ARTS1))
    dl = oracle.dedisp_delays(1536, F_LOW, 300.0 / 1536, TSAMP, [500.0])
    st = oracle.series_stats(oracle.dedisperse(out, dl))
    t_arr = int(round(0.04 / TSAMP))     # the pulse reaches the top of the band at 0.04 s
    assert abs(int(st["peak_t"][0]) - t_arr) <= 2
    assert st["snr"][0] > 8
