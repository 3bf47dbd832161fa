"""Pipeline-level properties of the oracle on the synthetic ARTS-like beam
(CPU only): what Section V-A reports qualitatively for the simulated data."""
from __future__ import annotations

import math

import numpy as np
import pytest

import dedisperse as dd
import oracle
import synth


@pytest.fixture(scope="module")
def arts1():
    x, inj = synth.arts_beam_u8(1536, 12500, synth.rng_for(1, 0), with_truth=True)
    out, fl = oracle.pipeline(x, synth.STEPS_ARTS1, want_flags=True)
    return x, inj, out, fl


def test_dispersed_pulse_stays_detectable(arts1):
    """After TD 3.25 + FD 2.75 the DM-500 pulse still dedisperses above the
    detection threshold of 8 (Section V-A)."""
    x, inj, out, fl = arts1
    t0 = int(round(0.04 / synth.TSAMP_S))
    assert dd.snr(dd.dedisperse(out.astype(np.float64), 500.0), t0) >= 8.0


def test_broadband_impulses_removed_by_td(arts1):
    """TDSC targets bright broadband low-DM events: nearly every sample of the
    +8 sigma impulses is flagged by the time-domain step."""
    x, inj, out, fl = arts1
    cols = np.unique(np.concatenate([np.arange(s, min(12500, s + w))
                                     for s, w in zip(inj.impulse_starts, inj.impulse_widths)]))
    frac = (fl[:, cols] & 1).astype(bool).mean()
    assert frac > 0.95, frac


def test_narrowband_carriers_flagged_by_fd(arts1):
    """FDSC targets narrow-band RFI: the persistent carriers (+5..20 sigma of a
    single channel) are flagged by the frequency-domain step far more often than
    clean channels."""
    x, inj, out, fl = arts1
    persistent = inj.narrow_channels[:10]
    rate_rfi = (fl[persistent] & 2).astype(bool).mean()
    clean = np.setdiff1d(np.arange(1536), inj.narrow_channels)
    rate_clean = (fl[clean] & 2).astype(bool).mean()
    assert rate_rfi > 0.5 and rate_clean < 0.02, (rate_rfi, rate_clean)


def test_noise_only_left_essentially_untouched():
    """On pure noise a TD step at 3.25 sigma changes about 2*Q(3.25) = 0.115 %
    of the samples (the discretised clipped Gaussian is close to that)."""
    x = synth.arts_beam_u8(256, 12500, synth.rng_for(99, 0), n_narrow=0, n_impulse=0,
                           pulse_sigma=0.0)
    out, fl = oracle.pipeline(x, [synth.td(3.25)], want_flags=True)
    p = math.erfc(3.25 / math.sqrt(2.0))
    frac = (out != x).mean()
    assert abs(frac - p) < 0.25 * p, frac
    assert fl.astype(bool).mean() == pytest.approx(frac, rel=0.05)
