"""Test-only incoherent dedispersion and detection SNR (the search stage that
follows RFI mitigation, Section I and Eq. 2).  Used to check that mitigation
keeps an injected dispersed pulse detectable."""
from __future__ import annotations

import numpy as np

import synth


def dedisperse(x: np.ndarray, dm: float) -> np.ndarray:
    """Sum channels after shifting each one by its Eq. 2 delay relative to the
    top of the band; returns the DM time series (length T - max delay)."""
    C, T = x.shape
    f = synth.channel_freqs(C)
    delay = np.rint(synth.dispersion_delay_s(f, f[-1], dm) / synth.TSAMP_S).astype(np.int64)
    n = T - int(delay.max())
    out = np.zeros(n, dtype=np.float64)
    for c in range(C):
        out += x[c, delay[c]:delay[c] + n]
    return out


def snr(series: np.ndarray, at: int, guard: int = 3) -> float:
    """(peak near `at` - median) / robust std (from the median absolute deviation)."""
    med = np.median(series)
    mad = np.median(np.abs(series - med)) * 1.4826
    lo, hi = max(0, at - guard), min(series.size, at + guard + 1)
    return float((series[lo:hi].max() - med) / mad)
