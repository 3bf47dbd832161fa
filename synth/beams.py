"""Seeded synthetic beam generator shared by the tests and the benchmark.

This module draws random numbers and lays out arrays; it contains none of the
sigma-cut arithmetic.  It imitates the simulated set-up of the paper's accuracy
experiment (Section V-A): Gaussian noise per frequency channel, a faint
dispersed pulse, bright broadband low-DM impulses and narrow-band RFI channels,
on an ARTS-like band (300 MHz at L-band, 81.92 us sampling).  The dispersion
delay of the pulse follows Eq. 2 with the dispersion constant given there.

Layout of every beam is ``[channel][time]`` with time fastest; channel 0 is the
lowest frequency.  Seeds are ``SeedSequence([200103389, workload_id, beam_id])``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_ROOT = 200103389
K_DM = 4.15e3              # MHz^2 pc^-1 cm^3 s (Eq. 2)
F_LOW_MHZ = 1220.0
BANDWIDTH_MHZ = 300.0
TSAMP_S = 81.92e-6


def rng_for(workload_id: int, beam_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, workload_id, beam_id])))


def channel_freqs(nchan: int) -> np.ndarray:
    """Centre frequency (MHz) of each channel, channel 0 lowest."""
    return F_LOW_MHZ + (np.arange(nchan) + 0.5) * (BANDWIDTH_MHZ / nchan)


def dispersion_delay_s(freq_mhz: np.ndarray, f_ref_mhz: float, dm: float) -> np.ndarray:
    """Eq. 2: delay of frequency ``freq_mhz`` relative to ``f_ref_mhz``."""
    return K_DM * (np.asarray(freq_mhz, dtype=np.float64) ** -2 - f_ref_mhz ** -2) * dm


def pulse_track(nchan: int, nsamp: int, dm: float, t0_s: float) -> tuple[np.ndarray, np.ndarray]:
    """(channel, sample) pairs of a one-sample-wide dispersed pulse that reaches
    the top of the band at ``t0_s``; samples past the batch are dropped."""
    f = channel_freqs(nchan)
    t = t0_s + dispersion_delay_s(f, f[-1], dm)
    idx = np.rint(t / TSAMP_S).astype(np.int64)
    ch = np.arange(nchan)
    keep = (idx >= 0) & (idx < nsamp)
    return ch[keep], idx[keep]


@dataclasses.dataclass
class Injections:
    narrow_channels: np.ndarray          # channel indices carrying narrow-band RFI
    impulse_starts: np.ndarray           # start sample of each broadband impulse
    impulse_widths: np.ndarray
    pulse_channels: np.ndarray           # dispersed pulse path
    pulse_samples: np.ndarray


def _signal(nchan: int, nsamp: int, rng: np.random.Generator, *, n_narrow: int,
            n_impulse: int, impulse_sigma: float, pulse_sigma: float, dm: float,
            t0_s: float, bursty: bool) -> tuple[np.ndarray, Injections]:
    """Injected signal in units of each channel's noise sigma, float32 [C][T]."""
    sig = np.zeros((nchan, nsamp), dtype=np.float32)
    t = np.arange(nsamp, dtype=np.float64)
    n_narrow = min(n_narrow, nchan)
    narrow = rng.choice(nchan, size=n_narrow, replace=False) if n_narrow else np.zeros(0, np.int64)
    for j, c in enumerate(narrow):
        amp = rng.uniform(5.0, 20.0)
        if j < (n_narrow + 1) // 2:          # persistent carrier
            sig[c] += np.float32(amp)
        else:                                # sinusoidally modulated carrier
            period = rng.uniform(50.0, 2000.0)
            phase = rng.uniform(0.0, 2.0 * np.pi)
            sig[c] += (amp * 0.5 * (1.0 + np.sin(2.0 * np.pi * t / period + phase))).astype(np.float32)
    if bursty:
        starts, widths = [], []
        for _ in range(10):
            centre = rng.integers(0, max(1, nsamp - 200))
            for _ in range(int(rng.integers(5, 21))):
                starts.append(centre + int(rng.integers(0, 200)))
                widths.append(int(rng.integers(1, 6)))
        starts = np.asarray(starts, dtype=np.int64)
        widths = np.asarray(widths, dtype=np.int64)
    else:
        starts = rng.integers(0, nsamp, size=n_impulse).astype(np.int64)
        widths = rng.integers(1, 6, size=n_impulse).astype(np.int64)
    for s, w in zip(starts, widths):
        sig[:, s:min(nsamp, s + w)] += np.float32(impulse_sigma)
    pc, ps = pulse_track(nchan, nsamp, dm, t0_s) if pulse_sigma else (np.zeros(0, np.int64),) * 2
    sig[pc, ps] += np.float32(pulse_sigma)
    return sig, Injections(narrow, starts, widths, pc, ps)


def arts_beam_u8(nchan: int, nsamp: int, rng: np.random.Generator, *, n_narrow: int = 20,
                 n_impulse: int = 30, impulse_sigma: float = 8.0, pulse_sigma: float = 3.0,
                 dm: float = 500.0, t0_s: float = 0.04, bursty: bool = False,
                 with_truth: bool = False):
    """uint8 beam: per-channel mean ~U[60,100], std ~U[6,12], plus injections
    scaled by each channel's std, rounded and clipped to [0, 255]."""
    mu = rng.uniform(60.0, 100.0, size=(nchan, 1)).astype(np.float32)
    sd = rng.uniform(6.0, 12.0, size=(nchan, 1)).astype(np.float32)
    noise = rng.standard_normal((nchan, nsamp), dtype=np.float32)
    sig, inj = _signal(nchan, nsamp, rng, n_narrow=n_narrow, n_impulse=n_impulse,
                       impulse_sigma=impulse_sigma, pulse_sigma=pulse_sigma, dm=dm,
                       t0_s=t0_s, bursty=bursty)
    x = mu + sd * (noise + sig)
    out = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    return (out, inj) if with_truth else out


def arts_beam_f32(nchan: int, nsamp: int, rng: np.random.Generator, *, n_narrow: int = 20,
                  n_impulse: int = 30, impulse_sigma: float = 8.0, pulse_sigma: float = 3.0,
                  dm: float = 500.0, t0_s: float = 0.04, bursty: bool = False,
                  with_truth: bool = False):
    """float32 beam: N(0,1) noise plus injections in units of sigma = 1."""
    noise = rng.standard_normal((nchan, nsamp), dtype=np.float32)
    sig, inj = _signal(nchan, nsamp, rng, n_narrow=n_narrow, n_impulse=n_impulse,
                       impulse_sigma=impulse_sigma, pulse_sigma=pulse_sigma, dm=dm,
                       t0_s=t0_s, bursty=bursty)
    out = noise + sig
    return (out, inj) if with_truth else out
