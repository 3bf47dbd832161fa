"""Named synthetic workloads (shapes, dtypes, step lists) and their beams.

A step is ``(domain, k, replace, bin_size)`` with domain ``"td"`` or ``"fd"``,
replace ``"mean"`` or ``"median"`` and ``bin_size`` the number of consecutive
channels per frequency bin (0 means one bin spanning every channel).  The
thresholds are the ones the paper uses: 3.25 sigma in time and 2.75 sigma in
frequency with 32-channel bins (Fig. 5), 4.00 sigma (Fig. 7), three iterations
in production (Section V-B).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .beams import arts_beam_f32, arts_beam_u8, rng_for


@dataclasses.dataclass(frozen=True)
class Step:
    domain: str          # "td" | "fd"
    k: float
    replace: str = "mean"
    bin_size: int = 32


def td(k, replace="mean"):
    return Step("td", float(k), replace, 0)


def fd(k, bin_size=32, replace="mean"):
    return Step("fd", float(k), replace, int(bin_size))


STEPS_ARTS1 = (td(3.25), fd(2.75, 32))
STEPS_ARTS40_MEAN = (td(4.0), td(3.5), td(3.25), fd(3.0, 32), fd(2.75, 32))
STEPS_ARTS40_MEDIAN = tuple(dataclasses.replace(s, replace="median") for s in STEPS_ARTS40_MEAN)
STEPS_STRESS = (td(4.0, "median"), td(3.5, "median"), td(3.25, "median"), td(3.25, "median"),
                fd(3.0, 32, "median"), fd(2.75, 32, "median"), fd(2.75, 32, "median"))
UNEVEN_SHAPES = ((1536, 12500), (384, 25000), (4096, 8192), (768, 16384))


@dataclasses.dataclass
class BeamSpec:
    dtype: str           # "u8" | "f32"
    nchan: int
    nsamp: int
    workload_id: int
    beam_id: int
    bursty: bool = False
    narrow_fraction: float | None = None   # fraction of channels with narrow-band RFI


def make_beam(spec: BeamSpec) -> np.ndarray:
    rng = rng_for(spec.workload_id, spec.beam_id)
    n_narrow = 20 if spec.narrow_fraction is None else int(round(spec.narrow_fraction * spec.nchan))
    gen = arts_beam_u8 if spec.dtype == "u8" else arts_beam_f32
    return gen(spec.nchan, spec.nsamp, rng, n_narrow=n_narrow, bursty=spec.bursty)


def arts1_specs():
    """One ARTS-like beam, 1536 channels x 12500 samples, uint8."""
    return [BeamSpec("u8", 1536, 12500, 1, 0)]


def arts40_specs(nbeams: int = 40):
    """40 such beams with per-beam seeds."""
    return [BeamSpec("u8", 1536, 12500, 2, b) for b in range(nbeams)]


def uneven72_specs():
    """64 uint8 beams (16 per shape) and 8 float32 beams (2 per shape), shapes round-robin."""
    out = [BeamSpec("u8", c, t, 3, b) for b, (c, t) in
           ((b, UNEVEN_SHAPES[b % 4]) for b in range(64))]
    out += [BeamSpec("f32", c, t, 3, 64 + b) for b, (c, t) in
            ((b, UNEVEN_SHAPES[b % 4]) for b in range(8))]
    return out


def stress16_specs(nbeams: int = 16, nchan: int = 4096, nsamp: int = 65536):
    """float32 N(0,1) beams, 5 % of channels carrying narrow-band RFI, bursty impulses."""
    return [BeamSpec("f32", nchan, nsamp, 5, b, bursty=True, narrow_fraction=0.05)
            for b in range(nbeams)]
