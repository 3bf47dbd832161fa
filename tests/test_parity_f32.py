"""GPU parity of the float32 path against the CPU oracle: outputs (bit
patterns) and flag bits must be identical.  Covers the register-resident TD
kernel, the fused TD-apply + FD kernel with every fast bin size, and the wide
fallback kernels (rows / time samples whose values span more than the fast
window, replacement values below it, bins the fast path does not take)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rf():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    import paper_2001_03389_amd as m
    m.lib()  # fails loudly when the HIP library is missing
    return m


def gpu_run(rf, beams, steps, *, flags=True, inplace=False, nsamp=None, plan=False):
    import torch
    dev = torch.device("cuda:0")
    ins = [torch.from_numpy(np.ascontiguousarray(b)).to(dev) for b in beams]
    outs = ins if inplace else [torch.full_like(x, 1234.5 if x.dtype == torch.float32 else 90) for x in ins]
    fls = [torch.full(x.shape, 0xA5, dtype=torch.uint8, device=dev) for x in ins] if flags else None
    if plan:
        p = rf.Plan(ins, steps, outputs=outs, flags=fls, nsamp=nsamp)
        rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls, nsamp=nsamp, plan=p)
        torch.cuda.synchronize()
        counts = p.flag_counts()
        p.close()
    else:
        rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls, nsamp=nsamp)
        torch.cuda.synchronize()
        counts = None
    o = [x.cpu().numpy() for x in outs]
    f = [x.cpu().numpy() for x in fls] if flags else None
    return o, f, counts


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def check_against_oracle(beams, steps, out, fl, nsamp=None, counts=None):
    for i, b in enumerate(beams):
        T = b.shape[1] if nsamp is None else (nsamp[i] if isinstance(nsamp, list) else nsamp)
        want, wf = oracle.pipeline(b, steps, want_flags=True, nsamp=T)
        got = out[i][:, :T]
        bad = bits(got) != bits(want[:, :T])
        if bad.any():
            r, c = np.argwhere(bad)[0]
            raise AssertionError(f"beam {i}: {int(bad.sum())} outputs differ, first at ({r},{c}): "
                                 f"got {got[r, c]!r} want {want[r, c]!r}")
        if fl is not None:
            np.testing.assert_array_equal(fl[i][:, :T], wf[:, :T], err_msg=f"beam {i} flags")
            if T < b.shape[1]:
                assert (fl[i][:, T:] == 0xA5).all(), "flags written past nsamp"
        if counts is not None:
            for j in range(min(len(steps), 8)):
                assert counts[i][j] == int(((wf[:, :T] >> j) & 1).sum()), (i, j)


def rand_steps(rng, C, n):
    divs = [d for d in range(1, C + 1) if C % d == 0]
    out = []
    for _ in range(n):
        dom = "td" if rng.random() < 0.5 else "fd"
        k = float(rng.choice([0.0, 0.5, 1.0, 1.5, 2.0, 2.75, 3.25, 4.0, rng.uniform(0.2, 3.5)]))
        rep = "mean" if rng.random() < 0.6 else "median"
        fast = [d for d in divs if d in (8, 16, 32, 64)]
        if dom == "fd" and fast and rng.random() < 0.7:
            B = int(rng.choice(fast))
        else:
            B = int(rng.choice(divs))
        out.append((dom, k, rep, B if dom == "fd" else 0))
    return out


def rand_values(rng, C, stride, kind):
    if kind == 0:
        return rng.standard_normal((C, stride))
    if kind == 1:      # bandpass-like: per-channel offsets and widths
        return rng.normal(50, 3, (C, 1)) + rng.normal(0, 1, (C, stride)) * rng.uniform(0.5, 4, (C, 1))
    if kind == 2:      # small integers as floats (many exact ties)
        return rng.integers(-3, 4, (C, stride)).astype(np.float64)
    if kind == 3:      # wide dynamic range: the wide kernels
        return rng.standard_normal((C, stride)) * np.exp2(rng.integers(-40, 40, (C, stride)))
    x = rng.standard_normal((C, stride))  # N(0,1) with sprinkled zeros, -0, tiny values
    m = rng.random((C, stride))
    x[m < 0.02] = 0.0
    x[(m >= 0.02) & (m < 0.03)] = -0.0
    x[(m >= 0.03) & (m < 0.032)] = 1e-30
    return x


@pytest.mark.parametrize("seed", range(24))
def test_random_small_beams_f32(rf, seed):
    """Several float32 beams per call, ragged tiles, padded strides, random
    step lists over fast and wide bin sizes, flags on."""
    rng = np.random.default_rng(900 + seed)
    C = int(rng.choice([1, 3, 8, 16, 32, 64, 96, 128, 256, 384]))
    steps = rand_steps(rng, C, int(rng.integers(1, 6)))
    beams, nsamp = [], []
    for _ in range(int(rng.integers(1, 4))):
        T = int(rng.choice([1, 3, 5, 17, 64, 100, 257, 1000, 5000]))
        stride = T + int(rng.choice([0, 0, 1, 3, 8]))
        x = rand_values(rng, C, stride, int(rng.integers(0, 5)))
        beams.append(x.astype(np.float32))
        nsamp.append(T)
    say(f"seed={seed} C={C} shapes={[b.shape for b in beams]} nsamp={nsamp} steps={steps}")
    out, fl, _ = gpu_run(rf, beams, steps, nsamp=nsamp)
    check_against_oracle(beams, steps, out, fl, nsamp=nsamp)


@pytest.mark.parametrize("case", ["constant", "zeros", "signed-zeros", "denormals", "huge", "tiny-and-huge",
                                  "k0", "khuge", "t1", "c1", "tie-k4-n17", "single-spike",
                                  "tiny-mean", "td-only", "fd-only-wide-bin"])
def test_edge_cases_f32(rf, case):
    rng = np.random.default_rng(11)
    steps = [synth.td(3.25), synth.td(3.25, "median"), synth.fd(2.75, 32), synth.fd(2.0, 32, "median")]
    C, T = 64, 300
    if case == "constant":
        x = np.full((C, T), 0.1, np.float32)
    elif case == "zeros":
        x = np.zeros((C, T), np.float32)
    elif case == "signed-zeros":
        x = np.where(rng.random((C, T)) < 0.5, -0.0, 0.0).astype(np.float32)
        x[5, 7] = 1.0
    elif case == "denormals":
        x = (rng.integers(-50, 50, (C, T)) * np.float32(1e-45)).astype(np.float32)
        x[3, 3] = np.float32(3e-40)
    elif case == "huge":
        x = (rng.standard_normal((C, T)) * 1e37).astype(np.float32)
        x[0, 0] = np.float32(3.4e38)
        x[1, 1] = np.float32(-3.4e38)
    elif case == "tiny-and-huge":
        x = rng.standard_normal((C, T)).astype(np.float32)
        x[:, ::7] *= np.float32(1e-20)
        x[::5, 3] = np.float32(1e20)
    elif case == "k0":
        x = rng.standard_normal((C, T)).astype(np.float32)
        steps = [synth.td(0.0), synth.fd(0.0, 32), synth.td(0.0, "median"), synth.fd(0.0, 8, "median")]
    elif case == "khuge":
        x = rng.standard_normal((C, T)).astype(np.float32)
        steps = [synth.td(1e9), synth.fd(3e6, 32), synth.td(2.0 ** 20), synth.fd(2.0 ** -70, 16)]
    elif case == "t1":
        x = rng.standard_normal((C, 1)).astype(np.float32)
    elif case == "c1":
        x = rng.standard_normal((1, T)).astype(np.float32)
        steps = [synth.td(1.0), synth.fd(1.0, 1), synth.fd(0.0, 0)]
    elif case == "tie-k4-n17":
        # |x - mu| == 4 sigma exactly for the single non-zero value of a row of 17
        # (population sigma): an exact tie, not an outlier
        x = np.zeros((8, 17), np.float32)
        x[:, 5] = np.float32(0.375)
        steps = [synth.td(4.0), synth.td(4.0, "median")]
    elif case == "single-spike":
        x = np.zeros((C, T), np.float32)
        x[3, 100] = np.float32(255.0)
    elif case == "tiny-mean":
        # means far below the largest value: replacements below the fast window
        x = rng.standard_normal((C, T)).astype(np.float32)
        x[:, 0] = np.float32(1e12)
        x[:, 1] = np.float32(-1e12)
    elif case == "td-only":
        x = rng.standard_normal((C, T)).astype(np.float32)
        steps = [synth.td(3.0), synth.td(2.5, "median"), synth.td(2.0)]
    else:
        x = rng.standard_normal((96, T)).astype(np.float32)
        steps = [synth.fd(2.5, 96), synth.fd(2.25, 48, "median"), synth.fd(2.0, 0)]
    say(f"edge {case} shape={x.shape} steps={steps}")
    out, fl, _ = gpu_run(rf, [x], steps)
    check_against_oracle([x], steps, out, fl)


def median_rows(T, rng):
    """Rows whose lower medians the value-bin select settles, or hands to the
    radix select: Gaussian, skewed, bimodal (the median between the modes),
    integers with ties far beyond a bin's capacity at the median, a majority
    of signed zeros, one huge spike, bandpass-like integer levels, all zeros
    and a constant row."""
    rows = [rng.standard_normal(T),
            rng.exponential(1.0, T),
            np.where(rng.random(T) < 0.5, -5.0, 5.0) + rng.standard_normal(T) * 0.1,
            rng.integers(0, 4, T).astype(np.float64),
            np.where(rng.random(T) < 0.5, -0.0, 0.0) + (rng.random(T) < 0.2) * rng.standard_normal(T),
            np.r_[rng.standard_normal(T - 1), 3.0e37],
            np.clip(np.round(rng.normal(80, 8, T)), 0, 255),
            rng.standard_normal(T) * 1e-3 + 7.0,
            np.zeros(T),                       # a range of width zero
            np.full(T, 3.5)]                   # one bin holding every value
    return np.stack(rows).astype(np.float32)


@pytest.mark.parametrize("T", [65536, 4099])
def test_td_median_rows_f32(rf, T):
    """Row medians at the stress row length and a ragged one, for median
    steps first and after a mean step: every output bit against the oracle."""
    x = median_rows(T, np.random.default_rng(T))
    for steps in ([synth.td(3.0, "median"), synth.td(2.5, "median"), synth.td(2.0, "median")],
                  [synth.td(3.0), synth.td(2.0, "median"), synth.td(1.5, "median")]):
        say(f"median rows T={T} steps={steps}")
        out, fl, _ = gpu_run(rf, [x], steps)
        check_against_oracle([x], steps, out, fl)


@pytest.mark.parametrize("shape", synth.UNEVEN_SHAPES, ids=[f"{c}x{t}" for c, t in synth.UNEVEN_SHAPES])
def test_uneven_shapes_f32_full(rf, shape):
    """The float32 beams of the batched uneven workload at full size, TD 3.25 +
    FD 2.75 with 32-channel bins, mean: every output and flag."""
    C, T = shape
    spec = synth.BeamSpec("f32", C, T, 3, 64 + synth.UNEVEN_SHAPES.index(shape))
    x = synth.make_beam(spec)
    say(f"uneven f32 {shape}")
    out, fl, counts = gpu_run(rf, [x], synth.STEPS_ARTS1, plan=True)
    check_against_oracle([x], synth.STEPS_ARTS1, out, fl, counts=counts)


@pytest.mark.parametrize("inplace", [False, True])
def test_stress_steps_reduced_f32(rf, inplace):
    """The stress step list (4 TD + 3 FD, median, 32-channel bins) on a
    4096-channel bursty beam with 4096 samples: every output and flag."""
    spec = synth.BeamSpec("f32", 4096, 4096, 5, 0, bursty=True, narrow_fraction=0.05)
    x = synth.make_beam(spec)
    say(f"stress reduced inplace={inplace}")
    out, fl, counts = gpu_run(rf, [x], synth.STEPS_STRESS, inplace=inplace, plan=not inplace)
    check_against_oracle([x], synth.STEPS_STRESS, out, fl, counts=counts)


def test_stress_full_size_sampled_f32(rf):
    """A full stress beam (4096 x 65536 float32): the 4 TD steps alone checked
    on sampled rows (TD is per row), the 3 FD steps alone on sampled time
    samples (FD is per time sample)."""
    spec = synth.stress16_specs(1)[0]
    x = synth.make_beam(spec)
    td_steps = [s for s in synth.STEPS_STRESS if s.domain == "td"]
    fd_steps = [s for s in synth.STEPS_STRESS if s.domain == "fd"]
    say("stress full size, TD only")
    out, fl, _ = gpu_run(rf, [x], td_steps)
    rng = np.random.default_rng(3)
    for r in rng.choice(x.shape[0], 6, replace=False):
        want, wf = oracle.pipeline(x[r:r + 1], td_steps, want_flags=True)
        np.testing.assert_array_equal(bits(out[0][r:r + 1]), bits(want), err_msg=f"row {r}")
        np.testing.assert_array_equal(fl[0][r:r + 1], wf, err_msg=f"row {r} flags")
    say("stress full size, FD only")
    out, fl, _ = gpu_run(rf, [x], fd_steps)
    for t in rng.choice(x.shape[1], 64, replace=False):
        col = np.ascontiguousarray(x[:, t:t + 1])
        want, wf = oracle.pipeline(col, fd_steps, want_flags=True)
        np.testing.assert_array_equal(bits(out[0][:, t:t + 1]), bits(want), err_msg=f"sample {t}")
        np.testing.assert_array_equal(fl[0][:, t:t + 1], wf, err_msg=f"sample {t} flags")


def test_mixed_dtype_batch_matches_single_calls(rf):
    """uint8 and float32 beams of different shapes in one call give the same
    bytes as one beam per call."""
    rng = np.random.default_rng(21)
    beams = [rng.normal(80, 10, (128, 1000)).clip(0, 255).astype(np.uint8),
             rng.standard_normal((256, 777)).astype(np.float32),
             rng.normal(60, 8, (64, 3000)).clip(0, 255).astype(np.uint8),
             (rng.standard_normal((96, 2048)) * 3).astype(np.float32)]
    steps = [synth.td(3.0), synth.td(2.5, "median"), synth.fd(2.5, 32), synth.fd(2.25, 32, "median")]
    out, fl, _ = gpu_run(rf, beams, steps)
    for i, b in enumerate(beams):
        o1, f1, _ = gpu_run(rf, [b], steps)
        np.testing.assert_array_equal(out[i].view(np.uint8), o1[0].view(np.uint8), err_msg=f"beam {i}")
        np.testing.assert_array_equal(fl[i], f1[0], err_msg=f"beam {i} flags")
    check_against_oracle([beams[1], beams[3]], steps, [out[1], out[3]], [fl[1], fl[3]])


@pytest.mark.parametrize("case", ["td-tiny", "fd-tiny", "both-tiny", "tiny-and-wide", "tiny-mean-rows",
                                  "long-rows-tiny"])
def test_second_window_paths_f32(rf, case):
    """Rows and time samples with a few values 2^24..2^48 below their largest
    (the two-window kernels), mixed with values further down (wide kernels)."""
    rng = np.random.default_rng(77)
    C, T = 128, 2000
    x = rng.standard_normal((C, T))
    if case in ("td-tiny", "both-tiny", "tiny-and-wide"):
        m = rng.random((C, T)) < 0.002
        x[m] *= 2.0 ** -30
    if case in ("fd-tiny", "both-tiny"):
        cols = rng.choice(T, 40, replace=False)
        x[rng.integers(0, C, 40), cols] *= 2.0 ** -35
    if case == "tiny-and-wide":
        x[rng.random((C, T)) < 0.0005] *= 2.0 ** -70
    if case == "tiny-mean-rows":
        x *= 1e-6
        x[:, 0] = 8.0
        x[:, 1] = -8.0
    if case == "long-rows-tiny":
        C, T = 32, 40000
        x = rng.standard_normal((C, T))
        x[rng.random((C, T)) < 0.0005] *= 2.0 ** -33
    x = x.astype(np.float32)
    for steps in ([synth.td(3.25), synth.td(3.0, "median"), synth.fd(2.75, 32), synth.fd(2.5, 32, "median")],
                  [synth.td(2.5, "median"), synth.fd(2.25, 16), synth.fd(2.0, 16, "median")]):
        say(f"second window {case} {x.shape} steps={steps}")
        out, fl, counts = gpu_run(rf, [x], steps, plan=True)
        check_against_oracle([x], steps, out, fl, counts=counts)
