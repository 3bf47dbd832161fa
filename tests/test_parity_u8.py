"""GPU parity of the uint8 path against the CPU oracle: outputs and flag bits
must be bit-identical (the method is exact; see include/rfim.h)."""
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
    outs = ins if inplace else [torch.full_like(x, 0x5A) for x in ins]
    fls = [torch.full(x.shape, 0xA5, dtype=torch.uint8, device=dev) for x in ins] if flags else None
    ns = nsamp if nsamp is not None else None
    if plan:
        p = rf.Plan(ins, steps, outputs=outs, flags=fls, nsamp=ns)
        rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls, nsamp=ns, plan=p)
        torch.cuda.synchronize()
        counts = p.flag_counts()
        p.close()
    else:
        rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls, nsamp=ns)
        torch.cuda.synchronize()
        counts = None
    o = [x.cpu().numpy() for x in outs]
    f = [x.cpu().numpy() for x in fls] if flags else None
    return o, f, counts


def check_against_oracle(beams, steps, out, fl, nsamp=None, counts=None):
    for i, b in enumerate(beams):
        T = b.shape[1] if nsamp is None else (nsamp[i] if isinstance(nsamp, list) else nsamp)
        want, wf = oracle.pipeline(b, steps, want_flags=True, nsamp=T)
        np.testing.assert_array_equal(out[i][:, :T], want[:, :T], err_msg=f"beam {i} output")
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
        out.append((dom, k, rep, int(rng.choice(divs)) if dom == "fd" else 0))
    return out


@pytest.mark.parametrize("seed", range(24))
def test_random_small_beams(rf, seed):
    """Several beams of different shapes in one call, ragged time tiles,
    padded and odd row strides, random step lists, flags on."""
    rng = np.random.default_rng(700 + seed)
    C = int(rng.choice([1, 3, 4, 7, 32, 64, 96, 100]))
    steps = rand_steps(rng, C, int(rng.integers(1, 6)))
    beams, nsamp = [], []
    for _ in range(int(rng.integers(1, 4))):
        T = int(rng.choice([1, 3, 5, 17, 64, 100, 257, 1000]))
        stride = T + int(rng.choice([0, 0, 1, 3, 8]))
        kind = rng.integers(0, 3)
        if kind == 0:
            x = rng.integers(0, 256, size=(C, stride))
        elif kind == 1:
            x = rng.normal(80, 10, size=(C, stride)).clip(0, 255)
        else:
            x = rng.integers(0, 3, size=(C, stride)) * 100
        beams.append(x.astype(np.uint8))
        nsamp.append(T)
    say(f"seed={seed} C={C} shapes={[b.shape for b in beams]} nsamp={nsamp} steps={steps}")
    out, fl, _ = gpu_run(rf, beams, steps, nsamp=nsamp)
    check_against_oracle(beams, steps, out, fl, nsamp=nsamp)


@pytest.mark.parametrize("inplace", [False, True])
def test_arts1_full_beam(rf, inplace):
    """1536 x 12500 uint8 ARTS-like beam, TD 3.25 then FD 2.75 with 32-channel
    bins, mean replacement: every output byte and flag bit."""
    x = synth.make_beam(synth.arts1_specs()[0])
    say(f"arts1 inplace={inplace}")
    out, fl, counts = gpu_run(rf, [x], synth.STEPS_ARTS1, inplace=inplace, plan=not inplace)
    check_against_oracle([x], synth.STEPS_ARTS1, out, fl, counts=counts)


def test_arts1_single_bin(rf):
    """FD with one bin of all 1536 channels (no bandpass binning)."""
    x = synth.make_beam(synth.arts1_specs()[0])[:, :3000].copy()
    steps = [synth.td(3.25), synth.fd(2.75, 0)]
    say("arts1 one-bin FD")
    out, fl, _ = gpu_run(rf, [x], steps)
    check_against_oracle([x], steps, out, fl)


@pytest.mark.parametrize("steps", [synth.STEPS_ARTS40_MEAN, synth.STEPS_ARTS40_MEDIAN],
                         ids=["mean", "median"])
def test_arts40_full_size_beam(rf, steps):
    """A full-size beam of the 40-beam workload: 3 TD + 2 FD steps."""
    x = synth.make_beam(synth.arts40_specs()[3])
    say(f"arts40 beam 3 steps={steps}")
    out, fl, counts = gpu_run(rf, [x], steps, plan=True)
    check_against_oracle([x], steps, out, fl, counts=counts)


def test_arts40_batch_matches_single_calls(rf):
    """All 40 beams in one call give, beam by beam, the same bytes as one beam
    per call, and sampled beams match the oracle."""
    import torch
    specs = synth.arts40_specs()
    beams = [synth.make_beam(s) for s in specs]
    say("arts40 batch of 40")
    out, fl, _ = gpu_run(rf, beams, synth.STEPS_ARTS40_MEAN)
    for i in (0, 17, 39):
        o1, f1, _ = gpu_run(rf, [beams[i]], synth.STEPS_ARTS40_MEAN)
        np.testing.assert_array_equal(out[i], o1[0])
        np.testing.assert_array_equal(fl[i], f1[0])
    check_against_oracle([beams[39]], synth.STEPS_ARTS40_MEAN, [out[39]], [fl[39]])
    del torch


@pytest.mark.parametrize("case", ["constant", "zeros", "all255", "k0", "khuge", "t1", "c1",
                                  "two-values", "single-spike"])
def test_edge_cases(rf, case):
    rng = np.random.default_rng(5)
    steps = [synth.td(3.25), synth.td(3.25, "median"), synth.fd(2.75, 4), synth.fd(2.0, 4, "median")]
    if case == "constant":
        x = np.full((8, 300), 77, np.uint8)
    elif case == "zeros":
        x = np.zeros((8, 300), np.uint8)
    elif case == "all255":
        x = np.full((8, 300), 255, np.uint8)
    elif case == "k0":
        x = rng.integers(0, 256, size=(8, 300)).astype(np.uint8)
        steps = [synth.td(0.0), synth.fd(0.0, 4), synth.td(0.0, "median"), synth.fd(0.0, 2, "median")]
    elif case == "khuge":
        x = rng.integers(0, 256, size=(8, 300)).astype(np.uint8)
        steps = [synth.td(1e9), synth.fd(3e6, 4), synth.td(2.0 ** 20), synth.fd(2.0 ** -70, 4)]
    elif case == "t1":
        x = rng.integers(0, 256, size=(8, 1)).astype(np.uint8)
    elif case == "c1":
        x = rng.integers(0, 256, size=(1, 300)).astype(np.uint8)
        steps = [synth.td(1.0), synth.fd(1.0, 1), synth.fd(0.0, 0)]
    elif case == "two-values":
        x = (rng.integers(0, 2, size=(8, 300)) * 255).astype(np.uint8)
    else:
        x = np.zeros((8, 300), np.uint8)
        x[3, 100] = 255
    say(f"edge {case}")
    out, fl, _ = gpu_run(rf, [x], steps)
    check_against_oracle([x], steps, out, fl)


@pytest.mark.parametrize("frac", [0.0, 0.001, 0.02, 0.1, 0.3])
def test_td_iterations_with_shrinking_spread(rf, frac):
    """Rows whose spread collapses after the first cut (a fraction of samples
    at 255 over a narrow background): later TD steps cut deep inside the first
    step's interval, which the kernel must handle exactly."""
    rng = np.random.default_rng(int(frac * 1000) + 3)
    x = rng.normal(40, 3, size=(64, 12500)).clip(0, 255)
    hit = rng.random(x.shape) < frac
    x[hit] = 255
    x[::7, :] = rng.normal(90, 20, size=(10, 12500)).clip(0, 255)   # some plain wide rows
    x = x.astype(np.uint8)
    steps = [synth.td(4.0), synth.td(3.5), synth.td(3.25), synth.td(2.0), synth.fd(2.75, 32)]
    say(f"shrinking spread frac={frac}")
    out, fl, counts = gpu_run(rf, [x], steps, plan=True)
    check_against_oracle([x], steps, out, fl, counts=counts)


@pytest.mark.parametrize("seed", range(6))
def test_flag_counts_rows_across_work_groups(rf, seed):
    """Per-step flag counts with beams whose channel counts are not multiples
    of four: the TD statistics kernel sums the counts of the rows it handles
    together (up to four) before adding them to the beam's counter, so some
    groups of rows span two beams and the last one is short."""
    rng = np.random.default_rng(900 + seed)
    C = int(rng.choice([1, 3, 5, 6, 7]))
    steps = [synth.td(float(rng.choice([1.5, 2.0, 2.75]))), synth.td(2.0, "median"), synth.td(1.5),
             synth.fd(2.0, C)]
    beams = []
    for _ in range(int(rng.integers(2, 6))):
        T = int(rng.choice([64, 300, 1000, 4097]))
        beams.append(rng.normal(100, 15, size=(C, T)).clip(0, 255).astype(np.uint8))
    say(f"seed={seed} C={C} shapes={[b.shape for b in beams]} steps={steps}")
    out, fl, counts = gpu_run(rf, beams, steps, plan=True)
    check_against_oracle(beams, steps, out, fl, counts=counts)


@pytest.mark.parametrize("T", [15360, 15377, 15393, 31000, 40003])
def test_long_rows(rf, T):
    """Rows longer than one 16 KB chunk of the TD statistics pass, with odd
    row strides so that rows start at every byte offset.  Near-constant rows
    (one value in all but 0.3 % of samples), constant rows and a dense comb
    of outliers: the replacement means depend on every count being exact."""
    rng = np.random.default_rng(T)
    C = 64
    x = rng.normal(80, 10, size=(C, T + 1))
    for r in range(0, 8):                      # near-constant rows
        x[r] = 77 + (r & 1) * 100
        hit = rng.random(T + 1) < 0.003
        x[r, hit] = rng.integers(0, 256, size=int(hit.sum()))
    x[8] = 255
    x[9] = 0
    x[10, :: 5] = 250                          # a dense outlier comb
    x[11:20] += rng.normal(0, 40, size=(9, T + 1)) * (rng.random((9, T + 1)) < 0.02)
    x = x.clip(0, 255).astype(np.uint8)
    for steps in (synth.STEPS_ARTS40_MEAN, synth.STEPS_ARTS40_MEDIAN):
        say(f"long rows T={T} stride={T + 1} steps={steps}")
        out, fl, counts = gpu_run(rf, [x], steps, nsamp=[T], plan=True)
        check_against_oracle([x], steps, out, fl, nsamp=[T], counts=counts)


def test_td_and_fd_entry_points(rf):
    """rfim_td_sigma_cut and rfim_fd_sigma_cut are the one-step pipelines."""
    import torch
    x = synth.make_beam(synth.arts1_specs()[0])[:, :2000].copy()
    dev = torch.device("cuda:0")
    xi = torch.from_numpy(x).to(dev)
    o1 = torch.empty_like(xi)
    f1 = torch.zeros_like(xi)
    rf.rfim_td_sigma_cut([xi], 3.25, "median", outputs=[o1], flags=[f1])
    o2 = torch.empty_like(xi)
    f2 = torch.zeros_like(xi)
    rf.rfim_fd_sigma_cut([xi], 2.75, 32, "mean", outputs=[o2], flags=[f2])
    torch.cuda.synchronize()
    w1, wf1 = oracle.pipeline(x, [synth.td(3.25, "median")], True)
    w2, wf2 = oracle.pipeline(x, [synth.fd(2.75, 32)], True)
    np.testing.assert_array_equal(o1.cpu().numpy(), w1)
    np.testing.assert_array_equal(f1.cpu().numpy(), wf1)
    np.testing.assert_array_equal(o2.cpu().numpy(), w2)
    np.testing.assert_array_equal(f2.cpu().numpy(), wf2)


def test_interleaved_step_list(rf):
    """TD, FD, TD, FD: two runs of [TD][FD]; the second run ORs its flag bits."""
    rng = np.random.default_rng(8)
    x = rng.normal(90, 12, size=(64, 777)).clip(0, 255).astype(np.uint8)
    x[10, :] = 250
    x[:, 300:303] = 255
    steps = [synth.td(2.5), synth.fd(2.25, 16, "median"), synth.td(2.0, "median"), synth.fd(2.0, 8)]
    out, fl, _ = gpu_run(rf, [x], steps)
    check_against_oracle([x], steps, out, fl)
    out2, _, _ = gpu_run(rf, [x], steps, flags=False)
    np.testing.assert_array_equal(out2[0], out[0])


def test_flag_counts_beyond_eight_steps(rf):
    """Per-step flag counts of a 12-step list (no flag array: bits stop at 8
    steps, counts do not) on a uint8 and a float32 beam in one call.  The
    oracle runs the list one step at a time, each step on the previous one's
    output, which is the pipeline's definition."""
    import torch
    rng = np.random.default_rng(12)
    xu = rng.normal(90, 12, size=(96, 1500)).clip(0, 255).astype(np.uint8)
    xu[7, :] = 250
    xu[:, 400:402] = 255
    xf = rng.standard_normal((64, 2000)).astype(np.float32)
    xf[3] += 7.0
    steps = [synth.td(2.5), synth.fd(2.25, 16), synth.td(2.0, "median"), synth.fd(2.0, 32, "median"),
             synth.td(1.75), synth.td(1.5, "median"), synth.fd(1.75, 8), synth.fd(1.5, 0),
             synth.td(1.25), synth.fd(1.25, 16, "median"), synth.td(1.0), synth.fd(1.0, 32)]
    dev = torch.device("cuda:0")
    ins = [torch.from_numpy(xu).to(dev), torch.from_numpy(xf).to(dev)]
    outs = [torch.empty_like(x) for x in ins]
    p = rf.Plan(ins, steps, outputs=outs)
    rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=p)
    torch.cuda.synchronize()
    counts = p.flag_counts()
    p.close()
    for b, x in enumerate((xu, xf)):
        cur, want = x, []
        for st in steps:
            cur, f = oracle.pipeline(cur, [st], want_flags=True)
            want.append(int((f & 1).sum()))
        np.testing.assert_array_equal(outs[b].cpu().numpy().view(np.uint8), cur.view(np.uint8))
        assert counts[b] == want, (b, counts[b], want)
