"""GPU parity against the oracle for the exact calls the benchmark, the
single-beam and serve measurements time, and for every launch configuration
the planner or the auto-tuner can choose on the workloads' real shapes.

Each test runs the call the way the measurement runs it (same shapes, same
step list, flags off when the measurement has them off, a plan, the same
stream), asserts through rfim_plan_describe which tile and FD code path ran,
and compares bytes (and per-step flag counts) with the oracle.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle_pool
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
    m.lib()
    return m


def oracle_counts(flags, nsteps):
    return [int(((flags >> j) & 1).sum()) for j in range(nsteps)]


# ---------------------------------------------------------------- 40-beam call
SAMPLED = (0, 13, 26, 39)


@pytest.fixture(scope="module")
def arts40():
    specs = synth.arts40_specs()
    beams = [synth.make_beam(s) for s in specs]
    say("oracle: 40-beam workload, beams", SAMPLED, "mean and median lists")
    jobs = [(beams[i], list(st), True, None) for st in (synth.STEPS_ARTS40_MEAN, synth.STEPS_ARTS40_MEDIAN)
            for i in SAMPLED]
    res = oracle_pool.pipelines(jobs)
    ref = {"mean": res[:len(SAMPLED)], "median": res[len(SAMPLED):]}
    return beams, ref


@pytest.mark.parametrize("replace", ["mean", "median"])
def test_arts40_bench_call(rf, arts40, replace):
    """The benchmark's 40-beam step: all beams in one rfim_pipeline_run with a
    plan, out of place, flags off, on the current stream.  At 1536 channels
    with flags off the planner takes 32-sample tiles and the 8-lanes-per-time-
    sample 32-channel FD path; sampled beams must equal the oracle byte for
    byte and every sampled beam's per-step flag count the oracle's."""
    import torch
    beams, ref = arts40
    steps = synth.STEPS_ARTS40_MEAN if replace == "mean" else synth.STEPS_ARTS40_MEDIAN
    dev = torch.device("cuda:0")
    ins = [torch.from_numpy(b).to(dev) for b in beams]
    outs = [torch.full_like(x, 0x5A) for x in ins]
    plan = rf.Plan(ins, steps, outputs=outs)
    for i in SAMPLED:
        d = plan.describe(i, 0)
        assert d["tile_samples"] == 32 and d["fd_path"] == "u8_bin32_g8", d
    stream = torch.cuda.current_stream()
    for rep in range(2):   # the benchmark repeats the call on the same buffers
        say(f"arts40 {replace} call {rep}")
        rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan, stream=stream)
        torch.cuda.synchronize()
        counts = plan.flag_counts()
        for n, i in enumerate(SAMPLED):
            want, wf = ref[replace][n]
            np.testing.assert_array_equal(outs[i].cpu().numpy(), want, err_msg=f"beam {i}")
            assert counts[i] == oracle_counts(wf, len(steps)), (i, counts[i])
    plan.close()


def test_single_beam_call_and_graph(rf):
    """The single-beam and serve call: 1536 x 12500, TD 3.25 + FD 2.75,
    flags off, through a plan and through the plan's HIP graph."""
    import torch
    x = synth.make_beam(synth.BeamSpec("u8", 1536, 12500, 1, 0))
    steps = list(synth.STEPS_ARTS1)
    want, wf = oracle_pool.pipelines([(x, steps, True, None)])[0]
    dev = torch.device("cuda:0")
    xi = torch.from_numpy(x).to(dev)
    o = torch.full_like(xi, 0x5A)
    s = torch.cuda.Stream()
    plan = rf.Plan([xi], steps, outputs=[o])
    d = plan.describe(0, 0)
    assert d["tile_samples"] == 32 and d["fd_path"] == "u8_bin32_g8", d
    rf.rfim_pipeline_run([xi], steps, outputs=[o], plan=plan, stream=s)
    s.synchronize()
    np.testing.assert_array_equal(o.cpu().numpy(), want)
    assert plan.flag_counts()[0] == oracle_counts(wf, 2)
    plan.capture([xi], outputs=[o], stream=s)
    for rep in range(3):
        o.fill_(0)
        torch.cuda.synchronize()
        plan.replay(stream=s)
        s.synchronize()
        np.testing.assert_array_equal(o.cpu().numpy(), want, err_msg=f"replay {rep}")
        assert plan.flag_counts()[0] == oracle_counts(wf, 2)
    plan.close()


# ------------------------------------------------- uneven workload, real shapes
# (index in the 72-descriptor workload, expected tile and FD path with flags
# off / on at the default tuning)
UNEVEN_U8 = {
    "1536x12500": (0, (32, "u8_bin32_g8"), (16, "u8_bin32_g16")),
    "384x25000": (1, (64, "u8_bin32_g4"), (64, "u8_bin32_g4")),
    "4096x8192": (2, (8, "u8_vec"), (4, "u8_vec")),
    "768x16384": (3, (64, "u8_bin32_g4"), (32, "u8_bin32_g8")),
}


@pytest.fixture(scope="module")
def uneven_u8():
    specs = synth.uneven72_specs()
    beams = {k: synth.make_beam(specs[v[0]]) for k, v in UNEVEN_U8.items()}
    say("oracle: uneven-workload uint8 shapes")
    res = oracle_pool.pipelines([(beams[k], list(synth.STEPS_ARTS1), True, None) for k in UNEVEN_U8])
    return beams, dict(zip(UNEVEN_U8, res))


def run_one(rf, x, steps, flags, tune_cache=None):
    import torch
    dev = torch.device("cuda:0")
    xi = torch.from_numpy(x).to(dev)
    o = torch.full_like(xi, 0x5A)
    fl = [torch.full(xi.shape, 0xA5, dtype=torch.uint8, device=dev)] if flags else None
    plan = rf.Plan([xi], steps, outputs=[o], flags=fl, tune_cache=tune_cache)
    d = plan.describe(0, 0)
    rf.rfim_pipeline_run([xi], steps, outputs=[o], flags=fl, plan=plan)
    torch.cuda.synchronize()
    counts = plan.flag_counts()[0]
    plan.close()
    return d, o.cpu().numpy(), (fl[0].cpu().numpy() if flags else None), counts


@pytest.mark.parametrize("flags", [False, True], ids=["flags-off", "flags-on"])
@pytest.mark.parametrize("shape", list(UNEVEN_U8))
def test_uneven_u8_full_size(rf, uneven_u8, shape, flags):
    beams, ref = uneven_u8
    steps = list(synth.STEPS_ARTS1)
    x = beams[shape]
    say(f"uneven u8 {shape} flags={flags}")
    d, out, fl, counts = run_one(rf, x, steps, flags)
    tt, path = UNEVEN_U8[shape][2 if flags else 1]
    assert (d["tile_samples"], d["fd_path"]) == (tt, path), d
    want, wf = ref[shape]
    np.testing.assert_array_equal(out, want)
    if flags:
        np.testing.assert_array_equal(fl, wf)
    assert counts == oracle_counts(wf, len(steps))


# ---------------------------------------------- every auto-tuner candidate
U8_CANDIDATES = [(cap, lds) for cap in (16, 32, 64) for lds in (51200, 102400)]
F32_CANDIDATES = [(lds, cap) for lds in (40960, 81920, 163840) for cap in (8, 64)]


@pytest.mark.parametrize("flags", [False, True], ids=["flags-off", "flags-on"])
@pytest.mark.parametrize("shape", ["1536x12500", "4096x8192"])
@pytest.mark.parametrize("cand", U8_CANDIDATES, ids=[f"cap{c}-lds{l // 1024}k" for c, l in U8_CANDIDATES])
def test_tuner_candidate_u8(rf, uneven_u8, tmp_path, cand, shape, flags):
    """Each uint8 candidate of the auto-tuner, forced through the tuning cache,
    on full-size beams: the plan must pick it up and give the oracle's bytes."""
    beams, ref = uneven_u8
    steps = list(synth.STEPS_ARTS1)
    x = beams[shape]
    cache = str(tmp_path / "tune.json")
    shp = [rf.shape_beam("u8", x.shape[0], x.shape[1], flags=flags)]
    rf.tune_store(cache, shp, steps, (cand[0], 81920, 64, cand[1]))
    say(f"tuner u8 cand={cand} {shape} flags={flags}")
    d, out, fl, counts = run_one(rf, x, steps, flags, tune_cache=cache)
    assert d["tile_samples"] <= cand[0] and d["lds_bytes"] <= cand[1], d
    want, wf = ref[shape]
    np.testing.assert_array_equal(out, want)
    if flags:
        np.testing.assert_array_equal(fl, wf)
    assert counts == oracle_counts(wf, len(steps))


@pytest.fixture(scope="module")
def uneven_f32():
    specs = synth.uneven72_specs()
    beams = {"1536x12500": synth.make_beam(specs[64]), "4096x8192": synth.make_beam(specs[66])}
    assert beams["1536x12500"].shape == (1536, 12500) and beams["4096x8192"].shape == (4096, 8192)
    say("oracle: uneven-workload float32 shapes")
    res = oracle_pool.pipelines([(b, list(synth.STEPS_ARTS1), True, None) for b in beams.values()])
    return beams, dict(zip(beams, res))


@pytest.mark.parametrize("flags", [False, True], ids=["flags-off", "flags-on"])
@pytest.mark.parametrize("shape", ["1536x12500", "4096x8192"])
@pytest.mark.parametrize("cand", F32_CANDIDATES, ids=[f"lds{l // 1024}k-cap{c}" for l, c in F32_CANDIDATES])
def test_tuner_candidate_f32(rf, uneven_f32, tmp_path, cand, shape, flags):
    beams, ref = uneven_f32
    steps = list(synth.STEPS_ARTS1)
    x = beams[shape]
    cache = str(tmp_path / "tune.json")
    shp = [rf.shape_beam("f32", x.shape[0], x.shape[1], flags=flags)]
    rf.tune_store(cache, shp, steps, (64, cand[0], cand[1], 51200))
    say(f"tuner f32 cand={cand} {shape} flags={flags}")
    d, out, fl, counts = run_one(rf, x, steps, flags, tune_cache=cache)
    assert d["fd_path"] in ("f32_fast", "f32_wide"), d
    if d["fd_path"] == "f32_fast":
        assert d["tile_samples"] <= cand[1], d
    want, wf = ref[shape]
    np.testing.assert_array_equal(out.view(np.uint32), want.view(np.uint32))
    if flags:
        np.testing.assert_array_equal(fl, wf)
    assert counts == oracle_counts(wf, len(steps))


# ------------------------------------- the uneven call, autotuned, as a graph
def test_uneven72_autotuned_graph_vs_oracle(rf, tmp_path):
    """The benchmark's 72-descriptor call: auto-tuned plan, captured into a
    HIP graph and replayed (eager work in between); one descriptor of every
    shape and dtype is checked against the oracle after each replay."""
    import torch
    specs = synth.uneven72_specs()
    beams = [synth.make_beam(s) for s in specs]
    steps = list(synth.STEPS_ARTS1)
    check = [0, 1, 2, 3, 64, 65, 66, 67]
    say("oracle: one descriptor per shape and dtype of the uneven call")
    ref = oracle_pool.pipelines([(beams[i], steps, True, None) for i in check])
    dev = torch.device("cuda:0")
    ins = [torch.from_numpy(b).to(dev) for b in beams]
    outs = [torch.empty_like(x) for x in ins]
    shapes = [rf.shape_beam("u8" if b.dtype == np.uint8 else "f32", *b.shape) for b in beams]
    cache = str(tmp_path / "tune.json")
    say("autotune uneven72")
    rf.autotune(shapes, steps, cache)
    plan = rf.Plan(ins, steps, outputs=outs, tune_cache=cache)
    stream = torch.cuda.Stream()
    plan.capture(ins, outputs=outs, stream=stream)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        say(f"uneven72 replay {rep}")
        plan.replay(stream=stream)
        stream.synchronize()
        counts = plan.flag_counts()
        for n, i in enumerate(check):
            want, wf = ref[n]
            got = outs[i].cpu().numpy()
            np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8), err_msg=f"replay {rep} beam {i}")
            assert counts[i] == oracle_counts(wf, len(steps)), (rep, i)
    plan.close()


# --------------------------------------- the float32 stress beam at full size
@pytest.fixture(scope="module")
def stress_beam():
    spec = synth.stress16_specs()[0]
    x = synth.make_beam(spec)
    rng = np.random.default_rng(77)
    T = x.shape[1]
    # tile edges, the ends and random time samples
    cols = sorted(set([0, 1, 3, 4, 63, 64, 65, T - 65, T - 4, T - 1] + list(rng.integers(0, T, size=54))))
    say(f"oracle: full-size stress beam, all rows through the TD steps, {len(cols)} time samples through FD")
    td = [s for s in synth.STEPS_STRESS if s.domain == "td"]
    fd = [s for s in synth.STEPS_STRESS if s.domain == "fd"]
    want, wf, td_counts = oracle_pool.td_then_fd_columns(x, td, fd, cols)
    return x, cols, want, wf, td_counts


@pytest.mark.parametrize("inplace", [False, True], ids=["out-of-place", "in-place"])
def test_stress_full_pipeline_sampled(rf, stress_beam, inplace):
    """One 4096 x 65536 float32 beam of the stress workload through the whole
    7-step list (4 TD + 3 FD, median) as the benchmark runs it (flags off),
    checked against the oracle at sampled time samples (every channel), and
    the per-step flag counts of the TD steps against the oracle's."""
    import torch
    x, cols, want, wf, td_counts = stress_beam
    steps = list(synth.STEPS_STRESS)
    dev = torch.device("cuda:0")
    xi = torch.from_numpy(x).to(dev)
    o = xi if inplace else torch.full_like(xi, 7.0)
    plan = rf.Plan([xi], steps, outputs=[o])
    d = plan.describe(0, 0)
    say(f"stress inplace={inplace} {d}")
    rf.rfim_pipeline_run([xi], steps, outputs=[o], plan=plan)
    torch.cuda.synchronize()
    counts = plan.flag_counts()[0]
    got = o[:, cols].cpu().numpy()
    plan.close()
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    assert counts[:4] == td_counts            # TD steps: every sample of the beam
    for j in range(4, 7):                      # FD steps: the sampled time samples are a lower bound
        assert counts[j] >= int(((wf >> j) & 1).sum())
    del xi, o
    torch.cuda.empty_cache()


# ------------------------------------- TD rows per work-group (tuning axis)
@pytest.mark.parametrize("rows", [2, 8])
def test_td_rows_per_group_full_size(rf, uneven_u8, tmp_path, rows):
    """The uint8 TD pass with 2 or 8 rows per work-group, forced through the
    tuning cache, on full-size beams of two uneven shapes (flags on and off)."""
    beams, ref = uneven_u8
    steps = list(synth.STEPS_ARTS1)
    for shape in ("1536x12500", "768x16384"):
        for flags in (False, True):
            x = beams[shape]
            cache = str(tmp_path / f"tune_{shape}_{flags}.json")
            shp = [rf.shape_beam("u8", x.shape[0], x.shape[1], flags=flags)]
            rf.tune_store(cache, shp, steps, (64, 81920, 64, 51200, 0, rows))
            assert rf.tune_lookup(cache, shp, steps)[5] == rows
            say(f"td rows {rows} {shape} flags={flags}")
            _, out, fl, counts = run_one(rf, x, steps, flags, tune_cache=cache)
            want, wf = ref[shape]
            np.testing.assert_array_equal(out, want)
            if flags:
                np.testing.assert_array_equal(fl, wf)
            assert counts == oracle_counts(wf, len(steps))


@pytest.mark.parametrize("rows", [2, 4, 8])
def test_td_rows_groups_spanning_beams(rf, tmp_path, rows):
    """Work-groups of 2, 4 or 8 rows over beams whose channel counts are not
    multiples of the group (groups spanning beams, short last group): TD-only
    lists, outputs and per-beam counts against the oracle."""
    import torch
    steps = [synth.td(3.0), synth.td(2.5, "median"), synth.td(2.75)]
    shapes = [(5, 3001), (63, 2000), (130, 777), (1, 4096), (250, 1500), (7, 9000)]
    xs = [synth.make_beam(synth.BeamSpec("u8", C, T, 7, i)) for i, (C, T) in enumerate(shapes)]
    ref = oracle_pool.pipelines([(x, steps, True, None) for x in xs])
    cache = str(tmp_path / "tune.json")
    shp = [rf.shape_beam("u8", C, T) for C, T in shapes]
    rf.tune_store(cache, shp, steps, (64, 81920, 64, 51200, 0, rows))
    ins = [torch.from_numpy(x).cuda() for x in xs]
    outs = [torch.full_like(x, 0x5A) for x in ins]
    plan = rf.Plan(ins, steps, outputs=outs, tune_cache=cache)
    say(f"td rows {rows}: six beams")
    rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan)
    torch.cuda.synchronize()
    counts = plan.flag_counts()
    plan.close()
    for i, (want, wf) in enumerate(ref):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), want, err_msg=f"beam {i}")
        assert counts[i] == oracle_counts(wf, len(steps)), i
