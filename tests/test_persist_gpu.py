"""The uint8 persistent beam-major schedule (one launch per run of [TD][FD]
steps: work-groups take work items from a device counter, each beam's TD row
groups before its tiles, a tile waiting on its beam's completion counter)
against the oracle through the C ABI, chosen through the tuning cache as the
auto-tuner would: byte-exact outputs, flags and per-step counts; in a
captured graph; and the bounded wait's error path, forced from the host."""
from __future__ import annotations

import os
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


def counts_of(flags, nsteps):
    return [int(((flags >> j) & 1).sum()) for j in range(nsteps)]


def persistent_plan(rf, tmp_path, ins, steps, outs, fls=None):
    """A plan whose tuning-cache entry selects the persistent schedule."""
    cache = str(tmp_path / "tune.json")
    shapes = [rf.shape_beam("u8", x.shape[0], x.shape[1], row_stride=x.stride(0) if x.shape[0] > 1 else None,
                            flags=fls is not None) for x in ins]
    rf.tune_store(cache, shapes, steps, (64, 81920, 64, 51200, 1))
    assert rf.tune_lookup(cache, shapes, steps)[4] == 1
    plan = rf.Plan(ins, steps, outputs=outs, flags=fls, tune_cache=cache)
    plan.set_timing(True)
    return plan


def ran_persistent(rf, plan):
    n, _ = plan.kernel_times(rf.RFIM_KERNEL_PERSIST_U8)
    m, _ = plan.kernel_times(rf.RFIM_KERNEL_FUSED_U8)
    return n > 0 and m == 0


@pytest.mark.parametrize("replace", ["mean", "median"])
def test_persistent_40_beams(rf, tmp_path, replace):
    import torch
    specs = synth.arts40_specs()
    beams = [synth.make_beam(s) for s in specs]
    steps = synth.STEPS_ARTS40_MEAN if replace == "mean" else synth.STEPS_ARTS40_MEDIAN
    sampled = (0, 13, 26, 39)
    say(f"oracle: 40-beam workload ({replace}), beams {sampled}")
    ref = oracle_pool.pipelines([(beams[i], list(steps), True, None) for i in sampled])
    ins = [torch.from_numpy(b).cuda() for b in beams]
    outs = [torch.full_like(x, 0x5A) for x in ins]
    plan = persistent_plan(rf, tmp_path, ins, steps, outs)
    for rep in range(2):
        say(f"persistent 40-beam {replace} call {rep}")
        rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan)
        torch.cuda.synchronize()
        counts = plan.flag_counts()
        for n, i in enumerate(sampled):
            want, wf = ref[n]
            np.testing.assert_array_equal(outs[i].cpu().numpy(), want, err_msg=f"beam {i}")
            assert counts[i] == counts_of(wf, len(steps)), i
    assert ran_persistent(rf, plan)
    plan.close()


LISTS = {
    "td-fd": [synth.td(4.0), synth.td(3.25, "median"), synth.fd(3.0, 32), synth.fd(2.75, 32, "median")],
    "td-only": [synth.td(3.0), synth.td(2.5)],
    "fd-only": [synth.fd(2.75, 32), synth.fd(2.5, 0)],
    "interleaved": [synth.td(3.25), synth.fd(2.75, 32), synth.td(3.0, "median"), synth.fd(2.5, 64)],
}


@pytest.mark.parametrize("flags", [False, True], ids=["flags-off", "flags-on"])
@pytest.mark.parametrize("name", list(LISTS))
def test_persistent_uneven_small(rf, tmp_path, name, flags):
    """Six beams of uneven shapes in one call: odd strides, short last
    tiles, and for the TD-only list channel counts that are not multiples of
    four (row groups that end inside a beam)."""
    import torch
    steps = LISTS[name]
    if name == "td-only":   # row groups of four rows that end inside a beam
        shapes = [(63, 1000, 1003), (130, 777, 777), (97, 2500, 2504), (5, 333, 340), (1, 4097, 4100),
                  (250, 1500, 1501)]
    else:                   # FD bins of 32 and 64 channels
        shapes = [(64, 1000, 1003), (192, 777, 777), (128, 2500, 2504), (256, 333, 340), (64, 4097, 4100),
                  (320, 1500, 1501)]
    rng = np.random.default_rng(len(name) * 7 + flags)
    xs, ins, outs, fls = [], [], [], []
    for C, T, S in shapes:
        x = np.zeros((C, S), dtype=np.uint8)
        x[:, :T] = synth.make_beam(synth.BeamSpec("u8", C, T, 6, int(rng.integers(0, 1000))))
        xs.append(x)
        xi = torch.from_numpy(x).cuda()
        ins.append(xi)
        outs.append(torch.full_like(xi, 0x5A))
        fls.append(torch.full_like(xi, 0xA5))
    nsamp = [T for _, T, _ in shapes]
    say(f"oracle: {name} flags={flags}")
    ref = oracle_pool.pipelines([(x, steps, True, T) for x, T in zip(xs, nsamp)])
    cache = str(tmp_path / "tune.json")
    sh = [rf.shape_beam("u8", C, T, row_stride=S, flags=flags) for C, T, S in shapes]
    rf.tune_store(cache, sh, steps, (64, 81920, 64, 51200, 1))
    plan = rf.Plan(ins, steps, outputs=outs, flags=fls if flags else None, nsamp=nsamp, tune_cache=cache)
    plan.set_timing(True)
    rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls if flags else None, nsamp=nsamp, plan=plan)
    torch.cuda.synchronize()
    counts = plan.flag_counts()
    assert ran_persistent(rf, plan)
    plan.close()
    for i, (C, T, S) in enumerate(shapes):
        want, wf = ref[i]
        got = outs[i].cpu().numpy()
        np.testing.assert_array_equal(got[:, :T], want[:, :T], err_msg=f"beam {i}")
        if flags:
            np.testing.assert_array_equal(fls[i].cpu().numpy()[:, :T], wf[:, :T], err_msg=f"flags {i}")
        assert counts[i] == counts_of(wf[:, :T], len(steps)), i


UNEVEN = {"1536x12500": 0, "384x25000": 1, "4096x8192": 2, "768x16384": 3}


def test_persistent_uneven_full_size_graph(rf, tmp_path):
    """One uint8 beam of each shape of the uneven workload in one persistent
    call, captured into a graph and replayed three times (eager work in
    between), every replay against the oracle."""
    import torch
    specs = synth.uneven72_specs()
    beams = [synth.make_beam(specs[i]) for i in UNEVEN.values()]
    steps = list(synth.STEPS_ARTS1)
    say("oracle: one uint8 beam per shape of the uneven workload")
    ref = oracle_pool.pipelines([(b, steps, True, None) for b in beams])
    ins = [torch.from_numpy(b).cuda() for b in beams]
    outs = [torch.empty_like(x) for x in ins]
    plan = persistent_plan(rf, tmp_path, ins, steps, outs)
    plan.set_timing(False)
    s = torch.cuda.Stream()
    plan.capture(ins, outputs=outs, stream=s)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        say(f"persistent graph replay {rep}")
        plan.replay(stream=s)
        s.synchronize()
        counts = plan.flag_counts()
        for i, (want, wf) in enumerate(ref):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), want, err_msg=f"replay {rep} beam {i}")
            assert counts[i] == counts_of(wf, len(steps))
    plan.close()


def test_persistent_wait_runs_out(rf, tmp_path):
    """A tile's wait for its beam's TD row groups is bounded.  Raising the
    awaited count past what the row groups reach (from the host) makes every
    wait run out: the launch still ends, and the plan's next flag-count read
    reports RFIM_ERR_DEVICE once; a plan without the raise then runs clean."""
    import torch
    x = synth.make_beam(synth.BeamSpec("u8", 256, 3000, 6, 1))
    steps = [synth.td(3.25), synth.fd(2.75, 32)]
    xi = torch.from_numpy(x).cuda()
    o = torch.empty_like(xi)
    os.environ["RFIM_WAIT_EXTRA"] = "1"
    os.environ["RFIM_SPIN_LIMIT"] = "64"
    try:
        plan = persistent_plan(rf, tmp_path, [xi], steps, [o])
    finally:
        del os.environ["RFIM_WAIT_EXTRA"]
        del os.environ["RFIM_SPIN_LIMIT"]
    rf.rfim_pipeline_run([xi], steps, outputs=[o], plan=plan)
    torch.cuda.synchronize()
    with pytest.raises(rf.RfimError) as e:
        plan.flag_counts()
    assert e.value.status == rf.RFIM_ERR_DEVICE
    plan.flag_counts()   # reported once
    plan.close()
    want, _ = oracle_pool.pipelines([(x, steps, False, None)])[0]
    plan = persistent_plan(rf, tmp_path, [xi], steps, [o])
    rf.rfim_pipeline_run([xi], steps, outputs=[o], plan=plan)
    torch.cuda.synchronize()
    plan.flag_counts()
    np.testing.assert_array_equal(o.cpu().numpy(), want)
    plan.close()


def test_autotuner_times_both_schedules(rf, tmp_path):
    """The auto-tuner's table holds candidates of both uint8 schedules, all
    bit-identical to the default (it fails otherwise), and its choice gives
    the oracle's bytes."""
    import json
    import torch
    beams = [synth.make_beam(synth.BeamSpec("u8", 1536, 12500, 1, b)) for b in range(4)]
    steps = list(synth.STEPS_ARTS1)
    shapes = [rf.shape_beam("u8", 1536, 12500) for _ in beams]
    cache = str(tmp_path / "tune.json")
    rf.autotune(shapes, steps, cache)
    doc = json.load(open(cache))
    (entry,) = doc.values()
    scheds = {row[2] for row in entry["table"]}
    assert scheds == {0, 1}, entry["table"]
    ref = oracle_pool.pipelines([(b, steps, False, None) for b in beams])
    ins = [torch.from_numpy(b).cuda() for b in beams]
    outs = [torch.empty_like(x) for x in ins]
    plan = rf.Plan(ins, steps, outputs=outs, tune_cache=cache)
    rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan)
    torch.cuda.synchronize()
    for i, (want, _) in enumerate(ref):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), want)
    plan.close()
