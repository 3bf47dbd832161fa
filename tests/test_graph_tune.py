"""GPU: the HIP-graph form of a plan and the auto-tuner.  A captured graph
is replayed several times with eager work and synchronisation in between;
every replay must give the oracle's bytes, flags and flag counts, as must a
graph replayed on other buffers and the plan the auto-tuner's cache entry
selects."""
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
    m.lib()
    return m


def mixed_beams():
    rng = np.random.default_rng(44)
    return [rng.normal(80, 10, (256, 3000)).clip(0, 255).astype(np.uint8),
            rng.standard_normal((128, 2500)).astype(np.float32),
            rng.normal(70, 9, (64, 1777)).clip(0, 255).astype(np.uint8),
            (rng.standard_normal((96, 5000)) * 2).astype(np.float32)]


STEPS = [synth.td(3.5), synth.td(3.0, "median"), synth.fd(2.75, 32), synth.fd(2.5, 32, "median")]


def oracle_refs(host):
    refs = [oracle.pipeline(h, STEPS, want_flags=True) for h in host]
    counts = [[int(((f >> j) & 1).sum()) for j in range(len(STEPS))] for _, f in refs]
    return [o.view(np.uint8) for o, _ in refs], [f for _, f in refs], counts


def test_graph_replays_match_eager(rf):
    import torch
    dev = torch.device("cuda:0")
    host = mixed_beams()
    ins = [torch.from_numpy(h).to(dev) for h in host]
    outs_e = [torch.empty_like(x) for x in ins]
    fl_e = [torch.zeros(x.shape, dtype=torch.uint8, device=dev) for x in ins]
    want, want_f, want_counts = oracle_refs(host)
    pe = rf.Plan(ins, STEPS, outputs=outs_e, flags=fl_e)
    rf.rfim_pipeline_run(ins, STEPS, outputs=outs_e, flags=fl_e, plan=pe)
    torch.cuda.synchronize()
    assert pe.flag_counts() == want_counts
    for i in range(len(host)):
        np.testing.assert_array_equal(outs_e[i].cpu().numpy().view(np.uint8), want[i], err_msg=f"eager beam {i}")
        np.testing.assert_array_equal(fl_e[i].cpu().numpy(), want_f[i], err_msg=f"eager beam {i} flags")
    pe.close()

    outs = [torch.empty_like(x) for x in ins]
    fls = [torch.zeros(x.shape, dtype=torch.uint8, device=dev) for x in ins]
    pg = rf.Plan(ins, STEPS, outputs=outs, flags=fls)
    stream = torch.cuda.Stream()
    pg.capture(ins, outputs=outs, flags=fls, stream=stream)
    for rep in range(4):
        say(f"replay {rep}")
        for o in outs:
            o.fill_(0)          # eager work between replays
        for f in fls:
            f.fill_(0x5A)
        torch.cuda.synchronize()
        pg.replay(stream=stream)
        stream.synchronize()
        got = [o.cpu().numpy().view(np.uint8) for o in outs]
        for i in range(len(host)):
            np.testing.assert_array_equal(got[i], want[i], err_msg=f"replay {rep} beam {i}")
            np.testing.assert_array_equal(fls[i].cpu().numpy(), want_f[i], err_msg=f"replay {rep} beam {i} flags")
        assert pg.flag_counts() == want_counts
    pg.close()


def test_graph_replay_on_other_buffers(rf):
    """A graph captured on one set of buffers, replayed on buffers of the same
    shapes holding other data, gives that data's eager result; buffers of
    another shape are refused before anything is launched."""
    import torch
    dev = torch.device("cuda:0")
    host_a = mixed_beams()
    rng = np.random.default_rng(45)
    host_b = [rng.normal(60, 12, h.shape).clip(0, 255).astype(np.uint8) if h.dtype == np.uint8
              else (rng.standard_normal(h.shape) * 3).astype(np.float32) for h in host_a]
    ins_a = [torch.from_numpy(h).to(dev) for h in host_a]
    ins_b = [torch.from_numpy(h).to(dev) for h in host_b]
    outs_a = [torch.empty_like(x) for x in ins_a]
    outs_b = [torch.empty_like(x) for x in ins_b]
    want_b, _, _ = oracle_refs(host_b)
    p = rf.Plan(ins_a, STEPS, outputs=outs_a)
    stream = torch.cuda.Stream()
    p.capture(ins_a, outputs=outs_a, stream=stream)
    for rep in range(3):
        say(f"replay_on {rep}")
        for o in outs_b:
            o.fill_(0)
        torch.cuda.synchronize()
        p.replay_on(ins_b, outputs=outs_b, stream=stream)
        stream.synchronize()
        for i in range(len(host_b)):
            np.testing.assert_array_equal(outs_b[i].cpu().numpy().view(np.uint8), want_b[i],
                                          err_msg=f"replay {rep} beam {i}")
    wrong = [torch.empty((x.shape[0], x.shape[1] - 4), dtype=x.dtype, device=dev) for x in ins_b]
    with pytest.raises(rf.RfimError):
        p.replay_on(wrong, outputs=[torch.empty_like(w) for w in wrong], stream=stream)
    p.close()


def test_autotune_cache_gives_identical_plan(rf, tmp_path):
    import torch
    dev = torch.device("cuda:0")
    host = mixed_beams()
    ins = [torch.from_numpy(h).to(dev) for h in host]
    shapes = [rf.shape_beam("u8" if h.dtype == np.uint8 else "f32", *h.shape) for h in host]
    cache = str(tmp_path / "tune.json")
    say("autotune")
    ms = rf.autotune(shapes, STEPS, cache)
    assert ms > 0
    params = rf.tune_lookup(cache, shapes, STEPS)
    assert params is not None
    say(f"tuned {params} {ms:.3f} ms")
    want, _, want_counts = oracle_refs(host)
    for tc in (None, cache):
        outs = [torch.empty_like(x) for x in ins]
        p = rf.Plan(ins, STEPS, outputs=outs, tune_cache=tc)
        rf.rfim_pipeline_run(ins, STEPS, outputs=outs, plan=p)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            np.testing.assert_array_equal(o.cpu().numpy().view(np.uint8), want[i], err_msg=f"tune={tc} beam {i}")
        assert p.flag_counts() == want_counts
        p.close()
    # the cache entry records every candidate's time
    import json
    entry = next(iter(json.load(open(cache)).values()))
    assert entry["candidates"] == len(entry["table"]) > 1
