"""GPU: the serve loop in its three forms delivers, for every admitted
arrival, exactly the bytes of a direct pipeline run on that batch (and of
the oracle), with latency statistics for every completion."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

STEPS = [synth.td(3.25), synth.fd(2.75, 32)]
C, T = 256, 3000


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


@pytest.mark.parametrize("mode", ["per_call", "batched", "graph"])
def test_serve_outputs_match_direct_runs(rf, mode):
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    pool = [rng.normal(80, 10, (C, T)).clip(0, 255).astype(np.uint8) for _ in range(6)]
    for p in pool:
        p[rng.integers(0, C, 3), :] = 250           # narrow-band channels
        p[:, rng.integers(0, T, 4)] = 240           # broadband impulses
    src = [torch.from_numpy(p).to(dev) for p in pool]
    want = []
    for x in src:
        o = torch.empty_like(x)
        rf.rfim_pipeline_run([x], STEPS, outputs=[o])
        want.append(o)
    torch.cuda.synchronize()
    say(f"serve mode={mode}")
    s = rf.Serve(STEPS, dtype="u8", nchan=C, nsamp=T, ring_depth=2, max_batch=4,
                 hbm_budget=16 * C * T, max_wait_s=0.0005, deadline_s=1.0, mode=mode)
    outs, which = [], []
    for i in range(12):
        d = torch.full_like(src[0], 7)
        assert s.submit(i % 6, src[i % 6], arrival_s=s.now(), dst=d)
        outs.append(d)
        which.append(i % 6)
        s.poll(s.now())
    while s.stats()["completed"] < 12:
        s.poll(s.now())
    s.drain(s.now())
    torch.cuda.synchronize()
    st = s.stats()
    say(st)
    assert st["completed"] == 12 and st["admitted"] == 12 and st["rejected_budget"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"] < 10
    if mode == "per_call":
        assert st["launches"] == 12
    for d, w in zip(outs, which):
        assert torch.equal(d, want[w])
    got0 = outs[0].cpu().numpy()
    np.testing.assert_array_equal(got0, oracle.pipeline(pool[0], STEPS)[0])
    s.close()


@pytest.mark.parametrize("mode", ["per_call", "graph"])
def test_serve_host_sourced_batches(rf, mode):
    """Batches submitted from pinned host memory are copied in on the serve
    stream and mitigated exactly like device-resident ones."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(37)
    pool = [rng.normal(90, 8, (C, T)).clip(0, 255).astype(np.uint8) for _ in range(3)]
    for p in pool:
        p[rng.integers(0, C, 2), :] = 245
    host = [torch.from_numpy(p).pin_memory() for p in pool]   # new pinned allocations
    want = []
    for p in pool:
        x = torch.from_numpy(p).to(dev)
        o = torch.empty_like(x)
        rf.rfim_pipeline_run([x], STEPS, outputs=[o])
        want.append(o)
    torch.cuda.synchronize()
    say(f"serve host-sourced mode={mode}")
    s = rf.Serve(STEPS, dtype="u8", nchan=C, nsamp=T, ring_depth=2, max_batch=3,
                 hbm_budget=8 * C * T, max_wait_s=0.0005, deadline_s=1.0, mode=mode)
    outs = []
    for i in range(6):
        d = torch.full((C, T), 9, dtype=torch.uint8, device=dev)
        assert s.submit(i % 3, host[i % 3], arrival_s=s.now(), dst=d)
        outs.append(d)
        s.poll(s.now())
    while s.stats()["completed"] < 6:
        s.poll(s.now())
    s.drain(s.now())
    torch.cuda.synchronize()
    st = s.stats()
    say(st)
    assert st["completed"] == 6 and st["rejected_budget"] == 0
    for i, d in enumerate(outs):
        assert torch.equal(d, want[i % 3])
    s.close()
