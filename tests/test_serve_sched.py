"""Serve-loop scheduling on the CPU with the mock executor (a launch of k
arrivals takes launch_s + k * beam_s on one in-order device): admission by
the slot pool and per-beam ring, batch forming by size and waiting time,
latency accounting and percentiles, deadline misses, backlog under overload."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2001_03389_amd as rf

STEPS = [("td", 3.25, "mean", 0), ("fd", 2.75, "mean", 32)]
BATCH_BYTES = 1536 * 12500


def mock(**kw):
    args = dict(mock=True, mock_launch_s=0.001, mock_beam_s=0.0005, hbm_budget=8 * BATCH_BYTES,
                ring_depth=2, max_batch=4, max_wait_s=0.002, deadline_s=0.010, mode="batched")
    args.update(kw)
    return rf.Serve(STEPS, **args)


def test_single_arrival_latency_is_the_modelled_cost():
    s = mock(max_batch=1)
    assert s.submit(0, arrival_s=1.0)
    s.poll(1.0)                     # launches at 1.0, done at 1.0015
    st = s.stats()
    assert st["launches"] == 1 and st["completed"] == 0
    s.poll(1.0015)
    st = s.stats()
    assert st["completed"] == 1
    assert st["p50_s"] == pytest.approx(0.0015) and st["max_s"] == pytest.approx(0.0015)


def test_batch_waits_for_fullness_or_max_wait():
    s = mock(max_batch=4, max_wait_s=0.002)
    for b in range(3):
        assert s.submit(b, arrival_s=0.0)
    s.poll(0.001)                   # 3 < 4 and waited 1 ms < 2 ms: no launch
    assert s.stats()["launches"] == 0
    s.poll(0.002)                   # waited 2 ms: partial batch of 3 goes
    st = s.stats()
    assert st["launches"] == 1 and st["mean_batch"] == 3
    s.drain(0.002)
    st = s.stats()
    assert st["completed"] == 3
    # all three finish together at 0.002 + 0.001 + 3 * 0.0005
    assert st["p50_s"] == pytest.approx(0.0045) and st["max_s"] == pytest.approx(0.0045)


def test_full_batch_launches_immediately():
    s = mock(max_batch=2, max_wait_s=1.0)
    s.submit(0, arrival_s=0.0)
    s.submit(1, arrival_s=0.0)
    s.poll(0.0)
    assert s.stats()["launches"] == 1


def test_ring_depth_and_pool_budget_refuse():
    s = mock(hbm_budget=3 * BATCH_BYTES, ring_depth=2, max_wait_s=10.0)
    assert s.submit(7, arrival_s=0.0)
    assert s.submit(7, arrival_s=0.0)
    assert not s.submit(7, arrival_s=0.0)          # beam 7's ring is full
    assert s.submit(8, arrival_s=0.0)
    assert not s.submit(9, arrival_s=0.0)          # pool of 3 slots is full
    st = s.stats()
    assert st["rejected_ring"] == 1 and st["rejected_budget"] == 1 and st["admitted"] == 3
    s.drain(0.0)
    assert s.stats()["in_flight"] == 0
    assert s.submit(9, arrival_s=1.0)              # slots came back


def test_pool_smaller_than_one_batch_is_a_budget_error():
    with pytest.raises(rf.RfimError) as e:
        mock(hbm_budget=BATCH_BYTES - 1)
    assert e.value.status == rf.RFIM_ERR_BUDGET


def test_percentiles_nearest_rank_and_deadline_misses():
    s = mock(max_batch=1, mock_launch_s=0.0, mock_beam_s=0.001, deadline_s=0.0035, hbm_budget=200 * BATCH_BYTES,
             ring_depth=200)
    # 10 arrivals at t=0 on one beam: in-order device, latencies 1..10 ms
    for _ in range(10):
        s.submit(0, arrival_s=0.0)
    s.drain(0.0)
    st = s.stats()
    assert st["completed"] == 10
    assert st["p50_s"] == pytest.approx(0.005)
    assert st["p99_s"] == pytest.approx(0.010)
    assert st["deadline_misses"] == 7              # 4 ms .. 10 ms


def test_per_call_form_launches_one_per_arrival():
    s = mock(mode="per_call", max_batch=8)
    for b in range(5):
        s.submit(b, arrival_s=0.0)
    s.poll(0.0)
    st = s.stats()
    assert st["launches"] == 5 and st["mean_batch"] == 1


@pytest.mark.parametrize("beams,ok", [(20, True), (400, False)])
def test_poisson_load_sustained_or_backlogged(beams, ok):
    """Poisson arrivals, mean interval 1.024 s per beam, over 30 s of fake
    time; capacity 1 / beam_s = 200 arrivals/s.  20 beams (~20/s) keep the
    latency at the batch cost; 400 beams (~390/s) overload the device."""
    rng = np.random.default_rng(5)
    s = mock(mock_launch_s=0.001, mock_beam_s=0.005, max_batch=8, max_wait_s=0.001, deadline_s=0.1,
             hbm_budget=64 * BATCH_BYTES, ring_depth=3)
    events = []
    for b in range(beams):
        t = rng.exponential(1.024)
        while t < 30.0:
            events.append((t, b))
            t += rng.exponential(1.024)
    events.sort()
    # the harness polls every millisecond and on every arrival
    i = 0
    for tick in range(30001):
        now = tick * 0.001
        while i < len(events) and events[i][0] <= now:
            s.poll(events[i][0])
            s.submit(events[i][1], arrival_s=events[i][0])
            i += 1
        s.poll(now)
    s.drain(30.0)
    st = s.stats()
    if ok:
        assert st["rejected_budget"] == 0 and st["rejected_ring"] == 0
        assert st["p99_s"] < 0.1 and st["deadline_misses"] == 0
    else:
        assert st["rejected_budget"] > 0 or st["deadline_misses"] > 0


def test_submit_checks_batch_tensors():
    """The binding refuses a batch of the wrong size, dtype or layout before
    anything is copied (the C side copies nchan * nsamp elements)."""
    import torch
    s = mock(nchan=32, nsamp=8, hbm_budget=64 * 256)
    for bad in (torch.zeros(31, 8, dtype=torch.uint8), torch.zeros(32, 8, dtype=torch.float32),
                torch.zeros(8, 32, dtype=torch.uint8).t()):
        with pytest.raises(ValueError):
            s.submit(0, bad, arrival_s=0.0)
    with pytest.raises(ValueError):   # dst must be a device tensor
        s.submit(0, arrival_s=0.0, dst=torch.zeros(32, 8, dtype=torch.uint8))
    s.close()
