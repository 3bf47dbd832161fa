"""GPU parity of masked TD steps (RFIM_TD_MASKED, uint8 beams) against the
oracle: outputs, flag bits and per-step counts bit-identical, in the two-pass
and the persistent schedule; float32 beams are refused."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

from test_parity_u8 import check_against_oracle, gpu_run

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


def rand_masked_steps(rng, C, n):
    divs = [d for d in range(1, C + 1) if C % d == 0]
    out = []
    for _ in range(n):
        u = rng.random()
        dom = "td_masked" if u < 0.55 else ("td" if u < 0.75 else "fd")
        k = float(rng.choice([0.0, 0.5, 1.0, 1.5, 2.0, 2.75, 3.25, rng.uniform(0.2, 3.5)]))
        rep = "mean" if rng.random() < 0.6 else "median"
        out.append((dom, k, rep, int(rng.choice(divs)) if dom == "fd" else 0))
    return out


@pytest.mark.parametrize("seed", range(16))
def test_masked_random_small_beams(rf, seed):
    """Several beams per call, ragged tiles, padded strides, step lists mixing
    masked runs with TD and FD steps, flags on."""
    rng = np.random.default_rng(9100 + seed)
    C = int(rng.choice([1, 3, 4, 7, 32, 64, 100]))
    steps = rand_masked_steps(rng, C, int(rng.integers(1, 7)))
    beams, nsamp = [], []
    for _ in range(int(rng.integers(1, 4))):
        T = int(rng.choice([1, 2, 5, 17, 64, 257, 1000, 5000]))
        stride = T + int(rng.choice([0, 1, 3, 8]))
        kind = rng.integers(0, 3)
        if kind == 0:
            x = rng.integers(0, 256, size=(C, stride))
        elif kind == 1:
            x = rng.normal(80, 10, size=(C, stride)).clip(0, 255)
            x[rng.random(x.shape) < 0.02] = 250
        else:
            x = rng.integers(0, 3, size=(C, stride)) * 100
        beams.append(x.astype(np.uint8))
        nsamp.append(T)
    say(f"masked seed={seed} C={C} shapes={[b.shape for b in beams]} nsamp={nsamp} steps={steps}")
    out, fl, _ = gpu_run(rf, beams, steps, nsamp=nsamp)
    check_against_oracle(beams, steps, out, fl, nsamp=nsamp)


MASKED_STEPS = {
    "mean": [("td_masked", 4.0, "mean", 0), ("td_masked", 3.5, "mean", 0), ("td_masked", 3.25, "mean", 0),
             ("fd", 3.0, "mean", 32), ("fd", 2.75, "mean", 32)],
    "median": [("td_masked", 4.0, "median", 0), ("td_masked", 3.5, "median", 0),
               ("td_masked", 3.25, "median", 0), ("fd", 3.0, "median", 32), ("fd", 2.75, "median", 32)],
    "runs": [("td_masked", 2.5, "mean", 0), ("td", 2.5, "mean", 0), ("td_masked", 2.0, "median", 0),
             ("td_masked", 2.0, "mean", 0), ("fd", 2.75, "mean", 32), ("td_masked", 1.5, "mean", 0),
             ("td_masked", 1.5, "mean", 0)],
}


@pytest.mark.parametrize("which", sorted(MASKED_STEPS))
def test_masked_full_size_beam(rf, which):
    """A full-size 1536 x 12500 beam of the 40-beam workload, with a plan and
    per-step flag counts."""
    x = synth.make_beam(synth.arts40_specs()[5])
    steps = MASKED_STEPS[which]
    say(f"masked arts40 beam 5 steps={steps}")
    out, fl, counts = gpu_run(rf, [x], steps, plan=True)
    check_against_oracle([x], steps, out, fl, counts=counts)


def test_masked_rows_all_set_aside(rf):
    """Rows whose every sample is cut by the first masked step (values 0 and 2,
    k = 0: the mean 1 is no sample's value), constant rows, one-sample rows:
    later masked steps see no sample and leave the row as it is."""
    rng = np.random.default_rng(9200)
    C, T = 64, 3001
    x = rng.integers(0, 2, size=(C, T)).astype(np.uint8) * 2
    x[:, 0], x[:, 1] = 0, 2
    x[8:16] = 7                                    # constant rows
    x[16:24, : T // 2] = 0                         # half zeros, half twos
    x[16:24, T // 2:] = 2
    steps = [("td_masked", 0.0, "mean", 0), ("td_masked", 0.0, "median", 0), ("td_masked", 1.0, "mean", 0)]
    say("masked rows all set aside")
    out, fl, counts = gpu_run(rf, [x], steps, plan=True)
    check_against_oracle([x], steps, out, fl, counts=counts)
    y = rng.integers(0, 256, size=(5, 1)).astype(np.uint8)
    out, fl, _ = gpu_run(rf, [y], steps)
    check_against_oracle([y], steps, out, fl)


def test_masked_persistent_schedule(rf, tmp_path):
    """The persistent beam-major schedule runs the same TD decisions."""
    import torch
    beams = [synth.make_beam(s) for s in synth.arts40_specs()[:3]]
    steps = MASKED_STEPS["runs"]
    ins = [torch.from_numpy(b).cuda() for b in beams]
    outs = [torch.full_like(x, 0x5A) for x in ins]
    fls = [torch.full(x.shape, 0xA5, dtype=torch.uint8, device=x.device) for x in ins]
    cache = str(tmp_path / "tune.json")
    shapes = [rf.shape_beam("u8", x.shape[0], x.shape[1], flags=True) for x in ins]
    rf.tune_store(cache, shapes, steps, (64, 81920, 64, 51200, 1))
    plan = rf.Plan(ins, steps, outputs=outs, flags=fls, tune_cache=cache)
    plan.set_timing(True)
    say("masked persistent schedule, 3 beams")
    rf.rfim_pipeline_run(ins, steps, outputs=outs, flags=fls, plan=plan)
    torch.cuda.synchronize()
    assert plan.kernel_times(rf.RFIM_KERNEL_PERSIST_U8)[0] > 0
    counts = plan.flag_counts()
    check_against_oracle(beams, steps, [o.cpu().numpy() for o in outs], [f.cpu().numpy() for f in fls],
                         counts=counts)
    plan.close()


def test_masked_float32_refused(rf):
    import torch
    f = torch.zeros((4, 64), dtype=torch.float32, device="cuda")
    u = torch.zeros((4, 64), dtype=torch.uint8, device="cuda")
    for ins in ([f], [u, f]):
        with pytest.raises(rf.RfimError) as e:
            rf.rfim_pipeline_run(ins, [("td_masked", 3.0, "mean", 0)], outputs=[torch.empty_like(x) for x in ins])
        assert e.value.status == rf.RFIM_ERR_UNSUPPORTED
    torch.cuda.synchronize()
