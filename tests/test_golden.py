"""Hand-worked cases of the sigma cuts (tests/golden/, each with its
derivation from Section IV): the oracle on the CPU, and the HIP path through
the C ABI on the GPU, must both reproduce them exactly."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from golden_cases import load_cases

CASES = load_cases()
IDS = [c[0] for c in CASES]


def test_fixtures_present():
    assert len(CASES) >= 14


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_oracle_reproduces_hand_cases(case):
    _, x, steps, out, fl = case
    got, gfl = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got.view(np.uint8), out.view(np.uint8))
    np.testing.assert_array_equal(gfl, fl)


@pytest.mark.gpu
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_hip_path_reproduces_hand_cases(case):
    import torch
    import paper_2001_03389_amd as rf
    assert torch.cuda.is_available(), "needs a GPU"
    rf.lib()
    _, x, steps, out, fl = case
    dev = torch.device("cuda:0")
    xi = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    o = torch.empty_like(xi)
    f = torch.full(x.shape, 0xA5, dtype=torch.uint8, device=dev)
    rf.rfim_pipeline_run([xi], steps, outputs=[o], flags=[f])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o.cpu().numpy().view(np.uint8), out.view(np.uint8))
    np.testing.assert_array_equal(f.cpu().numpy(), fl)
