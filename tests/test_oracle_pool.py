"""CPU: the split oracle evaluation the full-size GPU parity tests use (TD
steps on row blocks, FD steps on selected time samples) equals the oracle's
plain pipeline restricted to those time samples."""
import numpy as np

import oracle
import oracle_pool
import synth


def test_td_then_fd_columns_equals_pipeline():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((96, 700)).astype(np.float32)
    x[5] += 9.0
    x[:, 100:103] += 6.0
    td = [synth.td(3.0, "median"), synth.td(2.5)]
    fd = [synth.fd(2.75, 32, "median"), synth.fd(2.5, 16)]
    want, wf = oracle.pipeline(x, td + fd, want_flags=True)
    cols = [0, 1, 100, 101, 350, 699]
    out, fl, tdc = oracle_pool.td_then_fd_columns(x, td, fd, cols, row_block=40)
    np.testing.assert_array_equal(out.view(np.uint32), want[:, cols].view(np.uint32))
    np.testing.assert_array_equal(fl, wf[:, cols])
    assert tdc == [int(((wf >> j) & 1).sum()) for j in range(2)]


def test_pipelines_in_workers_match_direct_calls():
    rng = np.random.default_rng(4)
    xs = [rng.integers(0, 256, size=(64, 300)).astype(np.uint8) for _ in range(3)]
    steps = list(synth.STEPS_ARTS40_MEDIAN)
    res = oracle_pool.pipelines([(x, steps, True, None) for x in xs])
    for x, (o, f) in zip(xs, res):
        w, wf = oracle.pipeline(x, steps, want_flags=True)
        np.testing.assert_array_equal(o, w)
        np.testing.assert_array_equal(f, wf)
