"""Runs independent oracle calls in worker processes (test infrastructure).

The oracle is single-threaded; full-size parity references are many
independent oracle calls (beams, or row blocks for TD steps and column blocks
for FD steps, which the definitions keep independent: a TD step's statistics
never leave their row and an FD step's never leave their time sample).
Workers are spawned fresh, never forked, so a process that already holds the
GPU is not duplicated; they import only numpy and the oracle.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pipeline(args):
    import oracle
    x, steps, want_flags, nsamp = args
    return oracle.pipeline(x, steps, want_flags, nsamp=nsamp)


def pipelines(jobs):
    """[(x, steps, want_flags, nsamp)] -> [oracle.pipeline(...) result], in order."""
    if len(jobs) == 1:
        return [_pipeline(jobs[0])]
    with ProcessPoolExecutor(max_workers=min(_workers(), len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_pipeline, jobs))


def td_then_fd_columns(x, td_steps, fd_steps, cols, row_block=256):
    """Oracle output of [TD steps][FD steps] on beam x at the time samples
    `cols` only: the TD steps on every row (row blocks in parallel), then the
    FD steps on the selected time samples.  Returns (out[:, cols],
    flags[:, cols], td_counts) with flag bits numbered over the whole list and
    td_counts[j] the number of samples of the whole beam TD step j replaced."""
    C = x.shape[0]
    jobs = [(np.ascontiguousarray(x[r:r + row_block]), list(td_steps), True, None) for r in range(0, C, row_block)]
    res = pipelines(jobs)
    post_td = np.concatenate([o for o, _ in res], axis=0)
    td_flags = np.concatenate([f for _, f in res], axis=0)
    sub = np.ascontiguousarray(post_td[:, cols])
    out, fdf = _pipeline((sub, list(fd_steps), True, None))
    fl = td_flags[:, cols] | (fdf.astype(np.uint8) << len(td_steps))
    td_counts = [int(((td_flags >> j) & 1).sum()) for j in range(len(td_steps))]
    return out, fl.astype(np.uint8), td_counts
