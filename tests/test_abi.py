"""The C-ABI library loads and exports every entry point of include/rfim.h;
host-side argument validation answers without touching a GPU (CPU only)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import paper_2001_03389_amd as rf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rfim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rfim_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = rf.lib()
    names = header_functions()
    assert "rfim_pipeline_run" in names and "rfim_td_sigma_cut" in names and "rfim_fd_sigma_cut" in names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    assert rf.status_string(0) == "ok"
    assert "invalid" in rf.status_string(-1)
    assert re.match(r"^\d+\.\d+\.\d+$", rf.version())


def _beam(nchan=4, nsamp=8, stride=None, dtype=rf.RFIM_U8, inp=4096, out=4096, flags=None):
    b = rf.rfim_beam()
    b.dtype, b.reserved = dtype, 0
    b.nchan, b.nsamp, b.row_stride = nchan, nsamp, stride if stride is not None else nsamp
    b.in_, b.out, b.flags = inp, out, flags
    return b


def _run(beams, steps):
    arr = (rf.rfim_beam * len(beams))(*beams)
    st = rf.make_steps(steps)
    return rf.lib().rfim_pipeline_run(arr, len(beams), st, len(steps), None, None)


@pytest.mark.parametrize("beam,steps", [
    (dict(nchan=0), [("td", 3.0, "mean", 0)]),
    (dict(nsamp=0), [("td", 3.0, "mean", 0)]),
    (dict(stride=4), [("td", 3.0, "mean", 0)]),
    (dict(), [("td", -1.0, "mean", 0)]),
    (dict(), [("td", float("nan"), "mean", 0)]),
    (dict(), [("td", float("inf"), "mean", 0)]),
    (dict(nchan=6), [("fd", 3.0, "mean", 4)]),
    (dict(dtype=7), [("td", 3.0, "mean", 0)]),
    (dict(inp=0), [("td", 3.0, "mean", 0)]),
    (dict(inp=4096, out=4100), [("td", 3.0, "mean", 0)]),          # partial overlap
    (dict(flags=1 << 20), [("td", 3.0, "mean", 0)] * 9),            # > 8 steps with flags
    (dict(flags=4096 + 8, inp=4096, out=4096), [("td", 3.0, "mean", 0)]),  # flags overlap data
])
def test_invalid_arguments_rejected_on_host(beam, steps):
    assert _run([_beam(**beam)], steps) == rf.RFIM_ERR_INVALID_ARG


def test_bad_step_codes_rejected():
    st = (rf.rfim_step * 1)()
    st[0].domain, st[0].replace, st[0].k, st[0].bin_size = 5, 0, 1.0, 0
    arr = (rf.rfim_beam * 1)(_beam())
    assert rf.lib().rfim_pipeline_run(arr, 1, st, 1, None, None) == rf.RFIM_ERR_INVALID_ARG
    st[0].domain, st[0].replace = 0, 9
    assert rf.lib().rfim_pipeline_run(arr, 1, st, 1, None, None) == rf.RFIM_ERR_INVALID_ARG


def test_masked_steps_refused_for_float32_on_host():
    """Masked TD steps run on uint8 beams only; a call with any float32 beam is
    refused before anything is enqueued."""
    st = [("td_masked", 3.0, "mean", 0)]
    assert _run([_beam(dtype=rf.RFIM_F32)], st) == rf.RFIM_ERR_UNSUPPORTED
    assert _run([_beam(inp=1 << 20, out=1 << 21), _beam(dtype=rf.RFIM_F32)], st) == rf.RFIM_ERR_UNSUPPORTED
    assert _run([_beam()], [("td_masked", -1.0, "mean", 0)]) == rf.RFIM_ERR_INVALID_ARG


def test_header_step_codes_match_the_binding():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "rfim.h")).read()
    m = re.search(r"typedef enum \{([^}]*)\} rfim_domain;", hdr)
    vals = {k: int(v) for k, v in re.findall(r"(RFIM_\w+) = (\d+)", m.group(1))}
    assert vals == {"RFIM_TD": rf.RFIM_TD, "RFIM_FD": rf.RFIM_FD, "RFIM_TD_MASKED": rf.RFIM_TD_MASKED}


def test_plan_create_rejects_bad_shapes():
    arr = (rf.rfim_beam * 1)(_beam(nchan=6))
    st = rf.make_steps([("fd", 2.0, "mean", 4)])
    h = ctypes.c_void_p()
    assert rf.lib().rfim_plan_create(arr, 1, st, 1, None, ctypes.byref(h)) == rf.RFIM_ERR_INVALID_ARG
    assert not h.value

