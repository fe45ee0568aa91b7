"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/sgml.h declares, validates arguments, and its
host-only schedule equals the oracle's expansion of Algorithm 3."""
import ctypes
import os
import re

import pytest

from oracle.core import schedule as oracle_schedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgml.h")


def _sgml():
    from paper_1703_07206_amd import sgml
    return sgml


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgml_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_entry_point():
    sg = _sgml()
    L = sg.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_workspace_bytes_validates_problems():
    sg = _sgml()
    ok = sg.workspace_bytes(2, 5)
    assert ok > 0 and ok % 256 == 0
    assert sg.workspace_bytes(2, 5, precision=sg.MIXED) > ok
    assert sg.workspace_bytes(2, 1) == 0            # too small a grid
    assert sg.workspace_bytes(2, 14) == 0           # beyond the supported 2D size
    assert sg.workspace_bytes(3, 11) == 0           # beyond the supported 3D size
    assert sg.workspace_bytes(4, 5) == 0            # bad dimension
    assert sg.workspace_bytes(2, 5, stencil=7) == 0  # bad stencil
    # workspace grows linearly with the node count (compact levels)
    big = sg.workspace_bytes(2, 12)
    assert big / (4097 ** 2) < 48


@pytest.mark.parametrize("n", [2, 3, 5, 9, 12])
@pytest.mark.parametrize("n_r", [1, 2, 0])
@pytest.mark.parametrize("sched", [0, 1])
def test_schedule_matches_oracle(n, n_r, sched):
    sg = _sgml()
    assert sg.schedule(n, n_r, sched) == oracle_schedule(n, n_r, sched)


def test_status_strings_and_argument_errors():
    sg = _sgml()
    L = sg.lib()
    assert sg.status_string(0) == "ok"
    assert "diverged" in sg.status_string(-5)
    ln = ctypes.c_int(0)
    assert L.sgml_schedule(0, 2, 0, None, None, 0, ctypes.byref(ln)) == sg.E_ARG
    assert L.sgml_schedule(5, 2, 7, None, None, 0, ctypes.byref(ln)) == sg.E_ARG
    assert L.sgml_schedule(5, 2, 0, None, None, 0, ctypes.byref(ln)) == sg.OK and ln.value == 15
    prob = sg.make_problem(2, 5)
    h = ctypes.c_void_p()
    # no workspace / misaligned workspace are rejected before any device call
    assert L.sgml_plan_create(ctypes.byref(prob), 0, None, 1 << 20, ctypes.byref(h)) == sg.E_WORKSPACE
    assert L.sgml_plan_create(ctypes.byref(prob), 0, 16, 1 << 30, ctypes.byref(h)) == sg.E_WORKSPACE
    assert L.sgml_plan_create(ctypes.byref(prob), 5, None, 0, ctypes.byref(h)) == sg.E_ARG
    bad = sg.make_problem(2, 1)
    assert L.sgml_plan_create(ctypes.byref(bad), 0, None, 0, ctypes.byref(h)) == sg.E_SHAPE
    assert L.sgml_solve(None, None, None, None, None, None, None) == sg.E_ARG
