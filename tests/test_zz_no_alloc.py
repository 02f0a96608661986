"""The allocation-free diagnostics entry point (fblts_diagnostics_noalloc,
called through the C ABI) returns exactly what fblts_diagnostics returns, on
two calls in a row on one GPU, the second on a smaller mesh; the shared
scratch array keeps nothing that changes the second result."""
import ctypes as C

import numpy as np
import pytest

import paper_2405_10505_amd as F
from paper_2405_10505_amd.inputs import meshgen, workloads

pytestmark = pytest.mark.gpu

FIELDS = ("mass", "abs_vorticity", "abs_vorticity_scale", "energy", "min_h", "time", "n_nonfinite", "step")


def _noalloc(s):
    d = F.fblts_diag()
    rc = F.lib().fblts_diagnostics_noalloc(s.handle, C.byref(d))
    assert rc == F.FBLTS_OK, F.lib().fblts_last_error()
    return d.as_dict()


def _solver(w, steps):
    s = F.Solver(F.Mesh(w.mesh), w.dt, M=w.M, linear=w.linear)
    s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
    if w.cd is not None and not w.linear:
        s.set_drag(w.cd)
    s.set_state(w.h0, w.u0)
    s.step(steps)
    return s


def test_noalloc_diagnostics_equal_the_allocating_call():
    big = workloads.small_cvt(n=2000, seed=12)      # nonlinear with drag
    small = workloads.config1()                      # 1,024 cells, linear
    assert small.mesh.n_cells < big.mesh.n_cells
    for w, steps in ((big, 7), (small, 3)):
        s = _solver(w, steps)
        # the allocation-free call first, on a solver that has not allocated
        # its own reduction buffers yet
        a = _noalloc(s)
        b = s.diagnostics()
        for k in FIELDS:
            assert a[k] == b[k], (w.name, k, a[k], b[k])
        assert a["step"] == steps and a["mass"] > 0
    # a third call after both, on the larger mesh again
    s = _solver(big, 2)
    a, b = _noalloc(s), s.diagnostics()
    assert all(a[k] == b[k] for k in FIELDS)


def test_noalloc_diagnostics_reports_nonfinite_states():
    m = meshgen.hex_periodic(8, 8, 1.0e4, f0=1e-4, depth=1000.0)
    s = F.Solver(F.Mesh(m), 60.0, M=1, scheme=F.SCHEME_FBRK32, linear=True)
    s.set_regions(np.full(m.n_cells, 3, np.int8), binary=False)
    h = np.full(m.n_cells, 1000.0)
    h[5] = np.nan
    s.set_state(h, np.zeros(m.n_edges))
    d = F.fblts_diag()
    assert F.lib().fblts_diagnostics_noalloc(s.handle, C.byref(d)) == F.FBLTS_ENONFINITE
    assert d.n_nonfinite == 1
    assert s.diagnostics(allow_nonfinite=True)["n_nonfinite"] == 1
