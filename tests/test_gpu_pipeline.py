"""The pipelined FB-LTS step (FBLTS_OPT_PIPELINE, the default): the first fine
substep runs beside the coarse stages 2 and 3 on arrays of its own, the coarse
stages hand over their interface-one predictions and the interface-two and
interior values the third fine stage reads, and each substep's last momentum
pass carries the next prediction or the final correction and assembly.  The
arithmetic is that of the sequential pass list item by item, so trajectories
must equal it bit for bit: across M (1 to 16), interface widths, degenerate
fine sets, linear physics, both operator splittings, the gravity-wave system,
the moving storm, both momentum-pass forms, the persistent launch, and direct
and graph-replayed launches.  Its launch count is 9M + 3 per coarse step (q_v
fused) against 10M + 10."""
import dataclasses

import numpy as np
import pytest

import paper_2405_10505_amd as F
from paper_2405_10505_amd import autotune
from paper_2405_10505_amd.inputs import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvt():
    w = workloads.small_cvt()
    return w, F.Mesh(w.mesh)


def _solver(fm, w, pipeline, M=None, dt=None, fine=None, r=2, split=0, physics=None, storm=None, fuse=1,
            cells=0, persistent=0, graph=True):
    kw = dict(physics=physics) if physics is not None else dict(linear=w.linear)
    M = w.M if M is None else M
    s = F.Solver(fm, w.dt if dt is None else dt, M=M, split=split, r_layers=r, **kw)
    s.set_regions(np.where(w.fine_mask if fine is None else fine, 0, 1), binary=True)
    if w.cd is not None and not w.linear and physics != F.PHYS_GRAVITY_WAVE:
        s.set_drag(w.cd)
    s.set_state(w.h0, w.u0)
    if storm is not None:
        s.set_cyclone(w.mesh.x_edge, w.mesh.normal_edge, **storm.cyclone_kwargs())
    s.set_option(F.OPT_PIPELINE, pipeline)
    autotune.apply(s, dict(fuse_vertex=fuse, block=256 if persistent else 64, edge_cells=cells,
                           persistent=persistent))
    s.set_graph(graph)
    return s


def _same(steps, fm, w, **kw):
    out = []
    for pipeline in (0, 1):
        s = _solver(fm, w, pipeline, **kw)
        s.step(steps)
        h, u = s.get_state()
        out.append((h, u, s.diagnostics(), s.info()))
    (h0, u0, d0, i0), (h1, u1, d1, i1) = out
    assert d1["n_nonfinite"] == 0
    assert np.array_equal(h0, h1) and np.array_equal(u0, u1)
    return i0, i1


@pytest.mark.parametrize("fuse", [1, 0])
def test_pipeline_equals_sequential_step(cvt, fuse):
    w, fm = cvt
    i0, i1 = _same(9, fm, w, fuse=fuse)
    M = w.M
    if fuse:
        assert i0["launches_per_step"] == 10 * M + 10 and i1["launches_per_step"] == 9 * M + 3
    else:
        assert i0["launches_per_step"] == 13 * M + 13 and i1["launches_per_step"] == 12 * M + 4
    assert i0["cell_substeps_per_step"] == i1["cell_substeps_per_step"]


@pytest.mark.parametrize("M", [1, 2, 3, 16])
def test_pipeline_across_substep_counts(cvt, M):
    """Below the configuration's M the fine step is held at the configuration's
    (the coarse step M times it); above it the coarse step is held."""
    w, fm = cvt
    _same(7, fm, w, M=M, dt=w.dt if M >= w.M else w.dt / w.M * M)


def test_pipeline_thicker_interfaces(cvt):
    w, fm = cvt
    _same(7, fm, w, r=3)


def test_pipeline_single_fine_cell(cvt):
    w, fm = cvt
    fine = np.zeros(w.mesh.n_cells, bool)
    fine[int(np.argmin(w.mesh.area_cell))] = True
    # every other cell is coarse: the coarse step is the global fine limit
    _same(7, fm, w, fine=fine, M=3, dt=w.dt / w.M)


def test_pipeline_direct_launches(cvt):
    w, fm = cvt
    _same(6, fm, w, graph=False)


def test_pipeline_linear_inertia_gravity_waves():
    w = workloads.config1()
    _same(9, F.Mesh(w.mesh), w)


@pytest.mark.parametrize("split", [1, 2])
def test_pipeline_operator_splitting(cvt, split):
    w, fm = cvt
    _same(5, fm, w, split=split)


def test_pipeline_gravity_wave_system(cvt):
    w, fm = cvt
    _same(5, fm, w, physics=F.PHYS_GRAVITY_WAVE)


@pytest.mark.parametrize("cells", [0, 1])
def test_pipeline_sphere_with_moving_storm(cells):
    w = workloads.small_sphere()
    storm = dataclasses.replace(w.meta["storm"], rm=400e3)
    _same(6, F.Mesh(w.mesh), w, storm=storm, cells=cells)


def test_pipeline_persistent_launch(cvt):
    """Pipelined passes (two-segment launches, folded work) inside the
    cooperative launch against the sequential per-pass launches."""
    w, fm = cvt
    s = _solver(fm, w, 0)
    s.step(6)
    h0, u0 = s.get_state()
    s = _solver(fm, w, 1, persistent=1)
    s.step(6)
    h1, u1 = s.get_state()
    assert np.array_equal(h0, h1) and np.array_equal(u0, u1)


def test_ensembles_run_the_sequential_step():
    w = workloads.small_cvt(n=1500, seed=13)
    ens = F.Ensemble([F.Mesh(w.mesh)], [np.where(w.fine_mask, 0, 1)], [2], w.dt, M=w.M, linear=False)
    ens.set_option(F.OPT_PIPELINE, 0)
    with pytest.raises(F.FBLTSError):
        ens.set_option(F.OPT_PIPELINE, 1)


def test_on_off_options_take_zero_or_one(cvt):
    w, fm = cvt
    s = _solver(fm, w, 1)
    for opt in (F.OPT_PIPELINE, F.OPT_FUSE_VERTEX, F.OPT_EDGE_CELLS):
        with pytest.raises(F.FBLTSError):
            s.set_option(opt, 2)
        with pytest.raises(F.FBLTSError):
            s.set_option(opt, -1)
    # a refused value leaves the solver's options as they were
    s.step(2)
    assert s.info()["launches_per_step"] == 9 * w.M + 3
