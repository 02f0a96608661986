"""C ABI host-side checks (no GPU): the library loads, exports every declared
symbol, validates meshes, and layers regions exactly like the oracle."""
import os
import re

import numpy as np
import pytest

import paper_2405_10505_amd as F
from oracle import regions, trisk
from paper_2405_10505_amd.inputs import meshgen, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fblts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fblts_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    syms = declared_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(L, s), s
    # and the binding declares a signature for each of them
    assert set(syms) == set(F._SIGS), set(syms) ^ set(F._SIGS)


def test_version_and_error_string():
    assert F.lib().fblts_version() >= 100
    with pytest.raises(F.FBLTSError) as e:
        F._check(F.lib().fblts_mesh_create(None, None))
    assert e.value.code == F.FBLTS_EINVAL


def test_autotune_argument_checks_need_no_device():
    L = F.lib()
    for args in ((None, F.HANDLE_SOLVER, 5, 1), (None, F.HANDLE_ENSEMBLE, 5, 1)):
        rc = L.fblts_autotune(*args, None, None, None, 0, None)
        assert rc == F.FBLTS_EINVAL and b"NULL" in L.fblts_last_error()


@pytest.fixture(scope="module")
def hexm():
    return meshgen.hex_periodic(16, 16, 1.0e4)


def _bad(mesh, **kw):
    return mesh.copy_with(**kw)


@pytest.mark.parametrize("mutate,msg", [
    (lambda m: dict(cells_on_edge=np.where(np.arange(m.n_edges * 2).reshape(-1, 2) == 5, 10 ** 6, m.cells_on_edge)),
     "cells_on_edge"),
    (lambda m: dict(kite_areas_on_vertex=m.kite_areas_on_vertex * np.where(np.arange(m.n_vertices)[:, None] == 3, 1.5, 1.0)),
     "kite"),
    (lambda m: dict(dc_edge=np.where(np.arange(m.n_edges) == 7, -1.0, m.dc_edge)), "dc_edge"),
    (lambda m: dict(bottom_depth=np.where(np.arange(m.n_cells) == 2, 0.0, m.bottom_depth)), "bottom_depth"),
    (lambda m: dict(vertices_on_edge=m.vertices_on_edge[:, ::-1].copy()), "orientation"),
    (lambda m: dict(edges_on_cell=np.concatenate([m.edges_on_cell[:6][::-1], m.edges_on_cell[6:]])),
     "counter-clockwise"),
])
def test_mesh_validation_rejects(hexm, mutate, msg):
    bad = _bad(hexm, **mutate(hexm))
    with pytest.raises(F.FBLTSError) as e:
        F.Mesh(bad)
    assert e.value.code == F.FBLTS_EINVAL
    assert msg in str(e.value) or "vertex j" in str(e.value)


@pytest.mark.parametrize("name", ["small_cvt", "config1", "small_sphere"])
def test_plan_ranges_cover_the_regions(name):
    """fblts_plan (host): region counts equal the oracle's layering; the coarse
    advancement covers the coarse region and reaches into the fine region by
    fewer cells at later stages; a fine substep covers the fine region and its
    third stage the interface accumulations; linear stencils are never wider
    than nonlinear ones."""
    w = getattr(workloads, name)()
    fm = F.Mesh(w.mesh)
    ref, _ = regions.layer(trisk.OMesh(w.mesh), w.fine_mask, 2)
    p = fm.plan(np.where(w.fine_mask, 0, 1), nonlinear=True)
    pl = fm.plan(np.where(w.fine_mask, 0, 1), nonlinear=False)
    assert [p["n_fine"], p["n_if1"], p["n_if2"], p["n_int"]] == [int(np.sum(ref == k)) for k in range(4)]
    cells, e = w.mesh.cells_on_edge, ref[w.mesh.cells_on_edge].min(axis=1)   # an edge's region: its finer cell
    assert [p["n_fine_e"], p["n_if1_e"], p["n_if2_e"], p["n_int_e"]] == [int(np.sum(e == k)) for k in range(4)]
    nF, nFE = p["n_fine"], p["n_fine_e"]
    nIF, nIFE = nF + p["n_if1"] + p["n_if2"], nFE + p["n_if1_e"] + p["n_if2_e"]
    for q in (p, pl):
        cb, eb = q["coarse_cell_begin"], q["coarse_edge_begin"]
        assert cb[0] <= cb[1] <= cb[2] <= nF and eb[0] <= eb[1] <= eb[2] <= nFE
        fc, fe = q["fine_cell_end"], q["fine_edge_end"]
        assert min(fc) >= nF and fe[0] >= nFE and fe[1] >= nFE
        assert fc[2] >= nIF and fe[2] >= nIFE
        assert all(x <= p["n_cells"] for x in fc) and all(x <= p["n_edges"] for x in fe)
    assert all(a >= b for a, b in zip(pl["coarse_cell_begin"], p["coarse_cell_begin"]))
    assert all(a <= b for a, b in zip(pl["fine_cell_end"], p["fine_cell_end"]))


def test_layering_matches_oracle_and_rejects_bad_labels():
    w = workloads.small_cvt()
    fm = F.Mesh(w.mesh)
    lab, layer = fm.layer_regions(np.where(w.fine_mask, 0, 1), binary=True, r=2)
    ref, depth = regions.layer(trisk.OMesh(w.mesh), w.fine_mask, 2)
    assert np.array_equal(lab, ref)
    assert np.array_equal(-layer[w.fine_mask], depth[w.fine_mask])
    # fine next to interface two violates the one-region-apart rule
    bad = lab.copy()
    cells = w.mesh.cells_on_edge
    e = np.nonzero((lab[cells[:, 0]] == 0) & (lab[cells[:, 1]] == 1))[0][0]
    bad[cells[e, 1]] = 2
    with pytest.raises(F.FBLTSError) as exc:
        fm.layer_regions(bad, binary=False)
    assert exc.value.code == F.FBLTS_EREGION
    with pytest.raises(F.FBLTSError):
        fm.layer_regions(np.full(w.mesh.n_cells, 7, np.int8), binary=False)


def test_binding_rejects_wrong_array_sizes():
    """The C ABI takes plain pointers; the binding checks every array's length
    before the library reads or writes through it (no GPU needed to reach the
    checks: they fail before any library call)."""
    import paper_2405_10505_amd as F
    from paper_2405_10505_amd.inputs import meshgen
    m = meshgen.hex_periodic(8, 8, 1.0e4)
    fm = F.Mesh(m)
    with pytest.raises(ValueError):
        fm.layer_regions(np.zeros(m.n_cells + 1, np.int8))
    with pytest.raises(ValueError):
        F._ptr(np.zeros(5), np.float64, 4, "h")
    with pytest.raises(ValueError):
        F._host(np.zeros(3), np.int8, 4, "labels")
