"""GPU parity: the HIP library against the FP64 oracle (runs on an MI355X).

Tolerances (FP64, different rounding order only):
  * single tendency evaluations: max |gpu - oracle| <= 1e-13 * max |oracle|;
  * trajectories after 100 coarse steps: relative L2 <= 1e-10 per field;
  * conserved totals over 100 steps: mass <= 1e-13 relative, absolute
    vorticity <= 1e-13 of sum |eta| A_v (Theorems 1 and 2);
  * integer work (region labels) and library-internal reductions (M = 1 vs
    FB-RK(3,2), graph vs direct launches, repeated runs, ensemble member vs
    single solver): bitwise.
"""
import numpy as np
import pytest

import paper_2405_10505_amd as F
from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import workloads

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def c1():
    w = workloads.config1()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab, F.Mesh(w.mesh)


@pytest.fixture(scope="module")
def cvt():
    w = workloads.small_cvt()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab, F.Mesh(w.mesh)


def _solver(fm, w, scheme=F.SCHEME_FBLTS, M=None, dt=None, lab=None, graph=False, drag=True):
    s = F.Solver(fm, dt if dt is not None else w.dt, M=M or w.M, scheme=scheme, linear=w.linear)
    if lab is None:
        lab = np.where(w.fine_mask, 0, 1)
        s.set_regions(lab, binary=True)
    else:
        s.set_regions(lab, binary=False)
    if drag and w.cd is not None and not w.linear:
        s.set_drag(w.cd)
    s.set_state(w.h0, w.u0)
    if graph:
        s.set_graph(True)
    return s


def _phys(w, drag=True):
    return trisk.Physics(linear=w.linear, cd=w.cd if (drag and not w.linear) else None)


@pytest.mark.parametrize("name", ["c1", "cvt"])
def test_tendencies_match_oracle(name, request):
    w, om, lab, fm = request.getfixturevalue(name)
    s = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1)
    r = np.random.default_rng(3)
    u = 0.5 * r.normal(size=om.E)
    h = om.H + 2.0 * r.normal(size=om.N)
    ph = _phys(w)
    gp = s.tendency(0, h, u)
    gf = s.tendency(1, h, u)
    assert rel_max(gp, trisk.psi(om, u, h, ph)) <= 1e-13
    assert rel_max(gf, trisk.phi(om, u, h, ph)) <= 1e-13


def test_region_labels_bitwise(cvt):
    w, om, lab, fm = cvt
    got, _ = fm.layer_regions(np.where(w.fine_mask, 0, 1), binary=True, r=2)
    assert np.array_equal(got, lab)


@pytest.mark.parametrize("name,M,steps", [("c1", 2, 100), ("c1", 4, 100), ("cvt", 4, 100), ("cvt", 2, 60)])
def test_fblts_trajectory_and_conservation(name, M, steps, request):
    w, om, lab, fm = request.getfixturevalue(name)
    dt = w.dt * M / w.M
    s = _solver(fm, w, M=M, dt=dt)
    d0 = s.diagnostics()
    s.step(steps)
    hg, ug = s.get_state()
    d1 = s.diagnostics()
    ph = _phys(w)
    u, h = w.u0.copy(), w.h0.copy()
    for _ in range(steps):
        u, h = schemes.fblts_step(om, u, h, dt, M, ph, lab)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["abs_vorticity"] - d0["abs_vorticity"]) <= 1e-13 * d1["abs_vorticity_scale"]
    od = trisk.diagnostics(om, u, h, ph)
    assert abs(d1["mass"] - od["mass"]) <= 1e-13 * abs(od["mass"])
    assert abs(d1["energy"] - od["energy"]) <= 1e-10 * abs(od["energy"])


@pytest.mark.parametrize("scheme", [F.SCHEME_FBRK32, F.SCHEME_RK4])
@pytest.mark.parametrize("name", ["c1", "cvt"])
def test_global_schemes_match_oracle(scheme, name, request):
    w, om, lab, fm = request.getfixturevalue(name)
    dt = w.dt / w.M
    s = _solver(fm, w, scheme=scheme, M=1, dt=dt)
    s.step(50)
    hg, ug = s.get_state()
    ph = _phys(w)
    u, h = w.u0.copy(), w.h0.copy()
    step = schemes.fbrk32_step if scheme == F.SCHEME_FBRK32 else schemes.rk4_step
    for _ in range(50):
        u, h = step(om, u, h, dt, ph)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10


@pytest.mark.parametrize("name", ["c1", "cvt"])
def test_m1_all_coarse_all_fine_bitwise_on_gpu(name, request):
    """Section 2.2: M = 1 is FB-RK(3,2); no fine cells: FB-RK(dt); all fine: M steps of FB-RK(dt/M)."""
    w, om, lab, fm = request.getfixturevalue(name)
    dt = w.dt / w.M
    ref = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1, dt=dt)
    ref.step(5)
    hr, ur = ref.get_state()
    m1 = _solver(fm, w, M=1, dt=dt, lab=lab)
    m1.step(5)
    h1, u1 = m1.get_state()
    assert np.array_equal(h1, hr) and np.array_equal(u1, ur)
    allc = _solver(fm, w, M=3, dt=dt, lab=np.full(om.N, 3, np.int8))
    allc.step(5)
    h2, u2 = allc.get_state()
    assert np.array_equal(h2, hr) and np.array_equal(u2, ur)
    allf = _solver(fm, w, M=3, dt=3 * dt, lab=np.zeros(om.N, np.int8))
    allf.step(5)
    ref3 = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1, dt=3 * dt / 3)
    ref3.step(15)
    h3, u3 = allf.get_state()
    hr3, ur3 = ref3.get_state()
    assert np.array_equal(h3, hr3) and np.array_equal(u3, ur3)


@pytest.mark.parametrize("name", ["c1", "cvt"])
def test_graph_replay_and_determinism_bitwise(name, request):
    w, om, lab, fm = request.getfixturevalue(name)
    a = _solver(fm, w)
    b = _solver(fm, w, graph=True)
    c = _solver(fm, w)
    for _ in range(4):
        a.step(3)
        b.step(3)
        c.step(3)
        ha, ua = a.get_state()
        hb, ub = b.get_state()
        hc, uc = c.get_state()
        assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
        assert np.array_equal(ha, hc) and np.array_equal(ua, uc)


def test_device_tensors_roundtrip(cvt):
    torch = pytest.importorskip("torch")
    w, om, lab, fm = cvt
    s = _solver(fm, w)
    ht = torch.tensor(w.h0, device="cuda", dtype=torch.float64)
    ut = torch.tensor(w.u0 + 0.01, device="cuda", dtype=torch.float64)
    s.set_state(ht, ut)
    ho = torch.empty_like(ht)
    uo = torch.empty_like(ut)
    s.get_state(ho, uo)
    assert torch.equal(ho, ht) and torch.equal(uo, ut)
    s.step(2)
    s.get_state(ho, uo)
    hn, un = s.get_state()
    assert np.array_equal(ho.cpu().numpy(), hn) and np.array_equal(uo.cpu().numpy(), un)


def test_nonfinite_reported(cvt):
    w, om, lab, fm = cvt
    s = _solver(fm, w)
    h = w.h0.copy()
    h[7] = np.nan
    s.set_state(h, w.u0)
    with pytest.raises(F.FBLTSError) as e:
        s.diagnostics()
    assert e.value.code == F.FBLTS_ENONFINITE


@pytest.mark.parametrize("fuse,bs,cells", [(0, 256, 0), (1, 64, 0), (0, 128, 0), (1, 128, 0), (1, 256, 1),
                                           (0, 64, 1)])
@pytest.mark.parametrize("name", ["c1", "cvt"])
def test_launch_options_bitwise(name, fuse, bs, cells, request):
    """Tuning options change the launch structure only: results are bitwise equal
    (the generated meshes' weights are exactly the kite-fraction walks)."""
    w, om, lab, fm = request.getfixturevalue(name)
    ref = _solver(fm, w)
    ref.step(4)
    s = _solver(fm, w)
    s.set_option(F.OPT_FUSE_VERTEX, fuse)
    s.set_option(F.OPT_BLOCK, bs)
    s.set_option(F.OPT_EDGE_CELLS, cells)
    s.step(4)
    hr, ur = ref.get_state()
    hs, us = s.get_state()
    assert np.array_equal(hr, hs) and np.array_equal(ur, us)


def test_autotuner_restores_state_and_picks_a_candidate(cvt, tmp_path):
    import json
    from paper_2405_10505_amd import autotune
    w, om, lab, fm = cvt
    s = _solver(fm, w)
    s.step(3)
    h0, u0 = s.get_state()
    d0 = s.diagnostics()
    path = str(tmp_path / "tune.json")
    choice = autotune.autotune(s, steps=5, repeats=1, cache_path=path)
    key = lambda c: (c["fuse_vertex"], c["block"], c["edge_cells"], c["persistent"])   # noqa: E731
    assert key(choice) in autotune.CANDIDATES
    assert choice["from_cache"] == 0 and choice["ms_per_step"] > 0
    timed = [key(c) for c in choice["candidates"]]
    # every per-pass schedule, the persistent launch, then (where the mesh
    # allows it) every schedule of the cells variant
    assert len(timed) in (10, 16) and timed == autotune.CANDIDATES[:len(timed)]
    assert choice["ms_per_step"] == min(c["ms_per_step"] for c in choice["candidates"])
    h1, u1 = s.get_state()
    assert np.array_equal(h0, h1) and np.array_equal(u0, u1)
    d1 = s.diagnostics()
    assert (d1["time"], d1["step"]) == (d0["time"], d0["step"])
    # the cache is JSON with one entry, and a second call reads it without timing
    entries = json.load(open(path))
    assert len(entries) == 1 and list(entries.values())[0]["block"] == choice["block"]
    again = autotune.autotune(s, cache_path=path)
    assert again["from_cache"] == 1 and again["candidates"] == []
    assert key(again) == key(choice)
    # stepping after tuning continues the trajectory bit for bit
    ref = _solver(fm, w)
    ref.step(5)
    s.step(2)
    hr, ur = ref.get_state()
    h2, u2 = s.get_state()
    assert np.array_equal(hr, h2) and np.array_equal(ur, u2)


def test_autotuner_rejects_foreign_cache_files(cvt, tmp_path):
    w, om, lab, fm = cvt
    s = _solver(fm, w)
    path = tmp_path / "other.json"
    path.write_text('{\n "solver": {\n  "block": 64\n }\n}\n')
    with pytest.raises(F.FBLTSError) as e:
        s.autotune(steps=1, repeats=1, cache_path=str(path))
    assert e.value.code == F.FBLTS_EINVAL and "schedule cache" in str(e.value)
    assert path.read_text().startswith('{\n "solver"')   # left untouched


def test_dispatch_timing_mode_counts_launches_and_keeps_results(cvt):
    """Timing mode launches directly with dispatch-recorded events: same bits, one timed launch per pass."""
    w, om, lab, fm = cvt
    ref = _solver(fm, w)
    ref.step(3)
    s = _solver(fm, w)
    s.set_timing(True)
    s.step(3)
    ms, launches = s.kernel_time(0)
    info = s.info()
    assert ms > 0
    # pipelined step: 3 stages x (coarse + M fine), the first two stages of
    # fine substep 0 sharing the coarse stages 2 and 3's launches
    assert launches % 3 == 0 and launches // 3 == 3 * (1 + w.M) - 2
    for cls in (1, 3):
        m2, n2 = s.kernel_time(cls)
        assert m2 > 0 and n2 > 0
    s.set_timing(False)
    hr, ur = ref.get_state()
    hs, us = s.get_state()
    assert np.array_equal(hr, hs) and np.array_equal(ur, us)
    assert info["launches_per_step"] > 0
    # the sequential step: one momentum launch per stage
    s.set_option(F.OPT_PIPELINE, 0)
    s.set_timing(True)
    s.step(3)
    assert s.kernel_time(0)[1] == 3 * 3 * (1 + w.M)
    s.set_timing(False)


def test_edge_cells_rejected_for_foreign_weights(cvt):
    """A mesh whose stored weights are not the kite-fraction walks cannot use the
    cell-walk momentum pass; the default pass still runs on it."""
    w, om, lab, fm = cvt
    bad = w.mesh.copy_with(weights_on_edge=w.mesh.weights_on_edge * (1 + 1e-9))
    s = F.Solver(F.Mesh(bad), w.dt, M=w.M)
    s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
    with pytest.raises(F.FBLTSError) as e:
        s.set_option(F.OPT_EDGE_CELLS, 1)
    assert e.value.code == F.FBLTS_EINVAL
    s.set_state(w.h0, w.u0)
    s.step(1)


def test_edge_cells_on_the_sphere_with_cyclone_bitwise():
    import dataclasses
    w = workloads.small_sphere()
    fm = F.Mesh(w.mesh)
    storm = dataclasses.replace(w.meta["storm"], rm=400e3)
    out = []
    for cells in (0, 1):
        s = F.Solver(fm, w.dt, M=w.M)
        s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
        s.set_drag(w.cd)
        s.set_state(w.h0, w.u0)
        s.set_cyclone(w.mesh.x_edge, w.mesh.normal_edge, **storm.cyclone_kwargs())
        s.set_option(F.OPT_EDGE_CELLS, cells)
        s.step(5)
        out.append(s.get_state())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("G", [1, 3, 8])
def test_multi_step_graphs_bitwise(cvt, G):
    """Several coarse steps per captured graph: any mix of multi-step and single
    step replays gives the bits of direct launches."""
    w, om, lab, fm = cvt
    a = _solver(fm, w)
    b = _solver(fm, w, graph=True)
    b.set_option(F.OPT_GRAPH_STEPS, G)
    for n in (11, 2, 7):
        a.step(n)
        b.step(n)
        ha, ua = a.get_state()
        hb, ub = b.get_state()
        assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
    with pytest.raises(F.FBLTSError):
        b.set_option(F.OPT_GRAPH_STEPS, 0)
