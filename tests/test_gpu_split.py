"""GPU parity of the gravity-wave system and the operator-split FB-LTS
(Sections 2.4, 3.2 and 4.2) against the oracle (runs on an MI355X).

Tolerances as for the unsplit path (FP64, different rounding order):
  * single tendencies (fast Phi, slow Phi): max |gpu - oracle| <= 1e-13 max |oracle|;
  * trajectories: relative L2 <= 1e-10 per field; total mass to 1e-13;
  * reductions that hold bitwise in the oracle (M = 1, all-coarse, all-fine with
    per-substep slow terms) and graph replays: bitwise;
  * temporal order of FB-LTS on the aquaplanet gravity wave: fitted slope in [1.8, 2.3].
"""
import math

import numpy as np
import pytest

import paper_2405_10505_amd as F
from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def aqua():
    w = workloads.aquaplanet()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab, F.Mesh(w.mesh)


@pytest.fixture(scope="module")
def cvt():
    w = workloads.small_cvt()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab, F.Mesh(w.mesh)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solver(fm, w, lab=None, scheme=F.SCHEME_FBLTS, M=None, dt=None, physics=F.PHYS_NONLINEAR, split=0,
            drag=True, graph=False, h0=None, u0=None):
    s = F.Solver(fm, dt or w.dt, M=M or w.M, scheme=scheme, physics=physics, split=split)
    if lab is None:
        s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
    else:
        s.set_regions(lab, binary=False)
    if drag and w.cd is not None and physics == F.PHYS_NONLINEAR:
        s.set_drag(w.cd)
    s.set_state(w.h0 if h0 is None else h0, w.u0 if u0 is None else u0)
    s.set_graph(graph)
    return s


def _state(om, seed):
    r = np.random.default_rng(seed)
    return 0.3 * r.normal(size=om.E), om.H * (1 + 0.01 * r.normal(size=om.N))


def test_gravity_wave_tendencies_match_oracle(aqua):
    w, om, lab, fm = aqua
    s = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1, physics=F.PHYS_GRAVITY_WAVE)
    u, h = _state(om, 1)
    ph = trisk.Physics(gravity_wave=True)
    ref_p, ref_f = trisk.psi(om, u, h, ph), trisk.phi_fast(om, u, h, ph)
    assert np.max(np.abs(s.tendency(0, h, u) - ref_p)) <= 1e-13 * np.max(np.abs(ref_p))
    assert np.max(np.abs(s.tendency(1, h, u) - ref_f)) <= 1e-13 * np.max(np.abs(ref_f))


def test_slow_tendency_matches_oracle(cvt):
    w, om, lab, fm = cvt
    s = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1)
    r = np.random.default_rng(2)
    wind = (10 * r.normal(size=om.E), 10 * r.normal(size=om.E), 1e-3 * (1.0 + r.uniform(size=om.E)))
    s.set_wind(*wind)
    u, h = _state(om, 3)
    ref = trisk.phi_slow(om, u, h, trisk.Physics(cd=w.cd, wind=wind))
    assert np.max(np.abs(s.tendency(2, h, u) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_gravity_wave_fblts_matches_oracle(aqua):
    w, om, lab, fm = aqua
    steps = 20
    s = _solver(fm, w, lab=lab, physics=F.PHYS_GRAVITY_WAVE)
    d0 = s.diagnostics()
    s.step(steps)
    hg, ug = s.get_state()
    d1 = s.diagnostics()
    ph = trisk.Physics(gravity_wave=True)
    u, h = w.u0.copy(), w.h0.copy()
    for _ in range(steps):
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])


@pytest.mark.parametrize("split", [1, 2])
def test_split_fblts_matches_oracle(cvt, split):
    w, om, lab, fm = cvt
    steps = 30
    s = _solver(fm, w, lab=lab, split=split)
    d0 = s.diagnostics()
    s.step(steps)
    hg, ug = s.get_state()
    d1 = s.diagnostics()
    ph = trisk.Physics(cd=w.cd)
    u, h = w.u0.copy(), w.h0.copy()
    for _ in range(steps):
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab, split=split)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["abs_vorticity"] - d0["abs_vorticity"]) <= 1e-13 * d1["abs_vorticity_scale"]


def test_split_fbrk32_matches_oracle(cvt):
    w, om, lab, fm = cvt
    dt = w.dt / w.M
    s = _solver(fm, w, scheme=F.SCHEME_FBRK32, M=1, dt=dt, split=1)
    s.step(40)
    hg, ug = s.get_state()
    ph = trisk.Physics(cd=w.cd)
    u, h = w.u0.copy(), w.h0.copy()
    for _ in range(40):
        u, h = schemes.fbrk32_step(om, u, h, dt, ph, split=True)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10


def test_split_with_moving_cyclone_matches_oracle():
    import dataclasses
    w = workloads.small_sphere()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    storm = dataclasses.replace(w.meta["storm"], rm=400e3)
    fm = F.Mesh(w.mesh)
    s = _solver(fm, w, lab=lab, split=1)
    s.set_cyclone(w.mesh.x_edge, w.mesh.normal_edge, **storm.cyclone_kwargs())
    steps = 20
    s.step(steps)
    hg, ug = s.get_state()
    u, h = w.u0.copy(), w.h0.copy()
    for k in range(steps):
        ph = trisk.Physics(cd=w.cd, wind=storm.edge_forcing(w.mesh, k * w.dt))
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab, split=1)
    assert np.linalg.norm(u) > 1e-3
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10
    assert rel_l2(ug, u) <= 1e-10


def test_split_reductions_bitwise_on_gpu(cvt):
    w, om, lab, fm = cvt
    u0, h0 = _state(om, 4)
    dt = w.dt / w.M

    def run(n, **kw):
        s = _solver(fm, w, h0=h0, u0=u0, **kw)
        s.step(n)
        return s.get_state()

    ref = run(4, scheme=F.SCHEME_FBRK32, M=1, dt=dt, split=1)
    for split in (1, 2):
        got = run(4, lab=lab, M=1, dt=dt, split=split)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        got = run(4, lab=np.full(om.N, 3, np.int8), M=3, dt=dt, split=split)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    ref3 = run(12, scheme=F.SCHEME_FBRK32, M=1, dt=dt / 3, split=1)
    got = run(4, lab=np.zeros(om.N, np.int8), M=3, dt=dt, split=2)
    assert np.array_equal(got[0], ref3[0]) and np.array_equal(got[1], ref3[1])


@pytest.mark.parametrize("kw", [dict(split=2), dict(physics=F.PHYS_GRAVITY_WAVE)])
def test_graph_replay_bitwise_fast_modes(cvt, kw):
    w, om, lab, fm = cvt
    a = _solver(fm, w, lab=lab, **kw)
    b = _solver(fm, w, lab=lab, graph=True, **kw)
    for _ in range(3):
        a.step(3)
        b.step(3)
        ha, ua = a.get_state()
        hb, ub = b.get_state()
        assert np.array_equal(ha, hb) and np.array_equal(ua, ub)


def test_aquaplanet_convergence_on_gpu(aqua):
    """Section 2.3's experiment on the device: FB-LTS (M = 4) errors against RK4
    at dt = 10 s, for coarse steps dt, dt/2, dt/4; the same figures as the oracle's."""
    w, om, lab, fm = aqua
    T = 4 * 3600.0
    ref = _solver(fm, w, scheme=F.SCHEME_RK4, M=1, dt=10.0, physics=F.PHYS_GRAVITY_WAVE,
                  lab=np.full(om.N, 3, np.int8))
    ref.step(int(round(T / 10.0)))
    _, href = ref.get_state()
    dts = [T / round(T / (w.dt / k)) for k in (1, 2, 4)]
    errs = []
    for dt in dts:
        s = _solver(fm, w, lab=lab, dt=dt, physics=F.PHYS_GRAVITY_WAVE, graph=True)
        s.step(int(round(T / dt)))
        _, h = s.get_state()
        errs.append(math.sqrt(np.mean((h - href) ** 2)))
    slope = float(np.polyfit(np.log(dts), np.log(errs), 1)[0])
    assert 1.8 <= slope <= 2.3, errs


def test_split_argument_errors(cvt):
    w, om, lab, fm = cvt
    for kw in (dict(physics=F.PHYS_LINEAR, split=1), dict(scheme=F.SCHEME_RK4, split=1),
               dict(scheme=F.SCHEME_FBRK32, split=2), dict(split=3), dict(physics=3)):
        with pytest.raises(F.FBLTSError) as e:
            F.Solver(fm, w.dt, M=w.M, **kw)
        assert e.value.code == F.FBLTS_EINVAL
    s = _solver(fm, w, lab=lab, split=1)
    with pytest.raises(F.FBLTSError) as e:
        s.adjoint_forward(2, 1)
    assert e.value.code == F.FBLTS_EINVAL
