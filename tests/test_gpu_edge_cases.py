"""GPU parity on the degenerate and extreme cases of the FB-LTS step (runs on
an MI355X): many fine substeps (M = 16), thicker interfaces (r = 3), a fine
set of a single cell, a fine band that wraps around the periodic domain, linear
physics on the sphere, and a state at rest (steady).  Tolerances as in the main
parity tests: relative L2 <= 1e-10 after the trajectory, total mass to 1e-13.
A uniform flow with quadratic drag also follows its closed form on the GPU."""
import numpy as np
import pytest

import paper_2405_10505_amd as F
from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import workloads

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _compare(w, fine, M, steps, r=2, linear=None, dt=None, h0=None, u0=None):
    linear = w.linear if linear is None else linear
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, fine, r)
    dt = dt or w.dt
    h0 = w.h0 if h0 is None else h0
    u0 = w.u0 if u0 is None else u0
    fm = F.Mesh(w.mesh)
    s = F.Solver(fm, dt, M=M, linear=linear, r_layers=r)
    s.set_regions(np.where(fine, 0, 1), binary=True)
    cd = w.cd if (w.cd is not None and not linear) else None
    if cd is not None:
        s.set_drag(cd)
    s.set_state(h0, u0)
    d0 = s.diagnostics()
    s.step(steps)
    hg, ug = s.get_state()
    d1 = s.diagnostics()
    ph = trisk.Physics(linear=linear, cd=cd)
    u, h = u0.copy(), h0.copy()
    for _ in range(steps):
        u, h = schemes.fblts_step(om, u, h, dt, M, ph, lab)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    return hg, ug, h, u, om, lab


def test_many_substeps_m16():
    # the M = 4 fine set at its coarse step, split into 16 substeps
    w = workloads.small_cvt()
    hg, ug, h, u, om, _ = _compare(w, w.fine_mask, 16, 10)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10 and rel_l2(ug, u) <= 1e-10


def test_thicker_interfaces_r3():
    w = workloads.small_cvt()
    hg, ug, h, u, om, lab = _compare(w, w.fine_mask, w.M, 20, r=3)
    assert np.count_nonzero(lab == 1) > 0 and np.count_nonzero(lab == 2) > 0
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10 and rel_l2(ug, u) <= 1e-10


def test_single_fine_cell():
    w = workloads.small_cvt()
    fine = np.zeros(w.mesh.n_cells, bool)
    fine[int(np.argmin(w.mesh.dc_edge[w.mesh.edges_on_cell[w.mesh.edges_on_cell_off[:-1]]]))] = True
    # every other cell is coarse, so the coarse step is the global fine limit
    hg, ug, h, u, om, lab = _compare(w, fine, 3, 20, dt=w.dt / w.M)
    assert np.count_nonzero(lab == 0) == 1
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10 and rel_l2(ug, u) <= 1e-10


def test_fine_band_wrapping_the_periodic_domain():
    w = workloads.config1()
    x = w.mesh.x_cell[:, 0]
    L = w.mesh.lx
    fine = (x < 0.15 * L) | (x > 0.85 * L)     # a column band across x = 0
    hg, ug, h, u, om, lab = _compare(w, fine, 2, 50)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10 and rel_l2(ug, u) <= 1e-10


def test_linear_physics_on_the_sphere():
    w = workloads.small_sphere()
    r = np.random.default_rng(4)
    h0 = w.mesh.bottom_depth + 0.5 * np.exp(-0.5 * ((np.arange(w.mesh.n_cells) % 97) / 20.0) ** 2)
    u0 = 0.01 * r.normal(size=w.mesh.n_edges)
    hg, ug, h, u, om, _ = _compare(w, w.fine_mask, w.M, 20, linear=True, h0=h0, u0=u0)
    assert rel_l2(hg - om.H, h - om.H) <= 1e-10 and rel_l2(ug, u) <= 1e-10


def test_rest_state_stays_at_rest():
    w = workloads.small_cvt()
    fm = F.Mesh(w.mesh)
    s = F.Solver(fm, w.dt, M=w.M, linear=False)
    s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
    s.set_drag(w.cd)
    s.set_state(w.mesh.bottom_depth, np.zeros(w.mesh.n_edges))
    s.step(20)
    h, u = s.get_state()
    assert np.max(np.abs(u)) <= 1e-12
    assert np.max(np.abs(h - w.mesh.bottom_depth)) <= 1e-9


def test_inertial_oscillation_with_quadratic_drag_closed_form():
    """The GPU FB-LTS step on a uniform flow with quadratic drag over uniform
    depth (regular hexagon, fine band, M = 4) follows the closed form
    V0 exp(-i f t) / (1 + C_D |V0| t / H) to second order, and matches the
    oracle on the same run."""
    import math
    from paper_2405_10505_amd.inputs import meshgen
    m = meshgen.hex_periodic(16, 16, 1.0e4, depth=10.0)
    om = trisk.OMesh(m)
    H, cd, f, T = 10.0, 2.5e-3, 1e-4, 7200.0
    U0 = np.array([1.3, -0.6])
    s_ = 1.0 / (1.0 + cd / H * np.hypot(*U0) * T)
    c, sn = math.cos(f * T), math.sin(f * T)
    V = s_ * np.array([c * U0[0] + sn * U0[1], -sn * U0[0] + c * U0[1]])
    fine = np.zeros(om.N, bool)
    fine[:64] = True
    lab, _ = regions.layer(om, fine, 2)
    fm = F.Mesh(m)
    errs = []
    for n in (48, 96):
        s = F.Solver(fm, T / n, M=4, linear=False)
        s.set_regions(np.where(fine, 0, 1), binary=True)
        s.set_drag(np.full(om.N, cd))
        s.set_state(np.full(om.N, H), m.normal_edge @ U0)
        s.step(n)
        hg, ug = s.get_state()
        errs.append(np.max(np.abs(ug - m.normal_edge @ V)) / np.hypot(*U0))
    assert errs[1] < 2e-5, errs
    assert 3.4 < errs[0] / errs[1] < 4.6, errs
    ph = trisk.Physics(linear=False, cd=np.full(om.N, cd))
    u, h = m.normal_edge @ U0, np.full(om.N, H)
    for _ in range(96):
        u, h = schemes.fblts_step(om, u, h, T / 96, 4, ph, lab)
    assert rel_l2(hg, h) <= 1e-10 and rel_l2(ug, u) <= 1e-10
