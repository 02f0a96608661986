"""Pins of the oracle's time integrators and FB-LTS step (CPU).

Independent references: the exact semi-discrete solution exp(L t) y0 of the
linear configuration-1 problem (order of accuracy), textbook imaginary-axis
stability bounds of RK4 (2 sqrt 2) and RK(3,2) (sqrt 3), the paper's printed
time-step ratios (Table meshes, Section 2.1), the paper's statements that
M = 1 reduces FB-LTS to FB-RK(3,2) and that FB-LTS conserves mass (Theorem 1)
and absolute vorticity (Theorem 2), and the appendix's consistency of the
interface predictions for constant tendencies.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import meshgen, workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_fb_weights_are_the_papers():
    assert tuple(schemes.BETA) == tuple(GOLD["fb_weights"]["value"])


@pytest.fixture(scope="module")
def c1():
    w = workloads.config1()
    om = trisk.OMesh(w.mesh)
    lab, depth = regions.layer(om, w.fine_mask, 2)
    return w, om, lab


def test_config1_region_counts(c1):
    w, om, lab = c1
    assert np.bincount(lab, minlength=4).tolist() == [256, 128, 128, 512]


def _linear_matrix(om, ph):
    N, E = om.N, om.E
    cols = []
    for j in range(N + E):
        y = np.zeros(N + E)
        y[j] = 1.0
        u, eta = y[N:], y[:N]
        cols.append(np.concatenate([trisk.psi(om, u, om.H + eta, ph), trisk.phi(om, u, om.H + eta, ph)]))
    return np.array(cols).T


@pytest.fixture(scope="module")
def exact_c1(c1):
    w, om, lab = c1
    ph = trisk.Physics(linear=True)
    L = sp.csc_matrix(_linear_matrix(om, ph))
    T = 6000.0
    y0 = np.concatenate([w.h0 - om.H, w.u0])
    return T, expm_multiply(L * T, y0)


def _errors(w, om, step, dts, T, yT, lab):
    out = []
    IF = (lab == 1) | (lab == 2)
    for dt in dts:
        u, h = w.u0.copy(), w.h0.copy()
        for _ in range(int(round(T / dt))):
            u, h = step(u, h, dt)
        eh = h - om.H - yT[:om.N]
        eu = u - yT[om.N:]
        out.append((math.sqrt(np.mean(eh ** 2)), math.sqrt(np.mean(eu ** 2)), math.sqrt(np.mean(eh[IF] ** 2))))
    return np.array(out)


@pytest.mark.parametrize("scheme,order", [("fbrk32", 2), ("fblts2", 2), ("fblts4", 2), ("rk4", 4)])
def test_temporal_order_against_exact_solution(c1, exact_c1, scheme, order):
    w, om, lab = c1
    T, yT = exact_c1
    ph = trisk.Physics(linear=True)
    if scheme == "fbrk32":
        step = lambda u, h, dt: schemes.fbrk32_step(om, u, h, dt, ph)
    elif scheme == "rk4":
        step = lambda u, h, dt: schemes.rk4_step(om, u, h, dt, ph)
    else:
        M = int(scheme[-1])
        step = lambda u, h, dt: schemes.fblts_step(om, u, h, dt, M, ph, lab)
    err = _errors(w, om, step, [60.0, 30.0, 15.0], T, yT, lab)
    slopes = np.log2(err[:-1] / err[1:])
    # h (all cells), u (all edges), h on interface cells: paper Section 2.3 (second order everywhere)
    assert np.all(slopes[-1] > order - 0.1), slopes
    assert np.all(slopes[-1] < order + 0.2), slopes


def _step_matrix(om, ph, fn, dt):
    N, E = om.N, om.E
    cols = []
    for j in range(N + E):
        y = np.zeros(N + E)
        y[j] = 1.0
        u, h = fn(om, y[N:], om.H + y[:N], dt, ph)
        cols.append(np.concatenate([h - om.H, u]))
    return np.array(cols).T


def _rho(om, ph, fn, dt):
    return np.max(np.abs(np.linalg.eigvals(_step_matrix(om, ph, fn, dt))))


@pytest.fixture(scope="module")
def hex12():
    m = meshgen.hex_periodic(12, 12, 1.0e4)
    om = trisk.OMesh(m)
    ph = trisk.Physics(linear=True)
    wmax = np.max(np.abs(np.linalg.eigvals(_linear_matrix(om, ph))))
    return om, ph, wmax


def test_rk4_and_rk32_imaginary_axis_limits(hex12):
    om, ph, wmax = hex12
    for fn, bound in ((schemes.rk4_step, 2 * math.sqrt(2)), (schemes.rk32_step, math.sqrt(3))):
        dt = bound / wmax
        assert _rho(om, ph, fn, 0.995 * dt) <= 1 + 1e-12
        assert _rho(om, ph, fn, 1.005 * dt) > 1 + 1e-9


def test_fbrk32_stability_gain_matches_paper(hex12):
    """FB-RK(3,2) admits ~1.35x the RK4 step and 1.6-2.3x the RK(3,2) step (Table meshes, Section 2.1)."""
    om, ph, wmax = hex12
    lo, hi = 0.0, 6.0 / wmax
    for _ in range(22):
        mid = 0.5 * (lo + hi)
        if _rho(om, ph, schemes.fbrk32_step, mid) <= 1 + 1e-12:
            lo = mid
        else:
            hi = mid
    r_rk4 = lo / (2 * math.sqrt(2) / wmax)
    r_rk32 = lo / (math.sqrt(3) / wmax)
    assert abs(r_rk4 - GOLD["dt_ratio_fblts_fine_over_rk4_delbay2km"]["value"]) < 0.05, r_rk4
    g = GOLD["fbrk32_dt_gain_vs_rk32"]["value"]
    assert g[0] <= r_rk32 <= GOLD["dt_ratio_fblts_over_lts3_delbay2km"]["value"] + 0.05, r_rk32


@pytest.mark.parametrize("linear", [True, False])
def test_m1_all_coarse_all_fine_reductions(c1, linear):
    w, om, lab = c1
    ph = trisk.Physics(linear=linear)
    u, h = w.u0.copy(), w.h0.copy()
    ref = schemes.fbrk32_step(om, u, h, 60.0, ph)
    got = schemes.fblts_step(om, u, h, 60.0, 1, ph, lab)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    coarse = np.full(om.N, 3, np.int8)
    got = schemes.fblts_step(om, u, h, 60.0, 3, ph, coarse)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    fine = np.zeros(om.N, np.int8)
    got = schemes.fblts_step(om, u, h, 60.0, 3, ph, fine)
    uu, hh = u, h
    for _ in range(3):
        uu, hh = schemes.fbrk32_step(om, uu, hh, 60.0 / 3, ph)
    assert np.array_equal(uu, got[0]) and np.array_equal(hh, got[1])


@pytest.fixture(scope="module")
def cvt_small():
    w = workloads.small_cvt()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab


@pytest.mark.parametrize("M", [2, 4])
def test_theorem1_mass_and_theorem2_vorticity(cvt_small, M):
    w, om, lab = cvt_small
    assert set(np.unique(lab)) == {0, 1, 2, 3}
    ph = trisk.Physics(linear=False, cd=w.cd)
    u, h = w.u0.copy(), w.h0.copy()
    d0 = trisk.diagnostics(om, u, h, ph)
    for _ in range(40):
        u, h = schemes.fblts_step(om, u, h, w.dt * M / w.M, M, ph, lab)
    d1 = trisk.diagnostics(om, u, h, ph)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert abs(d1["abs_vorticity"] - d0["abs_vorticity"]) <= 1e-13 * d1["abs_vorticity_scale"]
    # negative control: interface left uncorrected (step 4 skipped)
    u, h = w.u0.copy(), w.h0.copy()
    for _ in range(40):
        u, h = schemes.fblts_step(om, u, h, w.dt * M / w.M, M, ph, lab, correct_interface=False)
    d2 = trisk.diagnostics(om, u, h, ph)
    assert abs(d2["mass"] - d0["mass"]) > 1e-11 * d0["mass"]


@pytest.mark.parametrize("M", [2, 3])
def test_theorem2_local_vorticity_f0_linear(c1, M):
    """f = 0, linear: every velocity update is a gradient of one cell field, so zeta_v never changes."""
    w, _, lab = c1
    m = w.mesh.copy_with(f_vertex=np.zeros(w.mesh.n_vertices), f_edge=np.zeros(w.mesh.n_edges))
    om = trisk.OMesh(m)
    ph = trisk.Physics(linear=True)
    u, h = w.u0.copy(), w.h0.copy()
    z0 = trisk.relative_vorticity(om, u)
    scale = np.max(trisk.relative_vorticity(om, np.abs(u)) * 0 + (np.abs(om.dc[om.eov] * u[om.eov]).sum(1) / om.Av))
    for _ in range(30):
        u, h = schemes.fblts_step(om, u, h, 60.0, M, ph, lab)
    assert np.max(np.abs(trisk.relative_vorticity(om, u) - z0)) <= 1e-13 * scale
    u2, h2 = w.u0.copy(), w.h0.copy()
    for _ in range(30):
        u2, h2 = schemes.fblts_step(om, u2, h2, 60.0, M, ph, lab, correct_interface=False)
    assert np.max(np.abs(trisk.relative_vorticity(om, u2) - z0)) > 1e-10 * scale


def test_rest_state_is_steady(cvt_small):
    w, om, lab = cvt_small
    ph = trisk.Physics(linear=False, cd=w.cd)
    u = np.zeros(om.E)
    h = om.H.copy()
    for _ in range(3):
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab)
    # exact up to the rounding of the FB averages (b h + (1-b) h need not equal h bitwise)
    assert np.max(np.abs(u)) < 1e-12
    assert np.max(np.abs(h - om.H) / om.H) < 1e-14


@pytest.mark.parametrize("M", [1, 2, 3, 4, 8])
def test_predictions_exact_for_constant_tendency(M):
    """Appendix: with coarse data from a constant tendency s, eq. preds returns the fine stage values."""
    r = np.random.default_rng(M)
    hn = r.normal(size=50)
    s = r.normal(size=50)
    dt = 0.7
    d = dt / M
    for k in range(M):
        H0, H1, H2, H3 = schemes.predictions(hn, hn + dt * s / 3, hn + dt * s / 2, hn + dt * s, M, k)
        tol = 1e-14 * (np.abs(hn).max() + dt * np.abs(s).max())
        np.testing.assert_allclose(H0, hn + k * d * s, atol=tol)
        np.testing.assert_allclose(H1, hn + (k + 1 / 3) * d * s, atol=tol)
        np.testing.assert_allclose(H2, hn + (k + 1 / 2) * d * s, atol=tol)
        np.testing.assert_allclose(H3, hn + (k + 1) * d * s, atol=tol)
    # M = 1: exact pass-through of the coarse data
    H0, H1, H2, H3 = schemes.predictions(hn, hn + 1.0, hn + 2.0, hn + 3.0, 1, 0)
    assert np.array_equal(H0, hn) and np.array_equal(H1, hn + 1.0) and np.array_equal(H2, hn + 2.0)


@pytest.mark.parametrize("scheme", ["fbrk32", "fblts"])
def test_inertial_oscillation_with_quadratic_drag_closed_form(scheme):
    """A uniform flow over uniform depth H on the regular hexagon stays uniform,
    with h = H, and its velocity obeys dV/dt = -f k x V - (C_D / H) |V| V.  In
    complex form V(t) = V0 exp(-i f t) / (1 + C_D |V0| t / H): the speed decays
    as the quadratic law fixes and the direction turns at the inertial rate.
    FB-RK(3,2) and FB-LTS (M = 4, fine band with two interface layers) converge
    to it at second order."""
    m = meshgen.hex_periodic(16, 16, 1.0e4, depth=10.0)
    om = trisk.OMesh(m)
    H, cd, f, T = 10.0, 2.5e-3, 1e-4, 7200.0
    U0 = np.array([1.3, -0.6])
    ph = trisk.Physics(linear=False, cd=np.full(om.N, cd))
    s = 1.0 / (1.0 + cd / H * np.hypot(*U0) * T)
    c, sn = math.cos(f * T), math.sin(f * T)
    V = s * np.array([c * U0[0] + sn * U0[1], -sn * U0[0] + c * U0[1]])
    mask = np.zeros(om.N, bool)
    mask[:64] = True
    lab, _ = regions.layer(om, mask, 2)
    errs = []
    for n in (48, 96):
        dt = T / n
        u, h = m.normal_edge @ U0, np.full(om.N, H)
        for _ in range(n):
            if scheme == "fbrk32":
                u, h = schemes.fbrk32_step(om, u, h, dt, ph)
            else:
                u, h = schemes.fblts_step(om, u, h, dt, 4, ph, lab)
        errs.append(np.max(np.abs(u - m.normal_edge @ V)) / np.hypot(*U0))
    assert errs[1] < 2e-5, errs
    assert 3.4 < errs[0] / errs[1] < 4.6, errs


def test_theorems_on_the_sphere_with_a_moving_storm():
    """Theorems 1 and 2 on the small spherical mesh (f varies with latitude)
    with quadratic drag and the moving cyclone's wind stress: FB-LTS (M = 4)
    keeps the total mass to 1e-13 relative and the absolute vorticity to
    1e-13 of its scale over 10 coarse steps; with the interface left
    uncorrected the mass drifts."""
    w = workloads.small_sphere()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    assert {0, 1, 2} <= set(np.unique(lab).tolist())
    storm = w.meta["storm"]

    def run(correct):
        u, h = w.u0.copy(), w.h0.copy()
        for n in range(10):
            ph = trisk.Physics(linear=False, cd=w.cd, wind=storm.edge_forcing(w.mesh, n * w.dt))
            u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab, correct_interface=correct)
        return u, h

    ph0 = trisk.Physics(linear=False, cd=w.cd)
    d0 = trisk.diagnostics(om, w.u0, w.h0, ph0)
    u, h = run(True)
    d1 = trisk.diagnostics(om, u, h, ph0)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert abs(d1["abs_vorticity"] - d0["abs_vorticity"]) <= 1e-13 * d1["abs_vorticity_scale"]
    u, h = run(False)
    d2 = trisk.diagnostics(om, u, h, ph0)
    assert abs(d2["mass"] - d0["mass"]) > 1e-11 * d0["mass"]
