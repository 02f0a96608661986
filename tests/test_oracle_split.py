"""Pins of the operator splitting (Section 3.2), its per-substep variant
(Section 4.2) and the gravity-wave system (Section 2.3) in the oracle (CPU).

Independent references:
  * the splitting is a decomposition of Phi: fast + slow equals the full
    tendency of the pinned TRiSK operators;
  * order of accuracy: the paper states that the splitting introduces a
    first-order error (Section 3.2) and that FB-LTS without slow terms is
    second order (Section 2.3); measured against an RK4 reference at a small
    step on a rotating problem (split: order 1) and on the non-rotating
    aquaplanet gravity wave (FB-LTS: order 2, the paper's own experiment);
  * reductions that follow from the definitions: M = 1 and an all-coarse
    fine set reduce split FB-LTS to split FB-RK(3,2); with every cell fine,
    refreshing the slow terms per substep gives M split FB-RK(3,2) steps of
    dt/M (and freezing them for the whole step does not);
  * Theorems 1 and 2 (mass, absolute vorticity) also hold for the split step.
"""
import math

import numpy as np
import pytest

from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import meshgen, workloads


@pytest.fixture(scope="module")
def cvt_small():
    w = workloads.small_cvt()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    return w, om, lab


def _state(om, seed):
    r = np.random.default_rng(seed)
    return 0.3 * r.normal(size=om.E), om.H * (1 + 0.01 * r.normal(size=om.N))


def test_fast_plus_slow_is_the_full_tendency(cvt_small):
    w, om, lab = cvt_small
    u, h = _state(om, 1)
    r = np.random.default_rng(2)
    wind = (10 * r.normal(size=om.E), 10 * r.normal(size=om.E), 1e-3 * (1.0 + r.uniform(size=om.E)))
    for ph in (trisk.Physics(cd=w.cd), trisk.Physics(cd=w.cd, wind=wind), trisk.Physics()):
        full = trisk.phi(om, u, h, ph)
        parts = trisk.phi_fast(om, u, h, ph) + trisk.phi_slow(om, u, h, ph)
        assert np.max(np.abs(parts - full)) <= 1e-12 * np.max(np.abs(full))
        # the slow part is not negligible on this state
        assert np.max(np.abs(trisk.phi_slow(om, u, h, ph))) > 1e-3 * np.max(np.abs(full))


def test_gravity_wave_physics_is_the_fast_system(cvt_small):
    w, om, lab = cvt_small
    u, h = _state(om, 3)
    gw = trisk.Physics(gravity_wave=True)
    assert np.array_equal(trisk.phi(om, u, h, gw), trisk.phi_fast(om, u, h, gw))
    assert np.array_equal(trisk.psi(om, u, h, gw), trisk.psi(om, u, h, trisk.Physics()))
    # at rest the nonlinear tendency has no slow part: both systems agree bitwise
    z = np.zeros(om.E)
    assert np.array_equal(trisk.phi(om, z, h, gw), trisk.phi(om, z, h, trisk.Physics()))


@pytest.fixture(scope="module")
def rotating():
    """Periodic hexagonal mesh, f = 1e-3, H = 100 m, SSH bump plus a cellular flow, drag."""
    m = meshgen.hex_periodic(16, 16, 1.0e4, f0=1e-3, depth=100.0)
    om = trisk.OMesh(m)
    L = m.lx
    xc, xe = m.x_cell, m.x_edge
    h0 = om.H + 2.0 * np.exp(-((xc[:, 0] - 0.5 * L) ** 2 + (xc[:, 1] - 0.5 * L) ** 2) / (2 * (0.15 * L) ** 2))
    U = np.stack([np.sin(2 * np.pi * xe[:, 1] / L), np.cos(2 * np.pi * xe[:, 0] / L)], 1)
    u0 = np.einsum("ij,ij->i", U, m.normal_edge)
    fine = (xc[:, 0] > 0.3 * L) & (xc[:, 0] < 0.6 * L)
    lab, _ = regions.layer(om, fine, 2)
    ph = trisk.Physics(cd=np.full(om.N, 2.5e-3))
    return om, u0, h0, lab, ph


def _run(step, u0, h0, T, dt):
    u, h = u0.copy(), h0.copy()
    for _ in range(int(round(T / dt))):
        u, h = step(u, h, dt)
    return u, h


def _slope(dts, errs):
    return float(np.polyfit(np.log(dts), np.log(errs), 1)[0])


def test_splitting_is_first_order_unsplit_second(rotating):
    om, u0, h0, lab, ph = rotating
    T = 2400.0
    _, href = _run(lambda u, h, dt: schemes.rk4_step(om, u, h, dt, ph), u0, h0, T, 2.5)
    dts = [120.0, 60.0, 30.0]
    for split, lo, hi in ((0, 1.8, 2.3), (1, 0.9, 1.35), (2, 0.9, 1.35)):
        errs = []
        for dt in dts:
            _, h = _run(lambda u, h, d: schemes.fblts_step(om, u, h, d, 4, ph, lab, split=split), u0, h0, T, dt)
            errs.append(math.sqrt(np.mean((h - href) ** 2)))
        assert lo <= _slope(dts, errs) <= hi, (split, errs)


@pytest.mark.parametrize("split", [1, 2])
def test_split_reductions(cvt_small, split):
    w, om, lab = cvt_small
    ph = trisk.Physics(cd=w.cd)
    u, h = _state(om, 4)
    dt = w.dt / w.M
    ref = schemes.fbrk32_step(om, u, h, dt, ph, split=True)
    for cl, M in ((lab, 1), (np.full(om.N, 3), 3)):
        got = schemes.fblts_step(om, u, h, dt, M, ph, cl, split=split)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    # every cell fine: per-substep slow terms give M split FB-RK(3,2) steps of dt/M
    M = 3
    uu, hh = u, h
    for _ in range(M):
        uu, hh = schemes.fbrk32_step(om, uu, hh, dt / M, ph, split=True)
    got = schemes.fblts_step(om, u, h, dt, M, ph, np.zeros(om.N, int), split=split)
    same = np.array_equal(got[0], uu) and np.array_equal(got[1], hh)
    assert same == (split == 2)


def test_split_fine_with_one_substep_is_split_coarse(cvt_small):
    w, om, lab = cvt_small
    ph = trisk.Physics(cd=w.cd)
    u, h = _state(om, 5)
    a = schemes.fblts_step(om, u, h, w.dt, 1, ph, lab, split=1)
    b = schemes.fblts_step(om, u, h, w.dt, 1, ph, lab, split=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("split", [1, 2])
def test_split_conserves_mass_and_absolute_vorticity(cvt_small, split):
    w, om, lab = cvt_small
    ph = trisk.Physics(cd=w.cd)
    u, h = _state(om, 6)
    d0 = trisk.diagnostics(om, u, h, ph)
    for _ in range(5):
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab, split=split)
    d1 = trisk.diagnostics(om, u, h, ph)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["abs_vorticity"] - d0["abs_vorticity"]) <= 1e-13 * d0["abs_vorticity_scale"]


def test_aquaplanet_gravity_wave_fblts_second_order():
    """Section 2.3: FB-LTS (M = 4) on the non-rotating aquaplanet gravity wave,
    errors against RK4 at dt = 10 s, coarse steps dt, dt/2, dt/4."""
    w = workloads.aquaplanet()
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    assert np.all(np.bincount(lab, minlength=4) > 0)
    ph = trisk.Physics(gravity_wave=True)
    T = 4 * 3600.0
    _, href = _run(lambda u, h, dt: schemes.rk4_step(om, u, h, dt, ph), w.u0, w.h0, T, 10.0)
    dts = [T / round(T / (w.dt / k)) for k in (1, 2, 4)]
    errs = []
    for dt in dts:
        _, h = _run(lambda u, hh, d: schemes.fblts_step(om, u, hh, d, w.M, ph, lab), w.u0, w.h0, T, dt)
        errs.append(math.sqrt(np.mean((h - href) ** 2)))
    assert 1.8 <= _slope(dts, errs) <= 2.3, errs
