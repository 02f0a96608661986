"""GPU ensemble form: every member of a batched, multi-mesh ensemble equals the
single-member solver on the same inputs, bitwise (same kernels and operation
order), with and without hipGraph replay; and the batched members match the
oracle."""
import numpy as np
import pytest

import paper_2405_10505_amd as F
from oracle import regions, schemes, trisk
from paper_2405_10505_amd.inputs import forcing, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def two_meshes():
    a = workloads.small_cvt(n=2000, seed=12)
    b = workloads.small_cvt(n=1500, seed=13)
    return [a, b]


def _members(w, nm, k):
    fields, cds = workloads.ensemble_members(w.mesh, nm, seed_ssh0=500 + 50 * k)
    return [(w.h0 + fields[m], w.u0 + 0.0, np.full(w.mesh.n_cells, cds[m])) for m in range(nm)]


@pytest.mark.parametrize("graph", [False, True])
def test_members_equal_single_solver_bitwise(two_meshes, graph):
    ws = two_meshes
    dt = min(w.dt for w in ws)
    nms = [4, 2]
    fms = [F.Mesh(w.mesh) for w in ws]
    ens = F.Ensemble(fms, [np.where(w.fine_mask, 0, 1) for w in ws], nms, dt, M=4, linear=False)
    inputs = [_members(w, nm, k) for k, (w, nm) in enumerate(zip(ws, nms))]
    for k, mem in enumerate(inputs):
        for m, (h, u, cd) in enumerate(mem):
            ens.set_member(k, m, h, u, cd)
    ens.set_graph(graph)
    ens.step(6)
    diags = ens.diagnostics()
    assert len(diags) == sum(nms)
    for k, (w, mem) in enumerate(zip(ws, inputs)):
        for m, (h, u, cd) in enumerate(mem):
            s = F.Solver(fms[k], dt, M=4, linear=False)
            s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
            s.set_drag(cd)
            s.set_state(h, u)
            s.step(6)
            hs, us = s.get_state()
            he, ue = ens.get_member(k, m)
            assert np.array_equal(he, hs) and np.array_equal(ue, us), (k, m)
            d = s.diagnostics()
            de = diags[sum(nms[:k]) + m]
            # states are bitwise equal; the reduction tree groups entities by member
            # count, so the totals agree to rounding only
            assert abs(de["mass"] - d["mass"]) <= 1e-15 * abs(d["mass"])
            assert abs(de["energy"] - d["energy"]) <= 1e-14 * abs(d["energy"])


def test_member_matches_oracle(two_meshes):
    w = two_meshes[0]
    nm = 4
    fm = F.Mesh(w.mesh)
    ens = F.Ensemble([fm], [np.where(w.fine_mask, 0, 1)], [nm], w.dt, M=4, linear=False)
    mem = _members(w, nm, 0)
    for m, (h, u, cd) in enumerate(mem):
        ens.set_member(0, m, h, u, cd)
    ens.step(20)
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    for m in (0, 3):
        h, u, cd = mem[m]
        ph = trisk.Physics(linear=False, cd=cd)
        uo, ho = u.copy(), h.copy()
        for _ in range(20):
            uo, ho = schemes.fblts_step(om, uo, ho, w.dt, 4, ph, lab)
        he, ue = ens.get_member(0, m)
        assert np.linalg.norm(he - ho) / np.linalg.norm(ho - om.H) <= 1e-10
        assert np.linalg.norm(ue - uo) / np.linalg.norm(uo) <= 1e-10


@pytest.mark.parametrize("graph", [False, True])
def test_per_member_cyclones_equal_single_solver_bitwise(graph):
    """Perturbed forcing: members of one spherical mesh carry different storms
    (track, intensity, size, start time) or calm air; each equals the
    single-member solver with that storm (calm air: a zero wind field)."""
    import dataclasses
    w = workloads.small_sphere()
    fm = F.Mesh(w.mesh)
    base = dataclasses.replace(w.meta["storm"], rm=400e3)
    storms = [base.cyclone_kwargs(),
              dict(dataclasses.replace(base, dp=9000.0, rm=300e3, v_trans=8.0).cyclone_kwargs()),
              None,
              dict(base.cyclone_kwargs(), t0=3 * 3600.0)]
    nm = len(storms)
    lab = np.where(w.fine_mask, 0, 1)
    ens = F.Ensemble([fm], [lab], [nm], w.dt, M=w.M, linear=False)
    cds = [2.5e-3, 1.5e-3, 3e-3, 2e-3]
    for m in range(nm):
        ens.set_member(0, m, w.h0, w.u0, np.full(w.mesh.n_cells, cds[m]))
    for m, st in enumerate(storms):
        ens.set_cyclone(0, m, w.mesh.x_edge, w.mesh.normal_edge, st)
    ens.set_graph(graph)
    ens.step(8)
    for m, st in enumerate(storms):
        s = F.Solver(fm, w.dt, M=w.M, linear=False)
        s.set_regions(lab, binary=True)
        s.set_drag(np.full(w.mesh.n_cells, cds[m]))
        s.set_state(w.h0, w.u0)
        if st is None:
            # calm air: zero wind, the coefficient of zero wind speed
            z = np.zeros(w.mesh.n_edges)
            s.set_wind(z, z, forcing.wind_stress_coefficient(z, z))
        else:
            s.set_cyclone(w.mesh.x_edge, w.mesh.normal_edge, **st)
        s.step(8)
        hs, us = s.get_state()
        he, ue = ens.get_member(0, m)
        assert np.array_equal(hs, he) and np.array_equal(us, ue), m
    # the storms really differ
    a, b = ens.get_member(0, 0)[1], ens.get_member(0, 1)[1]
    assert np.max(np.abs(a - b)) > 1e-6


@pytest.mark.parametrize("kw", [dict(split=1), dict(split=2), dict(physics=F.PHYS_GRAVITY_WAVE)])
def test_split_and_gravity_wave_members_equal_single_solver_bitwise(two_meshes, kw):
    ws = two_meshes
    dt = min(w.dt for w in ws)
    nms = [2, 4]
    fms = [F.Mesh(w.mesh) for w in ws]
    labels = [np.where(w.fine_mask, 0, 1) for w in ws]
    ens = F.Ensemble(fms, labels, nms, dt, M=4, **kw)
    inputs = [_members(w, nm, k) for k, (w, nm) in enumerate(zip(ws, nms))]
    gw = kw.get("physics") == F.PHYS_GRAVITY_WAVE
    for k, mem in enumerate(inputs):
        for m, (h, u, cd) in enumerate(mem):
            ens.set_member(k, m, h, u, None if gw else cd)
    ens.set_graph(True)
    ens.step(5)
    for k, (w, mem) in enumerate(zip(ws, inputs)):
        for m, (h, u, cd) in enumerate(mem):
            s = F.Solver(fms[k], dt, M=4, **kw)
            s.set_regions(labels[k], binary=True)
            if not gw:
                s.set_drag(cd)
            s.set_state(h, u)
            s.step(5)
            hs, us = s.get_state()
            he, ue = ens.get_member(k, m)
            assert np.array_equal(hs, he) and np.array_equal(us, ue), (k, m)


def test_autotune_keeps_every_member_and_the_step_count(two_meshes):
    ws = two_meshes
    dt = min(w.dt for w in ws)
    nms = [4, 2]
    fms = [F.Mesh(w.mesh) for w in ws]
    labels = [np.where(w.fine_mask, 0, 1) for w in ws]
    inputs = [_members(w, nm, k) for k, (w, nm) in enumerate(zip(ws, nms))]

    def make():
        e = F.Ensemble(fms, labels, nms, dt, M=4, linear=False)
        for k, mem in enumerate(inputs):
            for m, (h, u, cd) in enumerate(mem):
                e.set_member(k, m, h, u, cd)
        e.set_graph(True)
        return e

    a = make()
    a.step(2)
    before = [[a.get_member(k, m) for m in range(nm)] for k, nm in enumerate(nms)]
    choice = a.autotune(steps=2, repeats=1)
    assert choice["candidates"] and choice["from_cache"] == 0
    assert all(d["step"] == 2 for d in a.diagnostics())
    for k, nm in enumerate(nms):
        for m in range(nm):
            h, u = a.get_member(k, m)
            assert np.array_equal(h, before[k][m][0]) and np.array_equal(u, before[k][m][1])
    a.step(3)
    b = make()
    b.step(5)
    for k, nm in enumerate(nms):
        for m in range(nm):
            ha, ua = a.get_member(k, m)
            hb, ub = b.get_member(k, m)
            assert np.array_equal(ha, hb) and np.array_equal(ua, ub), (k, m)


@pytest.mark.parametrize("nms", [[16, 32], [16]])
def test_wide_members_share_slots_and_equal_single_solver_bitwise(two_meshes, nms):
    """With 16 or more members per mesh the momentum pass shares each edge's
    edges_on_edge slots across its members' lanes; results stay bitwise."""
    ws = two_meshes[:len(nms)]
    dt = min(w.dt for w in ws)
    fms = [F.Mesh(w.mesh) for w in ws]
    ens = F.Ensemble(fms, [np.where(w.fine_mask, 0, 1) for w in ws], nms, dt, M=4, linear=False)
    inputs = [_members(w, nm, k) for k, (w, nm) in enumerate(zip(ws, nms))]
    for k, mem in enumerate(inputs):
        for m, (h, u, cd) in enumerate(mem):
            ens.set_member(k, m, h, u, cd)
    ens.set_graph(True)
    ens.step(5)
    for k, (w, mem) in enumerate(zip(ws, inputs)):
        for m in sorted({0, 7, nms[k] - 1}):
            h, u, cd = mem[m]
            s = F.Solver(fms[k], dt, M=4, linear=False)
            s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
            s.set_drag(cd)
            s.set_state(h, u)
            s.step(5)
            hs, us = s.get_state()
            he, ue = ens.get_member(k, m)
            assert np.array_equal(he, hs) and np.array_equal(ue, us), (k, m)


@pytest.fixture(scope="module")
def four_meshes(two_meshes):
    return two_meshes + [workloads.small_cvt(n=1000, seed=14), workloads.small_cvt(n=1800, seed=15)]


@pytest.mark.parametrize("nms,graph", [([16, 4, 8, 16], True), ([1, 2, 4, 8], False), ([16, 16, 32, 16], True)])
def test_four_meshes_every_segment_equals_single_solver_bitwise(four_meshes, nms, graph):
    """Four meshes in one launch per pass (every slot of the launch's segment
    table, uneven member counts, with and without the shared-slot momentum
    pass): sampled members of every mesh equal the single-member solver."""
    ws = four_meshes
    dt = min(w.dt for w in ws)
    fms = [F.Mesh(w.mesh) for w in ws]
    ens = F.Ensemble(fms, [np.where(w.fine_mask, 0, 1) for w in ws], nms, dt, M=4, linear=False)
    inputs = [_members(w, nm, k) for k, (w, nm) in enumerate(zip(ws, nms))]
    for k, mem in enumerate(inputs):
        for m, (h, u, cd) in enumerate(mem):
            ens.set_member(k, m, h, u, cd)
    ens.set_graph(graph)
    d0 = ens.diagnostics()
    ens.step(5)
    d1 = ens.diagnostics()
    for a, b in zip(d0, d1):
        assert abs(b["mass"] - a["mass"]) <= 1e-13 * abs(a["mass"])
    for k, (w, mem) in enumerate(zip(ws, inputs)):
        for m in sorted({0, nms[k] // 2, nms[k] - 1}):
            h, u, cd = mem[m]
            s = F.Solver(fms[k], dt, M=4, linear=False)
            s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
            s.set_drag(cd)
            s.set_state(h, u)
            s.step(5)
            hs, us = s.get_state()
            he, ue = ens.get_member(k, m)
            assert np.array_equal(he, hs) and np.array_equal(ue, us), (k, m)
