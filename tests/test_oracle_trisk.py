"""Pins of the oracle's TRiSK tendencies against identities and closed forms (CPU).

None of these re-derive the oracle's formulas: they check consequences fixed
by the mathematics -- telescoping of fluxes (Theorem 1's mechanism), the
divergence theorem, exact values on the regular hexagonal mesh, curl(grad)=0,
conservation of the discrete energy by the semi-discrete system, and the
constant-PV compatibility of the vorticity flux (eq. trisk_vorticity), the
energy neutrality of the Coriolis term, the energy skew-symmetry of the linear
operator, and the discrete inertia-gravity frequency of the regular hexagonal
mesh from its Bloch matrix (checked against an independent value) with its
steady geostrophic modes.
"""
import math

import numpy as np
import pytest

from oracle import trisk
from paper_2405_10505_amd.inputs import meshgen, workloads


@pytest.fixture(scope="module")
def hexm():
    return meshgen.hex_periodic(32, 32, 1.0e4)


@pytest.fixture(scope="module")
def cvt():
    w = workloads.small_cvt()
    return w.mesh


def _rand_state(om, seed, amp_u=0.7, amp_h=5.0):
    r = np.random.default_rng(seed)
    u = amp_u * r.normal(size=om.E)
    h = om.H + amp_h * r.normal(size=om.N)
    return u, h


def _unwrap_rel(m, x, origin):
    d = x - origin
    d[..., 0] -= m.lx * np.round(d[..., 0] / m.lx)
    d[..., 1] -= m.ly * np.round(d[..., 1] / m.ly)
    return d


@pytest.mark.parametrize("meshname", ["hexm", "cvt"])
@pytest.mark.parametrize("linear", [True, False])
def test_thickness_tendency_telescopes(meshname, linear, request):
    m = request.getfixturevalue(meshname)
    om = trisk.OMesh(m)
    u, h = _rand_state(om, 1)
    p = trisk.psi(om, u, h, trisk.Physics(linear=linear))
    assert abs(np.sum(om.A * p)) <= 1e-14 * np.sum(np.abs(om.A * p))


def test_divergence_theorem_on_cvt(cvt):
    """For a linear flow U(x) sampled at Voronoi-edge midpoints, sum n l u = (a+b) A exactly."""
    m = cvt
    om = trisk.OMesh(m)
    a, b, c, d = 2.0e-5, -0.7e-5, 1.3e-5, 0.4e-5
    x0 = m.x_cell[m.cells_on_edge[:, 0]]
    v0 = x0 + _unwrap_rel(m, m.x_vertex[m.vertices_on_edge[:, 0]], x0)
    v1 = x0 + _unwrap_rel(m, m.x_vertex[m.vertices_on_edge[:, 1]], x0)
    mid = 0.5 * (v0 + v1)
    U = np.stack([a * mid[:, 0] + c * mid[:, 1], d * mid[:, 0] + b * mid[:, 1]], 1)
    u = np.einsum("ij,ij->i", U, m.normal_edge)
    h = np.full(om.N, 1000.0)
    p = trisk.psi(om, u, h, trisk.Physics(linear=False))
    L = m.lx
    inner = np.all((m.x_cell > 0.25 * L) & (m.x_cell < 0.75 * L), axis=1)
    assert inner.sum() > 100
    np.testing.assert_allclose(p[inner], -1000.0 * (a + b), rtol=1e-9)


def test_hex_flux_of_linear_thickness(hexm):
    """Uniform U and h = h0 + alpha.x: Psi = -U.alpha (edge-mean thickness is exact on the hexagon)."""
    m = hexm
    om = trisk.OMesh(m)
    U = np.array([0.8, -0.3])
    alpha = np.array([1.0e-4, 2.5e-4])
    L = m.lx
    # unwrap around the domain centre; keep cells whose neighbours do not cross the seam
    ctr = np.array([0.5 * m.lx, 0.5 * m.ly])
    xc = ctr + _unwrap_rel(m, m.x_cell, ctr)
    h = 1000.0 + xc @ alpha
    u = m.normal_edge @ U
    p = trisk.psi(om, u, h, trisk.Physics(linear=False))
    inner = np.all(np.abs(xc - ctr) < 0.35 * np.array([m.lx, m.ly]), axis=1)
    np.testing.assert_allclose(p[inner], -(U @ alpha), rtol=1e-9)


def test_hex_uniform_flow_kinetic_energy_and_coriolis(hexm):
    """Uniform flow on the hexagon: K = |U|^2/2, zeta = 0, Phi_e = n_e.(-f k x U) = f t_e.U."""
    m = hexm
    om = trisk.OMesh(m)
    U = np.array([1.3, -0.6])
    u = m.normal_edge @ U
    np.testing.assert_allclose(trisk.kinetic_energy(om, u), 0.5 * U @ U, rtol=1e-12)
    assert np.max(np.abs(trisk.relative_vorticity(om, u))) < 1e-18
    f = 1e-4
    expect = m.tangent_edge @ U * f
    h = np.full(om.N, 1000.0)
    for linear in (True, False):
        got = trisk.phi(om, u, h, trisk.Physics(linear=linear))
        np.testing.assert_allclose(got, expect, atol=1e-12 * f * np.abs(U).max())


def test_hex_uniform_flow_drag_and_wind_stress(hexm):
    """Uniform flow U and uniform wind W over uniform depth h on the hexagon: the
    quadratic drag adds n_e . (-C_D |U| U / h) to Phi and the wind stress adds
    n_e . (C_W |W - U| (W - U) / h), the vector laws with the full speeds (the
    tangential components come from the TRiSK reconstruction, exact for uniform
    flow here); C_W is forcing data, like the wind."""
    m = hexm
    om = trisk.OMesh(m)
    U = np.array([1.3, -0.6])
    W = np.array([-7.0, 18.0])
    u = m.normal_edge @ U
    h = np.full(om.N, 37.0)
    cd = 2.5e-3
    base = trisk.phi(om, u, h, trisk.Physics(linear=False))
    drag = trisk.phi(om, u, h, trisk.Physics(linear=False, cd=np.full(om.N, cd))) - base
    expect = m.normal_edge @ (-cd * np.hypot(*U) * U / 37.0)
    np.testing.assert_allclose(drag, expect, rtol=1e-10, atol=1e-13 * np.abs(expect).max())
    cw = 1.7e-3
    ph = trisk.Physics(linear=False, wind=(m.normal_edge @ W, m.tangent_edge @ W, np.full(om.E, cw)))
    wind = trisk.phi(om, u, h, ph) - base
    expect = m.normal_edge @ (cw * np.hypot(*(W - U)) * (W - U) / 37.0)
    np.testing.assert_allclose(wind, expect, rtol=1e-10, atol=1e-13 * np.abs(expect).max())


def test_hex_linear_drag_coefficient_field(hexm):
    """A drag coefficient varying linearly in space, uniform flow U over
    uniform depth h on the regular hexagon: on every edge away from the
    periodic seam the drag term equals the vector law n_e . (-C_D(x_e) |U| U / h)
    with C_D evaluated at the edge's own midpoint x_e.  Each hexagon edge
    bisects the segment between its two cell centres, so the edge value of a
    linear field is exactly the mean of the two cell values, and any other
    reconstruction from the cells (one side, a geometric mean) misses it."""
    m = hexm
    om = trisk.OMesh(m)
    U = np.array([0.9, 1.7])
    u = m.normal_edge @ U
    h = np.full(om.N, 52.0)
    a, bx, by = 1.0e-3, 2.0e-3 / m.lx, 1.0e-3 / m.ly
    xc = m.x_cell
    cd = a + bx * xc[:, 0] + by * xc[:, 1]
    base = trisk.phi(om, u, h, trisk.Physics(linear=False))
    drag = trisk.phi(om, u, h, trisk.Physics(linear=False, cd=cd)) - base
    c0, c1 = m.cells_on_edge[:, 0], m.cells_on_edge[:, 1]
    d = xc[c1] - xc[c0]
    inner = np.all(np.abs(d) < 2.0 * m.dc_edge[:, None], axis=1)   # no periodic wrap between the cells
    assert inner.sum() > 0.9 * om.E
    xe = m.x_edge[inner]
    # the mesh property the reading relies on: the edge point is the midpoint of the cell centres
    np.testing.assert_allclose(xe, 0.5 * (xc[c0] + xc[c1])[inner], rtol=0, atol=1e-9 * m.lx)
    cde = a + bx * xe[:, 0] + by * xe[:, 1]
    expect = -cde * np.hypot(*U) * (m.normal_edge[inner] @ U) / 52.0
    np.testing.assert_allclose(drag[inner], expect, rtol=1e-10, atol=1e-13 * np.abs(expect).max())


def test_hex_uniform_state_diagnostics(hexm):
    """Uniform flow U over uniform thickness h (flat bottom H) on the regular
    hexagon, total area A: mass = A h, absolute vorticity = A f (zeta = 0),
    and the energy of Section 2.4 is A (g h (h/2 - H) + h |U|^2 / 2) in the
    nonlinear form and A (g (h - H)^2 / 2 + H |U|^2 / 2) in the linear one."""
    m = hexm
    om = trisk.OMesh(m)
    U = np.array([1.3, -0.6])
    u = m.normal_edge @ U
    H, hv, g, f = 1000.0, 1000.7, 9.81, 1e-4
    h = np.full(om.N, hv)
    A = float(np.sum(om.A))
    d = trisk.diagnostics(om, u, h, trisk.Physics(linear=False, g=g))
    assert abs(d["mass"] - A * hv) <= 1e-13 * A * hv
    assert abs(d["abs_vorticity"] - A * f) <= 1e-12 * A * f
    e = A * (g * hv * (0.5 * hv - H) + 0.5 * hv * (U @ U))
    assert abs(d["energy"] - e) <= 1e-11 * abs(e)
    d = trisk.diagnostics(om, u, h, trisk.Physics(linear=True, g=g))
    e = A * (0.5 * g * (hv - H) ** 2 + 0.5 * H * (U @ U))
    assert abs(d["energy"] - e) <= 1e-11 * abs(e)


@pytest.mark.parametrize("meshname", ["hexm", "cvt"])
def test_curl_of_gradient_vanishes(meshname, request):
    m = request.getfixturevalue(meshname)
    om = trisk.OMesh(m)
    B = np.random.default_rng(3).normal(size=om.N)
    g = trisk.gradient(om, B)
    z = trisk.relative_vorticity(om, g)
    scale = np.abs(g).max() * om.dc.max() / om.Av.min()
    assert np.abs(z).max() < 1e-14 * scale


def _energy(om, u, h, g):
    """TRiSK total energy: sum_e l d h_e u^2 / 2 + sum_i A g h (h/2 - H)."""
    he = 0.5 * (h[om.coe[:, 0]] + h[om.coe[:, 1]])
    return np.sum(0.5 * om.dv * om.dc * he * u * u) + np.sum(om.A * g * h * (0.5 * h - om.H))


@pytest.mark.parametrize("meshname", ["hexm", "cvt"])
def test_semi_discrete_energy_conserved(meshname, request):
    """dE/dt = grad E . (Phi, Psi) = 0 (complex-step directional derivative)."""
    m = request.getfixturevalue(meshname)
    om = trisk.OMesh(m)
    u, h = _rand_state(om, 5)
    ph = trisk.Physics(linear=False)
    P = trisk.psi(om, u, h, ph)
    F = trisk.phi(om, u, h, ph)
    eps = 1e-30
    dE = _energy(om, u + 1j * eps * F, h + 1j * eps * P, ph.g).imag / eps
    # scale: the size of the individual terms of grad E . (Phi, Psi)
    he = 0.5 * (h[om.coe[:, 0]] + h[om.coe[:, 1]])
    scale = np.sum(np.abs(om.dv * om.dc * he * u * F)) + np.sum(np.abs(om.A * ph.g * (h - om.H) * P))
    assert abs(dE) < 1e-13 * scale


@pytest.mark.parametrize("meshname", ["hexm", "cvt"])
def test_linear_operator_is_linearisation_at_rest(meshname, request):
    m = request.getfixturevalue(meshname)
    om = trisk.OMesh(m)
    r = np.random.default_rng(7)
    du = r.normal(size=om.E)
    deta = r.normal(size=om.N)
    eps = 1e-30
    nl = trisk.Physics(linear=False)
    lin = trisk.Physics(linear=True)
    jp = trisk.psi(om, 1j * eps * du, om.H + 1j * eps * deta, nl).imag / eps
    jf = trisk.phi(om, 1j * eps * du, om.H + 1j * eps * deta, nl).imag / eps
    np.testing.assert_allclose(trisk.psi(om, du, om.H + deta, lin), jp, rtol=1e-12, atol=1e-12 * np.abs(jp).max())
    np.testing.assert_allclose(trisk.phi(om, du, om.H + deta, lin), jf, rtol=1e-12, atol=1e-12 * np.abs(jf).max())


@pytest.mark.parametrize("meshname", ["hexm", "cvt"])
def test_constant_pv_compatibility(meshname, request):
    """If q_v = q0 everywhere, d(zeta_v)/dt = q0 d(h_v)/dt (PV stays uniform; eq. trisk_vorticity)."""
    m = request.getfixturevalue(meshname)
    om = trisk.OMesh(m)
    u, h = _rand_state(om, 9)
    q0 = 3.1e-7
    zeta = trisk.relative_vorticity(om, u)
    hv = trisk.vertex_thickness(om, h)
    m2 = m.copy_with(f_vertex=q0 * hv - zeta)
    om2 = trisk.OMesh(m2)
    ph = trisk.Physics(linear=False)
    dzeta = trisk.relative_vorticity(om2, trisk.phi(om2, u, h, ph))
    dhv = trisk.vertex_thickness(om2, trisk.psi(om2, u, h, ph))
    np.testing.assert_allclose(dzeta, q0 * dhv, atol=1e-12 * np.abs(q0 * dhv).max())


def test_drag_removes_energy(cvt):
    """Quadratic drag contributes sum_e l d F_e (-C_D |u| u / h_e) <= 0 to dE/dt."""
    om = trisk.OMesh(cvt)
    u, h = _rand_state(om, 11)
    cd = np.full(om.N, 2.5e-3)
    P = trisk.psi(om, u, h, trisk.Physics(linear=False))
    Fd = trisk.phi(om, u, h, trisk.Physics(linear=False, cd=cd))
    eps = 1e-30
    dE = _energy(om, u + 1j * eps * Fd, h + 1j * eps * P, 9.81).imag / eps
    assert dE < 0


def test_linear_energy_is_conserved_by_the_linear_operator(cvt):
    """Linear TRiSK conserves E = sum_i A_i g eta_i^2 / 2 + sum_e l_e d_e H_e u_e^2 / 2:
    g sum A eta Psi + sum l d H_e u Phi = 0 for any state (the divergence is the
    negative adjoint of the gradient and the PV flux is energy-neutral)."""
    om = trisk.OMesh(cvt)
    ph = trisk.Physics(linear=True)
    r = np.random.default_rng(11)
    u = r.normal(size=om.E)
    eta = r.normal(size=om.N)
    psi = trisk.psi(om, u, om.H + eta, ph)
    phi = trisk.phi(om, u, om.H + eta, ph)
    a = ph.g * np.sum(om.A * eta * psi)
    b = np.sum(om.dv * om.dc * om.He * u * phi)
    assert abs(a + b) <= 1e-13 * (np.sum(np.abs(ph.g * om.A * eta * psi)) + np.sum(np.abs(om.dv * om.dc * om.He * u * phi)))


def test_coriolis_term_is_energy_neutral(cvt):
    """sum_e l_e d_e u_e u_perp_e = 0: the tangential reconstruction through the
    antisymmetric weights does no work."""
    om = trisk.OMesh(cvt)
    u = np.random.default_rng(12).normal(size=om.E)
    up = trisk.perp(om, u)
    s = np.sum(om.dv * om.dc * u * up)
    assert abs(s) <= 1e-13 * np.sum(np.abs(om.dv * om.dc * u * up))


def _bloch(m, om, kvec, ph):
    """4x4 Bloch matrix of the linear operator on the regular hexagonal mesh for
    wavenumber kvec: one cell mode and three edge-orientation modes, each with
    phase exp(i k.x); the operator is applied to complex states."""
    ph_c = np.exp(1j * (m.x_cell @ kvec))
    ph_e = np.exp(1j * (m.x_edge @ kvec))
    ang = np.mod(np.arctan2(m.normal_edge[:, 1], m.normal_edge[:, 0]), np.pi)
    cls = np.round(ang / (np.pi / 3)).astype(int) % 3
    ref = np.stack([np.cos(np.arange(3) * np.pi / 3), np.sin(np.arange(3) * np.pi / 3)], 1)
    sgn = np.sign(np.einsum("ij,ij->i", m.normal_edge, ref[cls]))
    basis = [(ph_c, np.zeros(om.E, complex))] + [
        (np.zeros(om.N, complex), np.where(cls == c, sgn * ph_e, 0)) for c in range(3)]
    e0 = [int(np.nonzero(cls == c)[0][0]) for c in range(3)]
    Lk = np.zeros((4, 4), complex)
    out = [(trisk.psi(om, u, om.H + eta, ph), trisk.phi(om, u, om.H + eta, ph)) for eta, u in basis]
    scale = max(max(np.max(np.abs(dh)), np.max(np.abs(du))) for dh, du in out)
    for b, (dh, du) in enumerate(out):
        Lk[0, b] = dh[0] / ph_c[0]
        for c in range(3):
            Lk[1 + c, b] = du[e0[c]] / (sgn[e0[c]] * ph_e[e0[c]])
        # the result is the Bloch combination everywhere (translation invariance)
        rh = Lk[0, b] * ph_c
        ru = sum(Lk[1 + c, b] * basis[1 + c][1] for c in range(3))
        assert np.max(np.abs(dh - rh)) <= 1e-12 * scale
        assert np.max(np.abs(du - ru)) <= 1e-12 * scale
    return Lk, basis


def test_discrete_inertia_gravity_frequency_and_geostrophic_modes():
    """Configuration 1's mesh and wavenumber (2, 1): the Bloch eigenvalues of the
    linear TRiSK operator are {0, 0, +-i omega_d} with omega_d = 4.46348e-3 1/s
    (an independent Bloch computation done before this test; the continuous f-plane value is
    4.49233e-3), and the two zero-frequency (geostrophically balanced) modes are
    steady states of FB-RK(3,2)."""
    from oracle import schemes
    w = workloads.config1()
    m = w.mesh
    om = trisk.OMesh(m)
    ph = trisk.Physics(linear=True)
    kvec = np.array([2 * math.pi * 2 / m.lx, 2 * math.pi * 1 / m.ly])
    Lk, basis = _bloch(m, om, kvec, ph)
    lam = np.linalg.eigvals(Lk)
    lam = lam[np.argsort(np.abs(lam))]
    omega_c = math.sqrt(1e-4 ** 2 + 9.81 * 1000.0 * float(kvec @ kvec))
    assert abs(omega_c - 4.49233e-3) <= 5e-9
    assert np.max(np.abs(lam[:2])) <= 1e-12 * omega_c
    assert np.max(np.abs(lam[2:].real)) <= 1e-12 * omega_c
    assert abs(np.abs(lam[2].imag) - 4.46348e-3) <= 5e-9 and abs(lam[2] + lam[3]) <= 1e-12 * omega_c
    # a real zero mode: Re of the null vector's Bloch combination
    vals, vecs = np.linalg.eig(Lk)
    v = vecs[:, int(np.argmin(np.abs(vals)))]
    eta = np.real(v[0] * basis[0][0])
    u = np.real(sum(v[1 + c] * basis[1 + c][1] for c in range(3)))
    scale = 0.1 / max(np.max(np.abs(eta)), np.max(np.abs(u)))
    eta, u = eta * scale, u * scale
    uu, hh = u.copy(), om.H + eta
    for _ in range(10):
        uu, hh = schemes.fbrk32_step(om, uu, hh, 60.0, ph)
    assert np.max(np.abs(uu - u)) <= 1e-12 * np.max(np.abs(u)) + 1e-15
    assert np.max(np.abs(hh - om.H - eta)) <= 1e-9 * max(np.max(np.abs(eta)), 1e-3)
