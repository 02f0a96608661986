"""TRiSK shallow-water tendencies on a Voronoi C-grid (oracle, plain FP64 numpy).

Test infrastructure only (see the package header).

Thickness h lives on primal cells, the normal velocity u on edges, potential
vorticity on vertices (paper, Section 2.2, Fig. ``trisk``).  The semi-discrete
system is u_e' = Phi_e(u, h), h_i' = Psi_i(u, h) (eq. ``semi_discrete_sys``).

* Psi (eq. ``trisk_thickness``): Psi_i = -(1/A_i) sum_{e in E_i} n_{e,i} l_e F_e,
  with the thickness flux F_e = h_e u_e and h_e the mean of the two cells.
* Phi: the normal component of eq. ``nonlinear_swe``,
  -(curl u + f) k x u - grad(|u|^2/2) - g grad(h + z_b), written as
      Phi_e = q_hat_e F_perp_e - (B_c1 - B_c0)/d_e,   B = K + g (h - H)
  where the PV flux q_hat F_perp is the TRiSK mapping of the primal flux
  (eq. ``trisk_vorticity``; F_perp_e = (1/d_e) sum w_{e,e'} l_e' F_e', the
  energy-conserving edge PV average q_hat = (q_e + q_e')/2), z_b = -H.
  Quadratic bottom drag and wind stress follow eq. ``hurricane_model``.
* The linear operator (configurations with "linearized SWE") is the exact
  linearisation of the above about the state of rest u = 0, h = H.

Readings where the paper is silent (h_e, q_hat, K, the weights): the
energy-conserving TRiSK definitions of the method the paper cites (Ringler et
al. 2010).  Inside Phi(u, h*) every thickness is the FB-averaged one.

Pins (tests/test_oracle_trisk.py): sum_i A_i Psi_i = 0; exact divergence of a
linear flow; K = |U|^2/2 and the Coriolis force of a uniform flow on the
regular hexagonal mesh; curl(grad) = 0; the energy identity
sum l d F Phi + sum A B Psi = 0; B and F as the gradients of the discrete
energy; constant-PV compatibility of the vorticity flux; the linear operator's
energy skew-symmetry; the drag and wind-stress vector laws for uniform flow
and wind on the regular hexagon, and drag's energy sign; the edge value of a
drag coefficient that varies linearly in space (exact at the edge midpoints of
the hexagon).  The wind-stress coefficient C_W arrives with the wind as forcing
data per edge (the paper takes it from Garratt's law), like C_D per cell.
"""
from __future__ import annotations

import numpy as np


class OMesh:
    """Incidence lists of a mesh, in the layout the formulas below read."""

    def __init__(self, m):
        self.N = int(m.n_cells)
        self.E = int(m.n_edges)
        self.V = int(m.n_vertices)
        self.coe = np.asarray(m.cells_on_edge, dtype=np.int64).reshape(-1, 2)
        self.voe = np.asarray(m.vertices_on_edge, dtype=np.int64).reshape(-1, 2)
        self.cov = np.asarray(m.cells_on_vertex, dtype=np.int64).reshape(-1, 3)
        self.eov = np.asarray(m.edges_on_vertex, dtype=np.int64).reshape(-1, 3)
        self.kite = np.asarray(m.kite_areas_on_vertex, dtype=np.float64).reshape(-1, 3)
        self.dc = np.asarray(m.dc_edge, dtype=np.float64)
        self.dv = np.asarray(m.dv_edge, dtype=np.float64)
        self.A = np.asarray(m.area_cell, dtype=np.float64)
        self.Av = np.asarray(m.area_triangle, dtype=np.float64)
        self.fv = np.asarray(m.f_vertex, dtype=np.float64)
        self.fe = np.asarray(m.f_edge, dtype=np.float64)
        self.H = np.asarray(m.bottom_depth, dtype=np.float64)
        eoc_off = np.asarray(m.edges_on_cell_off, dtype=np.int64)
        eoc = np.asarray(m.edges_on_cell, dtype=np.int64)
        # (cell i, edge e, n_{e,i}) incidence: n_{e,i} = +1 when n_e points out of i
        self.ce_cell = np.repeat(np.arange(self.N), np.diff(eoc_off))
        self.ce_edge = eoc
        self.ce_sign = np.where(self.coe[eoc, 0] == self.ce_cell, 1.0, -1.0)
        # edges_on_edge triples (e, e', w_{e,e'})
        eoe_off = np.asarray(m.edges_on_edge_off, dtype=np.int64)
        self.ee_e = np.repeat(np.arange(self.E), np.diff(eoe_off))
        self.ee_e2 = np.asarray(m.edges_on_edge, dtype=np.int64)
        self.ee_w = np.asarray(m.weights_on_edge, dtype=np.float64)
        # circulation sign: +1 at v1 (c0 -> c1 is counter-clockwise about v1), -1 at v0
        self.He = 0.5 * (self.H[self.coe[:, 0]] + self.H[self.coe[:, 1]])


def _sum_to(index, values, n):
    """out[k] = sum of values[j] over index[j] == k (values real or complex)."""
    if np.iscomplexobj(values):
        return (np.bincount(index, values.real, n) + 1j * np.bincount(index, values.imag, n))
    return np.bincount(index, values, n)


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def edge_thickness(om, h):
    """h_e = (h_c0 + h_c1)/2."""
    return 0.5 * (h[om.coe[:, 0]] + h[om.coe[:, 1]])


def divergence_term(om, F):
    """Psi_i = -(1/A_i) sum_{e in E_i} n_{e,i} l_e F_e   (eq. trisk_thickness)."""
    s = _sum_to(om.ce_cell, om.ce_sign * om.dv[om.ce_edge] * F[om.ce_edge], om.N)
    return -s / om.A


def relative_vorticity(om, u):
    """zeta_v = (1/A_v) sum_{e in E_v} s_{e,v} d_e u_e (counter-clockwise circulation)."""
    circ = _sum_to(om.voe[:, 1], om.dc * u, om.V) - _sum_to(om.voe[:, 0], om.dc * u, om.V)
    return circ / om.Av


def vertex_thickness(om, h):
    """h_v = (1/A_v) sum_{i in C_v} kite_{i,v} h_i."""
    return (om.kite * h[om.cov]).sum(axis=1) / om.Av


def perp(om, x):
    """x_perp_e = (1/d_e) sum_{e'} w_{e,e'} l_e' x_e'  (TRiSK tangential map)."""
    return _sum_to(om.ee_e, om.ee_w * om.dv[om.ee_e2] * x[om.ee_e2], om.E) / om.dc


def pv_flux(om, F, q_edge):
    """q_hat F_perp: (1/d_e) sum_{e'} w_{e,e'} l_e' F_e' (q_e + q_e')/2."""
    t = om.ee_w * om.dv[om.ee_e2] * F[om.ee_e2] * 0.5 * (q_edge[om.ee_e] + q_edge[om.ee_e2])
    return _sum_to(om.ee_e, t, om.E) / om.dc


def kinetic_energy(om, u):
    """K_i = (1/A_i) sum_{e in E_i} (l_e d_e / 4) u_e^2."""
    t = 0.25 * om.dv[om.ce_edge] * om.dc[om.ce_edge] * u[om.ce_edge] ** 2
    return _sum_to(om.ce_cell, t, om.N) / om.A


def gradient(om, B):
    """(B_c1 - B_c0)/d_e."""
    return (B[om.coe[:, 1]] - B[om.coe[:, 0]]) / om.dc


# ----------------------------------------------------------------------------
# tendencies
# ----------------------------------------------------------------------------

class Physics:
    """Model switches: linear or nonlinear TRiSK, gravity, drag, wind.

    ``gravity_wave=True`` keeps only the fast terms of eq. ``fast_terms``
    (Section 3.2): Psi = -div(h u) and Phi = -g grad(h + z_b) with
    z_b = -H; the system of eq. ``grav_wave_model`` (Section 2.3).
    """

    def __init__(self, linear=False, g=9.81, cd=None, wind=None, gravity_wave=False):
        self.linear = linear
        self.gravity_wave = gravity_wave
        self.g = g
        self.cd = cd            # per-cell quadratic drag coefficient C_D (nonlinear only)
        # wind forcing at edges (nonlinear only): (uW_normal[E], uW_tangential[E],
        # C_W[E]), the wind and the wind-stress coefficient of eq. hurricane_model
        self.wind = wind


def psi(om, u, h, ph):
    """Thickness tendency Psi(u, h) (eq. trisk_thickness)."""
    if ph.linear:
        F = om.He * u
    else:
        F = edge_thickness(om, h) * u
    return divergence_term(om, F)


def phi_fast(om, u, h, ph):
    """Fast momentum tendency of eq. fast_terms: -g grad(h + z_b), z_b = -H."""
    return -gradient(om, ph.g * (h - om.H))


def phi_slow(om, u, h, ph):
    """Slow momentum tendency (Section 3.2): everything in Phi but the pressure
    gradient, i.e. the PV flux, -grad K, drag and wind stress, evaluated at (u, h)."""
    he = edge_thickness(om, h)
    F = he * u
    q = (relative_vorticity(om, u) + om.fv) / vertex_thickness(om, h)
    q_edge = 0.5 * (q[om.voe[:, 0]] + q[om.voe[:, 1]])
    out = pv_flux(om, F, q_edge) - gradient(om, kinetic_energy(om, u))
    return out + forcing_terms(om, u, he, ph)


def forcing_terms(om, u, he, ph):
    """Quadratic bottom drag and wind stress of eq. hurricane_model at edges."""
    out = np.zeros_like(u)
    if ph.cd is None and ph.wind is None:
        return out
    up = perp(om, u)
    if ph.cd is not None:
        cde = 0.5 * (ph.cd[om.coe[:, 0]] + ph.cd[om.coe[:, 1]])
        speed = np.sqrt(u * u + up * up)
        out = out - cde * speed * u / he
    if ph.wind is not None:
        wn, wt, cw = ph.wind
        rel = np.sqrt((wn - u) ** 2 + (wt - up) ** 2)
        out = out + cw * rel * (wn - u) / he
    return out


def phi(om, u, h, ph):
    """Momentum tendency Phi(u, h); h is whatever thickness the stage passes."""
    if ph.gravity_wave:
        return phi_fast(om, u, h, ph)
    if ph.linear:
        # linearisation about rest: F = H_e u, q = f_v / H_v, B = g (h - H)
        F = om.He * u
        q = om.fv / vertex_thickness(om, om.H)
        B = ph.g * (h - om.H)
    else:
        he = edge_thickness(om, h)
        F = he * u
        q = (relative_vorticity(om, u) + om.fv) / vertex_thickness(om, h)
        B = kinetic_energy(om, u) + ph.g * (h - om.H)
    q_edge = 0.5 * (q[om.voe[:, 0]] + q[om.voe[:, 1]])
    out = pv_flux(om, F, q_edge) - gradient(om, B)
    if not ph.linear and (ph.cd is not None or ph.wind is not None):
        up = perp(om, u)
        if ph.cd is not None:
            cde = 0.5 * (ph.cd[om.coe[:, 0]] + ph.cd[om.coe[:, 1]])
            speed = np.sqrt(u * u + up * up)
            out = out - cde * speed * u / he
        if ph.wind is not None:
            wn, wt, cw = ph.wind
            rel = np.sqrt((wn - u) ** 2 + (wt - up) ** 2)
            out = out + cw * rel * (wn - u) / he
    return out


# ----------------------------------------------------------------------------
# diagnostics (Section 2.4: discrete mass and absolute vorticity)
# ----------------------------------------------------------------------------

def neumaier_sum(x):
    """Compensated sum in index order."""
    s = 0.0
    c = 0.0
    for v in np.asarray(x, dtype=np.float64).tolist():
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


def diagnostics(om, u, h, ph):
    """mass = sum A_i h_i; abs_vorticity = sum A_v (zeta_v + f_v); energy; min h; non-finite count."""
    eta = relative_vorticity(om, u) + om.fv
    if ph.linear:
        energy = 0.5 * neumaier_sum(om.He * om.dv * om.dc * u * u) + \
            0.5 * neumaier_sum(ph.g * om.A * (h - om.H) ** 2)
    else:
        energy = neumaier_sum(0.5 * om.dv * om.dc * edge_thickness(om, h) * u * u) + \
            neumaier_sum(om.A * ph.g * h * (0.5 * h - om.H))
    return dict(
        mass=neumaier_sum(om.A * h),
        abs_vorticity=neumaier_sum(om.Av * eta),
        abs_vorticity_scale=neumaier_sum(om.Av * np.abs(eta)),
        energy=energy,
        min_h=float(np.min(h)),
        n_nonfinite=int(np.count_nonzero(~np.isfinite(h)) + np.count_nonzero(~np.isfinite(u))),
    )
