"""Time integrators: FB-RK(3,2), RK4, RK(3,2) and the FB-LTS step (oracle).

Test infrastructure only (see the package header).

* FB-RK(3,2) is eq. ``fbrk32`` (Section 2.1) with the FB weights
  beta = (0.531, 0.531, 0.313) of that section.
* RK4 is the classical four-stage scheme on the joint state (u, h), the
  global comparison scheme of Sections 2.4 and 4.
* RK(3,2) (Wicker-Skamarock, the base of FB-RK(3,2), Section 2.1) is only used
  by the stability-ratio tests.
* ``fblts_step`` is Section 2.2 written as a plain definition: the coarse
  advancement (step 1) is evaluated on every cell and edge, the interface
  prediction (step 2, eq. ``preds`` and ``hstar_preds``) on interface one, the
  fine advancement (step 3, eq. ``fine_fbrk32``) on the fine region with the
  interface-one predictions and the interface-two / interior aliases the
  paper lists under eq. ``if_correction``, and the interface correction
  (step 4, eq. ``if_correction``) as h^n + (dt/M) * (sum over k of the
  stage-2 tendencies, accumulated in increasing k).

Readings where the paper leaves a choice: the prediction coefficients are FP64
quotients of integers (k/M, (M-k)/M, 1/M, (M-k-1)/M); velocity stage 3 of the
coarse advancement is also evaluated on interface two, where it is unused.

Pins (tests/test_oracle_schemes.py): second-order convergence of FB-RK(3,2)
and FB-LTS against the exact semi-discrete solution exp(L t) y0; the RK4
imaginary-axis stability bound 2*sqrt(2); the M = 1 / all-coarse / all-fine
reductions to FB-RK(3,2) (Section 2.2); Theorem 1 (mass) and Theorem 2
(absolute vorticity, global and, with f = 0, at every vertex) with a negative
control; the prediction exactness for constant tendencies (appendix); steady
rest state.
"""
from __future__ import annotations

import numpy as np

from . import trisk

BETA = (0.531, 0.531, 0.313)

F_LABEL, IF1_LABEL, IF2_LABEL, INT_LABEL = 0, 1, 2, 3


def momentum_tendency(om, ph, slow=None):
    """Phi as a function of (u, h): the full Phi, or, under the operator
    splitting of eq. ``splitting`` (Section 3.2), Phi_fast(u, h) plus the slow
    tendency ``slow`` frozen at an earlier state."""
    if slow is None:
        return lambda uu, hh: trisk.phi(om, uu, hh, ph)
    return lambda uu, hh: trisk.phi_fast(om, uu, hh, ph) + slow


def fbrk32_stages(om, u, h, dt, ph, beta=BETA, split=False):
    """The three FB-RK(3,2) stages of eq. fbrk32; returns (h1, h2, h3, u1, u2, u3).

    ``split``: Lie-Trotter operator splitting (eq. ``splitting``): the slow
    terms are evaluated once at (u, h) and added to the fast Phi of every stage."""
    b1, b2, b3 = beta
    Phi = momentum_tendency(om, ph, trisk.phi_slow(om, u, h, ph) if split else None)
    h1 = h + (dt / 3.0) * trisk.psi(om, u, h, ph)
    hs = b1 * h1 + (1.0 - b1) * h
    u1 = u + (dt / 3.0) * Phi(u, hs)
    h2 = h + (dt / 2.0) * trisk.psi(om, u1, h1, ph)
    hss = b2 * h2 + (1.0 - b2) * h
    u2 = u + (dt / 2.0) * Phi(u1, hss)
    h3 = h + dt * trisk.psi(om, u2, h2, ph)
    hsss = b3 * h3 + (1.0 - 2.0 * b3) * h2 + b3 * h
    u3 = u + dt * Phi(u2, hsss)
    return h1, h2, h3, u1, u2, u3


def fbrk32_step(om, u, h, dt, ph, beta=BETA, split=False):
    h1, h2, h3, u1, u2, u3 = fbrk32_stages(om, u, h, dt, ph, beta, split)
    return u3, h3


def rk4_step(om, u, h, dt, ph):
    """Classical RK4 on (u, h) with the same tendencies."""
    def f(uu, hh):
        return trisk.phi(om, uu, hh, ph), trisk.psi(om, uu, hh, ph)
    ku1, kh1 = f(u, h)
    ku2, kh2 = f(u + 0.5 * dt * ku1, h + 0.5 * dt * kh1)
    ku3, kh3 = f(u + 0.5 * dt * ku2, h + 0.5 * dt * kh2)
    ku4, kh4 = f(u + dt * ku3, h + dt * kh3)
    u_new = u + (dt / 6.0) * (ku1 + 2.0 * ku2 + 2.0 * ku3 + ku4)
    h_new = h + (dt / 6.0) * (kh1 + 2.0 * kh2 + 2.0 * kh3 + kh4)
    return u_new, h_new


def rk32_step(om, u, h, dt, ph):
    """Wicker-Skamarock RK(3,2): y1 = y + dt/3 f(y), y2 = y + dt/2 f(y1), y3 = y + dt f(y2)."""
    def f(uu, hh):
        return trisk.phi(om, uu, hh, ph), trisk.psi(om, uu, hh, ph)
    a, b = f(u, h)
    u1, h1 = u + dt / 3.0 * a, h + dt / 3.0 * b
    a, b = f(u1, h1)
    u2, h2 = u + dt / 2.0 * a, h + dt / 2.0 * b
    a, b = f(u2, h2)
    return u + dt * a, h + dt * b


def edge_labels(om, cell_label):
    """An edge between two regions belongs to the one closest to the fine region."""
    return np.minimum(cell_label[om.coe[:, 0]], cell_label[om.coe[:, 1]])


def fblts_step(om, u, h, dt, M, ph, cell_label, beta=BETA, correct_interface=True, split=0):
    """One FB-LTS coarse step (Section 2.2) in definition mode.

    ``cell_label``: 0 = fine, 1 = interface one, 2 = interface two,
    3 = interior coarse.  ``correct_interface=False`` is the negative control
    of the conservation tests: interface one and two keep the uncorrected
    coarse values instead of step 4.

    ``split``: 0 = unsplit; 1 = the operator splitting of Section 3.2 (eq.
    ``splitting``): the slow momentum terms are evaluated once at t^n and held
    for the whole step, every stage adds them to the fast terms of eq.
    ``fast_terms``; 2 = the variant proposed in Section 4.2: the fine
    advancement re-evaluates the slow terms at t^{n,k} before each substep k
    from the substep's starting state (fine values, interface-one predictions
    and the time-level-n aliases elsewhere), the coarse advancement keeps the
    t^n values.
    """
    b1, b2, b3 = beta
    cl = np.asarray(cell_label)
    el = edge_labels(om, cl)
    Fc, IF1c, IFc = cl == F_LABEL, cl == IF1_LABEL, (cl == IF1_LABEL) | (cl == IF2_LABEL)
    Fe, IF1e, IFe = el == F_LABEL, el == IF1_LABEL, (el == IF1_LABEL) | (el == IF2_LABEL)

    # step 1: coarse advancement (tilde values on the interface, bar values on the interior)
    h1, h2, h3, u1, u2, u3 = fbrk32_stages(om, u, h, dt, ph, beta, split=split > 0)
    slow_n = trisk.phi_slow(om, u, h, ph) if split else None

    # step 3 arrays; on interface two and the interior they hold the coarse
    # aliases listed under eq. if_correction (time-level independent)
    H0, H1, H2, H3 = h.copy(), h1.copy(), h2.copy(), h3.copy()
    U0, U1, U2 = u.copy(), u1.copy(), u2.copy()
    acc_h = np.zeros_like(h)
    acc_u = np.zeros_like(u)
    delta = dt / M
    for k in range(M):
        # step 2: interface prediction on interface one (eq. preds, plus h^{n,k+1})
        H0[IF1c], H1[IF1c], H2[IF1c], H3[IF1c] = predictions(
            h[IF1c], h1[IF1c], h2[IF1c], h3[IF1c], M, k)
        U0[IF1e], U1[IF1e], U2[IF1e], _ = predictions(
            u[IF1e], u1[IF1e], u2[IF1e], u3[IF1e], M, k)
        # step 3: fine advancement with dt/M (eq. fine_fbrk32)
        if split == 2 and k > 0:
            Phi = momentum_tendency(om, ph, trisk.phi_slow(om, U0, H0, ph))
        else:
            Phi = momentum_tendency(om, ph, slow_n)
        p = trisk.psi(om, U0, H0, ph)
        H1[Fc] = H0[Fc] + (delta / 3.0) * p[Fc]
        hs = b1 * H1 + (1.0 - b1) * H0
        f = Phi(U0, hs)
        U1[Fe] = U0[Fe] + (delta / 3.0) * f[Fe]
        p = trisk.psi(om, U1, H1, ph)
        H2[Fc] = H0[Fc] + (delta / 2.0) * p[Fc]
        hs = b2 * H2 + (1.0 - b2) * H0
        f = Phi(U1, hs)
        U2[Fe] = U0[Fe] + (delta / 2.0) * f[Fe]
        p = trisk.psi(om, U2, H2, ph)
        H3[Fc] = H0[Fc] + delta * p[Fc]
        acc_h[IFc] = acc_h[IFc] + p[IFc]
        hs = b3 * H3 + (1.0 - 2.0 * b3) * H2 + b3 * H0
        f = Phi(U2, hs)
        U3F = U0 + delta * f
        acc_u[IFe] = acc_u[IFe] + f[IFe]
        H0[Fc] = H3[Fc]
        U0[Fe] = U3F[Fe]

    # step 4: interface correction, and assembly of t^{n+1}
    h_new = h3.copy()
    u_new = u3.copy()
    h_new[Fc] = H0[Fc]
    u_new[Fe] = U0[Fe]
    if correct_interface:
        h_new[IFc] = h[IFc] + delta * acc_h[IFc]
        u_new[IFe] = u[IFe] + delta * acc_u[IFe]
    return u_new, h_new


def predictions(hn, h1, h2, h3, M, k):
    """Interface-one predictions of eq. preds for substep k (plus h^{n,k+1})."""
    a = float(k) / float(M)
    one_minus_a = float(M - k) / float(M)
    c = float(M - k - 1) / float(M)
    ap = float(k + 1) / float(M)
    invM = 1.0 / M
    return (a * h3 + one_minus_a * hn,
            a * h3 + invM * h1 + c * hn,
            a * h3 + invM * h2 + c * hn,
            ap * h3 + c * hn)
