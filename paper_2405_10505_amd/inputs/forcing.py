"""Analytic cyclone wind at edge points (input forcing for the wind-stress term).

The paper drives its storm-surge runs with observed hurricane winds; those are
not available, so the synthetic stand-in is an analytic Holland (1980)
gradient-wind vortex moving along a great circle.  The wind vector at a point
x (unit vector, sphere radius R) at time t:

  c(t)  storm centre: c0 rotated about the track axis by angle omega_track t
  r     great-circle distance from c(t) to x, R atan2(|x cross c|, x.c)
        (well conditioned near the eye, unlike R acos(x.c))
  V(r)  = sqrt((B/rho_a)(Rm/r)^B dp exp(-(Rm/r)^B) + (r f/2)^2) - r |f|/2
  W     = sign(f_c) V(r) (x cross r_hat)  +  v_trans (V/V_max) tau_hat
          (r_hat: unit tangent at x pointing away from c; tau_hat: the track
          direction at c projected onto x's tangent plane)

and its edge components wind_normal = W.n_e, wind_tangential = W.t_e.  The
wind-stress coefficient of eq. hurricane_model comes with the wind: the paper
takes it from Garratt (1977), C_W = (rho_air / rho_water)(0.75 + 0.067 |W|)
1e-3 (his 10 m drag law in kinematic form), evaluated from the wind speed at
the edge.  The library evaluates the same vortex and coefficient on the device
at the start of each coarse step (time t0 + k dt for the k-th step after the
storm is set); this numpy version feeds the oracle and checks the device
evaluation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

OMEGA = 7.292e-5
RHO_WATER = 1000.0


def wind_stress_coefficient(wn, wt, rho_air=1.15, rho_water=RHO_WATER):
    """C_W at edges from the wind components there (Garratt's law, kinematic form)."""
    return (rho_air / rho_water) * (0.75 + 0.067 * np.sqrt(wn * wn + wt * wt)) * 1e-3


@dataclass
class Holland:
    c0: np.ndarray          # initial centre (unit vector)
    axis: np.ndarray        # unit normal of the track's great circle
    v_trans: float = 5.0    # translation speed (m/s)
    dp: float = 6000.0      # central pressure deficit (Pa)
    rm: float = 40e3        # radius of maximum wind (m)
    B: float = 1.5          # Holland shape parameter
    rho_air: float = 1.15
    radius: float = 6.371229e6
    omega: float = OMEGA
    t0: float = 0.0

    @property
    def omega_track(self):
        return self.v_trans / self.radius

    def centre(self, t):
        ang = self.omega_track * (t + self.t0)
        k = self.axis
        c = self.c0
        return c * math.cos(ang) + np.cross(k, c) * math.sin(ang) + k * (k @ c) * (1 - math.cos(ang))

    def speed(self, r, f):
        r = np.maximum(r, 1.0)
        a = (self.rm / r) ** self.B
        return np.sqrt(self.B / self.rho_air * a * self.dp * np.exp(-a) + (r * f / 2) ** 2) - r * np.abs(f) / 2

    def wind(self, x, t):
        """Wind vectors [n,3] at unit vectors x [n,3]."""
        c = self.centre(t)
        cosang = x @ c
        sinang = np.linalg.norm(np.cross(x, c), axis=1)
        r = self.radius * np.arctan2(sinang, cosang)
        f = 2 * self.omega * x[:, 2]
        fc = 2 * self.omega * c[2]
        V = self.speed(r, f)
        vmax = float(self.speed(np.array([self.rm]), np.array([fc]))[0])
        ct = c[None, :] - cosang[:, None] * x            # towards the centre, tangent at x
        nrm = np.linalg.norm(ct, axis=1)
        safe = nrm > 0
        rhat = np.zeros_like(x)
        rhat[safe] = -ct[safe] / nrm[safe, None]
        swirl = np.cross(x, rhat) * (V * (1.0 if fc >= 0 else -1.0))[:, None]
        tau = np.cross(self.axis, c)
        tx = tau[None, :] - (x @ tau)[:, None] * x
        tn = np.linalg.norm(tx, axis=1)
        tx = tx / np.maximum(tn, 1e-300)[:, None]
        return swirl + (self.v_trans * V / vmax)[:, None] * tx

    def cyclone_kwargs(self):
        """The storm's parameters under the library's names (fblts_cyclone)."""
        return dict(center=self.c0, axis=self.axis, v_trans=self.v_trans, dp=self.dp, rm=self.rm, b=self.B,
                    rho_air=self.rho_air, radius=self.radius, omega=self.omega, t0=self.t0)

    def edge_components(self, mesh, t):
        x = mesh.x_edge / np.linalg.norm(mesh.x_edge, axis=1, keepdims=True)
        W = self.wind(x, t)
        return np.einsum("ij,ij->i", W, mesh.normal_edge), np.einsum("ij,ij->i", W, mesh.tangent_edge)

    def edge_forcing(self, mesh, t, rho_water=RHO_WATER):
        """(wind_normal, wind_tangential, C_W) at the edges at time t."""
        wn, wt = self.edge_components(mesh, t)
        return wn, wt, wind_stress_coefficient(wn, wt, self.rho_air, rho_water)


def seeded_track(seed, target=None, start_distance=None, radius=6.371229e6):
    """A storm heading for `target` (unit vector) from `start_distance` (rad) away
    at a seeded bearing; without a target, a random start and heading."""
    r = np.random.Generator(np.random.PCG64(seed))
    if target is None:
        c0 = r.normal(size=3)
        c0 /= np.linalg.norm(c0)
        d = r.normal(size=3)
        d -= (d @ c0) * c0
        d /= np.linalg.norm(d)
        axis = np.cross(c0, d)
        return Holland(c0=c0, axis=axis / np.linalg.norm(axis), radius=radius)
    tg = np.asarray(target, float) / np.linalg.norm(target)
    d = r.normal(size=3)
    d -= (d @ tg) * tg
    d /= np.linalg.norm(d)
    c0 = math.cos(start_distance) * tg + math.sin(start_distance) * d
    axis = np.cross(c0, tg)            # rotating c0 about this axis moves it towards the target
    return Holland(c0=c0, axis=axis / np.linalg.norm(axis), radius=radius)
