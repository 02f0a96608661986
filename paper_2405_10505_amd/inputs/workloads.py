"""Seeded synthetic workloads: meshes, initial states, drag, region masks.

Inputs only: nothing here evaluates a tendency or takes a time step.  The
recipes (shapes, distributions, seeds) stand in for the paper's Delaware Bay
meshes and hurricane forcing, which are not available; every random number is
drawn from ``numpy.random.Generator(PCG64(seed))``.

* ``config1``: periodic regular hexagonal mesh 32 x 32, dc = 10 km, H = 1000 m,
  f = 1e-4, linear; inertia-gravity plane wave a = 0.1 m, wavenumber (2, 1);
  a band of 8 full rows (start row from the seed) marked fine; M = 2.
* ``config2``: planar periodic variable-resolution CVT, 50k cells, 2 -> 8 km
  over a Gaussian patch, 50 Lloyd iterations; depth 4000 m minus six Gaussian
  seamount bumps (min 50 m); nonlinear with quadratic drag; at rest with three
  Gaussian SSH bumps; fine cells chosen from the local CFL number; M = 4.
* ``ensemble_members``: per-member SSH perturbations and drag coefficients.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import meshgen

G = 9.81
NU_MAX_FBRK32 = 1.58   # measured gravity-wave Courant limit of FB-RK(3,2) on the hex mesh


@dataclass
class Workload:
    name: str
    mesh: meshgen.Mesh
    h0: np.ndarray
    u0: np.ndarray
    fine_mask: np.ndarray
    dt: float
    M: int
    linear: bool
    cd: np.ndarray | None = None
    steps: int = 200
    meta: dict = field(default_factory=dict)


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# configuration 1: linear inertia-gravity wave on the periodic hexagonal mesh
# ----------------------------------------------------------------------------

def igw_state(mesh, t, amp=0.1, kx_n=2, ky_n=1, H=1000.0, f=1e-4, g=G):
    """Continuous f-plane inertia-gravity plane wave sampled on the mesh.

    eta = a cos(theta), u = a/(H |k|^2) (omega cos(theta) k + f sin(theta) k_perp),
    theta = k.x - omega t, omega^2 = f^2 + g H |k|^2; u_e = n_e . u(x_e).
    """
    k = np.array([2 * math.pi * kx_n / mesh.lx, 2 * math.pi * ky_n / mesh.ly])
    kperp = np.array([-k[1], k[0]])
    k2 = float(k @ k)
    om = math.sqrt(f * f + g * H * k2)
    th_c = mesh.x_cell @ k - om * t
    th_e = mesh.x_edge @ k - om * t
    h = H + amp * np.cos(th_c)
    A = amp / (H * k2)
    uvec = A * (om * np.cos(th_e)[:, None] * k[None, :] + f * np.sin(th_e)[:, None] * kperp[None, :])
    u = np.einsum("ij,ij->i", uvec, mesh.normal_edge)
    return h, u, om


def band_mask(nx, ny, rows, seed):
    j0 = int(rng_for(seed).integers(0, ny))
    rows_idx = (j0 + np.arange(rows)) % ny
    mask = np.zeros(nx * ny, dtype=bool)
    for j in rows_idx:
        mask[j * nx:(j + 1) * nx] = True
    return mask


def config1(M=2, dt=60.0, steps=200, seed=1):
    mesh = meshgen.hex_periodic(32, 32, 1.0e4, f0=1e-4, depth=1000.0)
    h0, u0, om = igw_state(mesh, 0.0)
    mask = band_mask(32, 32, 8, seed)
    return Workload("hex32_igw_linear", mesh, h0, u0, mask, dt, M, True, None, steps,
                    dict(omega=om, seed=seed))


# ----------------------------------------------------------------------------
# configuration 2: nonlinear, variable resolution, CFL-selected fine region
# ----------------------------------------------------------------------------

def _periodic_r2(x, y, cx, cy, lx, ly):
    dx = np.abs(x - cx); dx = np.minimum(dx, lx - dx)
    dy = np.abs(y - cy); dy = np.minimum(dy, ly - dy)
    return dx * dx + dy * dy


def seamount_depth(mesh, seed=3, n_bumps=6):
    r = rng_for(seed)
    x, y = mesh.x_cell[:, 0], mesh.x_cell[:, 1]
    H = np.full(mesh.n_cells, 4000.0)
    for _ in range(n_bumps):
        cx, cy = r.uniform(0, mesh.lx), r.uniform(0, mesh.ly)
        amp = r.uniform(1000.0, 3950.0)
        w = r.uniform(30e3, 120e3)
        H -= amp * np.exp(-_periodic_r2(x, y, cx, cy, mesh.lx, mesh.ly) / (2 * w * w))
    return np.maximum(H, 50.0)


def ssh_bumps(mesh, seed=4, n=3, amp=0.5, width=50e3):
    r = rng_for(seed)
    x, y = mesh.x_cell[:, 0], mesh.x_cell[:, 1]
    eta = np.zeros(mesh.n_cells)
    for _ in range(n):
        cx, cy = r.uniform(0, mesh.lx), r.uniform(0, mesh.ly)
        eta += amp * np.exp(-_periodic_r2(x, y, cx, cy, mesh.lx, mesh.ly) / (2 * width * width))
    return eta


def cfl_fine_mask(mesh, M, nu=0.6 * NU_MAX_FBRK32, g=G, margin=1.0):
    """Fine cells: those whose gravity-wave Courant number at the coarse step exceeds margin * nu.

    dt_fine = nu * min_i(dx_i / c_i), dt_coarse = M dt_fine; c_i = sqrt(g H_i),
    dx_i = the shortest dual edge of the cell.  margin < 1 moves the cells
    closest to the threshold into the fine set, so that the coarse region
    keeps a stability margin at the coarse step.
    """
    dx = np.full(mesh.n_cells, np.inf)
    np.minimum.at(dx, mesh.cells_on_edge[:, 0], mesh.dc_edge)
    np.minimum.at(dx, mesh.cells_on_edge[:, 1], mesh.dc_edge)
    c = np.sqrt(g * mesh.bottom_depth)
    dt_f = nu * float(np.min(dx / c))
    dt_c = M * dt_f
    fine = c * dt_c / dx > margin * nu
    return fine, dt_c, dt_f


_MESH_CACHE = {}


def cvt_mesh(n=50000, seed=2, iters=50):
    key = (n, seed, iters)
    if key not in _MESH_CACHE:
        # optional on-disk cache (directory in FBLTS_MESH_CACHE) of the generated mesh
        cache_dir = os.environ.get("FBLTS_MESH_CACHE")
        path = os.path.join(cache_dir, "cvt_%d_%d_%d.npz" % key) if cache_dir else None
        if path and os.path.exists(path):
            _MESH_CACHE[key] = meshgen.Mesh.load(path)
        else:
            _MESH_CACHE[key] = meshgen.cvt_planar_periodic(n, meshgen.gaussian_patch_dx, iters=iters, seed=seed)
            if path:
                os.makedirs(cache_dir, exist_ok=True)
                _MESH_CACHE[key].save(path)
    return _MESH_CACHE[key]


def config2(n=50000, M=4, steps=200, seed_mesh=2, seed_depth=3, seed_ic=4, iters=50, cd=2.5e-3):
    base = cvt_mesh(n, seed_mesh, iters)
    H = seamount_depth(base, seed_depth)
    mesh = base.copy_with(bottom_depth=H)
    h0 = H + ssh_bumps(mesh, seed_ic)
    u0 = np.zeros(mesh.n_edges)
    fine, dt_c, dt_f = cfl_fine_mask(mesh, M)
    return Workload("cvt%dk_nonlinear_drag" % (n // 1000), mesh, h0, u0, fine, dt_c, M, False,
                    np.full(mesh.n_cells, cd), steps,
                    dict(dt_fine=dt_f, n_fine=int(fine.sum()), seeds=(seed_mesh, seed_depth, seed_ic)))


def small_cvt(n=2000, M=4, seed=12, iters=20):
    """A small irregular mesh with the configuration-2 recipe (fast CPU tests)."""
    return config2(n=n, M=M, seed_mesh=seed, iters=iters)


def ensemble_members(mesh, n_members, seed_ssh0=1000, seed_cd=8, sigma=0.05, corr=50e3,
                     cd_range=(1e-3, 4e-3), n_modes=64):
    """Per-member SSH perturbations (smooth random fields, std sigma) and drag coefficients."""
    r_cd = rng_for(seed_cd)
    cds = r_cd.uniform(cd_range[0], cd_range[1], size=n_members)
    x, y = mesh.x_cell[:, 0], mesh.x_cell[:, 1]
    fields = []
    for m in range(n_members):
        r = rng_for(seed_ssh0 + m)
        # random Fourier features with a Gaussian spectrum of correlation length corr,
        # restricted to wavenumbers periodic on the domain
        kx = np.round(r.normal(0, mesh.lx / (2 * math.pi * corr), n_modes)) * 2 * math.pi / mesh.lx
        ky = np.round(r.normal(0, mesh.ly / (2 * math.pi * corr), n_modes)) * 2 * math.pi / mesh.ly
        ph = r.uniform(0, 2 * math.pi, n_modes)
        fld = np.sqrt(2.0 / n_modes) * np.cos(np.outer(x, kx) + np.outer(y, ky) + ph).sum(axis=1)
        fields.append(sigma * fld)
    return fields, cds


# ----------------------------------------------------------------------------
# configuration 3: spherical coastline-refined CVT, bathymetry field, cyclone
# ----------------------------------------------------------------------------

def _smoothstep(x):
    x = np.clip(x, 0.0, 1.0)
    return x * x * (3.0 - 2.0 * x)


class Coastline:
    """Seeded perturbed small circle (angular radius 20 deg, 6 Fourier modes)."""

    def __init__(self, seed, radius_deg=20.0, modes=6, amp=0.04):
        r = rng_for(seed)
        c0 = r.normal(size=3)
        c0[2] = abs(c0[2]) + 0.5          # keep the storm region in the northern hemisphere
        self.c0 = c0 / np.linalg.norm(c0)
        e1 = np.cross(self.c0, [0.0, 0.0, 1.0])
        self.e1 = e1 / np.linalg.norm(e1)
        self.e2 = np.cross(self.c0, self.e1)
        self.rho0 = math.radians(radius_deg)
        self.a = r.uniform(0, amp, size=modes)
        self.ph = r.uniform(0, 2 * math.pi, size=modes)

    def angular_distance(self, x):
        theta = np.arccos(np.clip(x @ self.c0, -1, 1))
        phi = np.arctan2(x @ self.e2, x @ self.e1)
        m = np.arange(1, self.a.size + 1)
        rho = self.rho0 * (1 + (self.a[None, :] * np.cos(np.outer(phi, m) + self.ph[None, :])).sum(axis=1))
        return np.abs(theta - rho)


def sphere_dx_factory(coast, n_target, radius=meshgen.EARTH_RADIUS, dx_fine=6e3, dx_coarse=60e3, nq=200000):
    """dx(x) = fine + (coarse - fine) smoothstep(d / D), D solved for n_target cells."""
    q = meshgen.fibonacci_sphere(nq)
    dq = coast.angular_distance(q) * radius
    area = 4 * math.pi * radius ** 2 / nq

    def count(D):
        dx = dx_fine + (dx_coarse - dx_fine) * _smoothstep(dq / D)
        return np.sum(area / (math.sqrt(3) / 2 * dx * dx))

    lo, hi = 1e3, 2e7
    for _ in range(80):
        mid = math.sqrt(lo * hi)
        if count(mid) < n_target:
            lo = mid
        else:
            hi = mid
    D = 0.5 * (lo + hi)

    def dx(x):
        return dx_fine + (dx_coarse - dx_fine) * _smoothstep(coast.angular_distance(x) * radius / D)
    return dx, D


def gaussian_field_sphere(x, seed, mean, std, corr, radius=meshgen.EARTH_RADIUS, n_modes=256):
    """Smooth random field on the sphere: random Fourier features of the embedding coordinates."""
    r = rng_for(seed)
    k = r.normal(0, 1.0 / corr, size=(n_modes, 3))
    ph = r.uniform(0, 2 * math.pi, n_modes)
    fld = np.sqrt(2.0 / n_modes) * np.cos((x * radius) @ k.T + ph).sum(axis=1)
    return mean + std * fld


_SPHERE_CACHE = {}


def sphere_mesh(n=400000, seed_coast=5, iters=20, dx_fine=6e3, dx_coarse=60e3, progress=None):
    """Spherical CVT refined near the seeded coastline.

    Multilevel construction: generators drawn with density ~ dx^-2 at
    n0 = (n + 30) / 16 points (or n when that is small), density-weighted Lloyd
    iterations (density dx^-4), then per level the Delaunay edge midpoints are
    added (N -> 4N - 6, halving the spacing everywhere) and the Lloyd sweeps are
    repeated; the final generators are sorted along a Morton curve."""
    key = (n, seed_coast, iters, dx_fine, dx_coarse)
    if key in _SPHERE_CACHE:
        return _SPHERE_CACHE[key]
    coast = Coastline(seed_coast)
    # optional on-disk cache (directory in FBLTS_MESH_CACHE) of the generated mesh
    cache_dir = os.environ.get("FBLTS_MESH_CACHE")
    cache_file = None
    if cache_dir:
        cache_file = os.path.join(cache_dir, "sphere_%d_%d_%d_%g_%g.npz" % key)
        if os.path.exists(cache_file):
            m = meshgen.Mesh.load(cache_file)
            m.meta["coast"] = coast
            _SPHERE_CACHE[key] = m
            return m
    dx, D = sphere_dx_factory(coast, n, dx_fine=dx_fine, dx_coarse=dx_coarse)
    levels = 0
    n0 = n
    while n0 > 80000:
        n0 = (n0 + 6) // 4
        levels += 1
    r = rng_for(seed_coast + 1000)
    pts = []
    need = n0
    while need > 0:
        cand = meshgen._normalize(r.normal(size=(need * 8, 3)))
        acc = r.uniform(size=cand.shape[0]) < (dx_fine / dx(cand)) ** 2
        got = cand[acc][:need]
        pts.append(got)
        need -= got.shape[0]
    pts = np.concatenate(pts)
    density = lambda x: dx(x) ** -4   # noqa: E731
    for lev in range(levels + 1):
        if lev > 0:
            pts = meshgen.refine_midpoints(pts)
        its = iters if lev == 0 else max(3, iters // 4)
        for it in range(its):
            pts = meshgen.lloyd_sphere(pts, density, 1)
            if progress:
                progress("sphere level %d (%d points) Lloyd %d/%d" % (lev, pts.shape[0], it + 1, its))
    pts = pts[meshgen.morton_order_sphere(pts)]
    m = meshgen.sphere_from_generators(pts)
    m.meta.update(kind="sphere", n=m.n_cells, seed=seed_coast, iters=iters, levels=levels, D=D)
    if cache_file:
        os.makedirs(cache_dir, exist_ok=True)
        m.save(cache_file)
    m.meta["coast"] = coast
    _SPHERE_CACHE[key] = m
    return m


def config3(n=400000, M=8, seed_coast=5, seed_bathy=6, seed_track=7, iters=20, cd=2.5e-3, dx_fine=6e3,
            dx_coarse=60e3, progress=None):
    """Spherical CVT refined 60 -> 6 km near a seeded coastline, bathymetry field in [10, 5000] m,
    quadratic drag, Holland cyclone wind stress along a seeded great-circle track, M = 8."""
    from . import forcing
    base = sphere_mesh(n, seed_coast, iters, dx_fine, dx_coarse, progress)
    xc = base.x_cell / base.sphere_radius
    H = np.clip(gaussian_field_sphere(xc, seed_bathy, 3000.0, 1500.0, 500e3), 10.0, 5000.0)
    mesh = base.copy_with(bottom_depth=H)
    h0 = H.copy()
    u0 = np.zeros(mesh.n_edges)
    fine, dt_c, dt_f = cfl_fine_mask(mesh, M)
    coast = base.meta["coast"]
    # the storm starts 6 degrees outside the mean coastline and heads for its centre
    storm = forcing.seeded_track(seed_track, target=coast.c0, start_distance=coast.rho0 + math.radians(6.0),
                                 radius=base.sphere_radius)
    steps = int(math.ceil(2 * 86400.0 / dt_c))      # two simulated days
    return Workload("sphere%dk_cyclone" % (round(mesh.n_cells / 1000)), mesh, h0, u0, fine, dt_c, M, False,
                    np.full(mesh.n_cells, cd), steps, dict(dt_fine=dt_f, n_fine=int(fine.sum()), storm=storm,
                                                         seeds=(seed_coast, seed_bathy, seed_track)))


def small_sphere(n=3000, M=4, iters=20):
    """Configuration-3 recipe at test size: the same construction with the
    resolution range scaled to the cell count (200 -> 600 km)."""
    return config3(n=n, M=M, iters=iters, dx_fine=200e3, dx_coarse=600e3)


# ----------------------------------------------------------------------------
# aquaplanet gravity wave (the paper's temporal-convergence experiment)
# ----------------------------------------------------------------------------

def aquaplanet(n=2000, M=4, depth=1000.0, amp=1.0, width=600e3, seed=9, iters=20,
               dx_fine=100e3, dx_coarse=800e3):
    """Non-rotating aquaplanet at rest with constant depth and a Gaussian SSH bump
    (Section 2.3): the coastline-refined spherical CVT with f = 0 everywhere, the
    fine set from the local CFL number, the external gravity-wave system."""
    base = sphere_mesh(n, 5, iters, dx_fine, dx_coarse)
    mesh = base.copy_with(f_vertex=np.zeros(base.n_vertices), f_edge=np.zeros(base.n_edges),
                          bottom_depth=np.full(base.n_cells, depth))
    r = rng_for(seed)
    c = meshgen._normalize(r.normal(size=3))
    xc = mesh.x_cell / mesh.sphere_radius
    d = np.arctan2(np.linalg.norm(np.cross(xc, c), axis=1), xc @ c) * mesh.sphere_radius
    h0 = depth + amp * np.exp(-0.5 * (d / width) ** 2)
    u0 = np.zeros(mesh.n_edges)
    fine, dt_c, dt_f = cfl_fine_mask(mesh, M)
    return Workload("aquaplanet%dk" % round(mesh.n_cells / 1000), mesh, h0, u0, fine, dt_c, M, False, None, 0,
                    dict(dt_fine=dt_f, n_fine=int(fine.sum()), centre=c))
