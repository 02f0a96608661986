"""Seeded synthetic Voronoi C-grid meshes in MPAS-style arrays.

This module only builds *inputs*: mesh connectivity and geometry of the kind
the TRiSK discretisation consumes (primal Voronoi cells carrying thickness,
edges carrying the normal velocity, triangular dual cells at the vertices;
the paper's Fig. ``trisk``).  It holds none of the time-stepping or tendency
arithmetic; both the HIP library and the CPU oracle read the arrays it writes.

Conventions (all 0-based):

* ``cells_on_edge[e] = (c0, c1)``; the unit normal ``n_e`` points c0 -> c1, so
  the outward sign of edge e for cell i is ``n_{e,i} = +1`` for c0 and -1 for
  c1 (paper, Section 2.4, the sign ``n_{e,i}`` in the mass-conservation proof).
* ``t_e = k x n_e``; ``vertices_on_edge[e] = (v0, v1)`` with t_e pointing
  v0 -> v1.  Traversing the dual edge c0 -> c1 is counter-clockwise about v1.
* Cells list their edges and vertices counter-clockwise; vertex j of a cell
  lies between its edge j and edge j+1.
* ``kite_areas_on_vertex[v, j]`` is the area of cell ``cells_on_vertex[v, j]``
  inside the dual triangle of v.  ``area_cell`` and ``area_triangle`` are the
  kite sums, so the kite fractions R_{i,v} of a cell add up to one.
* ``weights_on_edge`` are the dimensionless TRiSK tangential-reconstruction
  weights w_{e,e'} (Thuburn et al. 2009; Ringler et al. 2010, the TRiSK scheme
  the paper builds on), aligned with ``edges_on_edge``: the tangential velocity
  is u_perp_e = (1/d_e) sum_{e'} w_{e,e'} l_{e'} u_{e'}.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay, ConvexHull

EARTH_RADIUS = 6.371229e6
OMEGA = 7.292e-5


@dataclass
class Mesh:
    """MPAS-style mesh arrays (SI units; int32 connectivity, float64 geometry)."""

    n_cells: int
    n_edges: int
    n_vertices: int
    cells_on_edge: np.ndarray        # [E,2]
    vertices_on_edge: np.ndarray     # [E,2]
    edges_on_cell_off: np.ndarray    # [N+1]
    edges_on_cell: np.ndarray        # [sum]
    vertices_on_cell_off: np.ndarray  # [N+1]
    vertices_on_cell: np.ndarray     # [sum]
    edges_on_edge_off: np.ndarray    # [E+1]
    edges_on_edge: np.ndarray        # [sum]
    weights_on_edge: np.ndarray      # [sum]
    edges_on_vertex: np.ndarray      # [V,3]
    cells_on_vertex: np.ndarray      # [V,3]
    kite_areas_on_vertex: np.ndarray  # [V,3]
    dc_edge: np.ndarray
    dv_edge: np.ndarray
    area_cell: np.ndarray
    area_triangle: np.ndarray
    f_vertex: np.ndarray
    f_edge: np.ndarray
    bottom_depth: np.ndarray
    is_sphere: int = 0
    sphere_radius: float = 0.0
    # positions / orientation (not needed by the solver; used by generators)
    x_cell: np.ndarray = None        # [N,2] planar or [N,3] sphere
    x_edge: np.ndarray = None
    x_vertex: np.ndarray = None
    normal_edge: np.ndarray = None   # [E,2] or [E,3] unit n_e
    tangent_edge: np.ndarray = None  # t_e = k x n_e
    lx: float = 0.0
    ly: float = 0.0
    meta: dict = field(default_factory=dict)

    def desc_arrays(self):
        """Arrays in the order and dtypes of the library's mesh descriptor."""
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        return dict(
            cells_on_edge=i32(self.cells_on_edge.reshape(-1)),
            vertices_on_edge=i32(self.vertices_on_edge.reshape(-1)),
            edges_on_cell_off=i32(self.edges_on_cell_off),
            edges_on_cell=i32(self.edges_on_cell),
            vertices_on_cell_off=i32(self.vertices_on_cell_off),
            vertices_on_cell=i32(self.vertices_on_cell),
            edges_on_edge_off=i32(self.edges_on_edge_off),
            edges_on_edge=i32(self.edges_on_edge),
            weights_on_edge=f64(self.weights_on_edge),
            edges_on_vertex=i32(self.edges_on_vertex.reshape(-1)),
            cells_on_vertex=i32(self.cells_on_vertex.reshape(-1)),
            kite_areas_on_vertex=f64(self.kite_areas_on_vertex.reshape(-1)),
            dc_edge=f64(self.dc_edge), dv_edge=f64(self.dv_edge),
            area_cell=f64(self.area_cell), area_triangle=f64(self.area_triangle),
            f_vertex=f64(self.f_vertex), f_edge=f64(self.f_edge),
            bottom_depth=f64(self.bottom_depth),
        )

    def save(self, path):
        """Write the arrays and scalar fields to an .npz file (no pickled objects;
        ``meta`` entries that are not plain numbers or strings are dropped)."""
        arrays, scalars = {}, {}
        for k, v in self.__dict__.items():
            if isinstance(v, np.ndarray):
                arrays[k] = v
            elif k != "meta" and v is not None:
                scalars[k] = v
        meta = {k: v for k, v in self.meta.items() if isinstance(v, (int, float, str))}
        np.savez(path, __scalars__=np.array(json.dumps(scalars)), __meta__=np.array(json.dumps(meta)), **arrays)

    @staticmethod
    def load(path):
        with np.load(path, allow_pickle=False) as z:
            d = {k: z[k] for k in z.files if not k.startswith("__")}
            d.update(json.loads(str(z["__scalars__"])))
            meta = json.loads(str(z["__meta__"]))
        return Mesh(meta=meta, **d)

    def copy_with(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Mesh(**d)


# ----------------------------------------------------------------------------
# small geometry helpers
# ----------------------------------------------------------------------------

def _shoelace(*pts):
    """Signed area of the planar polygon with vertices pts (each [...,2])."""
    a = 0.0
    n = len(pts)
    for k in range(n):
        p, q = pts[k], pts[(k + 1) % n]
        a = a + (p[..., 0] * q[..., 1] - q[..., 0] * p[..., 1])
    return 0.5 * a


def _circumcenter2(a, b, c):
    ax, ay = a[:, 0], a[:, 1]
    bx, by = b[:, 0] - ax, b[:, 1] - ay
    cx, cy = c[:, 0] - ax, c[:, 1] - ay
    d = 2.0 * (bx * cy - by * cx)
    b2 = bx * bx + by * by
    c2 = cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    return np.stack([ax + ux, ay + uy], axis=1)


def _kite_lookup(cov, kites, cells, verts):
    """Kite area of (cell, vertex) pairs, looked up from the per-vertex lists."""
    nv = cov.shape[0]
    key = cov.reshape(-1).astype(np.int64) * nv + np.repeat(np.arange(nv), 3)
    order = np.argsort(key)
    q = cells.astype(np.int64) * nv + verts
    pos = np.searchsorted(key[order], q)
    if np.any(key[order][np.minimum(pos, key.size - 1)] != q):
        raise RuntimeError("cell/vertex incidence mismatch")
    return kites.reshape(-1)[order][pos]


def _trisk_weights(n_cells, eoc_off, eoc, voc, coe, cov, kites, area_cell):
    """edges_on_edge CSR and the dimensionless TRiSK weights.

    For edge e and one of its cells i, walk the other edges of i
    counter-clockwise starting after e: e'_1 .. e'_{n-1}; v_m is the vertex
    between e'_{m-1} and e'_m (e'_0 = e).  Then
        w_{e,e'_m} = n_{e,i} n_{e'_m,i} (1/2 - sum_{p<=m} R_{i,v_p}),
    with R_{i,v} the kite fraction of cell i at vertex v.  The list of e holds
    c0's edges first, then c1's.
    """
    deg = np.diff(eoc_off)
    cell_of = np.repeat(np.arange(n_cells), deg)
    kite_cv = _kite_lookup(cov, kites, cell_of, voc)
    R_all = kite_cv / area_cell[cell_of]
    sgn_all = np.where(coe[eoc, 0] == cell_of, 1.0, -1.0)
    rec_e, rec_slot, rec_m, rec_e2, rec_w = [], [], [], [], []
    for n in np.unique(deg):
        cells = np.nonzero(deg == n)[0]
        base = eoc_off[cells][:, None] + np.arange(n)[None, :]
        E = eoc[base]
        R = R_all[base]
        S = sgn_all[base]
        for j0 in range(n):
            acc = np.zeros(cells.size)
            e = E[:, j0]
            slot = np.where(coe[e, 0] == cells, 0, 1)
            for m in range(1, n):
                acc = acc + R[:, (j0 + m - 1) % n]
                jm = (j0 + m) % n
                rec_e.append(e); rec_slot.append(slot)
                rec_m.append(np.full(cells.size, m)); rec_e2.append(E[:, jm])
                rec_w.append(S[:, j0] * S[:, jm] * (0.5 - acc))
    rec_e = np.concatenate(rec_e); rec_slot = np.concatenate(rec_slot)
    rec_m = np.concatenate(rec_m); rec_e2 = np.concatenate(rec_e2); rec_w = np.concatenate(rec_w)
    order = np.lexsort((rec_m, rec_slot, rec_e))
    n_edges = coe.shape[0]
    off = np.zeros(n_edges + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(rec_e, minlength=n_edges))
    return off.astype(np.int32), rec_e2[order].astype(np.int32), rec_w[order]


# ----------------------------------------------------------------------------
# planar doubly periodic Voronoi mesh from generators
# ----------------------------------------------------------------------------

def _periodic_delaunay(pts, lx, ly, margin):
    shifts, ids, allp = [], [], []
    n = pts.shape[0]
    # the unshifted originals come first, so point k < n is generator k
    for sx, sy in [(0, 0)] + [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]:
        if True:
            q = pts + np.array([sx * lx, sy * ly])
            if sx == 0 and sy == 0:
                keep = np.ones(n, dtype=bool)
            else:
                keep = ((q[:, 0] > -margin) & (q[:, 0] < lx + margin) &
                        (q[:, 1] > -margin) & (q[:, 1] < ly + margin))
            allp.append(q[keep])
            ids.append(np.nonzero(keep)[0])
    allp = np.concatenate(allp)
    ids = np.concatenate(ids)
    tri = Delaunay(allp)
    return allp, ids, tri


def lloyd_planar_periodic(pts, lx, ly, density, iters, margin):
    """Density-weighted Lloyd iterations on the doubly periodic plane.

    Each Delaunay edge (a,b) with adjacent circumcentres (c1,c2) gives the
    triangle (x_a, c1, c2) to cell a and (x_b, c1, c2) to cell b; mass and
    first moments are integrated with the centroid rule on those triangles.
    """
    n = pts.shape[0]
    pts = pts.copy()
    for _ in range(iters):
        allp, ids, tri = _periodic_delaunay(pts, lx, ly, margin)
        s = tri.simplices
        cc = _circumcenter2(allp[s[:, 0]], allp[s[:, 1]], allp[s[:, 2]])
        nb = tri.neighbors
        # each interior triangle pair once: (t, k) with neighbour across vertex k
        t_idx = np.repeat(np.arange(s.shape[0]), 3)
        k_idx = np.tile(np.arange(3), s.shape[0])
        t2 = nb[t_idx, k_idx]
        ok = (t2 >= 0) & (t2 > t_idx)
        t_idx, k_idx, t2 = t_idx[ok], k_idx[ok], t2[ok]
        a = s[t_idx, (k_idx + 1) % 3]
        b = s[t_idx, (k_idx + 2) % 3]
        c1 = cc[t_idx]
        c2 = cc[t2]
        mass = np.zeros(allp.shape[0])
        mx = np.zeros(allp.shape[0])
        my = np.zeros(allp.shape[0])
        for g in (a, b):
            pg = allp[g]
            ar = np.abs(_shoelace(pg, c1, c2))
            cen = (pg + c1 + c2) / 3.0
            rho = density(np.mod(cen[:, 0], lx), np.mod(cen[:, 1], ly))
            m = ar * rho
            mass += np.bincount(g, m, allp.shape[0])
            mx += np.bincount(g, m * cen[:, 0], allp.shape[0])
            my += np.bincount(g, m * cen[:, 1], allp.shape[0])
        own = np.arange(n)  # the first n points are the unshifted originals
        newp = np.stack([mx[own] / mass[own], my[own] / mass[own]], axis=1)
        pts = np.stack([np.mod(newp[:, 0], lx), np.mod(newp[:, 1], ly)], axis=1)
    return pts


def planar_periodic_from_generators(pts, lx, ly, f0=1e-4, depth=1000.0, margin=None):
    """Build the TRiSK mesh whose Voronoi generators are ``pts`` on [0,lx)x[0,ly)."""
    pts = np.asarray(pts, dtype=np.float64)
    n = pts.shape[0]
    if margin is None:
        margin = 4.0 * math.sqrt(lx * ly / n) * 3.0
    allp, ids, tri = _periodic_delaunay(pts, lx, ly, margin)
    s = tri.simplices.copy()
    # orient every triangle counter-clockwise
    area = _shoelace(allp[s[:, 0]], allp[s[:, 1]], allp[s[:, 2]])
    flip = area < 0
    s[flip] = s[flip][:, [0, 2, 1]]
    cc = _circumcenter2(allp[s[:, 0]], allp[s[:, 1]], allp[s[:, 2]])
    # ownership window: the periodic cell shifted by an odd fraction of the
    # spacing, so no circumcentre or edge midpoint of a lattice sits on its border
    h_sp = math.sqrt(lx * ly / n)
    ox, oy = -0.1372 * h_sp, -0.0917 * h_sp

    def inside(p):
        return (p[..., 0] >= ox) & (p[..., 0] < lx + ox) & (p[..., 1] >= oy) & (p[..., 1] < ly + oy)

    owned_t = np.nonzero(inside(cc))[0]
    nv = owned_t.shape[0]
    tri_key = {}
    for vi, t in enumerate(owned_t):
        tri_key[tuple(sorted(ids[s[t]].tolist()))] = vi

    def canon_tri(t):
        return tri_key[tuple(sorted(ids[s[t]].tolist()))]

    # Delaunay edges -> adjacent triangles
    edge_tris = {}
    for t in range(s.shape[0]):
        for k in range(3):
            a, b = int(s[t, (k + 1) % 3]), int(s[t, (k + 2) % 3])
            key = (a, b) if a < b else (b, a)
            edge_tris.setdefault(key, []).append(t)
    owned_e = []
    for (a, b), tl in edge_tris.items():
        mid = 0.5 * (allp[a] + allp[b])
        if inside(mid):
            if len(tl) != 2:
                raise RuntimeError("periodic Delaunay margin too small")
            owned_e.append((a, b, tl[0], tl[1]))
    ne = len(owned_e)
    coe = np.zeros((ne, 2), np.int32)
    voe = np.zeros((ne, 2), np.int32)
    dc = np.zeros(ne)
    dv = np.zeros(ne)
    nrm = np.zeros((ne, 2))
    tng = np.zeros((ne, 2))
    xe = np.zeros((ne, 2))
    cell_edges = [[] for _ in range(n)]   # (angle, e)
    for e, (a, b, t1, t2) in enumerate(owned_e):
        pa, pb = allp[a], allp[b]
        d = pb - pa
        L = math.hypot(d[0], d[1])
        nvec = d / L
        tvec = np.array([-nvec[1], nvec[0]])  # k x n
        C1, C2 = cc[t1], cc[t2]
        if np.dot(C2 - C1, tvec) < 0:
            t1, t2 = t2, t1
            C1, C2 = C2, C1
        coe[e] = (ids[a], ids[b])
        voe[e] = (canon_tri(t1), canon_tri(t2))
        dc[e] = L
        dv[e] = math.hypot(*(C2 - C1))
        nrm[e] = nvec
        tng[e] = tvec
        m = 0.5 * (pa + pb)
        xe[e] = (m[0] % lx, m[1] % ly)
        vm = 0.5 * (C1 + C2)
        ra, rb = vm - pa, vm - pb
        cell_edges[ids[a]].append((math.atan2(ra[1], ra[0]), e))
        cell_edges[ids[b]].append((math.atan2(rb[1], rb[0]), e))
    # vertices: positions, cells (ccw), kites
    cov = np.zeros((nv, 3), np.int32)
    kites = np.zeros((nv, 3))
    xv = np.zeros((nv, 2))
    cell_verts = [[] for _ in range(n)]   # (angle, v)
    for vi, t in enumerate(owned_t):
        p = [allp[s[t, k]] for k in range(3)]
        C = cc[t]
        xv[vi] = (C[0] % lx, C[1] % ly)
        for k in range(3):
            P0, P1, P2 = p[k], p[(k + 1) % 3], p[(k + 2) % 3]
            z = np.zeros(2)
            kite = _shoelace(z, 0.5 * (P1 - P0), C - P0, 0.5 * (P2 - P0))
            ci = int(ids[s[t, k]])
            cov[vi, k] = ci
            kites[vi, k] = kite
            dvec = C - P0
            cell_verts[ci].append((math.atan2(dvec[1], dvec[0]), vi))
    # edges on vertex: edge between cells_on_vertex j and j+1
    pair_edge = {}
    for e in range(ne):
        a, b = int(coe[e, 0]), int(coe[e, 1])
        pair_edge[(min(a, b), max(a, b), int(voe[e, 0]))] = e
        pair_edge[(min(a, b), max(a, b), int(voe[e, 1]))] = e
    eov = np.zeros((nv, 3), np.int32)
    for vi in range(nv):
        for j in range(3):
            a, b = int(cov[vi, j]), int(cov[vi, (j + 1) % 3])
            eov[vi, j] = pair_edge[(min(a, b), max(a, b), vi)]
    # cell ccw ordering: vertex j between edge j and j+1
    eoc_off = np.zeros(n + 1, np.int32)
    eoc, voc = [], []
    for i in range(n):
        es = sorted(cell_edges[i])
        vs = sorted(cell_verts[i])
        if len(es) != len(vs):
            raise RuntimeError("cell %d: %d edges vs %d vertices" % (i, len(es), len(vs)))
        ea = np.array([a for a, _ in es])
        va = np.array([a for a, _ in vs])
        # choose the vertex list rotation so that vertex j follows edge j ccw
        k0 = int(np.searchsorted(va, ea[0], side="right")) % len(vs)
        vs = vs[k0:] + vs[:k0]
        eoc.extend([e for _, e in es])
        voc.extend([v for _, v in vs])
        eoc_off[i + 1] = len(eoc)
    eoc = np.array(eoc, np.int32)
    voc = np.array(voc, np.int32)
    area_cell = np.zeros(n)
    np.add.at(area_cell, cov.reshape(-1), kites.reshape(-1))
    area_tri = kites.sum(axis=1)
    eoe_off, eoe, woe = _trisk_weights(n, eoc_off, eoc, voc, coe, cov, kites, area_cell)
    mesh = Mesh(
        n_cells=n, n_edges=ne, n_vertices=nv,
        cells_on_edge=coe, vertices_on_edge=voe,
        edges_on_cell_off=eoc_off, edges_on_cell=eoc,
        vertices_on_cell_off=eoc_off.copy(), vertices_on_cell=voc,
        edges_on_edge_off=eoe_off, edges_on_edge=eoe, weights_on_edge=woe,
        edges_on_vertex=eov, cells_on_vertex=cov, kite_areas_on_vertex=kites,
        dc_edge=dc, dv_edge=dv, area_cell=area_cell, area_triangle=area_tri,
        f_vertex=np.full(nv, f0), f_edge=np.full(ne, f0),
        bottom_depth=np.full(n, depth) if np.isscalar(depth) else np.asarray(depth, float),
        x_cell=pts.copy(), x_edge=xe, x_vertex=xv, normal_edge=nrm, tangent_edge=tng,
        lx=lx, ly=ly,
    )
    return mesh


def hex_periodic(nx, ny, dc, f0=1e-4, depth=1000.0):
    """Regular hexagonal doubly periodic mesh: nx*ny cells, centre spacing dc.

    Offset rows: L_x = nx*dc, L_y = ny*dc*sqrt(3)/2 (ny even).
    """
    if ny % 2:
        raise ValueError("ny must be even for a periodic hexagonal mesh")
    lx = nx * dc
    ly = ny * dc * math.sqrt(3.0) / 2.0
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = (i + 0.5 * (j % 2) + 0.25) * dc
    y = (j + 0.5) * dc * math.sqrt(3.0) / 2.0
    pts = np.stack([x.reshape(-1), y.reshape(-1)], axis=1)
    m = planar_periodic_from_generators(pts, lx, ly, f0=f0, depth=depth, margin=3.0 * dc)
    m.meta.update(kind="hex", nx=nx, ny=ny, dc=dc)
    return m


# ----------------------------------------------------------------------------
# variable-resolution planar CVT (synthetic stand-in for a regionally refined mesh)
# ----------------------------------------------------------------------------

def _hilbert_order(x, y, lx, ly, bits=16):
    """Permutation sorting points along a Hilbert curve (locality ordering)."""
    n = 1 << bits
    xi = np.clip((x / lx * n).astype(np.int64), 0, n - 1)
    yi = np.clip((y / ly * n).astype(np.int64), 0, n - 1)
    d = np.zeros_like(xi)
    s = n >> 1
    while s > 0:
        rx = ((xi & s) > 0).astype(np.int64)
        ry = ((yi & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate
        m = ry == 0
        flip = m & (rx == 1)
        xi = np.where(flip, s - 1 - xi, xi)
        yi = np.where(flip, s - 1 - yi, yi)
        xi2 = np.where(m, yi, xi)
        yi2 = np.where(m, xi, yi)
        xi, yi = xi2, yi2
        s >>= 1
    return np.argsort(d, kind="stable")


def cvt_planar_periodic(n, dx_fn_factory, iters=50, seed=2, f0=1e-4):
    """Density-weighted planar periodic CVT with ``n`` cells.

    ``dx_fn_factory(L)`` returns (dx(x,y) in metres, domain side L); the
    generators are drawn with density proportional to dx^-2 and relaxed with
    Lloyd iterations under the CVT density dx^-4.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    L, dx = dx_fn_factory(n, rng)
    lx = ly = L
    # rejection sampling from cell density ~ dx^-2
    dmin = dx(np.array([0.0]), np.array([0.0]))
    pts = []
    need = n
    grid = np.linspace(0, L, 256)
    gx, gy = np.meshgrid(grid, grid)
    dmin = float(np.min(dx(gx.reshape(-1), gy.reshape(-1))))
    while need > 0:
        cand = rng.uniform(0, L, size=(need * 4, 2))
        acc = rng.uniform(0, 1, size=need * 4) < (dmin / dx(cand[:, 0], cand[:, 1])) ** 2
        got = cand[acc][:need]
        pts.append(got)
        need -= got.shape[0]
    pts = np.concatenate(pts)
    dmax = float(np.max(dx(gx.reshape(-1), gy.reshape(-1))))
    density = lambda x, y: dx(x, y) ** -4
    pts = lloyd_planar_periodic(pts, lx, ly, density, iters, margin=4.0 * dmax)
    order = _hilbert_order(pts[:, 0], pts[:, 1], lx, ly)
    pts = pts[order]
    m = planar_periodic_from_generators(pts, lx, ly, f0=f0, margin=4.0 * dmax)
    m.meta.update(kind="cvt_planar", n=n, seed=seed, iters=iters, L=L)
    return m


def gaussian_patch_dx(n_target, rng, dx_coarse=8e3, dx_fine=2e3, sigma_frac=0.1):
    """dx(x) = coarse - (coarse-fine) exp(-|x-x0|^2/(2 sigma^2)), sigma = 0.1 L.

    L is solved so that the integral of 1/((sqrt(3)/2) dx^2) over the periodic
    square equals n_target; x0 is drawn from ``rng``.
    """
    u0 = rng.uniform(0.2, 0.8, size=2)

    def make(L):
        x0 = u0 * L
        sig = sigma_frac * L

        def dx(x, y):
            ddx = np.abs(x - x0[0]); ddx = np.minimum(ddx, L - ddx)
            ddy = np.abs(y - x0[1]); ddy = np.minimum(ddy, L - ddy)
            r2 = ddx * ddx + ddy * ddy
            return dx_coarse - (dx_coarse - dx_fine) * np.exp(-r2 / (2 * sig * sig))
        return dx

    def count(L):
        g = (np.arange(400) + 0.5) / 400 * L
        gx, gy = np.meshgrid(g, g)
        d = make(L)(gx, gy)
        return np.sum(1.0 / (math.sqrt(3) / 2 * d * d)) * (L / 400) ** 2

    lo, hi = 1e3, 1e8
    for _ in range(100):
        mid = math.sqrt(lo * hi)
        if count(mid) < n_target:
            lo = mid
        else:
            hi = mid
    L = 0.5 * (lo + hi)
    return L, make(L)


# ----------------------------------------------------------------------------
# spherical centroidal Voronoi mesh
# ----------------------------------------------------------------------------

def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _sph_tri_area(a, b, c):
    """Signed spherical-triangle area (unit sphere), positive if a,b,c ccw seen from outside."""
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def _arc(a, b):
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.einsum("ij,ij->i", a, b))


def lloyd_sphere(pts, density, iters):
    """Density-weighted Lloyd iterations on the unit sphere (via the convex hull)."""
    for _ in range(iters):
        hull = ConvexHull(pts)
        s = hull.simplices.copy()
        a, b, c = pts[s[:, 0]], pts[s[:, 1]], pts[s[:, 2]]
        nrm = np.cross(b - a, c - a)
        flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
        s[flip] = s[flip][:, [0, 2, 1]]
        a, b, c = pts[s[:, 0]], pts[s[:, 1]], pts[s[:, 2]]
        cc = _normalize(np.cross(b - a, c - a))
        npt = pts.shape[0]
        acc = np.zeros((npt, 3))
        for k in range(3):
            g = s[:, k]
            p0 = pts[g]
            p1 = 0.5 * (p0 + pts[s[:, (k + 1) % 3]])
            p2 = 0.5 * (p0 + pts[s[:, (k + 2) % 3]])
            for q1, q2 in ((p1, cc), (cc, p2)):
                q1n, q2n = _normalize(q1), _normalize(q2)
                ar = _sph_tri_area(p0, q1n, q2n)      # signed: exact decomposition for obtuse triangles
                cen = _normalize(p0 + q1n + q2n)
                w = ar * density(cen)
                for d in range(3):
                    acc[:, d] += np.bincount(g, w * cen[:, d], npt)
        pts = _normalize(acc)
    return pts


def refine_midpoints(pts):
    """Add the midpoint of every Delaunay edge: N -> 4N - 6 points, each triangle split into four."""
    s = ConvexHull(pts).simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return np.concatenate([pts, _normalize(pts[e[:, 0]] + pts[e[:, 1]])])


def sphere_from_generators(pts, radius=EARTH_RADIUS, omega=OMEGA, depth=4000.0):
    """TRiSK mesh of the spherical Voronoi diagram of unit vectors ``pts`` (vectorised)."""
    pts = _normalize(np.asarray(pts, dtype=np.float64))
    n = pts.shape[0]
    hull = ConvexHull(pts)
    s = hull.simplices.copy()
    a, b, c = pts[s[:, 0]], pts[s[:, 1]], pts[s[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    s[flip] = s[flip][:, [0, 2, 1]]
    a, b, c = pts[s[:, 0]], pts[s[:, 1]], pts[s[:, 2]]
    cc = _normalize(np.cross(b - a, c - a))
    nv = s.shape[0]
    # edges: each triangle side, deduplicated; every edge borders exactly two triangles
    u = np.concatenate([s[:, 1], s[:, 2], s[:, 0]])
    v = np.concatenate([s[:, 2], s[:, 0], s[:, 1]])
    tri = np.tile(np.arange(nv), 3)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = lo.astype(np.int64) * n + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    if np.any(ks[0::2] != ks[1::2]):
        raise RuntimeError("spherical Delaunay: an edge does not border exactly two triangles")
    coe = np.stack([lo[order][0::2], hi[order][0::2]], 1).astype(np.int32)
    t12 = np.stack([tri[order][0::2], tri[order][1::2]], 1)
    ekeys = ks[0::2]
    ne = coe.shape[0]
    pa, pb = pts[coe[:, 0]], pts[coe[:, 1]]
    xe = _normalize(pa + pb)
    nvec = _normalize(pb - pa - np.einsum("ij,ij->i", pb - pa, xe)[:, None] * xe)
    tvec = np.cross(xe, nvec)  # k x n with k the outward radial unit vector
    C1, C2 = cc[t12[:, 0]], cc[t12[:, 1]]
    sw = np.einsum("ij,ij->i", C2 - C1, tvec) < 0
    t12[sw] = t12[sw][:, ::-1]
    voe = t12.astype(np.int32)
    dc = _arc(pa, pb) * radius
    dv = _arc(cc[voe[:, 0]], cc[voe[:, 1]]) * radius
    cov = s.astype(np.int32)
    kites = np.zeros((nv, 3))
    for k in range(3):
        P0 = pts[s[:, k]]
        M1 = _normalize(P0 + pts[s[:, (k + 1) % 3]])
        M2 = _normalize(P0 + pts[s[:, (k + 2) % 3]])
        kites[:, k] = (_sph_tri_area(P0, M1, cc) + _sph_tri_area(P0, cc, M2)) * radius ** 2
    # edges on vertex: edge j joins cells_on_vertex j and j+1
    eov = np.zeros((nv, 3), np.int32)
    for j in range(3):
        x, y = cov[:, j].astype(np.int64), cov[:, (j + 1) % 3].astype(np.int64)
        q = np.minimum(x, y) * n + np.maximum(x, y)
        eov[:, j] = np.searchsorted(ekeys, q)
    # counter-clockwise edges of each cell: angle of the Voronoi-edge midpoint in the cell's tangent frame
    vmid = _normalize(cc[voe[:, 0]] + cc[voe[:, 1]])
    cell_of = np.concatenate([coe[:, 0], coe[:, 1]]).astype(np.int64)
    edge_of = np.concatenate([np.arange(ne), np.arange(ne)])
    p = pts[cell_of]
    ref = np.where(np.abs(p[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    ex = _normalize(np.cross(ref, p))
    ey = np.cross(p, ex)
    d = vmid[edge_of] - p
    ang = np.arctan2(np.einsum("ij,ij->i", d, ey), np.einsum("ij,ij->i", d, ex))
    o = np.lexsort((ang, cell_of))
    eoc = edge_of[o].astype(np.int32)
    deg = np.bincount(cell_of, minlength=n)
    eoc_off = np.zeros(n + 1, np.int32)
    eoc_off[1:] = np.cumsum(deg)
    # vertex j: the vertex shared by edges j and j+1 of the cell
    nxt = np.arange(eoc.size) + 1
    ends = eoc_off[1:] - 1
    nxt[ends] = eoc_off[:-1]
    e0, e1 = eoc, eoc[nxt]
    a0, a1 = voe[e0, 0], voe[e0, 1]
    b0, b1 = voe[e1, 0], voe[e1, 1]
    voc = np.where((a0 == b0) | (a0 == b1), a0, a1).astype(np.int32)
    area_cell = np.zeros(n)
    np.add.at(area_cell, cov.reshape(-1), kites.reshape(-1))
    area_tri = kites.sum(axis=1)
    eoe_off, eoe, woe = _trisk_weights(n, eoc_off, eoc, voc, coe, cov, kites, area_cell)
    lat_v = np.arcsin(np.clip(cc[:, 2], -1, 1))
    lat_e = np.arcsin(np.clip(xe[:, 2], -1, 1))
    return Mesh(
        n_cells=n, n_edges=ne, n_vertices=nv,
        cells_on_edge=coe, vertices_on_edge=voe,
        edges_on_cell_off=eoc_off, edges_on_cell=eoc,
        vertices_on_cell_off=eoc_off.copy(), vertices_on_cell=voc,
        edges_on_edge_off=eoe_off, edges_on_edge=eoe, weights_on_edge=woe,
        edges_on_vertex=eov, cells_on_vertex=cov, kite_areas_on_vertex=kites,
        dc_edge=dc, dv_edge=dv, area_cell=area_cell, area_triangle=area_tri,
        f_vertex=2 * omega * np.sin(lat_v), f_edge=2 * omega * np.sin(lat_e),
        bottom_depth=np.full(n, depth) if np.isscalar(depth) else np.asarray(depth, float),
        is_sphere=1, sphere_radius=radius,
        x_cell=pts * radius, x_edge=xe * radius, x_vertex=cc * radius,
        normal_edge=nvec, tangent_edge=tvec,
    )


def morton_order_sphere(pts, bits=16):
    """Permutation sorting unit vectors along a 3-D Morton curve (locality ordering)."""
    q = np.clip(((pts + 1.0) * 0.5 * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(pts.shape[0], dtype=np.int64)
    for bit in range(bits):
        for k in range(3):
            code |= ((q[:, k] >> bit) & 1) << (3 * bit + k)
    return np.argsort(code, kind="stable")


def fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    z = 1 - 2 * k / n
    r = np.sqrt(1 - z * z)
    phi = k * math.pi * (3 - math.sqrt(5))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
