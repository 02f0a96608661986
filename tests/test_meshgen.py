"""Mesh generator pins: topology, geometry and TRiSK weights (CPU).

The mesh arrays are inputs shared by the HIP library and the oracle; these
tests check them against facts independent of either: Euler characteristic,
exact areas of the regular hexagonal mesh, kite decompositions, antisymmetry
of the weights and the exact tangential reconstruction of a uniform flow on
the regular hexagonal mesh (Thuburn et al. 2009 / Ringler et al. 2010).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2405_10505_amd.inputs import meshgen, workloads


@pytest.fixture(scope="module")
def hexm():
    return meshgen.hex_periodic(32, 32, 1.0e4)


@pytest.fixture(scope="module")
def cvt():
    return workloads.cvt_mesh(2000, seed=12, iters=20)


def _wmat(m):
    rows = np.repeat(np.arange(m.n_edges), np.diff(m.edges_on_edge_off))
    return sp.csr_matrix((m.weights_on_edge, (rows, m.edges_on_edge)), shape=(m.n_edges, m.n_edges))


def test_hex_counts_and_exact_geometry(hexm):
    m = hexm
    assert (m.n_cells, m.n_edges, m.n_vertices) == (1024, 3072, 2048)
    assert np.all(np.diff(m.edges_on_cell_off) == 6)
    d = 1.0e4
    np.testing.assert_allclose(m.dc_edge, d, rtol=1e-12)
    np.testing.assert_allclose(m.dv_edge, d / math.sqrt(3.0), rtol=1e-12)
    np.testing.assert_allclose(m.area_cell, math.sqrt(3) / 2 * d * d, rtol=1e-12)
    np.testing.assert_allclose(m.area_triangle, math.sqrt(3) / 4 * d * d, rtol=1e-12)
    np.testing.assert_allclose(m.kite_areas_on_vertex, math.sqrt(3) / 12 * d * d, rtol=1e-12)


@pytest.mark.parametrize("name", ["hexm", "cvt"])
def test_euler_and_area_decomposition(name, request):
    m = request.getfixturevalue(name)
    assert m.n_vertices - m.n_edges + m.n_cells == 0          # torus
    L2 = m.lx * m.ly
    assert abs(m.area_cell.sum() / L2 - 1) < 1e-12
    assert abs(m.area_triangle.sum() / L2 - 1) < 1e-12
    # half of dc*dv per edge tiles the plane (primal/dual orthogonality)
    assert abs((m.dc_edge * m.dv_edge).sum() / 2 / L2 - 1) < 1e-12
    # each vertex: three distinct cells, three distinct edges; each edge two cells, two vertices
    assert np.all(np.sort(m.cells_on_vertex, axis=1)[:, 1:] != np.sort(m.cells_on_vertex, axis=1)[:, :-1])
    assert np.all(m.cells_on_edge[:, 0] != m.cells_on_edge[:, 1])
    assert np.all(m.vertices_on_edge[:, 0] != m.vertices_on_edge[:, 1])
    assert np.all(m.kite_areas_on_vertex > 0)


@pytest.mark.parametrize("name", ["hexm", "cvt"])
def test_orientation_conventions(name, request):
    m = request.getfixturevalue(name)
    # t_e = k x n_e points from v0 to v1
    xv = m.x_vertex
    d = xv[m.vertices_on_edge[:, 1]] - xv[m.vertices_on_edge[:, 0]]
    d[:, 0] -= m.lx * np.round(d[:, 0] / m.lx)
    d[:, 1] -= m.ly * np.round(d[:, 1] / m.ly)
    assert np.all(np.einsum("ij,ij->i", d, m.tangent_edge) > 0)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), m.dv_edge, rtol=1e-9)
    # edges_on_vertex[j] joins cells_on_vertex[j] and [j+1]
    for j in range(3):
        e = m.edges_on_vertex[:, j]
        a, b = m.cells_on_vertex[:, j], m.cells_on_vertex[:, (j + 1) % 3]
        pair = np.sort(m.cells_on_edge[e], axis=1)
        assert np.all(pair == np.sort(np.stack([a, b], 1), axis=1))


@pytest.mark.parametrize("name", ["hexm", "cvt"])
def test_weights_antisymmetric(name, request):
    W = _wmat(request.getfixturevalue(name))
    assert abs(W + W.T).max() < 1e-15


def test_hex_weight_values_and_uniform_reconstruction(hexm):
    m = hexm
    vals = np.unique(np.round(np.abs(m.weights_on_edge), 12))
    np.testing.assert_allclose(vals, [0.0, 1 / 6, 1 / 3], atol=1e-12)
    assert np.all(np.diff(m.edges_on_edge_off) == 10)
    W = _wmat(m)
    for U in (np.array([3.0, -1.7]), np.array([0.0, 1.0])):
        u = m.normal_edge @ U
        perp = (W @ (m.dv_edge * u)) / m.dc_edge
        np.testing.assert_allclose(perp, m.tangent_edge @ U, atol=1e-11 * np.abs(U).max())


def test_cvt_config2_recipe_shapes():
    m = workloads.cvt_mesh(2000, seed=12, iters=20)
    assert m.n_cells == 2000
    deg = np.diff(m.edges_on_cell_off)
    assert deg.min() >= 4 and deg.max() <= 9
    assert abs(m.n_edges - 3 * m.n_cells) == 0          # torus: E = 3N, V = 2N
    # resolution ranges over the Gaussian patch: 2 km fine, 8 km coarse
    assert m.dc_edge.min() < 3.5e3 and m.dc_edge.max() > 7e3
