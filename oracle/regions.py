"""LTS regions (oracle): layering a fine set into F, IF-1, IF-2 and INT.

Test infrastructure only (see the package header).

Section 2.2: cells of the fine region F advance with dt/M; the coarse region
is split into interface one (the cells bordering F), interface two (bordering
interface one) and the interior coarse cells.  The paper asks for "enough"
interface layers so that a tendency stencil never reaches more than one region
away; the reading used here is r cell layers each (r = 2, the stencil radius
the paper gives for TRiSK), counted by breadth-first search over the
cell-adjacency graph.  F^l (l = 1..5) are the fine cells within l*r layers of
the coarse region.

Pin (tests): on the periodic hexagonal mesh with a band of full rows marked
fine, the layer counts are whole rows (256 / 128 / 128 / 512 for the 32x32
mesh with an 8-row band).
"""
from __future__ import annotations

from collections import deque

import numpy as np


def cell_neighbours(om):
    nb = [[] for _ in range(om.N)]
    for c0, c1 in om.coe.tolist():
        nb[c0].append(c1)
        nb[c1].append(c0)
    return nb


def bfs_distance(nb, sources):
    """Hop distance from the set ``sources`` (0 on it), by breadth-first search."""
    n = len(nb)
    d = np.full(n, -1, dtype=np.int64)
    q = deque()
    for s in np.nonzero(sources)[0].tolist():
        d[s] = 0
        q.append(s)
    while q:
        x = q.popleft()
        for y in nb[x]:
            if d[y] < 0:
                d[y] = d[x] + 1
                q.append(y)
    return d


def layer(om, fine_mask, r=2):
    """4-level labels (0 F, 1 IF-1, 2 IF-2, 3 INT) and F^l depth from a fine mask.

    Returns (labels, fine_depth) where fine_depth[i] is the hop distance of a
    fine cell to the coarse region (1 for fine cells bordering it) and 0 on
    coarse cells; F^l = {fine cells with fine_depth <= l*r}.
    """
    fine_mask = np.asarray(fine_mask, dtype=bool)
    nb = cell_neighbours(om)
    lab = np.full(om.N, 3, dtype=np.int8)
    lab[fine_mask] = 0
    if fine_mask.all() or not fine_mask.any():
        depth = np.zeros(om.N, dtype=np.int64)
        return lab, depth
    d_coarse = bfs_distance(nb, fine_mask)     # distance of coarse cells from F
    lab[(~fine_mask) & (d_coarse >= 1) & (d_coarse <= r)] = 1
    lab[(~fine_mask) & (d_coarse > r) & (d_coarse <= 2 * r)] = 2
    d_fine = bfs_distance(nb, ~fine_mask)      # distance of fine cells from C
    depth = np.where(fine_mask, d_fine, 0)
    return lab, depth
