"""Launch-schedule autotuning for a Solver or an Ensemble (fblts_autotune).

The search runs in the library: it times coarse steps of every candidate
schedule (fused vertex evaluation on/off with block size 256/128/64 on
graph-replayed steps; the persistent cooperative launch with fused vertex
evaluation on/off; the momentum pass through the cells' edge lists where the
mesh allows it) and keeps the fastest.  All candidates produce identical bits, so tuning
never changes results; the state, model time and storm clock are restored
after the search.  Results can be cached in a JSON file keyed by the
workload's shape.
"""
from __future__ import annotations

from . import OPT_BLOCK, OPT_EDGE_CELLS, OPT_FUSE_VERTEX, OPT_PERSISTENT

# the library's candidate schedules, in search order:
# (fuse_vertex, block, edge_cells, persistent)
CANDIDATES = ([(fuse, bs, 0, 0) for fuse in (1, 0) for bs in (256, 128, 64)] +
              [(fuse, 256, 0, per_cu) for fuse in (1, 0) for per_cu in (1, 4)] +
              [(fuse, bs, 1, 0) for fuse in (1, 0) for bs in (256, 128, 64)])


def apply(obj, choice):
    """Set a known schedule (a dict with fuse_vertex, block, edge_cells and
    persistent) and enable graphs (used by the per-pass schedules)."""
    obj.set_option(OPT_FUSE_VERTEX, choice["fuse_vertex"])
    obj.set_option(OPT_BLOCK, choice["block"])
    obj.set_option(OPT_EDGE_CELLS, choice.get("edge_cells", 0))
    obj.set_option(OPT_PERSISTENT, choice.get("persistent", 0))
    obj.set_graph(True)


def autotune(obj, steps=20, repeats=3, cache_path=None, verbose=False):
    """Search and set the fastest schedule for obj and turn graph replay on (the
    schedules are timed with it); returns the chosen schedule (fuse_vertex,
    block, edge_cells, ms_per_step, from_cache, candidates)."""
    choice = obj.autotune(steps=steps, repeats=repeats, cache_path=cache_path)
    obj.set_graph(True)
    if verbose:
        for c in choice["candidates"]:
            print("autotune fuse=%d block=%d cells=%d: %.4f ms/step" % (
                c["fuse_vertex"], c["block"], c["edge_cells"], c["ms_per_step"]), flush=True)
    return choice
