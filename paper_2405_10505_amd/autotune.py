"""Launch-schedule autotuner for a Solver or an Ensemble.

Searches the library's tuning options (fused vertex evaluation on/off, block
size 64/128/256, momentum pass through the cells' edge lists on/off where the
mesh allows it), timing hipGraph-replayed coarse steps for each candidate,
and keeps the fastest.  All candidates produce identical bits, so tuning never
changes results; the state is saved before and restored after the search.
Results are cached in a JSON file keyed by the workload's shape.
"""
from __future__ import annotations

import json
import os
import time

from . import OPT_BLOCK, OPT_EDGE_CELLS, OPT_FUSE_VERTEX, Ensemble, FBLTSError, Solver

CANDIDATES = [(fuse, bs, cells) for cells in (0, 1) for fuse in (1, 0) for bs in (256, 128, 64)]


def _sync():
    import torch
    torch.cuda.synchronize()


def _key(obj):
    if isinstance(obj, Solver):
        i = obj.info()
        return "solver:N%d:E%d:F%d:scheme%d:M%d:phys%d:split%d" % (
            i["n_cells"], i["n_edges"], i["n_fine"], obj.params.scheme, obj.params.M, obj.params.physics,
            obj.params.split)
    i = obj.info()
    return "ensemble:mc%d:members%s:M%d:phys%d:split%d" % (i["member_cells"], "-".join(map(str, obj.members)),
                                                           obj.params.M, obj.params.physics, obj.params.split)


def _save(obj):
    if isinstance(obj, Solver):
        return obj.get_state()
    return [[obj.get_member(k, m) for m in range(nm)] for k, nm in enumerate(obj.members)]


def _restore(obj, saved):
    if isinstance(obj, Solver):
        obj.set_state(*saved)
        return
    for k, mem in enumerate(saved):
        for m, (h, u) in enumerate(mem):
            obj.set_member(k, m, h, u)


def apply(obj, choice):
    obj.set_option(OPT_FUSE_VERTEX, choice["fuse_vertex"])
    obj.set_option(OPT_BLOCK, choice["block"])
    obj.set_option(OPT_EDGE_CELLS, choice.get("edge_cells", 0))
    obj.set_graph(True)


def _cells_available(obj):
    try:
        obj.set_option(OPT_EDGE_CELLS, 1)
    except FBLTSError:
        return False
    obj.set_option(OPT_EDGE_CELLS, 0)
    return True


def autotune(obj, steps=20, repeats=3, cache_path=None, verbose=False):
    """Pick the fastest (fuse_vertex, block) for obj; returns the chosen options.

    Ensemble members keep their drag coefficients (they are not part of the
    saved state, and tuning does not touch them)."""
    key = _key(obj)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            apply(obj, cache[key])
            return cache[key]
    saved = _save(obj)
    results = []
    cells_ok = _cells_available(obj)
    for fuse, bs, cells in CANDIDATES:
        if cells and not cells_ok:
            continue
        choice = dict(fuse_vertex=fuse, block=bs, edge_cells=cells)
        apply(obj, choice)
        obj.step(2)                      # capture the graph and warm up
        _sync()
        best = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            obj.step(steps)
            _sync()
            best = min(best, (time.perf_counter() - t0) / steps)
        results.append((best, choice))
        if verbose:
            print("autotune %s fuse=%d block=%d cells=%d: %.4f ms/step" % (key, fuse, bs, cells, best * 1e3),
                  flush=True)
    _restore(obj, saved)
    best_t, choice = min(results, key=lambda r: r[0])
    choice = dict(choice, ms_per_step=best_t * 1e3,
                  candidates=[dict(c, ms_per_step=t * 1e3) for t, c in results])
    apply(obj, choice)
    if cache_path:
        cache[key] = choice
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return choice
