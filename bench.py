#!/usr/bin/env python3
"""Benchmark of the FB-LTS hot path on one MI355X.

Default workload: the 50k-cell planar variable-resolution CVT (2 -> 8 km
Gaussian patch, 50 Lloyd iterations, seamount bathymetry), nonlinear TRiSK
with quadratic drag, fine cells chosen from the local CFL number, M = 4, FP64.
One step = one FB-LTS coarse step (coarse advancement, M predicted fine
substeps, interface correction), replayed from a hipGraph with the state
resident in HBM.

value = cell-substeps/s = (N_coarse + M N_fine) * steps / wall time.
Also reported: the momentum (edge) pass against the HBM roofline, the
time-to-solution of global FB-RK(3,2) and RK4 at their own largest stable
steps (the paper's speedup definition), and the oracle timed on the host
(one thread, then one process per host core up to 16).

Other workloads: sphere400k (the ~400k-cell spherical coastline-refined CVT,
6 -> 60 km, bathymetry field, drag and a moving analytic cyclone, M = 8; by
default two simulated days), hex32, ensemble, adjoint, aquaplanet.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload cvt50k|sphere400k|hex32|ensemble|adjoint|aquaplanet]
                       [--split 0|1|2] [--schedule F,B[,C]] [--profile-steps N] [--no-cpu] [--no-compare]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-substeps/s & %HBM roofline: FB-LTS vs global FB-RK/RK4; ensemble member-steps/s"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps per sample (default 200; sphere400k: two days)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5, help="timing samples; the median is reported")
    ap.add_argument("--workload", default="cvt50k", choices=["cvt50k", "sphere400k", "hex32", "ensemble", "adjoint", "aquaplanet"])
    ap.add_argument("--split", type=int, default=0, choices=[0, 1, 2],
                    help="operator splitting: 0 unsplit, 1 slow terms per coarse step, 2 per fine substep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the global-scheme comparison and the LTS sweep")
    ap.add_argument("--no-extra", action="store_true",
                    help="cvt50k: skip the sphere400k and ensemble blocks of the JSON line")
    ap.add_argument("--schedule", default=None,
                    help="fixed launch schedule 'fuse_vertex,block[,edge_cells[,persistent]]' instead of autotuning "
                         "(e.g. 1,64,0)")
    ap.add_argument("--pipeline", type=int, default=None, choices=[0, 1],
                    help="FB-LTS step arrangement (FBLTS_OPT_PIPELINE) of the main solver; default: the library's")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many graph-replayed steps (for rocprofv3), no JSON")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "fblts_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2405_10505_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, kernel="edge"):
    """HBM bytes per launch of the momentum (kernel="edge") or thickness
    ("cell") pass from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "%s_pass_%s_counters.json" % (kernel, workload))
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def make_solver(F, w, scheme, dt, M, labels=None, graph=True, split=0, mask=None):
    import numpy as np
    if scheme == F.SCHEME_RK4 or w.linear:
        split = 0
    elif scheme == F.SCHEME_FBRK32:
        split = min(split, 1)
    s = F.Solver(F.Mesh(w.mesh) if not hasattr(w, "_fm") else w._fm, dt, M=M, scheme=scheme, linear=w.linear,
                 split=split)
    if labels is None:
        s.set_regions(np.where(w.fine_mask if mask is None else mask, 0, 1), binary=True)
    else:
        s.set_regions(labels, binary=False)
    if w.cd is not None and not w.linear:
        s.set_drag(w.cd)
    s.set_state(w.h0, w.u0)
    storm = w.meta.get("storm")
    if storm is not None and not w.linear:
        s.set_cyclone(w.mesh.x_edge, w.mesh.normal_edge, **storm.cyclone_kwargs())
    sched = getattr(w, "_schedule", None)
    if sched is not None:
        from paper_2405_10505_amd import autotune
        autotune.apply(s, sched)
    s.set_graph(graph)
    return s


def stable(F, w, scheme, dt, steps, umax=50.0, split=0, M=None, mask=None):
    """Run `steps` steps; stable if the state stays finite, h > 0 and |u| < umax.

    Global schemes run with every cell coarse; FB-LTS with the given fine set
    (default: the workload's) and M (dt is then the coarse step)."""
    import numpy as np
    if scheme == F.SCHEME_FBLTS:
        s = make_solver(F, w, scheme, dt, M or w.M, graph=True, split=split, mask=mask)
    else:
        s = make_solver(F, w, scheme, dt, 1, labels=np.full(w.mesh.n_cells, 3, np.int8), split=split)
    s.step(steps)
    d = s.diagnostics(allow_nonfinite=True)
    if d["n_nonfinite"] > 0 or not (d["min_h"] > 0):
        return False
    h, u = s.get_state()
    return bool(np.max(np.abs(u)) < umax)


def largest_stable_dt(F, w, scheme, dt0, steps=200, iters=8, split=0, M=None, mask=None, grow=1.3):
    """The paper's procedure: grow dt until the run becomes unstable, then bisect."""
    run = lambda dt: stable(F, w, scheme, dt, steps, split=split, M=M, mask=mask)   # noqa: E731
    lo, hi = None, None
    dt = dt0
    for _ in range(20):
        if run(dt):
            lo = dt
            dt *= grow
        else:
            hi = dt
            break
    if lo is None:   # shrink until stable
        hi = dt0
        dt = dt0
        for _ in range(20):
            dt /= grow
            if run(dt):
                lo = dt
                break
            hi = dt
    if hi is None or lo is None:
        return lo
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if run(mid):
            lo = mid
        else:
            hi = mid
    return lo


def time_samples(torch, s, steps, warmup, reps=5):
    """Median wall time (s) of `reps` runs of `steps` steps after `warmup`
    untimed steps, each run bracketed by device synchronisations; and the
    samples."""
    s.step(warmup)
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return float(sorted(out)[len(out) // 2]), out


def time_steps(torch, s, steps, warmup):
    return time_samples(torch, s, steps, warmup, reps=1)[0]


def copy_peak(torch, mib=1024, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy of `mib` MiB
    (read + write bytes per copy), best of `reps`, timed with HIP events."""
    x = torch.empty(mib << 17, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del x, y
    return 2.0 * (mib << 20) / best / 1e9


def pass_roofline(s, info, tsteps, workload, split=0):
    """Kernel timing of the momentum and thickness passes: the same solver
    continues for `tsteps` coarse steps launched directly (not from the graph:
    kernel durations are the same, launch overheads are outside them) with
    every stencil pass recording HIP events from its own dispatch, on the
    solver's stream.  Achieved bandwidth = compulsory bytes per launch (mesh
    and state arrays the pass's mathematics references, once per launch; no
    intermediates) / average launch duration; the per-pass model (which also
    counts the intermediates the passes exchange through memory) beside it."""
    s.set_timing(True)
    s.step(tsteps)
    edge_ms, edge_launches = s.kernel_time(0)
    cell_ms, cell_launches = s.kernel_time(1)
    vert_ms, _ = s.kernel_time(2)
    prep_ms, _ = s.kernel_time(3)
    s.set_timing(False)
    out = {}
    for key, ms, nl, comp, model, items in (
            ("edge", edge_ms, edge_launches, info["compulsory_bytes_edge_pass"], info["model_bytes_edge_pass"],
             info["edge_pass_items_per_step"]),
            ("cell", cell_ms, cell_launches, info["compulsory_bytes_cell_pass"], info["model_bytes_cell_pass"], None)):
        per_step = nl / tsteps
        bpl = comp / per_step
        ach = bpl / (ms * 1e-3) / 1e9
        d = dict(avg_launch_ms=ms, launches_per_step=per_step, compulsory_bytes_per_launch=bpl,
                 achieved_GBs=ach, frac=ach / HBM_PEAK_GBS,
                 per_pass_model=dict(bytes_per_launch=model / per_step,
                                     frac=model / per_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS))
        if items is not None:
            d["edges_per_launch"] = items / per_step
            d["compulsory_bytes_per_edge"] = comp / items
        traffic = traffic_from_profiles(workload, key) if split == 0 else None
        d["counter_bytes_per_launch"] = traffic
        d["counter_over_compulsory"] = traffic / bpl if traffic else None
        out[key] = d
    out["avg_ms"] = dict(edge=edge_ms, cell=cell_ms, vertex=vert_ms, prep=prep_ms)
    out["timing"] = "HIP events recorded by each dispatch, %d momentum-pass launches over %d coarse steps" % (
        edge_launches, tsteps)
    return out


# ------------------------------------------------ workloads built off the GPU
# The sphere and the ensemble's extra meshes take a while to generate; they are
# built in separate host processes (no GPU use) while the main workload runs.

def _build_workload(kind, n=None, seed=None):
    from paper_2405_10505_amd.inputs import workloads
    if kind == "sphere400k":
        return workloads.config3()
    return workloads.config2(n=n, seed_mesh=seed)


ENSEMBLE_SPECS = [(50000, 2, 64), (20000, 20, 16), (50000, 21, 16), (120000, 22, 16)]


def start_background_builds(kinds):
    import multiprocessing as mp
    pool = mp.get_context("spawn").Pool(min(4, len(kinds)))
    futs = {}
    for k in kinds:
        if k == "sphere400k":
            futs[k] = pool.apply_async(_build_workload, ("sphere400k",))
        else:
            n, seed = k
            futs[k] = pool.apply_async(_build_workload, ("cvt", n, seed))
    return pool, futs


# ------------------------------------------------------- the LTS time steps

LTS_SWEEP = [(2, 1.0), (3, 1.0), (4, 1.0), (2, 0.8), (3, 0.8), (4, 0.8), (2, 0.65), (3, 0.65), (4, 0.65), (6, 0.65)]


def lts_sweep(F, torch, w, rate_fb, rate_rk4, dt_fb, steps, reps, split=0):
    """FB-LTS time steps chosen the paper's way (Sec. 4.1: the largest stable
    step, grown until the run is unstable, then bisected).  The fine set comes
    from the local CFL number: fine = Courant number at the coarse step above
    margin x the most restrictive cell's at the fine step.  For each (M,
    margin) the largest stable coarse step is searched (from M times the global
    FB-RK(3,2) limit downwards) and timed.  The paper's rule then takes the
    largest fine step first and, among the settings within 2% of it, the
    largest M; the fastest setting is reported beside it."""
    from paper_2405_10505_amd.inputs import workloads
    rows = []
    for M, margin in LTS_SWEEP:
        mask = workloads.cfl_fine_mask(w.mesh, M, margin=margin)[0]
        t0 = time.perf_counter()
        dtc = largest_stable_dt(F, w, F.SCHEME_FBLTS, M * dt_fb, split=split, M=M, mask=mask, iters=5, grow=1.15)
        if dtc is None:
            continue
        s = make_solver(F, w, F.SCHEME_FBLTS, dtc, M, split=split, mask=mask)
        el, samples = time_samples(torch, s, steps, 5, reps)
        info = s.info()
        rate = dtc * steps / el
        rows.append(dict(M=M, margin=margin, n_fine=int(mask.sum()), dt_coarse=dtc, dt_fine=dtc / M,
                         ms_per_step=el / steps * 1e3, launches_per_step=info["launches_per_step"],
                         cell_substeps_per_step=info["cell_substeps_per_step"],
                         sim_seconds_per_wall_second=rate, speedup_vs_fbrk32=rate / rate_fb,
                         speedup_vs_rk4=rate / rate_rk4))
        log("LTS M=%d margin=%.2f: fine %d, dt %.2f/%.2f s, %.4f ms/step, %.2fx FB-RK(3,2), %.2fx RK4 (%.1fs)" % (
            M, margin, rows[-1]["n_fine"], dtc, dtc / M, rows[-1]["ms_per_step"], rows[-1]["speedup_vs_fbrk32"],
            rows[-1]["speedup_vs_rk4"], time.perf_counter() - t0))
    paper, fastest = paper_choice(rows)
    return rows, paper, fastest


def paper_choice(rows, tol=0.02):
    """The paper's order (Sec. 4.1) applied to searched (M, margin) rows: the
    largest stable fine step first (rows within tol of it count as equal), then
    the largest M among them (the larger margin on a tie); and the row with the
    fastest time to solution."""
    best_f = max(r["dt_fine"] for r in rows)
    near = [r for r in rows if r["dt_fine"] >= (1.0 - tol) * best_f]
    paper = max(near, key=lambda r: (r["M"], r["margin"]))
    fastest = max(rows, key=lambda r: r["sim_seconds_per_wall_second"])
    return paper, fastest


# ------------------------------------------------------------ extra blocks

def sphere_block(F, torch, w, steps, reps, split=0):
    """The HBM-resident workload: ms per coarse step (median of reps) and the
    momentum- and thickness-pass roofline of the compulsory model, with the
    counter traffic of the committed profiles when they match the kernels."""
    w._fm = F.Mesh(w.mesh)
    s = make_solver(F, w, F.SCHEME_FBLTS, w.dt, w.M, split=split)
    from paper_2405_10505_amd import autotune
    tune = autotune.autotune(s, steps=10, repeats=2)
    info = s.info()
    el, samples = time_samples(torch, s, steps, 5, reps)
    ms = el / steps * 1e3
    roof = pass_roofline(s, info, 5, "sphere400k", split)
    log("sphere400k: %.4f ms/step, %.3e cell-substeps/s; momentum pass %.1f%% of peak, thickness pass %.1f%%" % (
        ms, info["cell_substeps_per_step"] / ms * 1e3, 100 * roof["edge"]["frac"], 100 * roof["cell"]["frac"]))
    return dict(workload=w.name, n_cells=w.mesh.n_cells, n_fine=info["n_fine"], M=w.M, dt_coarse=w.dt,
                ms_per_step=ms, samples_ms=[t / steps * 1e3 for t in samples],
                cell_substeps_per_s=info["cell_substeps_per_step"] / ms * 1e3,
                launch_schedule=dict(fuse_vertex=tune["fuse_vertex"], block=tune["block"],
                                     edge_cells=tune.get("edge_cells", 0),
                                     persistent=tune.get("persistent", 0)),
                autotune_candidates=[dict(fuse_vertex=c["fuse_vertex"], block=c["block"], edge_cells=c["edge_cells"], persistent=c["persistent"], ms_per_step=c["ms_per_step"]) for c in tune.get("candidates", [])],
                roofline=roof)


def ensemble_block(F, torch, ws, steps, reps, schedule=None, check_all_meshes=True):
    """Configuration 4: 64 members on the 50k-cell mesh plus 16 members each on
    20k / 50k / 120k-cell meshes, one launch per pass covering all meshes,
    hipGraph replay, autotuned schedule; compared with looping the
    single-member solver over every member on the same GPU.  One member of
    every mesh is checked bitwise against a single-member solver."""
    import numpy as np
    from paper_2405_10505_amd import autotune
    from paper_2405_10505_amd.inputs import workloads
    dt = min(w.dt for w, _ in ws)   # one coarse step for all meshes: the most restrictive
    fms = [F.Mesh(w.mesh) for w, _ in ws]
    labels = [np.where(w.fine_mask, 0, 1) for w, _ in ws]
    ens = F.Ensemble(fms, labels, [nm for _, nm in ws], dt, M=4, linear=False)
    inputs = []
    for k, (w, nm) in enumerate(ws):
        fields, cds = workloads.ensemble_members(w.mesh, nm, seed_ssh0=1000 + 100 * k)
        inputs.append([(w.h0 + fields[m], w.u0, np.full(w.mesh.n_cells, cds[m])) for m in range(nm)])
        for m in range(nm):
            ens.set_member(k, m, *inputs[k][m])
    if schedule:
        tune = dict(schedule)
        autotune.apply(ens, tune)
    else:
        tune = autotune.autotune(ens, steps=10, repeats=2)
    info = ens.info()
    el, samples = time_samples(torch, ens, steps, 5, reps)
    members = sum(nm for _, nm in ws)
    ms = el / steps * 1e3
    log("ensemble: %.3f ms per coarse step for %d members, %.3e member-cells" % (ms, members, info["member_cells"]))
    # the same work as a loop of single-member solvers (time one member per mesh)
    loop_ms = 0.0
    per_mesh = []
    ls = max(20, steps // 2)
    for k, (w, nm) in enumerate(ws):
        s = F.Solver(fms[k], dt, M=4, linear=False)
        s.set_regions(labels[k], binary=True)
        s.set_drag(inputs[k][0][2])
        s.set_state(inputs[k][0][0], inputs[k][0][1])
        autotune.autotune(s, steps=10, repeats=2)
        e, _ = time_samples(torch, s, ls, 5, reps)
        t1 = e / ls * 1e3
        per_mesh.append(dict(n_cells=w.mesh.n_cells, members=nm, single_member_ms=t1))
        loop_ms += nm * t1
    # one member of every mesh (the last one) equals the single-member solver
    # after 10 steps of the ensemble (same kernels, same order)
    ens2 = F.Ensemble(fms, labels, [nm for _, nm in ws], dt, M=4, linear=False)
    for k, (w, nm) in enumerate(ws):
        for m in range(nm):
            ens2.set_member(k, m, *inputs[k][m])
    autotune.apply(ens2, tune)
    ens2.step(10)
    same = []
    for k, (w, nm) in enumerate(ws[:len(ws) if check_all_meshes else 1]):
        m = nm - 1
        chk = F.Solver(fms[k], dt, M=4, linear=False)
        chk.set_regions(labels[k], binary=True)
        chk.set_drag(inputs[k][m][2])
        chk.set_state(inputs[k][m][0], inputs[k][m][1])
        chk.step(10)
        he, ue = ens2.get_member(k, m)
        hc, uc = chk.get_state()
        same.append(bool(np.array_equal(he, hc) and np.array_equal(ue, uc)))
    log("ensemble: %.2fx a loop of single-member solvers; members equal single solvers: %s" % (loop_ms / ms, same))
    return dict(workload="ensemble_4meshes_112members_cvt", members=members, member_cells=info["member_cells"],
                dt=dt, M=4, ms_per_step=ms, samples_ms=[t / steps * 1e3 for t in samples],
                member_steps_per_s=members / ms * 1e3,
                cell_substeps_per_s=info["cell_substeps_per_step"] / ms * 1e3,
                model_GBs=info["model_bytes_per_step"] / ms * 1e3 / 1e9,
                launch_schedule=dict(fuse_vertex=tune["fuse_vertex"], block=tune["block"],
                                     edge_cells=tune.get("edge_cells", 0),
                                     persistent=tune.get("persistent", 0)),
                loop_of_single_member_solvers_ms_per_step=loop_ms, speedup_vs_member_loop=loop_ms / ms,
                autotune_candidates=[dict(fuse_vertex=c["fuse_vertex"], block=c["block"], edge_cells=c["edge_cells"], persistent=c["persistent"], ms_per_step=c["ms_per_step"]) for c in tune.get("candidates", [])],
                per_mesh=per_mesh, checked_member_per_mesh_equals_single_solver_bitwise=same)


def _oracle_run(w, steps, split, limit_s=20.0):
    """Advance the oracle (plain numpy FP64, definition mode) through up to
    `steps` FB-LTS coarse steps of workload w, stopping after limit_s seconds;
    returns (steps done, seconds)."""
    from oracle import regions, schemes, trisk
    om = trisk.OMesh(w.mesh)
    lab, _ = regions.layer(om, w.fine_mask, 2)
    storm = w.meta.get("storm")
    u, h = w.u0.copy(), w.h0.copy()
    t0 = time.perf_counter()
    n = 0
    while n < steps:
        wind = storm.edge_forcing(w.mesh, n * w.dt) if storm is not None else None
        ph = trisk.Physics(linear=w.linear, cd=w.cd if not w.linear else None, wind=wind)
        u, h = schemes.fblts_step(om, u, h, w.dt, w.M, ph, lab, split=split)
        n += 1
        if time.perf_counter() - t0 > limit_s:
            break
    return n, time.perf_counter() - t0


def _oracle_worker(task):
    """One host process of the all-cores oracle run (no GPU use)."""
    w, steps, split = task
    return _oracle_run(w, steps, split)


def cpu_baseline(w, steps, split=0):
    """The oracle on a bounded sample of the workload: one thread, then one
    copy per host core (separate processes, up to 16) running the same sample
    side by side for the whole host's throughput."""
    n, el = _oracle_run(w, steps, split)
    nf = int(w.fine_mask.sum())
    per_step = (w.mesh.n_cells - nf) + w.M * nf
    out = dict(value=per_step * n / el, unit="cell-substeps/s", cores=1, kind="oracle",
               sample="%d FB-LTS coarse steps of the %s workload (numpy, one thread), %.1f s" % (n, w.name, el))
    ncpu = min(16, len(os.sched_getaffinity(0)))
    if ncpu > 1:
        import dataclasses
        import multiprocessing as mp
        wp = dataclasses.replace(w)   # the workload's fields only (no library handles)
        for k in [k for k in vars(wp) if k.startswith("_")]:
            delattr(wp, k)
        with mp.get_context("spawn").Pool(ncpu) as pool:
            res = pool.map(_oracle_worker, [(wp, n, split)] * ncpu)
        out["all_cores"] = dict(value=sum(per_step * k / t for k, t in res), unit="cell-substeps/s", cores=ncpu,
                                sample="%d processes, each the same %d steps (numpy, one thread each), %.1f s" % (
                                    ncpu, n, max(t for _, t in res)))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2405_10505_amd as F
    from paper_2405_10505_amd.inputs import workloads

    if args.steps is None and args.workload != "sphere400k":
        args.steps = 200
    extra = args.workload == "cvt50k" and not args.no_extra and not args.profile_steps and args.split == 0
    pool = futs = None
    if extra:
        # the other workloads' meshes, built on host cores while this one runs
        pool, futs = start_background_builds(["sphere400k"] + [(n, sd) for n, sd, _ in ENSEMBLE_SPECS[1:]])
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "aquaplanet":
        return bench_aquaplanet(args)
    t = time.perf_counter()
    if args.workload == "hex32":
        w = workloads.config1()
    elif args.workload == "sphere400k":
        w = workloads.config3(progress=log)
    else:
        w = workloads.config2()
    if args.steps is None:
        args.steps = w.steps
    log("workload %s: N=%d E=%d fine=%d dt=%.3f M=%d (built in %.1fs)" % (
        w.name, w.mesh.n_cells, w.mesh.n_edges, int(w.fine_mask.sum()), w.dt, w.M, time.perf_counter() - t))
    w._fm = F.Mesh(w.mesh)
    s = make_solver(F, w, F.SCHEME_FBLTS, w.dt, w.M, split=args.split)
    if args.pipeline is not None:
        s.set_option(F.OPT_PIPELINE, args.pipeline)
    from paper_2405_10505_amd import autotune
    # later runs on the same workload (a profiled run after the timed one) replay
    # the schedule it chose: the cache is keyed by the workload's shape
    cache = os.environ.get("FBLTS_AUTOTUNE_CACHE", os.path.join(ROOT, ".fblts_cache", "autotune_schedules.json"))
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    if args.schedule:
        vals = [int(v) for v in args.schedule.split(",")]
        tune = dict(fuse_vertex=vals[0], block=vals[1], edge_cells=vals[2] if len(vals) > 2 else 0,
                    persistent=vals[3] if len(vals) > 3 else 0,
                    ms_per_step=float("nan"))
        autotune.apply(s, tune)
    else:
        tune = autotune.autotune(s, steps=20, repeats=3, cache_path=cache)
    log("launch schedule: fuse_vertex=%d block=%d edge_cells=%d persistent=%d (%.4f ms/step when tuned)" % (
        tune["fuse_vertex"], tune["block"], tune.get("edge_cells", 0), tune.get("persistent", 0),
        tune["ms_per_step"]))
    for c in tune.get("candidates", []):
        log("  candidate fuse_vertex=%d block=%d edge_cells=%d persistent=%d: %.4f ms/step" % (
            c["fuse_vertex"], c["block"], c["edge_cells"], c["persistent"], c["ms_per_step"]))
    info = s.info()
    if args.profile_steps:
        s.step(args.profile_steps)
        torch.cuda.synchronize()
        # calibration for the HBM byte counters: a plain 512 MiB device copy
        x = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("profile run done: %d steps, then 3 copies of 512 MiB" % args.profile_steps)
        return
    el, samples = time_samples(torch, s, args.steps, args.warmup, args.reps)
    ms = el / args.steps * 1e3
    value = info["cell_substeps_per_step"] * args.steps / el
    d = s.diagnostics()
    log("FB-LTS: %.4f ms/step (median of %d), %.3e cell-substeps/s, launches/step %d" % (
        ms, args.reps, value, info["launches_per_step"]))

    # roofline of the dominant kernel (momentum pass), compulsory byte model
    tsteps = max(5, min(50, args.steps // 4))
    pr = pass_roofline(s, info, tsteps, args.workload, args.split)
    e = pr["edge"]
    roof = dict(bound="hbm", achieved=e["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=e["frac"],
                traffic=e["counter_bytes_per_launch"], kernel="fblts::k_edge (momentum pass)",
                avg_launch_ms=e["avg_launch_ms"], timing=pr["timing"],
                byte_model="compulsory: mesh and state arrays the momentum pass's mathematics references, each "
                           "element once per launch; no thickness flux, q, K, B, h* or edge-prep record bytes",
                algorithmic_bytes_per_launch=e["compulsory_bytes_per_launch"],
                edges_per_launch=e["edges_per_launch"], algorithmic_bytes_per_edge=e["compulsory_bytes_per_edge"],
                traffic_over_algorithmic=e["counter_over_compulsory"],
                per_pass_model=e["per_pass_model"], thickness_pass=pr["cell"], avg_ms=pr["avg_ms"])
    roof["measured_copy_GBs"] = copy_peak(torch)
    roof["frac_of_measured_copy"] = roof["achieved"] / roof["measured_copy_GBs"]
    log("edge pass: %.4f ms avg, %.1f GB/s compulsory (%.1f%% of HBM peak, %.1f%% of a %.0f GB/s device copy); "
        "per-pass model %.1f%%" % (roof["avg_launch_ms"], roof["achieved"], 100 * roof["frac"],
                                   100 * roof["frac_of_measured_copy"], roof["measured_copy_GBs"],
                                   100 * e["per_pass_model"]["frac"]))
    whole = info["compulsory_bytes_per_step"] / (ms * 1e-3) / 1e9

    comp = None
    if not args.no_compare:
        dt_f = w.dt / w.M
        t0 = time.perf_counter()
        dt_fb = largest_stable_dt(F, w, F.SCHEME_FBRK32, dt_f, split=args.split)
        dt_rk4 = largest_stable_dt(F, w, F.SCHEME_RK4, dt_f)
        log("stable dt: FB-RK(3,2) %.3f s, RK4 %.3f s (search %.1fs)" % (dt_fb, dt_rk4, time.perf_counter() - t0))
        ks = max(20, args.steps // 2)
        res = {}
        for name, scheme, dt in (("fbrk32_own_limit", F.SCHEME_FBRK32, dt_fb),
                                 ("fbrk32_fine_dt", F.SCHEME_FBRK32, dt_f),
                                 ("rk4_own_limit", F.SCHEME_RK4, dt_rk4)):
            g = make_solver(F, w, scheme, dt, 1, labels=np.full(w.mesh.n_cells, 3, np.int8), split=args.split)
            autotune.autotune(g, steps=20, repeats=3)   # each scheme at its own best launch schedule
            e_, smp = time_samples(torch, g, ks, 5, args.reps)
            res[name] = dict(dt=dt, ms_per_step=e_ / ks * 1e3, sim_seconds_per_wall_second=dt * ks / e_,
                             samples_ms=[x / ks * 1e3 for x in smp])
        rate_fb = res["fbrk32_own_limit"]["sim_seconds_per_wall_second"]
        rate_rk4 = res["rk4_own_limit"]["sim_seconds_per_wall_second"]
        # every FB-LTS leg runs the launch schedule tuned for this workload
        w._schedule = dict(fuse_vertex=tune["fuse_vertex"], block=tune["block"],
                           edge_cells=tune.get("edge_cells", 0), persistent=tune.get("persistent", 0))
        # the recipe's fine set and M with its own largest stable coarse step
        dt_lts = largest_stable_dt(F, w, F.SCHEME_FBLTS, w.dt, split=args.split)
        g = make_solver(F, w, F.SCHEME_FBLTS, dt_lts, w.M, split=args.split)
        e_, smp = time_samples(torch, g, ks, 5, args.reps)
        recipe = dict(M=w.M, margin=1.0, n_fine=int(w.fine_mask.sum()), dt_coarse=dt_lts, dt_fine=dt_lts / w.M,
                      ms_per_step=e_ / ks * 1e3, sim_seconds_per_wall_second=dt_lts * ks / e_,
                      speedup_vs_fbrk32=dt_lts * ks / e_ / rate_fb, speedup_vs_rk4=dt_lts * ks / e_ / rate_rk4)
        log("FB-LTS recipe (M=%d): dt %.2f/%.2f s, %.2fx FB-RK(3,2), %.2fx RK4" % (
            w.M, dt_lts, dt_lts / w.M, recipe["speedup_vs_fbrk32"], recipe["speedup_vs_rk4"]))
        sweep = paper = fastest = None
        if args.split == 0 and args.workload == "cvt50k":
            sweep, paper, fastest = lts_sweep(F, torch, w, rate_fb, rate_rk4, dt_fb, ks, args.reps, args.split)
        w._schedule = None
        chosen = paper or recipe
        comp = dict(fblts=chosen, fblts_recipe=recipe, lts_sweep=sweep, fastest_of_sweep=fastest,
                    **res,
                    speedup_vs_rk4=chosen["speedup_vs_rk4"], speedup_vs_fbrk32=chosen["speedup_vs_fbrk32"],
                    choice=("the paper's order (Sec. 4.1): the largest stable fine step first, then the largest M "
                            "(fine steps within 2% count as equal); fine sets from the local CFL number with a "
                            "margin" if paper else "the recipe's fine set and M at the largest stable coarse step"),
                    definition="time-to-solution ratio for equal simulated time (paper eq. speedup)",
                    timing="median of %d samples of %d steps per leg" % (args.reps, ks),
                    splitting=("FB-LTS and FB-RK(3,2) split (slow terms %s), RK4 unsplit" % (
                        "per coarse step" if args.split == 1 else "per fine substep on the fine region")
                        if args.split else "none"))
        log("speedup (%s) vs RK4 %.2fx, vs global FB-RK(3,2) %.2fx" % (
            "paper's choice M=%d margin %.2f" % (chosen["M"], chosen["margin"]), comp["speedup_vs_rk4"],
            comp["speedup_vs_fbrk32"]))

    sphere = ensemble = None
    if extra:
        try:
            t0 = time.perf_counter()
            w3 = futs["sphere400k"].get()
            log("sphere400k built in the background (waited %.1fs)" % (time.perf_counter() - t0))
            sphere = sphere_block(F, torch, w3, 20, args.reps)
            del w3
            t0 = time.perf_counter()
            ws = [(w, ENSEMBLE_SPECS[0][2])] + [(futs[(n, sd)].get(), nm) for n, sd, nm in ENSEMBLE_SPECS[1:]]
            log("ensemble meshes built in the background (waited %.1fs)" % (time.perf_counter() - t0))
            ensemble = ensemble_block(F, torch, ws, 20, args.reps)
            del ws
        finally:
            pool.terminate()
            pool.join()
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, 50, split=args.split)
        log("oracle: %.3e cell-substeps/s (%s)" % (cpu["value"], cpu["sample"]))
        if "all_cores" in cpu:
            log("oracle on %d cores: %.3e cell-substeps/s (%s)" % (
                cpu["all_cores"]["cores"], cpu["all_cores"]["value"], cpu["all_cores"]["sample"]))

    out = dict(metric=METRIC, value=value, unit="cell-substeps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload=w.name, n_cells=w.mesh.n_cells, n_edges=w.mesh.n_edges,
                           n_vertices=w.mesh.n_vertices, n_fine=info["n_fine"], n_if1=info["n_if1"],
                           n_if2=info["n_if2"], n_int=info["n_int"], M=w.M, dt_coarse=w.dt,
                           physics="linear" if w.linear else "nonlinear+drag", scheme="FB-LTS",
                           split=["none", "slow terms per coarse step", "slow terms per fine substep"][args.split],
                           cell_substeps_per_step=info["cell_substeps_per_step"],
                           launches_per_step=info["launches_per_step"], hipgraph=True,
                           launch_schedule=dict(fuse_vertex=tune["fuse_vertex"], block=tune["block"],
                                                edge_cells=tune.get("edge_cells", 0),
                                     persistent=tune.get("persistent", 0))),
               timing=dict(samples_ms=[x / args.steps * 1e3 for x in samples], reps=args.reps,
                           statistic="median"),
               autotune_candidates=[dict(fuse_vertex=c["fuse_vertex"], block=c["block"], edge_cells=c["edge_cells"],
                                         persistent=c["persistent"], ms_per_step=c["ms_per_step"])
                                    for c in tune.get("candidates", [])],
               roofline=roof, cpu_baseline=cpu, comparison=comp, sphere400k=sphere, ensemble=ensemble,
               whole_step_compulsory_GBs=whole, compulsory_bytes_per_step=info["compulsory_bytes_per_step"],
               model_bytes_per_step=info["model_bytes_per_step"],
               diagnostics=dict(mass=d["mass"], min_h=d["min_h"]))
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """Configuration 4 alone (the same block the default run appends)."""
    import torch
    import paper_2405_10505_amd as F
    from paper_2405_10505_amd.inputs import workloads
    ws = []
    for n, seed, nm in ENSEMBLE_SPECS:
        t = time.perf_counter()
        w = workloads.config2(n=n, seed_mesh=seed)
        ws.append((w, nm))
        log("mesh %d (seed %d) built in %.1fs, fine %d, dt %.2f" % (n, seed, time.perf_counter() - t,
                                                                    int(w.fine_mask.sum()), w.dt))
    sched = None
    if args.schedule:
        vals = [int(v) for v in args.schedule.split(",")]
        sched = dict(fuse_vertex=vals[0], block=vals[1], edge_cells=vals[2] if len(vals) > 2 else 0,
                    persistent=vals[3] if len(vals) > 3 else 0)
    if args.profile_steps:
        # stepping dispatches only: the members are set before the profiled steps
        from paper_2405_10505_amd import autotune
        import numpy as np
        dt = min(w.dt for w, _ in ws)
        ens = F.Ensemble([F.Mesh(w.mesh) for w, _ in ws], [np.where(w.fine_mask, 0, 1) for w, _ in ws],
                         [nm for _, nm in ws], dt, M=4, linear=False)
        for k, (w, nm) in enumerate(ws):
            fields, cds = workloads.ensemble_members(w.mesh, nm, seed_ssh0=1000 + 100 * k)
            for m in range(nm):
                ens.set_member(k, m, w.h0 + fields[m], w.u0, np.full(w.mesh.n_cells, cds[m]))
        if sched:
            autotune.apply(ens, sched)
        else:
            autotune.autotune(ens, steps=10, repeats=2)
        ens.step(2)
        torch.cuda.synchronize()
        log("PROFILE_MARK set-up done; stepping %d ensemble steps" % args.profile_steps)
        ens.step(args.profile_steps)
        torch.cuda.synchronize()
        log("profile run done: %d ensemble steps" % args.profile_steps)
        return
    blk = ensemble_block(F, torch, ws, args.steps, args.reps, schedule=sched)
    out = dict(metric=METRIC, value=blk["member_steps_per_s"], unit="member-steps/s", n_gpus=1, steps=args.steps,
               warmup=5, ms_per_step=blk["ms_per_step"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=blk["workload"], members=blk["members"], member_cells=blk["member_cells"],
                           dt=blk["dt"], M=4, hipgraph=True, launch_schedule=blk["launch_schedule"]),
               ensemble=blk)
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Configuration 5: reverse mode through 200 FB-LTS coarse steps on the 50k-cell
    mesh, loss = sum of squared SSH at 50 gauge cells, gradients with respect to
    h0 and the per-cell drag coefficient, checkpoint every 20 steps; checked by
    central finite differences on 20 random directions."""
    import numpy as np
    import torch
    import paper_2405_10505_amd as F
    from paper_2405_10505_amd import autotune
    from paper_2405_10505_amd.inputs import workloads
    w = workloads.config2()
    fm = F.Mesh(w.mesh)
    n_steps, K = 200, 20
    rg = workloads.rng_for(9)
    gauges = np.sort(rg.choice(np.nonzero(w.fine_mask)[0], size=50, replace=False))
    H = w.mesh.bottom_depth
    s = F.Solver(fm, w.dt, M=w.M, linear=False)
    s.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
    s.set_drag(w.cd)
    s.set_state(w.h0, w.u0)
    if args.schedule:
        vals = [int(v) for v in args.schedule.split(",")]
        tune = dict(fuse_vertex=vals[0], block=vals[1], edge_cells=vals[2] if len(vals) > 2 else 0,
                    persistent=vals[3] if len(vals) > 3 else 0)
        autotune.apply(s, tune)
    else:
        tune = autotune.autotune(s, steps=10, repeats=2)
    if args.profile_steps:
        # one checkpointed forward and backward over profile_steps coarse steps
        # (for rocprofv3), no finite-difference check and no JSON
        s.set_state(w.h0, w.u0)
        s.adjoint_forward(args.profile_steps, K)
        hN, _ = s.get_state()
        ghN = np.zeros(w.mesh.n_cells)
        ghN[gauges] = 2 * (hN[gauges] - H[gauges])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.adjoint_backward(ghN, np.zeros(w.mesh.n_edges))
        torch.cuda.synchronize()
        log("profile run done: checkpointed forward and backward over %d steps (backward %.3f s)" % (
            args.profile_steps, time.perf_counter() - t1))
        return

    def loss_of(h0, cd):
        q = F.Solver(fm, w.dt, M=w.M, linear=False)
        q.set_regions(np.where(w.fine_mask, 0, 1), binary=True)
        q.set_drag(cd)
        q.set_state(h0, w.u0)
        autotune.apply(q, tune)
        q.step(n_steps)
        h, _ = q.get_state()
        return float(np.sum((h[gauges] - H[gauges]) ** 2))

    # forward alone (graph replay)
    s.set_state(w.h0, w.u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n_steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # forward with checkpoints + backward
    s.set_state(w.h0, w.u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adjoint_forward(n_steps, K)
    hN, uN = s.get_state()
    ghN = np.zeros(w.mesh.n_cells)
    ghN[gauges] = 2 * (hN[gauges] - H[gauges])
    t1 = time.perf_counter()
    gh0, gu0, gcd = s.adjoint_backward(ghN, np.zeros(w.mesh.n_edges))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    L0 = float(np.sum((hN[gauges] - H[gauges]) ** 2))
    log("adjoint: forward %.3f s, checkpointed forward %.3f s, backward %.3f s, L = %.6e" % (
        t_fwd, t1 - t0, t2 - t1, L0))
    # central finite differences on 20 random unit directions in (h0, C_D)
    rd = workloads.rng_for(10)
    errs, raw = [], []
    t3 = time.perf_counter()
    for k in range(20):
        vh = rd.normal(size=w.mesh.n_cells)
        vc = rd.normal(size=w.mesh.n_cells)
        nrm = np.sqrt(vh @ vh + (vc @ vc))
        vh, vc = vh / nrm, vc / nrm
        # the C_D part of the direction is scaled to C_D's size so both parts are resolved
        ref = gh0 @ vh + 1e-3 * (gcd @ vc)

        def fd(eps):
            return (loss_of(w.h0 + eps * vh, w.cd + eps * 1e-3 * vc) -
                    loss_of(w.h0 - eps * vh, w.cd - eps * 1e-3 * vc)) / (2 * eps)
        # fixed steps chosen in advance: central differences at eps = 1 and 1/2 and
        # their Richardson extrapolation (O(eps^4)).  The unit direction spreads eps
        # over 100k parameters (a few mm of thickness per cell), so the loss stays
        # in its linear regime while its FP64 round-off (h ~ 4000 m carries
        # ~1e-12 m) stays far below the signal.
        d1, d2 = fd(1.0), fd(0.5)
        rich = (4 * d2 - d1) / 3
        errs.append(abs(rich - ref) / max(abs(ref), 1e-300))
        raw.append(abs(d2 - ref) / max(abs(ref), 1e-300))
    t_fd = (time.perf_counter() - t3) / (20 * 4.0)   # one FD evaluation = one forward run
    log("finite-difference check, 20 directions: max rel err %.2e (median %.2e); plain central eps=0.5: max %.2e" % (
        max(errs), np.median(errs), max(raw)))
    n_params = 2 * w.mesh.n_cells
    out = dict(metric=METRIC, value=1.0 / (t2 - t0), unit="gradients/s", n_gpus=1, steps=n_steps, warmup=0,
               ms_per_step=(t2 - t0) / n_steps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="adjoint_cvt50k_200steps_50gauges", n_params=n_params, ckpt_every=K, M=w.M),
               forward_s=t_fwd, adjoint_total_s=t2 - t0, backward_s=t2 - t1,
               adjoint_over_forward=(t2 - t0) / t_fwd,
               fd_gradient_s_extrapolated=2 * n_params * t_fd,
               speedup_vs_fd_gradient=2 * n_params * t_fd / (t2 - t0),
               fd_check=dict(directions=20, scheme="Richardson-extrapolated central differences, eps = 1 and 0.5",
                             max_rel_err=max(errs), median_rel_err=float(np.median(errs)),
                             plain_central_max_rel_err=max(raw)))
    print(json.dumps(out), flush=True)


def bench_aquaplanet(args):
    """The paper's temporal-convergence experiment (Section 2.3) at a larger size:
    external gravity wave on a non-rotating, constant-depth aquaplanet (spherical
    coastline-refined CVT, ~40k cells, 25 -> 200 km), FB-LTS with M = 4 at coarse
    steps dt, dt/2, dt/4, dt/8 against RK4 at 10 s over 4 simulated hours; RMS
    thickness error, fitted order, and the FB-LTS throughput on this system."""
    import numpy as np
    import torch
    import paper_2405_10505_amd as F
    from paper_2405_10505_amd.inputs import workloads
    t = time.perf_counter()
    w = workloads.aquaplanet(n=40000, dx_fine=25e3, dx_coarse=200e3)
    fm = F.Mesh(w.mesh)
    lab4, _ = fm.layer_regions(np.where(w.fine_mask, 0, 1), binary=True, r=2)
    log("aquaplanet: N=%d fine=%d regions %s dt=%.1f (built in %.1fs)" % (
        w.mesh.n_cells, int(w.fine_mask.sum()), np.bincount(lab4, minlength=4).tolist(), w.dt,
        time.perf_counter() - t))

    def solver(scheme, dt, M, lab):
        s = F.Solver(fm, dt, M=M, scheme=scheme, physics=F.PHYS_GRAVITY_WAVE)
        s.set_regions(lab, binary=False)
        s.set_state(w.h0, w.u0)
        s.set_graph(True)
        return s

    T = 4 * 3600.0
    ref = solver(F.SCHEME_RK4, 10.0, 1, np.full(w.mesh.n_cells, 3, np.int8))
    ref.step(int(round(T / 10.0)))
    _, href = ref.get_state()
    rows = []
    for k in (1, 2, 4, 8):
        n = int(round(T / (w.dt / k)))
        dt = T / n
        s = solver(F.SCHEME_FBLTS, dt, w.M, lab4)
        s.step(n)
        _, h = s.get_state()
        rows.append(dict(dt_coarse=dt, steps=n, rms_error=float(np.sqrt(np.mean((h - href) ** 2)))))
        log("dt %.1f s: RMS error %.3e m" % (dt, rows[-1]["rms_error"]))
    order = float(np.polyfit(np.log([r["dt_coarse"] for r in rows]), np.log([r["rms_error"] for r in rows]), 1)[0])
    s = solver(F.SCHEME_FBLTS, w.dt, w.M, lab4)
    steps = args.steps or 200
    el = time_steps(torch, s, steps, args.warmup)
    info = s.info()
    value = info["cell_substeps_per_step"] * steps / el
    log("order %.3f; FB-LTS %.4f ms/step, %.3e cell-substeps/s" % (order, el / steps * 1e3, value))
    out = dict(metric="aquaplanet gravity wave: FB-LTS temporal order and cell-substeps/s", value=value,
               unit="cell-substeps/s", n_gpus=1, steps=steps, warmup=args.warmup, ms_per_step=el / steps * 1e3,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=w.name, n_cells=w.mesh.n_cells, n_fine=int(w.fine_mask.sum()), M=w.M,
                           physics="gravity wave (fast terms only)", reference="RK4, dt = 10 s",
                           simulated_seconds=T),
               convergence=dict(rows=rows, fitted_order=order), roofline=None, cpu_baseline=None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
