"""Benchmark of the hydro step on one MI355X.

A step is one pass of the whole hot path over the workload: primitives and
the Courant timestep, limited gradients, face fluxes (extrapolation, face
frame, exact Riemann solve, lab-frame flux) and the conservative update,
through ``mm_hydro_step``. The headline workload is the 3D Kelvin-Helmholtz
shear layer on 128^3 Poisson points with a bulk boost of ten sound speeds
and a comoving mesh, run in the mixed form with the learned Newton guess;
the double-precision path is timed beside it on the same inputs, and the
error of the headline form against it after one step (rest-frame L1 per
conserved component) is reported with the speedup. Inputs are resident in
HBM before any timed region.

Prints ONE JSON line: face fluxes per second of the whole step (value), the
roofline of the dominant kernel (the face-flux kernel, timed on its own with
HIP events on the library's stream) and the CPU oracle's rate on the host
(cpu_baseline). The same form is also timed with the entropy scheme for
cold flows (Section 3.5: entropy row, Mach switch at --mach-thresh) and
reported under "entropy"; the mesh-motion entry points (Section 4.1
generator velocities, volume rate, velocity replacement) are timed on the
same mesh under "mesh_motion". ``--workload rt3d`` times the step with
reflective walls and a static field (Section 8.8's setup, mirror cells
included in the cell and face counts). ``--workload riemann`` instead times the batched
exact solver on 2^24 independent Riemann problems (standard vs learned
guess).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Riemann face fluxes/sec, 3D 128³ Voronoi; mixed+learned vs FP64 at set error"
HBM_PEAK_GBS = 8000.0
WARM_S = 0.25          # seconds of untimed steps before each form is timed, at least
SET_ERROR = 1e-6   # rest-frame L1 per conserved component, mixed forms vs double


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flux_kernel_bytes(dim, n_cells, n_faces, mixed):
    """Algorithmic HBM bytes of one face-flux launch, itemised from what the
    step needs per face and per cell, each item read or written once (ideal
    reuse of the cell data):
      per face: the two cell indices L, R (int32); the area A, the face
                centroid g = f - r_L and the separation d = r_R - r_L in the
                path's precision (float in the mixed form); the face velocity
                w_f and the D + 2 fluxes written, in double;
      per cell: the primitives W (D + 2), their limited gradients
                ((D + 2) D) and the centroid offset s - r (D), in the path's
                precision.
    The library's own face record stores |d| and the normal in place of d
    (one value more): that counts as overhead against this figure, not as
    algorithmic bytes."""
    nv = dim + 2
    fp = 4 if mixed else 8
    per_face = 2 * 4 + (1 + 2 * dim) * fp + dim * 8 + nv * 8
    per_cell = (nv + nv * dim + dim) * fp
    return n_faces * per_face + n_cells * per_cell, per_face, per_cell


def host_cpu():
    """The host the CPU baseline ran on: logical CPUs and model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def l1_rest(a, b, boost):
    """Rest-frame L1 per component (momentum against the momentum vector's
    L1 norm), after the Galilean boost by -v0."""
    D = a.shape[0] - 2

    def unboost(Q):
        out = Q.copy()
        out[1:1 + D] = Q[1:1 + D] - Q[0][None] * boost[:, None]
        out[D + 1] = Q[D + 1] - np.sum(Q[1:1 + D] * boost[:, None], axis=0) + 0.5 * Q[0] * float(boost @ boost)
        return out
    a, b = unboost(a), unboost(b)
    num = np.sum(np.abs(a - b), axis=1)
    den = np.sum(np.abs(b), axis=1)
    den[1:1 + D] = np.sum(np.sqrt(np.sum(b[1:1 + D] ** 2, axis=0)))
    return num / np.where(den > 0, den, 1.0)


def make_context(mm, learned, m, wl, form, dev, mach_thresh=None, steps=0, alpha_s=None):
    mode = mm.MM_FP64 if form.startswith("fp64") else mm.MM_MIXED
    guess = mm.MM_GUESS_LEARNED if form.endswith("learned") else mm.MM_GUESS_STANDARD
    ent = {} if mach_thresh is None else {"entropy": mm.MM_ENTROPY_MACH, "mach_thresh": mach_thresh}
    if alpha_s is not None:
        ent = {"entropy": mm.MM_ENTROPY_ENERGY, "alpha_s": alpha_s}
    ctx = mm.Context(m.dim, wl.gamma, wl.cfl, mode=mode, guess=guess, device=dev, steps=steps, **ent)
    if guess == mm.MM_GUESS_LEARNED:
        params = learned.load(wl.gamma, dev)
        if params is None:
            raise RuntimeError("no trained network for this gamma: run python -m paper_0901_4107_amd.learned")
        ctx.mm_mlp_load(params)
    return ctx


def time_form(mm, learned, torch, wl, dmesh, form, steps, warmup, dev, mach_thresh=None, alpha_s=None):
    """Time `form` on the workload; with mach_thresh, the entropy scheme
    for cold flows (entropy row in Q, Mach switch at that threshold); with
    alpha_s, the same scheme with its energy switch."""
    from paper_0901_4107_amd.inputs.configs import with_entropy
    m = wl.mesh
    ctx = make_context(mm, learned, m, wl, form, dev, mach_thresh, alpha_s=alpha_s)
    ctx.mm_mesh_upload(dmesh)
    if wl.walls is not None:
        ctx.mm_set_walls(torch.from_numpy(wl.walls.ghost).to(dev), torch.from_numpy(wl.walls.src).to(dev),
                         wl.walls.axis)
    if wl.accel is not None:
        ctx.mm_set_gravity(torch.from_numpy(np.ascontiguousarray(wl.accel)).to(dev))
    ent = mach_thresh is not None or alpha_s is not None
    Q0 = torch.from_numpy(with_entropy(wl) if ent else np.ascontiguousarray(wl.Q)).to(dev)
    Q = Q0.clone()
    rec = ctx.recon_buffer(m.n_cells)
    F = ctx.flux_buffer(m.n_faces)
    stream = ctx.stream
    torch.cuda.synchronize()
    dt = ctx.mm_hydro_step(Q)          # Courant step of the initial state
    Q.copy_(Q0)
    # W untimed steps, then exactly K timed consecutive steps (Courant
    # timestep recomputed on the device each step), bracketed by device
    # synchronisation
    # W untimed steps, and at least WARM_S seconds of them: the clocks take
    # longer than a few steps to ramp
    t_warm = time.perf_counter()
    k = 0
    while k < warmup or time.perf_counter() - t_warm < WARM_S:
        ctx.mm_hydro_step(Q, sync=False)
        k += 1
        if k % 10 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    # totals over the domain: the mirror cells of walls are excluded
    keep = (slice(None) if wl.walls is None else
            torch.from_numpy(np.nonzero(wl.walls.interior)[0]).to(dev))
    tot0 = Q[:, keep].sum(dim=1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ctx.mm_hydro_step(Q, sync=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3 / steps
    ms = e0.elapsed_time(e1) / steps
    # conservation over the timed steps: change of the totals of m, p, E,
    # relative to the total mass, momentum magnitude and energy
    tot1 = Q[:, keep].sum(dim=1)
    D = m.dim
    scale = torch.abs(tot0).clone()
    scale[1:1 + D] = torch.sqrt(torch.sum(Q[1:1 + D][:, keep] ** 2, dim=0)).sum()
    cons = (torch.abs(tot1 - tot0) / scale).cpu().numpy()
    # the dominant kernel alone, on the initial state's records
    ctx.mm_gradients(Q0, rec)
    for _ in range(max(warmup, 10)):
        ctx.mm_face_fluxes(dt, rec, F)
    torch.cuda.synchronize()
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for k in range(steps):
        fev[2 * k].record(stream)
        ctx.mm_face_fluxes(dt, rec, F)
        fev[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    flux_ms = float(np.mean([fev[2 * k].elapsed_time(fev[2 * k + 1]) for k in range(steps)]))
    # one step from the initial state at the common timestep, for the error
    Q1 = Q0.clone()
    ctx.mm_reset_diag()
    ctx.mm_hydro_step(Q1, dt=dt)
    diag = ctx.mm_get_diag()
    return {"ms": ms, "wall_ms": wall_ms, "flux_ms": flux_ms, "dt": dt, "Q1": Q1.cpu().numpy(), "diag": diag,
            "conservation": [float(x) for x in cons],
            "workspace_gb": ctx._ws.numel() / 1e9}


def time_mesh_motion(mm, torch, wl, dmesh, steps, dev):
    """The mesh-motion entry points on the workload's mesh: generator
    velocities with the roundness correction (eta 0.25, chi 1), the volume
    rate, the replacement of the mesh's velocities (which rebuilds the
    face records and synchronises), and the whole mesh upload (median of 5,
    wall clock)."""
    m = wl.mesh
    ctx = mm.Context(m.dim, wl.gamma, wl.cfl, mode=mm.MM_MIXED, device=dev)
    ctx.mm_mesh_upload(dmesh)
    Q = torch.from_numpy(np.ascontiguousarray(wl.Q)).to(dev)
    w = torch.empty((m.dim, m.n_cells), dtype=torch.float64, device=dev)
    rate = torch.empty(m.n_cells, dtype=torch.float64, device=dev)
    stream = ctx.stream

    def events(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    vel_ms = events(lambda: ctx.mm_mesh_velocity(Q, w))
    rate_ms = events(lambda: ctx.mm_volume_rate(rate))
    ctx.mm_mesh_set_velocity(w)
    t = time.perf_counter()
    for _ in range(steps):
        ctx.mm_mesh_set_velocity(w)
    set_ms = (time.perf_counter() - t) * 1e3 / steps
    # the whole mesh upload (validation, side lists, records; it synchronises)
    up = []
    for _ in range(5):
        t = time.perf_counter()
        ctx.mm_mesh_upload(dmesh)
        up.append((time.perf_counter() - t) * 1e3)
    return {"mesh_velocity_ms": vel_ms, "volume_rate_ms": rate_ms, "set_velocity_wall_ms": set_ms,
            "upload_wall_ms": float(np.median(up)), "cells_per_s_mesh_velocity": m.n_cells / (vel_ms * 1e-3)}


def time_individual(mm, learned, torch, wl, dmesh, form, dt_courant, step_ms, dev):
    """Individual power-of-two timesteps (Section 7.2) on the workload: one
    full cycle of dt_max = 4 Courant steps of the initial state, with the
    number of levels raised until every cell's criterion fits a bin (the
    library answers MM_E_RANGE below that). Untimed: a first full cycle;
    timed: a second one from the same initial state. Compared with a global
    scheme whose step is the smallest occupied bin's (the paper's
    comparison: a global step at the smallest individual criterion), whose
    cost is estimated from the measured global step time, and with the
    Courant-step global path per unit of simulated time."""
    m = wl.mesh
    ctx = make_context(mm, learned, m, wl, form, dev, steps=mm.MM_STEPS_INDIVIDUAL)
    ctx.mm_mesh_upload(dmesh)
    Q0 = torch.from_numpy(np.ascontiguousarray(wl.Q)).to(dev)
    dt_max, levels = 4.0 * dt_courant, 6

    def cycle(Q):
        """One cycle in batches of up to 64 points (one synchronisation per
        batch); the smallest and largest bins seen at the batch ends."""
        ctx.mm_tb_begin(dt_max, levels)
        pts, faces, cells, b0, hi = 0, 0, 0, levels, 0
        while True:
            info = ctx.mm_tb_advance(Q, 1 << levels, 64)
            pts += info["points"]
            faces += info["total_faces"]
            cells += info["total_cells"]
            b0, hi = min(b0, info["min_bin"]), max(hi, info["max_bin"])
            if info["next_tick"] >= 1 << levels:
                return pts, faces, cells, b0, hi
    while True:
        try:
            cycle(Q0.clone())
            break
        except mm.MMError as e:
            if e.status != mm.MM_E_RANGE or levels >= 30:
                raise
            levels += 1
    Q = Q0.clone()
    torch.cuda.synchronize()
    tot0 = Q.sum(dim=1)
    t = time.perf_counter()
    pts, faces, cells, b0, hi = cycle(Q)
    torch.cuda.synchronize()
    cycle_ms = (time.perf_counter() - t) * 1e3
    tot1 = Q.sum(dim=1)
    D = m.dim
    scale = torch.abs(tot0).clone()
    scale[1:1 + D] = torch.sqrt(torch.sum(Q[1:1 + D] ** 2, dim=0)).sum()
    cons = (torch.abs(tot1 - tot0) / scale).cpu().numpy()
    glob_steps = 1 << (levels - b0)
    glob_ms = glob_steps * step_ms
    return {"form": form, "levels": levels, "dt_max": dt_max, "dt_courant": dt_courant,
            "smallest_bin": b0, "largest_bin": hi, "points_per_cycle": pts, "cycle_ms": cycle_ms,
            "ms_per_point": cycle_ms / pts, "face_fluxes_per_cycle": faces, "cell_openings_per_cycle": cells,
            "global_at_smallest_bin": {"steps": glob_steps, "face_fluxes": glob_steps * m.n_faces,
                                       "ms_estimated": glob_ms},
            "flux_ratio_vs_global_at_smallest_bin": glob_steps * m.n_faces / faces,
            "speedup_vs_global_at_smallest_bin": glob_ms / cycle_ms,
            "time_per_simulated_time_vs_courant_global": (cycle_ms / dt_max) / (step_ms / dt_courant),
            "conservation_rel_change": [float(x) for x in cons]}


def newton_summary(d):
    return {"iters_mean": d["newton_iters"] / max(1, d["faces"]),
            "wave_max_mean": d["wave_iter_max_sum"] / max(1, d["waves"]), "max": d["newton_max"],
            "vacuum": d["vacuum"], "positivity_fallback": d["positivity_fallback"],
            "fp64_fallback": d["fp64_fallback"], "guess_fallback": d["guess_fallback"]}


def bench_step(args):
    import torch
    from paper_0901_4107_amd import learned, mm
    from paper_0901_4107_amd.inputs import configs

    t0 = time.time()
    if args.workload == "kh3d":
        wl = configs.kh3d(n_points=(args.size or 128) ** 3, nthreads=args.threads)
    elif args.workload == "random3d":
        wl = configs.random3d(n_side=args.size or 64, nthreads=args.threads)
    elif args.workload == "rt3d":
        wl = configs.rt3d(n_side=args.size or 128, nthreads=args.threads)
    else:
        wl = configs.sedov3d(n_side=args.size or 256, nthreads=args.threads)
    m = wl.mesh
    log(f"workload {wl.name}: N={m.n_cells} F={m.n_faces} built in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    dmesh = mm.DeviceMesh.from_host(m, dev)
    # the headline form once untimed first: the first context of a process
    # ran 2-3% slower on fresh device memory (a 6 GiB allocation touched and
    # freed first took half of that away), later contexts reuse the freed
    # blocks
    time_form(mm, learned, torch, wl, dmesh, args.mode, 2, 1, dev)
    head = time_form(mm, learned, torch, wl, dmesh, args.mode, args.steps, args.warmup, dev)
    log(f"{args.mode}: {head['ms']:.3f} ms/step, flux kernel {head['flux_ms']:.3f} ms")
    mixed = args.mode.startswith("mixed")
    out = {
        "metric": METRIC if (args.workload == "kh3d" and m.n_cells == 128 ** 3)
        else f"face fluxes/sec of the whole step, {wl.name}; {args.mode}",
        "value": m.n_faces / (head["ms"] * 1e-3),
        "unit": "face-fluxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "wall_ms_per_step": head["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_cells": m.n_cells, "n_faces": m.n_faces, "form": args.mode,
                   "gamma": wl.gamma, "cfl": wl.cfl, "seed": wl.seed, "boost": list(map(float, wl.boost))},
        "flux_kernel": {"ms": head["flux_ms"], "face_fluxes_per_s": m.n_faces / (head["flux_ms"] * 1e-3)},
        "newton": newton_summary(head["diag"]),
        "conservation_rel_change": head["conservation"],
        "device_memory_gb": {"workspace": head["workspace_gb"],
                             "peak_allocated": torch.cuda.max_memory_allocated(dev) / 1e9},
    }
    nbytes, per_face, per_cell = flux_kernel_bytes(m.dim, m.n_cells, m.n_faces, mixed)
    achieved = nbytes / (head["flux_ms"] * 1e-3) / 1e9
    lrn = 'true' if args.mode.endswith('learned') else 'false'
    grv = 'true' if wl.accel is not None else 'false'
    kname = (f"k_face_flux_mixed<{m.dim}, {lrn}, 0, {grv}>" if mixed
             else f"k_face_flux64<{m.dim}, {lrn}, 0, {grv}>")
    from paper_0901_4107_amd.prof_summary import read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles"), kname, wl.name)
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                       "traffic_vs_algorithmic": None if traffic is None else traffic / nbytes,
                       "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, copy-scaled)",
                       "kernel": kname, "algorithmic_bytes": nbytes,
                       "bytes_per_face": per_face, "bytes_per_cell": per_cell}
    if args.mode == "mixed+learned" and not args.no_compare:
        std = time_form(mm, learned, torch, wl, dmesh, "mixed", args.steps, args.warmup, dev)
        log(f"mixed (standard guess): {std['ms']:.3f} ms/step, flux kernel {std['flux_ms']:.3f} ms")
        out["mixed_standard_guess"] = {"ms_per_step": std["ms"], "face_fluxes_per_s": m.n_faces / (std["ms"] * 1e-3),
                                       "flux_kernel_ms": std["flux_ms"], "newton": newton_summary(std["diag"]),
                                       "learned_step_speedup": std["ms"] / head["ms"],
                                       "learned_flux_kernel_speedup": std["flux_ms"] / head["flux_ms"]}
    if args.mode != "fp64" and not args.no_compare:
        base = time_form(mm, learned, torch, wl, dmesh, "fp64", args.steps, args.warmup, dev)
        log(f"fp64: {base['ms']:.3f} ms/step, flux kernel {base['flux_ms']:.3f} ms")
        err = l1_rest(head["Q1"], base["Q1"], np.asarray(wl.boost, dtype=np.float64))
        out["fp64"] = {"ms_per_step": base["ms"], "face_fluxes_per_s": m.n_faces / (base["ms"] * 1e-3),
                       "flux_kernel_ms": base["flux_ms"],
                       "flux_kernel_face_fluxes_per_s": m.n_faces / (base["flux_ms"] * 1e-3),
                       "newton": newton_summary(base["diag"])}
        out["speedup_vs_fp64"] = {"step": base["ms"] / head["ms"], "flux_kernel": base["flux_ms"] / head["flux_ms"],
                                  "l1_rest_frame_vs_fp64": [float(x) for x in err],
                                  "set_error": SET_ERROR, "within_set_error": bool(np.all(err <= SET_ERROR))}
    if not args.no_entropy:
        ent = time_form(mm, learned, torch, wl, dmesh, args.mode, args.steps, args.warmup, dev,
                        mach_thresh=args.mach_thresh)
        log(f"{args.mode} with the entropy scheme: {ent['ms']:.3f} ms/step, flux kernel {ent['flux_ms']:.3f} ms")
        out["entropy"] = {"form": args.mode, "mach_thresh": args.mach_thresh, "ms_per_step": ent["ms"],
                          "face_fluxes_per_s": m.n_faces / (ent["ms"] * 1e-3), "flux_kernel_ms": ent["flux_ms"],
                          "kept_fraction": ent["diag"]["entropy_kept"] / m.n_cells,
                          "step_time_vs_plain": ent["ms"] / head["ms"]}
        esw = time_form(mm, learned, torch, wl, dmesh, args.mode, args.steps, args.warmup, dev,
                        alpha_s=args.alpha_s)
        log(f"{args.mode} with the energy switch: {esw['ms']:.3f} ms/step")
        out["entropy_energy_switch"] = {"form": args.mode, "alpha_s": args.alpha_s, "ms_per_step": esw["ms"],
                                        "face_fluxes_per_s": m.n_faces / (esw["ms"] * 1e-3),
                                        "kept_fraction": esw["diag"]["entropy_kept"] / m.n_cells,
                                        "step_time_vs_plain": esw["ms"] / head["ms"]}
    if not args.no_entropy:
        out["mesh_motion"] = time_mesh_motion(mm, torch, wl, dmesh, args.steps, dev)
        log(f"mesh motion: {out['mesh_motion']}")
    if wl.walls is not None:
        out["config"]["walls"] = {"axis": wl.walls.axis, "mirror_cells": int(len(wl.walls.ghost)),
                                  "domain_cells": int(wl.walls.interior.sum()), "field": "uniform -0.1 along y"}
    if not args.no_individual and wl.walls is None and wl.accel is None:   # neither combines with a timeline
        ind = time_individual(mm, learned, torch, wl, dmesh, args.mode, head["dt"], head["ms"], dev)
        out["individual_timesteps"] = ind
        log(f"individual timesteps: {ind['points_per_cycle']} points, {ind['cycle_ms']:.2f} ms per cycle of "
            f"{2 ** ind['levels']} ticks; {ind['flux_ratio_vs_global_at_smallest_bin']:.1f}x fewer fluxes than a "
            f"global step at the smallest bin")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    return out


def cpu_baseline(wl):
    """The oracle's whole step on the whole workload: once on one thread, and
    three times on every thread OpenMP is given (the median), the results
    being the same bit for bit. `value` is the all-thread rate."""
    from oracle import oracle as O
    m = wl.mesh

    def one_step():
        t = time.time()
        if wl.walls is None and wl.accel is None:
            O.hydro_step(m, wl.gamma, wl.cfl, wl.Q)
        else:   # the same work as the device step: reflection, step with the field
            Q = wl.Q if wl.walls is None else O.reflect(wl.Q, wl.walls.ghost, wl.walls.src, wl.walls.axis)
            O.hydro_step_full(m, wl.gamma, wl.cfl, Q, accel=wl.accel)
        return time.time() - t

    all_threads = O.threads()
    try:
        O.set_threads(1)
        log("cpu baseline: oracle hydro step on the full workload, 1 thread")
        t1 = one_step()
        O.set_threads(all_threads)
        log(f"cpu baseline: the same on {all_threads} threads (median of 3)")
        tn = float(np.median([one_step() for _ in range(3)]))
    finally:
        O.set_threads(all_threads)
    return {"value": m.n_faces / tn, "unit": "face-fluxes/s", "cores": all_threads, "kind": "oracle",
            "sample": f"one full oracle hydro step on the whole {wl.name} workload ({m.n_faces} faces): "
                      f"{tn:.2f} s on {all_threads} threads (median of 3), {t1:.2f} s on 1 thread",
            "single_thread": {"value": m.n_faces / t1, "unit": "face-fluxes/s", "cores": 1, "seconds": t1},
            "all_threads_seconds": tn, "host": host_cpu()}


def bench_riemann(args):
    """2^24 independent Riemann problems: Newton iterations and throughput
    of the batched exact solver, standard vs learned guess, double and float."""
    import torch
    from paper_0901_4107_amd import learned, mm
    from paper_0901_4107_amd.inputs import configs

    gamma = 5.0 / 3.0
    n = args.size or (1 << 24)
    t0 = time.time()
    S = torch.from_numpy(configs.riemann_problems(n)).cuda()
    log(f"riemann workload: {n} problems built in {time.time() - t0:.1f}s")
    params = learned.load(gamma)
    res = {}
    for form in ("fp64", "fp64+learned", "mixed", "mixed+learned"):
        mode = mm.MM_FP64 if form.startswith("fp64") else mm.MM_MIXED
        guess = mm.MM_GUESS_LEARNED if form.endswith("learned") else mm.MM_GUESS_STANDARD
        ctx = mm.Context(3, gamma, mode=mode, guess=guess)
        if guess == mm.MM_GUESS_LEARNED:
            ctx.mm_mlp_load(params)
        out = torch.empty((n, 5), dtype=torch.float64, device="cuda")
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        ctx.mm_riemann_batch(S, out, it)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            ctx.mm_riemann_batch(S, out, None)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        itn = it.cpu().numpy()
        waves = np.max(np.pad(itn, (0, (-n) % 64)).reshape(-1, 64), axis=1)
        d = ctx.mm_get_diag()
        res[form] = {"ms": ms, "problems_per_s": n / (ms * 1e-3), "iters_mean": float(itn.mean()),
                     "iters_p99": float(np.percentile(itn, 99)), "wave_max_mean": float(waves.mean()),
                     "fp64_fallback": d["fp64_fallback"] // (args.steps + 1),
                     "guess_fallback": d["guess_fallback"] // (args.steps + 1)}
        log(f"{form}: {ms:.3f} ms, iterations mean {itn.mean():.3f} wave-max {waves.mean():.3f}")
    return {"metric": "Riemann problems/sec (2^24 problems, exact solver)",
            "value": res["mixed+learned"]["problems_per_s"], "unit": "problems/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": res["mixed+learned"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"riemann_{n}", "gamma": gamma}, "forms": res}


def calibrate_copy(mb):
    """A plain device copy of known size, for scaling the rocprof FETCH_SIZE
    and WRITE_SIZE counters."""
    import torch
    x = torch.ones(mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=25,
                    help="untimed steps first, and at least 0.25 s of them (with 3 steps the first form timed in a "
                         "process ran 2-4%% slow: the clocks ramp)")
    ap.add_argument("--workload", default="kh3d", choices=["kh3d", "random3d", "sedov3d", "rt3d", "riemann"])
    ap.add_argument("--size", type=int, default=0, help="points per axis (lattice) or cube root of the point count")
    ap.add_argument("--mode", default="mixed+learned", choices=["fp64", "fp64+learned", "mixed", "mixed+learned"])
    ap.add_argument("--no-compare", action="store_true", help="skip the double-precision comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-entropy", action="store_true", help="skip the run with the entropy scheme for cold flows")
    ap.add_argument("--mach-thresh", type=float, default=1.1, help="Mach switch of the entropy scheme")
    ap.add_argument("--no-individual", action="store_true", help="skip the individual-timestep cycle")
    ap.add_argument("--alpha-s", type=float, default=0.01,
                    help="energy switch of the entropy scheme: thermal below alpha_s times the kinetic energy")
    ap.add_argument("--threads", type=int, default=0, help="host threads for the mesh builder")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "libmm runs one process on one GPU; the step is not sharded across GPUs, so --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    out = bench_riemann(args) if args.workload == "riemann" else bench_step(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
