"""Benchmark of the hydro step on one MI355X.

A step is one pass of the whole hot path over the workload: primitives and
the Courant timestep, limited gradients, face fluxes (extrapolation, face
frame, exact Riemann solve, lab-frame flux) and the conservative update,
through ``mm_hydro_step``. The headline workload is the 3D Kelvin-Helmholtz
shear layer on 128^3 Poisson points with a bulk boost of ten sound speeds
and a comoving mesh; its inputs are resident in HBM before timing starts.

Prints ONE JSON line: face fluxes per second of the whole step (value), the
roofline of the dominant kernel (the face-flux kernel, timed on its own
with HIP events on the library's stream) and the CPU oracle's rate on the
host (cpu_baseline).
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flux_kernel_bytes(dim, n_cells, n_faces, mode):
    """Algorithmic HBM bytes of one face-flux launch: per face the two cell
    indices, the face geometry and velocity, and the flux written; per cell
    (each read once under ideal reuse) primitives, gradients and the
    centre-of-mass offset."""
    nv = dim + 2
    if mode == "fp64":
        per_face = 2 * 4 + (2 + 2 * dim) * 8 + dim * 8 + nv * 8
        per_cell = (nv + nv * dim + dim) * 8
    else:
        per_face = 2 * 4 + (2 + 2 * dim) * 4 + 2 * dim * 4 + 8 + dim * 8 + nv * 8
        per_cell = (nv + nv * dim) * 4 + dim * 8
    return n_faces * per_face + n_cells * per_cell, per_face, per_cell


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kh3d", choices=["kh3d", "random3d", "sedov3d"])
    ap.add_argument("--size", type=int, default=0, help="points per axis (lattice) or cube root of the point count")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--threads", type=int, default=0, help="host threads for the mesh builder")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_0901_4107_amd import mm
    from paper_0901_4107_amd.inputs import configs

    t0 = time.time()
    if args.workload == "kh3d":
        wl = configs.kh3d(n_points=(args.size or 128) ** 3, nthreads=args.threads)
    elif args.workload == "random3d":
        wl = configs.random3d(n_side=args.size or 64, nthreads=args.threads)
    else:
        wl = configs.sedov3d(n_side=args.size or 256, nthreads=args.threads)
    m = wl.mesh
    log(f"workload {wl.name}: N={m.n_cells} F={m.n_faces} built in {time.time() - t0:.1f}s")

    mode = mm.MM_FP64 if args.mode == "fp64" else mm.MM_MIXED
    dev = torch.device("cuda:0")
    ctx = mm.Context(m.dim, wl.gamma, wl.cfl, mode=mode, device=dev)
    dmesh = mm.DeviceMesh.from_host(m, dev)
    ctx.mm_mesh_upload(dmesh)
    Q0 = torch.from_numpy(np.ascontiguousarray(wl.Q)).to(dev)
    Q = Q0.clone()
    rec = ctx.recon_buffer(m.n_cells)
    F = ctx.flux_buffer(m.n_faces)
    stream = ctx.stream
    torch.cuda.synchronize()

    # timestep of the first step, used for the isolated flux-kernel timing
    dt = ctx.mm_hydro_step(Q)
    Q.copy_(Q0)

    # whole step: W untimed steps, then exactly K timed consecutive steps
    # (Courant timestep computed on the device each step), bracketed by
    # device synchronisation
    for _ in range(args.warmup):
        ctx.mm_hydro_step(Q, sync=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.mm_hydro_step(Q, sync=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3 / args.steps
    ms = e0.elapsed_time(e1) / args.steps

    # the dominant kernel alone: face fluxes
    ctx.mm_gradients(Q0, rec)
    for _ in range(args.warmup):
        ctx.mm_face_fluxes(dt, rec, F)
    torch.cuda.synchronize()
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    for k in range(args.steps):
        fev[2 * k].record(stream)
        ctx.mm_face_fluxes(dt, rec, F)
        fev[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    flux_ms = float(np.mean([fev[2 * k].elapsed_time(fev[2 * k + 1]) for k in range(args.steps)]))
    ctx.mm_reset_diag()
    ctx.mm_hydro_step(Q0.clone())
    diag = ctx.mm_get_diag()

    nbytes, per_face, per_cell = flux_kernel_bytes(m.dim, m.n_cells, m.n_faces, args.mode)
    achieved = nbytes / (flux_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": m.n_faces / (ms * 1e-3),
        "unit": "face-fluxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_cells": m.n_cells, "n_faces": m.n_faces, "mode": args.mode,
                   "guess": "standard", "gamma": wl.gamma, "cfl": wl.cfl, "seed": wl.seed},
        "flux_kernel": {"ms": flux_ms, "face_fluxes_per_s": m.n_faces / (flux_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_face_flux", "bytes_per_face": per_face, "bytes_per_cell": per_cell},
        "newton": {"iters_mean": diag["newton_iters"] / max(1, diag["faces"]),
                   "wave_max_mean": diag["wave_iter_max_sum"] / max(1, diag["waves"]),
                   "max": diag["newton_max"], "vacuum": diag["vacuum"],
                   "positivity_fallback": diag["positivity_fallback"], "fp64_fallback": diag["fp64_fallback"]},
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("cpu baseline: oracle hydro step on the full workload (1 thread)")
        t = time.time()
        O.hydro_step(m, wl.gamma, wl.cfl, wl.Q)
        el = time.time() - t
        out["cpu_baseline"] = {"value": m.n_faces / el, "unit": "face-fluxes/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full oracle hydro step on the whole {wl.name} workload "
                                         f"({m.n_faces} faces), single thread, {el:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
