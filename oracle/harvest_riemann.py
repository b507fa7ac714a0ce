"""Harvest the Riemann problems of the method's own runs, for the batch
workload of independent 1D problems (test infrastructure: the oracle takes
the steps; only the input generator reads what this writes).

The batch is to be drawn from histograms of the problems that the runs of
the random-state, boosted Kelvin-Helmholtz and point-explosion workloads
pose. This script runs those workloads with the oracle at 48^3, moving the
generators with the flow and rebuilding the tessellation every step (the
scheme's steps (i)-(vii), Section 3), and records at every tenth step the
face-frame Riemann problems of every face: the states extrapolated to the
face and half a step forward, in the face's frame, along its normal
(Section 3.3), exactly the problems the exact solver is given.

Each source is reduced to histograms of the quantities that fix a problem:
  x0 = ln(rho_R / rho_L), x1 = ln(P_R / P_L), x2 = (u_R - u_L) / (c_L + c_R)
jointly (a sparse 3D histogram: the Riemann solution's structure and
Newton's iteration count depend on these alone), with the scale
(ln rho_L, ln P_L) as a 2D histogram and the frame u_L / c_L as a 1D one
(where the face sits in the wave fan). Problems that generate vacuum or have
a vacuum side are counted apart (their share) and drawn uniformly in the
vacuum region by the generator.

    python -m oracle.harvest_riemann [--side 48] [--out PATH]

writes paper_0901_4107_amd/data/riemann_harvest.npz (numpy arrays, no
pickled objects): per source the joint, scale and frame histograms, the
number of problems and the vacuum share, and the bin edges.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_0901_4107_amd.inputs import build_mesh  # noqa: E402
from paper_0901_4107_amd.inputs import configs as C  # noqa: E402

OUT = os.path.join(ROOT, "paper_0901_4107_amd", "data", "riemann_harvest.npz")

# Bin edges. The ln ratios and the velocity jump take edges that are fine
# near zero (where the smooth parts of a flow put most faces) and coarse in
# the tails: +-(0.005 ... 16) for the ln ratios (pressure ratios to e^16),
# -12 ... 3 for the velocity jump in units of c_L + c_R (vacuum starts at
# 2/(gamma - 1) = 3 for gamma = 5/3). The scale takes steps of 1/2 in
# [-12, 12], the frame u_L / c_L steps of 1/4 in [-16, 16].
_TAIL = [0.005, 0.02, 0.05, 0.1, 0.2, 0.35, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 11.0, 16.0]
_RATIO = [-t for t in reversed(_TAIL)] + [0.0] + _TAIL
_JUMP = [-t for t in reversed(_TAIL[:-2] + [12.0])] + [0.0] + _TAIL[:11] + [2.5, 3.0]
EDGES = {
    "x0": np.array(_RATIO),
    "x1": np.array(_RATIO),
    "x2": np.array(_JUMP),
    "lr": np.arange(-12.0, 12.0 + 1e-9, 0.5),
    "lp": np.arange(-12.0, 12.0 + 1e-9, 0.5),
    "m": np.arange(-16.0, 16.0 + 1e-9, 0.25),
}


def note(msg):
    print(msg, flush=True)


def run(wl, steps, every, moving=True):
    """Oracle steps of a workload with the Courant timestep; the face-frame
    problems [6][F] of every `every`-th step (the first included)."""
    m, g = wl.mesh, wl.gamma
    Q = wl.Q.copy()
    pts = m.positions.copy()
    out = []
    for k in range(steps):
        W = O.prim(m.dim, g, m.volume, Q)
        if moving:
            m.with_velocity(np.ascontiguousarray(W[1:1 + m.dim]))   # w = v (Section 3.2)
        _, G, _ = O.gradients(m, W)
        dt = O.cfl_dt(m, g, wl.cfl, W)
        if k % every == 0:
            out.append(O.face_states(m, g, dt, W, G))
        F, _, _ = O.face_fluxes(m, g, dt, W, G)
        Q = O.apply_update(m, F, Q)
        if moving:
            pts = np.mod(pts + dt * W[1:1 + m.dim].T, 1.0)
            m = build_mesh(pts)
    return np.concatenate(out, axis=1)


def features(S, gamma):
    """(x0, x1, x2, ln rho_L, ln P_L, u_L / c_L) of problems without vacuum,
    and the share of vacuum problems."""
    rL, uL, PL, rR, uR, PR = S
    ok = (rL > 0) & (PL > 0) & (rR > 0) & (PR > 0)
    cL = np.sqrt(gamma * PL[ok] / rL[ok])
    cR = np.sqrt(gamma * PR[ok] / rR[ok])
    x2 = (uR[ok] - uL[ok]) / (cL + cR)
    keep = x2 < 2.0 / (gamma - 1.0)
    f = np.stack([np.log(rR[ok] / rL[ok]), np.log(PR[ok] / PL[ok]), x2, np.log(rL[ok]), np.log(PL[ok]),
                  uL[ok] / cL])[:, keep]
    return f, 1.0 - f.shape[1] / S.shape[1]


def histograms(f):
    """Joint histogram of (x0, x1, x2) and the histograms of the scale and of
    the frame; values beyond the edges go to the outermost bins."""
    def clip(v, e):
        return np.clip(v, e[0], np.nextafter(e[-1], -np.inf))
    joint, _ = np.histogramdd(np.stack([clip(f[0], EDGES["x0"]), clip(f[1], EDGES["x1"]),
                                        clip(f[2], EDGES["x2"])], axis=1),
                              bins=[EDGES["x0"], EDGES["x1"], EDGES["x2"]])
    scale, _, _ = np.histogram2d(clip(f[3], EDGES["lr"]), clip(f[4], EDGES["lp"]), bins=[EDGES["lr"], EDGES["lp"]])
    frame, _ = np.histogram(clip(f[5], EDGES["m"]), bins=EDGES["m"])
    return {"joint": joint.astype(np.uint32), "scale": scale.astype(np.uint32), "frame": frame.astype(np.uint32)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=48)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    s = args.side
    sources = {
        # the random-state workload: one step (it is a one-step workload)
        "random3d": (lambda: C.random3d(n_side=s, seed=2001), 1, 1),
        # the boosted shear layer, comoving mesh: 30 steps
        "kh3d": (lambda: C.kh3d(n_points=s ** 3, seed=2002), 30, 10),
        # the point explosion, moving mesh: until the blast has grown
        "sedov3d": (lambda: C.sedov3d(n_side=s, seed=2003), 160, 10),
    }
    arrays = {f"edges_{k}": e for k, e in EDGES.items()}
    arrays["gamma"] = np.array(5.0 / 3.0)
    arrays["side"] = np.array(s)
    for name, (make, steps, every) in sources.items():
        t = time.time()
        wl = make()
        S = run(wl, steps, every)
        f, vac = features(S, wl.gamma)
        for k, v in histograms(f).items():
            arrays[f"{name}_{k}"] = v
        arrays[f"{name}_problems"] = np.array(S.shape[1])
        arrays[f"{name}_vacuum_share"] = np.array(vac)
        note(f"{name}: {S.shape[1]} problems over {steps} steps, {int(np.count_nonzero(arrays[name + '_joint']))} "
             f"joint bins, vacuum share {vac:.2e}, {time.time() - t:.0f} s")
    np.savez_compressed(args.out, **arrays)
    note(f"wrote {args.out} ({os.path.getsize(args.out) / 1024:.0f} KB)")


if __name__ == "__main__":
    main()
