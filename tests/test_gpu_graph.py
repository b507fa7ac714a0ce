"""Steps captured into a HIP graph: mm_hydro_step without a host copy of
the timestep (the Courant step stays on the device, and every counter is
cleared by a kernel, not a memset) enqueues only kernels on the context's
stream, so a caller can capture several steps once and replay them. Each
replay, with eager work and synchronisations between replays, equals the
eager steps bit for bit, in double and in the mixed + learned form; the
replay's time per step is printed beside the eager one for a mesh small
enough to be bound by launches."""
import time

import numpy as np
import pytest
import torch

from paper_0901_4107_amd import learned, mm
from paper_0901_4107_amd.inputs.configs import kh3d

pytestmark = pytest.mark.gpu

STEPS = 3


def context(wl, mode, stream):
    guess = mm.MM_GUESS_LEARNED if mode == mm.MM_MIXED else mm.MM_GUESS_STANDARD
    ctx = mm.Context(3, wl.gamma, wl.cfl, mode=mode, guess=guess, stream=stream)
    if guess == mm.MM_GUESS_LEARNED:
        ctx.mm_mlp_load(learned.load(wl.gamma))
    ctx.mm_mesh_upload(mm.DeviceMesh.from_host(wl.mesh))
    return ctx


@pytest.mark.parametrize("mode", [mm.MM_FP64, mm.MM_MIXED])
def test_captured_steps_replay_like_eager(mode):
    wl = kh3d(n_points=32 ** 3, seed=941)
    side = torch.cuda.Stream()      # capture needs a stream of its own (default priority)
    with torch.cuda.stream(side):
        run(wl, mode, side)


def run(wl, mode, side):
    ctx = context(wl, mode, side)
    Q0 = torch.from_numpy(np.ascontiguousarray(wl.Q)).cuda()
    Qe = Q0.clone()
    for _ in range(STEPS):
        ctx.mm_hydro_step(Qe, sync=False)
    torch.cuda.synchronize()
    Qg = Q0.clone()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        for _ in range(STEPS):
            ctx.mm_hydro_step(Qg, sync=False)
    torch.cuda.synchronize()
    for rep in range(4):
        Qg.copy_(Q0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Qg, Qe), rep
        Qx = Q0.clone()                      # eager steps between the replays
        ctx.mm_hydro_step(Qx, sync=False)
        torch.cuda.synchronize()
    reps = 50
    t = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t) / (reps * STEPS)
    t = time.perf_counter()
    for _ in range(reps * STEPS):
        ctx.mm_hydro_step(Qx, sync=False)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t) / (reps * STEPS)
    print(f"mode {mode}, {wl.mesh.n_cells} cells: {t_eager * 1e3:.4f} ms per step eager, "
          f"{t_graph * 1e3:.4f} ms replayed", flush=True)
