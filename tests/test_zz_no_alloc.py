"""The allocation-free batch entry point (mm_riemann_batch_noalloc) against
the context entry point it varies (mm_riemann_batch): the same outputs and
iteration counts bit for bit, in every form, on two calls in a row whose
second is smaller than the first (the scratch keeps the first call's
contents), through the C ABI."""
import sys

import numpy as np
import pytest
import torch

from paper_0901_4107_amd import learned, mm

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def problems(n, seed):
    """Seeded 1D Riemann problems over wide ranges: densities and pressures
    log-uniform over six decades, velocities up to a few sound speeds, so
    that vacuum, strong shocks and strong rarefactions (the float form's
    hard problems) all occur."""
    rng = np.random.default_rng(seed)
    rho = 10.0 ** rng.uniform(-3, 3, (2, n))
    P = 10.0 ** rng.uniform(-3, 3, (2, n))
    c = np.sqrt(GAMMA * P / rho)
    u = rng.normal(0.0, 1.5, (2, n)) * c
    return np.ascontiguousarray(np.stack([rho[0], u[0], P[0], rho[1], u[1], P[1]]))


@pytest.mark.parametrize("mode", [mm.MM_FP64, mm.MM_MIXED])
@pytest.mark.parametrize("guess", [mm.MM_GUESS_STANDARD, mm.MM_GUESS_LEARNED])
def test_noalloc_equals_context_batch(mode, guess):
    params = learned.load(GAMMA) if guess == mm.MM_GUESS_LEARNED else None
    ctx = mm.Context(3, GAMMA, mode=mode, guess=guess)
    if params is not None:
        ctx.mm_mlp_load(params)
    # the first call spans two chunks of the scratch and a ragged tail; the
    # second is smaller and finds the first one's list in the scratch
    for n, seed in ((mm.MM_NOALLOC_CHUNK + (1 << 19) + 777, 11), (4099, 12)):
        print(f"noalloc: mode {mode} guess {guess} n {n}", flush=True)
        sys.stdout.flush()
        S = torch.from_numpy(problems(n, seed)).cuda()
        want = torch.empty((n, 5), dtype=torch.float64, device="cuda")
        want_it = torch.empty(n, dtype=torch.int32, device="cuda")
        ctx.mm_riemann_batch(S, want, want_it)
        got = torch.full((n, 5), float("nan"), dtype=torch.float64, device="cuda")
        got_it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        mm.mm_riemann_batch_noalloc(S, got, got_it, gamma=GAMMA, mode=mode, guess=guess, mlp_params=params)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert torch.equal(got_it, want_it)
        if mode == mm.MM_MIXED and n > 10000:
            assert ctx.mm_get_diag()["fp64_fallback"] > 0   # the scratch's hard list was used


def test_noalloc_refuses_bad_arguments():
    S = torch.from_numpy(problems(10, 3)).cuda()
    out = torch.empty((10, 5), dtype=torch.float64, device="cuda")
    L = mm.lib()
    import ctypes
    p = mm.mm_params(3, mm.MM_FP64, mm.MM_GUESS_LEARNED, 0, GAMMA, 0.4, 0.0, 0.0, None, 0, 0, 1.1, 0.0, 0.0)
    # the learned guess without parameters, n out of range, a bad gamma
    assert L.mm_riemann_batch_noalloc(ctypes.byref(p), 10, mm._ptr(S), mm._ptr(out), None, None) == mm.MM_E_ARG
    p.guess = mm.MM_GUESS_STANDARD
    assert L.mm_riemann_batch_noalloc(ctypes.byref(p), 0, mm._ptr(S), mm._ptr(out), None, None) == mm.MM_E_ARG
    assert L.mm_riemann_batch_noalloc(ctypes.byref(p), mm.MM_NOALLOC_MAX_BATCH + 1, mm._ptr(S), mm._ptr(out),
                                      None, None) == mm.MM_E_ARG
    p.gamma = 1.0
    assert L.mm_riemann_batch_noalloc(ctypes.byref(p), 10, mm._ptr(S), mm._ptr(out), None, None) == mm.MM_E_ARG
