"""The oracle's loops run on several host threads; every result is the same
bit for bit for any thread count (independent faces and cells, and per-cell
gathers in ascending face order, the order a single face loop adds them)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_4107_amd.inputs.configs import kh2d, kh3d, random3d


def _run(n_threads, wl):
    O.set_threads(n_threads)
    m = wl.mesh
    Q1, dt = O.hydro_step(m, wl.gamma, wl.cfl, wl.Q)
    W = O.prim(m.dim, wl.gamma, m.volume, wl.Q)
    G = O.gradients(m, W)
    F = O.face_fluxes(m, wl.gamma, dt, W, G[1])
    Qe = wl.Q.copy()
    O.apply_update(m, F[0] if isinstance(F, tuple) else F, Qe)
    return [Q1, np.array([dt]), W, *G, Qe]


@pytest.mark.parametrize("make", [lambda: random3d(n_side=14, seed=77), lambda: kh3d(n_points=12 ** 3, seed=78),
                                  lambda: kh2d(seed=79)])
def test_thread_count_does_not_change_results(make):
    wl = make()
    before = O.threads()
    try:
        one = _run(1, wl)
        many = _run(5, wl)
    finally:
        O.set_threads(before)
    for a, b in zip(one, many):
        assert np.array_equal(a, b, equal_nan=True)
