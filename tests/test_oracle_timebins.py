"""Pins of the oracle's individual power-of-two timesteps (Section 7.2):
cells in a nested hierarchy of step sizes dt_max / 2^k, each face
integrated over the smaller step of its two cells, inactive cells keeping
their records of their last active step, and the signal-speed criterion of
eq. EqnTiStepIndividual over the Voronoi neighbours.

Pinned against: the global step (one occupied bin is exactly the global
scheme); closed forms of the criterion on Cartesian lattices; the
invariants of the hierarchy (who is active, bins below the criterion, one
bin up at most and only in step, the next synchronisation point, every face
integrated exactly up to each activation of its cells); exact states that
must survive any bin pattern (a static density contrast in pressure
equilibrium, a uniform flow at full synchronisation); conservation; and a
Sedov blast against the global scheme at the smallest criterion."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import (conserved_from_primitive, kh2d, poisson_points, random3d,
                                                random_states, sedov3d)
from tests.util import blast_radius


def timeline_for(mesh, gam, cfl, Q, levels, spread=1.0):
    """A timeline whose smallest step is spread times the smallest
    criterion (just below it for spread = 1)."""
    W = O.prim(mesh.dim, gam, mesh.volume, Q)
    dmin = O.tb_criterion(mesh, gam, cfl, W).min()
    return O.Timeline(mesh, gam, cfl, np.ldexp(0.99 * dmin * spread, levels), levels)


@pytest.mark.parametrize("make", [lambda: random3d(n_side=10, seed=801), kh2d])
def test_single_bin_is_the_global_step(make):
    """With dt_max below every cell's criterion all cells sit in the top
    bin: one synchronisation point is the global step of length dt_max,
    bit for bit, and the next point is dt_max later."""
    wl = make()
    m, g, D = wl.mesh, wl.gamma, wl.mesh.dim
    dmin = O.tb_criterion(m, g, wl.cfl, O.prim(D, g, m.volume, wl.Q)).min()
    tl = O.Timeline(m, g, wl.cfl, 0.5 * dmin, 3)
    Q = wl.Q.copy()
    r = tl.step(Q)
    assert r["status"] == 0 and r["next"] == 8 and r["active"].all() and r["n_faces"] == m.n_faces
    assert np.all(tl.bin == 3)
    Qg, _ = O.hydro_step(m, g, wl.cfl, wl.Q, dt=0.5 * dmin)
    assert np.array_equal(Q, Qg)


def lattice(n):
    xs = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    return build_mesh(np.stack([X.ravel(), Y.ravel()], axis=1)), X.ravel()


def test_criterion_closed_forms_on_a_lattice():
    """Cartesian lattice of spacing h, c = 1 (rho = 1, P = 3/5, gamma =
    5/3), R = h / sqrt(pi): at rest every neighbour pair has signal speed
    2c, so dt = C h/2 (below C R/c); a uniform flow at 3c keeps the pairs at
    2c but the local bound falls to C R/(4c); colliding streams +-u (u =
    c/2, meeting at x = 1/2 and parting across the periodic edge) give the
    two columns at the meeting line dt = C h/(2c + 2u) and every other
    column C R/(c + u), the parting pairs (2c - 2u) binding nobody."""
    n, cfl, g = 16, 0.4, 5.0 / 3.0
    mesh, x = lattice(n)
    h = 1.0 / n
    R = h / np.sqrt(np.pi)
    N = mesh.n_cells

    def crit(vx):
        Q = conserved_from_primitive(mesh.volume, np.ones(N), np.stack([vx, np.zeros(N)]), np.full(N, 0.6), g)
        return O.tb_criterion(mesh, g, cfl, O.prim(2, g, mesh.volume, Q))
    c = np.sqrt(g * 0.6)
    assert np.allclose(crit(np.zeros(N)), cfl * h / (2 * c), rtol=1e-13)
    assert np.allclose(crit(np.full(N, 3.0 * c)), cfl * R / (4 * c), rtol=1e-13)
    u = 0.5 * c
    dt = crit(np.where(x < 0.5, u, -u))
    meet = np.abs(x - 0.5) < h
    assert meet.sum() == 2 * n
    assert np.allclose(dt[meet], cfl * h / (2 * c + 2 * u), rtol=1e-13)
    assert np.allclose(dt[~meet], cfl * R / (c + u), rtol=1e-13)


def bin_of(dt, tick, levels):
    """Largest b <= levels with tick 2^b <= dt, by direct comparison."""
    b = np.zeros(dt.shape, dtype=np.int64)
    for k in range(1, levels + 1):
        b[np.ldexp(tick, k) <= dt] = k
    return b


def test_hierarchy_invariants():
    """Two full cycles on random states over five levels, each point
    checked against the definitions: active cells are those whose step
    ends now; an active cell's new bin never exceeds its criterion's bin,
    rises by one at most and only where the higher bin starts a step, and
    takes the criterion's bin otherwise; the next point is the earliest end
    of any cell's step; a face is active exactly when one of its cells is;
    every face of an active cell has been integrated exactly up to now; each
    side of an active face is predicted over the time since that cell last
    became active plus half the face's step; totals are conserved."""
    rng = np.random.default_rng(802)
    mesh = build_mesh(poisson_points(1000, 3, rng))
    g, cfl, L = 5.0 / 3.0, 0.4, 5
    rho, vel, P = random_states(mesh.n_cells, 3, g, rng)
    Q = conserved_from_primitive(mesh.volume, rho, 0.5 * vel, P, g)
    tot0 = Q.sum(axis=1)
    tl = timeline_for(mesh, g, cfl, Q, L, spread=0.25)
    tick = tl.tick
    n, nf = mesh.n_cells, mesh.n_faces
    fL, fR = mesh.face_L, mesh.face_R
    cum = np.zeros(nf, dtype=np.int64)     # integrated ticks per face
    last = np.zeros(n, dtype=np.int64)
    seen_up = seen_down = False
    occupied = set()
    while tl.ti < 2 * 2 ** L:
        ti = tl.ti
        ends = tl.trec + (np.int64(1) << tl.bin.astype(np.int64))
        old = tl.bin.astype(np.int64)
        r = tl.step(Q)
        assert r["status"] == 0
        act = r["active"]
        assert np.array_equal(act, (ends == ti) | (ti == 0))
        last[act] = ti
        new = tl.bin.astype(np.int64)
        assert np.array_equal(new[~act], old[~act])
        bc = bin_of(O.tb_criterion(mesh, g, cfl, tl.W), tick, L)
        a = act
        assert np.all(new[a] <= bc[a])
        assert np.all(new[a] <= old[a] + 1)
        up = a & (new > old)
        assert np.all(ti % (np.int64(1) << new[up]) == 0)
        stay = a & ~up
        assert np.all((new[stay] == bc[stay]) | ((ti % (np.int64(1) << (old[stay] + 1))) != 0))
        seen_up |= bool(up.any())
        seen_down |= bool((a & (new < old)).any())
        occupied |= set(np.unique(new).tolist())
        assert r["next"] == (tl.trec + (np.int64(1) << new)).min()
        fa = r["face_dt"] > 0
        assert np.array_equal(fa, act[fL] | act[fR])
        assert np.all(cum[fa] == ti)
        bmin = np.minimum(new[fL], new[fR])
        assert np.array_equal(r["face_dt"][fa], np.ldexp(tick, bmin[fa]))
        for s, side in enumerate((fL, fR)):
            want = (ti - last[side[fa]]) * tick + 0.5 * r["face_dt"][fa]
            assert np.array_equal(r["pred"][s][fa], want)
        steps = r["face_dt"] / tick
        assert np.array_equal(steps, np.round(steps))
        cum += steps.astype(np.int64)
    assert np.all(cum == 2 * 2 ** L)
    assert seen_up and seen_down and len(occupied) >= 3
    assert np.allclose(Q.sum(axis=1), tot0, rtol=0, atol=1e-13 * np.abs(Q).sum())


def test_static_contact_stays_exact():
    """A density contrast at rest in pressure equilibrium is an exact
    steady state: with four occupied bins, after a full cycle the
    velocities are zero and the densities and pressures unchanged, to
    round-off."""
    rng = np.random.default_rng(806)
    mesh = build_mesh(poisson_points(800, 2, rng))
    g = 5.0 / 3.0
    x, y = mesh.positions.T
    rho = 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    Q = conserved_from_primitive(mesh.volume, rho, np.zeros((2, mesh.n_cells)), np.ones(mesh.n_cells), g)
    tl = timeline_for(mesh, g, 0.4, Q, 4)
    while tl.ti < 16:
        assert tl.step(Q)["status"] == 0
    assert len(np.unique(tl.bin)) >= 3
    W = O.prim(2, g, mesh.volume, Q)
    assert np.abs(W[1:3]).max() < 1e-13
    assert np.allclose(W[0], rho, rtol=1e-13, atol=0) and np.allclose(W[3], 1.0, rtol=1e-12, atol=0)


def test_uniform_flow_at_full_synchronisation():
    """A uniform flow stays uniform only if every face of every cell has
    been integrated over the same time: midway through a cycle with several
    bins it is not (faces of one cell have different steps), at the end of
    the cycle it is, to round-off."""
    rng = np.random.default_rng(804)
    mesh = build_mesh(poisson_points(1200, 3, rng))
    g = 5.0 / 3.0
    n = mesh.n_cells
    v0 = np.array([0.7, -0.3, 0.2])
    Q = conserved_from_primitive(mesh.volume, np.full(n, 1.2), np.tile(v0[:, None], (1, n)), np.full(n, 0.9), g)
    tl = timeline_for(mesh, g, 0.4, Q, 3)
    midway = None
    while tl.ti < 8:
        assert tl.step(Q)["status"] == 0
        if tl.ti == 4:
            midway = np.abs(O.prim(3, g, mesh.volume, Q)[1] - v0[0]).max()
    assert len(np.unique(tl.bin)) >= 2
    assert midway > 1e-6
    W = O.prim(3, g, mesh.volume, Q)
    assert np.allclose(W[0], 1.2, rtol=1e-13, atol=0) and np.allclose(W[4], 0.9, rtol=1e-12, atol=0)
    for k in range(3):
        assert np.allclose(W[1 + k], v0[k], rtol=0, atol=1e-13)


def test_blast_against_the_global_step():
    """Sedov blast on a 16^3 lattice to t = 0.06 with four levels below
    dt_max (Section 8's point explosion): the shell radius is within 2% of
    the run with a global step at the smallest criterion, with at least
    three times fewer flux computations (the paper reports 4.3 for its 2D
    case), and mass and energy are conserved to round-off."""
    wl = sedov3d(n_side=16, seed=4104)
    m, g = wl.mesh, wl.gamma
    Q, t, nfg = wl.Q.copy(), 0.0, 0
    while t < 0.06:
        dt = min(O.tb_criterion(m, g, wl.cfl, O.prim(3, g, m.volume, Q)).min(), 0.06 - t)
        Q, _ = O.hydro_step(m, g, wl.cfl, Q, dt)
        t += dt
        nfg += m.n_faces
    Rg, _ = blast_radius(m, O.prim(3, g, m.volume, Q)[0])
    tl = timeline_for(m, g, wl.cfl, wl.Q, 4)
    Qi, nfi = wl.Q.copy(), 0
    while tl.time < 0.06:
        r = tl.step(Qi)
        assert r["status"] == 0
        nfi += r["n_faces"]
    Ri, peak = blast_radius(m, O.prim(3, g, m.volume, Qi)[0])
    Rs = Rg * (tl.time / 0.06) ** 0.4       # the similarity scaling to the timeline's end
    assert abs(Ri / Rs - 1.0) < 0.02, (Ri, Rs)
    assert nfg / nfi >= 3.0
    assert abs(Qi[0].sum() - wl.Q[0].sum()) <= 1e-13 * wl.Q[0].sum()
    assert abs(Qi[4].sum() - wl.Q[4].sum()) <= 1e-12 * wl.Q[4].sum()


def test_criterion_below_one_tick_is_an_error():
    """A cell whose criterion is below the smallest step fits no bin: the
    point reports it and leaves Q untouched."""
    wl = random3d(n_side=8, seed=805)
    m, g = wl.mesh, wl.gamma
    dmin = O.tb_criterion(m, g, wl.cfl, O.prim(3, g, m.volume, wl.Q)).min()
    tl = O.Timeline(m, g, wl.cfl, 4.0 * dmin, 1)
    Q = wl.Q.copy()
    r = tl.step(Q)
    assert r["status"] == 1 and tl.ti == 0
    assert np.array_equal(Q, wl.Q)
