"""Pins of the oracle's coupling to an external static gravitational field
(Section 5.2, the standard approach applied to a field given per cell):
the half-step prediction of the velocities gains (dt/2) g, and the update
adds (dt/2)(m^n + m^(n+1)) g to the momentum and (dt/2)(p^n + p^(n+1)).g
to the energy.

Pinned against: free fall of a uniform state (closed form v = v0 + g t,
density and pressure unchanged); second-order convergence of the residual
velocities of an isothermal atmosphere in hydrostatic equilibrium; the
exact balance of the total momentum and energy with the source terms."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import conserved_from_primitive, poisson_points, random_states


@pytest.mark.parametrize("moving", [False, True])
def test_free_fall(moving):
    """A uniform state in a uniform field accelerates as a whole: after
    eight steps v = v0 + g t to round-off, with density and pressure
    unchanged; the generators either rest or move with the initial
    velocity (Galilean frames of the same fall)."""
    rng = np.random.default_rng(70)
    mesh = build_mesh(poisson_points(1200, 3, rng))
    gam = 5.0 / 3.0
    n = mesh.n_cells
    v0 = np.array([0.2, -0.1, 0.05])
    gvec = np.array([0.3, -0.5, 0.1])
    rho, P = 1.3, 0.7
    Q = conserved_from_primitive(mesh.volume, np.full(n, rho), np.tile(v0[:, None], (1, n)), np.full(n, P), gam)
    if moving:
        mesh.with_velocity(np.ascontiguousarray(np.tile(v0[:, None], (1, n))))
    acc = np.ascontiguousarray(np.tile(gvec[:, None], (1, n)))
    t = 0.0
    for _ in range(8):
        Q, dt, _ = O.hydro_step_full(mesh, gam, 0.4, Q, accel=acc)
        t += dt
    W = O.prim(3, gam, mesh.volume, Q)
    assert np.allclose(W[0], rho, rtol=1e-13, atol=0)
    assert np.allclose(W[4], P, rtol=1e-11, atol=0)
    for k in range(3):
        assert np.allclose(W[1 + k], v0[k] + gvec[k] * t, rtol=1e-12, atol=1e-14)


def atmosphere(n, g0=0.5, c2=1.0, gam=5.0 / 3.0):
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    mesh = build_mesh(np.stack([X.ravel(), Y.ravel()], axis=1))
    x = X.ravel()
    phi = -(g0 / (2 * np.pi)) * np.cos(2 * np.pi * x)   # Phi, with g = -dPhi/dx
    rho = np.exp(-phi / c2)                              # isothermal: P = rho c^2, dP/dx = rho g
    acc = np.ascontiguousarray(np.stack([-g0 * np.sin(2 * np.pi * x), np.zeros(mesh.n_cells)]))
    Q = conserved_from_primitive(mesh.volume, rho, np.zeros((2, mesh.n_cells)), rho * c2, gam)
    return mesh, Q, acc


def test_hydrostatic_atmosphere_converges_at_second_order():
    """An isothermal atmosphere in the periodic potential
    Phi = -(g0/2pi) cos(2 pi x) is in equilibrium: rho ~ exp(-Phi/c^2). On
    Cartesian lattices of 16^2 and 32^2 cells run to t = 0.2, the residual
    velocities are below 2e-3 c and fall by a factor of at least 3.5 when
    the spacing halves (second order)."""
    gam = 5.0 / 3.0
    res = []
    for n in (16, 32):
        mesh, Q, acc = atmosphere(n, gam=gam)
        t = 0.0
        while t < 0.2:
            W = O.prim(2, gam, mesh.volume, Q)
            dt = min(O.cfl_dt(mesh, gam, 0.4, W), 0.2 - t)
            Q, used, _ = O.hydro_step_full(mesh, gam, 0.4, Q, dt=dt, accel=acc)
            t += used
        res.append(np.abs(O.prim(2, gam, mesh.volume, Q)[1:3]).max())
    assert res[0] < 2e-3 and res[0] / res[1] > 3.5, res


def test_source_terms_balance_the_totals():
    """Random states and a random smooth field: the fluxes cancel in the
    totals, so the total momentum changes by sum (dt/2)(m^n + m^(n+1)) g
    and the total energy by sum (dt/2)(p^n + p^(n+1)).g, to round-off."""
    rng = np.random.default_rng(71)
    mesh = build_mesh(poisson_points(1500, 3, rng))
    gam = 5.0 / 3.0
    rho, vel, P = random_states(mesh.n_cells, 3, gam, rng)
    Q = conserved_from_primitive(mesh.volume, rho, 0.3 * vel, P, gam)
    pos = mesh.positions.T
    acc = np.ascontiguousarray(np.stack([np.sin(2 * np.pi * pos[1]), np.cos(2 * np.pi * pos[2]),
                                         0.5 * np.sin(2 * np.pi * pos[0])]))
    Qn, dt, _ = O.hydro_step_full(mesh, gam, 0.4, Q, accel=acc)
    Qh, _ = O.hydro_step(mesh, gam, 0.4, Q, dt=dt)
    assert not np.array_equal(Qn, Qh)
    mom = 0.5 * dt * (Q[0] + Qn[0])[None] * acc
    assert np.allclose(Qn[1:4].sum(axis=1) - Q[1:4].sum(axis=1), mom.sum(axis=1),
                       rtol=1e-10, atol=1e-13 * np.abs(Q[1:4]).sum())
    work = 0.5 * dt * np.sum((Q[1:4] + Qn[1:4]) * acc, axis=0)
    assert abs((Qn[4].sum() - Q[4].sum()) - work.sum()) <= 1e-12 * np.abs(Q[4]).sum()
    assert abs(Qn[0].sum() - Q[0].sum()) <= 1e-13 * Q[0].sum()
