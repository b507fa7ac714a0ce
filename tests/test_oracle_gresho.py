"""Pin of the moving-mesh scheme's Galilean invariance over many steps: the
Gresho vortex of Section 8.5 (rho = 1, gamma = 5/3, the piecewise
rotation and pressure profiles in equilibrium, 40^2 generators), run with
generators moving at the fluid velocity plus the roundness correction and
the tessellation rebuilt each step. With a uniform boost of 1 or 3 added,
the L1 error of the azimuthal velocity against the equilibrium profile,
measured in the boosted frame about the carried centre, is the same as
unboosted to 1e-9 (the paper: independent of the boost to machine
precision), while on a fixed mesh the boost raises it by a fifth (0.0089
to 0.0107)."""
import numpy as np

from oracle import oracle as O
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import conserved_from_primitive

GAMMA = 5.0 / 3.0


def profile(r):
    """Equilibrium azimuthal velocity and pressure of the vortex."""
    vphi = np.where(r < 0.2, 5 * r, np.where(r < 0.4, 2 - 5 * r, 0.0))
    P = np.where(r < 0.2, 5 + 12.5 * r ** 2,
                 np.where(r < 0.4, 9 + 12.5 * r ** 2 - 20 * r + 4 * np.log(np.maximum(5 * r, 1e-300)),
                          3 + 4 * np.log(2.0)))
    return vphi, P


def initial(nx, boost):
    h = 1.0 / nx
    xs = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    p = np.stack([X.ravel(), Y.ravel()], axis=1)
    d = p - 0.5
    r = np.hypot(d[:, 0], d[:, 1])
    vphi, P = profile(r)
    rs = np.maximum(r, 1e-300)
    vel = np.stack([-vphi * d[:, 1] / rs + boost, vphi * d[:, 0] / rs])
    mesh = build_mesh(p)
    return p, conserved_from_primitive(mesh.volume, np.ones(len(r)), vel, P, GAMMA)


def l1_vphi(mesh, Q, boost, t):
    W = O.prim(2, GAMMA, mesh.volume, Q)
    c = np.array([0.5 + boost * t, 0.5])
    d = np.mod(mesh.positions + mesh.centroid_off.T, 1.0) - c
    d -= np.round(d)
    r = np.hypot(d[:, 0], d[:, 1])
    vphi, _ = profile(r)
    vx = W[1] - boost
    return float(np.mean(np.abs((-vx * d[:, 1] + W[2] * d[:, 0]) / np.maximum(r, 1e-300) - vphi)))


def evolve(nx, boost, t_end, moving=True, step=None):
    """Runs to t_end; `step(mesh, Q, dt)` -> (Q, w) replaces the oracle's
    mesh velocity and step. Returns the L1 error and the step count."""
    p, Q = initial(nx, boost)
    t, k = 0.0, 0
    while t < t_end - 1e-14:
        mesh = build_mesh(p)
        W = O.prim(2, GAMMA, mesh.volume, Q)
        w = O.mesh_velocity(mesh, GAMMA, W) if moving else np.zeros((2, len(p)))
        mesh.with_velocity(np.ascontiguousarray(w))
        dt = min(O.cfl_dt(mesh, GAMMA, 0.4, W), t_end - t)
        if step is None:
            Q = O.hydro_step(mesh, GAMMA, 0.4, Q, dt=dt)[0]
        else:
            Q, w = step(mesh, Q, dt)
        p = np.mod(p + w.T * dt, 1.0)
        t += dt
        k += 1
    return l1_vphi(build_mesh(p), Q, boost, t_end), k


def test_boost_leaves_the_moving_mesh_error_unchanged():
    base, k = evolve(40, 0.0, 0.3)
    assert k > 150 and 1e-3 < base < 0.05
    for boost in (1.0, 3.0):
        l1, _ = evolve(40, boost, 0.3)
        assert abs(l1 / base - 1.0) < 1e-9, (boost, l1, base)


def test_boost_raises_the_fixed_mesh_error():
    base, _ = evolve(40, 0.0, 0.3, moving=False)
    l1, _ = evolve(40, 1.0, 0.3, moving=False)
    assert l1 > 1.1 * base, (l1, base)      # 0.0107 against 0.0089


def test_moving_mesh_error_falls_at_the_papers_rate():
    """The paper finds the moving-mesh L1 error of the vortex falling as
    N^-1.4 (N cells per dimension). To t = 0.3 it is 0.0106 on 40^2 and
    0.0041 on 80^2: a factor 2.61, N^-1.38 (from 20^2, where the vortex's
    inner ring spans four cells, the factor is only 1.96)."""
    l1_40, _ = evolve(40, 0.0, 0.3)
    l1_80, _ = evolve(80, 0.0, 0.3)
    assert 2.3 < l1_40 / l1_80 < 3.0, (l1_40, l1_80)
