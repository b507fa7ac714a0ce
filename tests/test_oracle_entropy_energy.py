"""Pins of the oracle's energy switch of the entropy scheme (Section 3.5,
eqs. eqnScrit1 and eqnScrit2): a cell keeps its advected entropy when its
expected new thermal energy is below alpha_s times the largest kinetic
energy of the cell and its neighbours, measured in the frame of the cell's
generator, or below beta_s M |g| R.

Pinned against: the plain scheme when both conditions are off (bit for
bit); the cold supersonic flow the scheme exists for; closed forms of the
decisions in a shear layer on a Cartesian lattice, with the mesh at rest
and moving with the stream (the frame of the kinetic energies); the
gravity condition's threshold on the cell radius in free fall."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import conserved_from_primitive, poisson_points, random_states, total_entropy
from tests.test_oracle_entropy import cold_flow, lattice_2d


def with_s(mesh, Q, g):
    W = O.prim(mesh.dim, g, mesh.volume, Q)
    return np.concatenate([Q, total_entropy(mesh.volume, W[0], W[-1], g)[None]])


def test_switch_off_is_the_plain_scheme():
    """alpha_s = beta_s = 0: no cell keeps, and the step equals the Mach
    switch with a threshold no face falls below, bit for bit."""
    rng = np.random.default_rng(901)
    mesh = build_mesh(poisson_points(1500, 3, rng))
    g = 5.0 / 3.0
    rho, vel, P = random_states(mesh.n_cells, 3, g, rng)
    Q = with_s(mesh, conserved_from_primitive(mesh.volume, rho, vel, P, g), g)
    Qa, dt, kept = O.hydro_step_energy(mesh, g, 0.4, Q, 0.0, 0.0)
    Qm, _, keptm = O.hydro_step_entropy(mesh, g, 0.4, Q, 0.0, dt=dt)
    assert not kept.any() and not keptm.any()
    assert np.array_equal(Qa, Qm)


def test_cold_supersonic_flow_stays_adiabatic():
    """The cold flow at about 77 sound speeds over a fixed lattice: its
    thermal energy is about 3e-4 of its kinetic energy, so with alpha_s =
    0.01 every cell keeps its entropy and P / rho^gamma stays within 1e-5 of
    its initial value over 30 steps, while mass and momentum are conserved."""
    g = 5.0 / 3.0
    mesh, Qp, Qe = cold_flow(32, g)
    tot0 = Qe[:3].sum(axis=1)
    for _ in range(30):
        Qp, dt = O.hydro_step(mesh, g, 0.4, Qp)
        Qe, _, kept = O.hydro_step_energy(mesh, g, 0.4, Qe, 0.01, dt=dt)
        assert kept.all()
    We = O.prim(2, g, mesh.volume, Qe[:4])
    Ae = We[3] / We[0] ** g
    assert np.abs(Ae / 1e-4 - 1.0).max() < 1e-5
    assert np.allclose(Qe[:3].sum(axis=1), tot0, rtol=1e-13, atol=1e-13)


def shear_layer(n, u, moving):
    """rho = 1, P = 1 on an n x n Cartesian lattice; v_x = u on the rows
    with 1/4 <= y < 3/4, at rest elsewhere; the generators at rest, or all
    moving with the stream (w = u)."""
    g = 5.0 / 3.0
    mesh, x, h = lattice_2d(n)
    y = mesh.positions[:, 1]
    stream = (y >= 0.25) & (y < 0.75)
    vel = np.stack([np.where(stream, u, 0.0), np.zeros(mesh.n_cells)])
    Q = conserved_from_primitive(mesh.volume, np.ones(mesh.n_cells), vel, np.ones(mesh.n_cells), g)
    if moving:
        mesh.with_velocity(np.ascontiguousarray(np.stack([np.full(mesh.n_cells, u), np.zeros(mesh.n_cells)])))
    # rows next to the other phase (across the two interfaces, periodic in y)
    edge = (np.abs(y - 0.25) < h) | (np.abs(y - 0.75) < h)
    return mesh, with_s(mesh, Q, g), stream, edge, g


@pytest.mark.parametrize("moving", [False, True])
def test_shear_layer_decisions(moving):
    """A tangential discontinuity at rest in pressure: the step leaves every
    thermal energy at P V/(gamma-1) = 1.5 V, and the kinetic energy in a
    cell's frame is 0 or u^2 V/2 = 2 V (u = 2). With the mesh at rest the
    stream cells and the rest cells next to the stream see 2 V; with the
    mesh moving with the stream, the rest cells and the stream cells next to
    them do. alpha_s = 1 keeps exactly those cells (1.5 < 2), alpha_s = 0.5
    none."""
    mesh, Q, stream, edge, g = shear_layer(16, 2.0, moving)
    hot = (~stream | edge) if moving else (stream | edge)
    _, dt, kept = O.hydro_step_energy(mesh, g, 0.4, Q, 1.0)
    W = O.prim(2, g, mesh.volume, O.hydro_step(mesh, g, 0.4, Q[:4], dt=dt)[0])
    assert np.allclose(W[3], 1.0, rtol=1e-12)
    assert hot.sum() not in (0, mesh.n_cells)
    assert np.array_equal(kept.astype(bool), hot)
    _, _, none = O.hydro_step_energy(mesh, g, 0.4, Q, 0.5, dt=dt)
    assert not none.any()


def test_gravity_condition_threshold():
    """A uniform state at rest in a uniform field (free fall keeps its
    thermal energy, 1.5 V for P = 1): with alpha_s off, eqnScrit2 keeps the
    cells with 1.5 V < beta_s M |g| R, i.e. R > 1.5 / (beta_s |g|) for
    rho = 1, with R the radius of the cell's area. beta_s is set so that the
    median radius is the threshold; cells within 1e-6 of it are not judged."""
    rng = np.random.default_rng(902)
    mesh = build_mesh(poisson_points(800, 2, rng))
    g = 5.0 / 3.0
    n = mesh.n_cells
    Q = with_s(mesh, conserved_from_primitive(mesh.volume, np.ones(n), np.zeros((2, n)), np.ones(n), g), g)
    gvec = np.array([0.3, -0.4])                       # |g| = 0.5
    acc = np.ascontiguousarray(np.tile(gvec[:, None], (1, n)))
    R = np.sqrt(mesh.volume / np.pi)
    Rs = np.median(R)
    beta = 1.5 / (0.5 * Rs)
    _, _, kept = O.hydro_step_energy(mesh, g, 0.4, Q, 0.0, beta, accel=acc)
    judged = np.abs(R / Rs - 1.0) > 1e-6
    assert np.array_equal(kept.astype(bool)[judged], (R > Rs)[judged])
    assert 0.4 < kept.mean() < 0.6
    # no field, no gravity condition
    _, _, none = O.hydro_step_energy(mesh, g, 0.4, Q, 0.0, beta)
    assert not none.any()
