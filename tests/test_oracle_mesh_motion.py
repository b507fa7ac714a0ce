"""Pins of the oracle's mesh motion: the generator velocities with the
roundness correction of Section 4.1 (eq. EqnShapeCorrVel) and the cell
volume rate of eq. eqnvolchange (Section 3.3).

Pinned against: finite differences of the volumes of rebuilt
tessellations; the face-velocity form of the same rate; the periodic box's
constant volume; one Lloyd iteration (the paper describes the correction as
one, or a fraction of one); convergence of repeated Lloyd iterations
towards a centroidal tessellation; the shape of the correction."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import (conserved_from_primitive, jittered_lattice, poisson_points,
                                                random_states)


@pytest.mark.parametrize("dim", [2, 3])
def test_volume_rate_against_rebuilt_meshes(dim):
    """eq. eqnvolchange against central differences of the volumes of the
    tessellations of r +- w h; the rates of a periodic box sum to zero."""
    rng = np.random.default_rng(30 + dim)
    pts = jittered_lattice(12 if dim == 3 else 24, dim, 0.2, rng)
    w = rng.normal(size=pts.shape) * 0.5
    mesh = build_mesh(pts).with_velocity(np.ascontiguousarray(w.T))
    rate = O.volume_rate(mesh)
    h = 1e-6
    fd = (build_mesh(pts + h * w).volume - build_mesh(pts - h * w).volume) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(rate - fd).max() < 1e-4 * scale
    assert abs(rate.sum()) < 1e-12 * np.abs(rate).sum()
    # the same rate from the face velocities, sum_j A_ij w_f . n_ij
    wf = O.face_velocity(mesh)
    n = mesh.face_sep / np.sqrt(np.sum(mesh.face_sep ** 2, axis=0))
    flux = mesh.face_area * np.sum(wf * n, axis=0)
    alt = np.zeros(mesh.n_cells)
    np.add.at(alt, mesh.face_L, flux)
    np.add.at(alt, mesh.face_R, -flux)
    assert np.abs(rate - alt).max() < 1e-12 * scale


def state(mesh, dim, seed, still=False):
    rng = np.random.default_rng(seed)
    g = 5.0 / 3.0
    rho, vel, P = random_states(mesh.n_cells, dim, g, rng)
    if still:
        vel[:] = 0.0
    W = np.concatenate([rho[None], vel, P[None]])
    return W, g


def test_one_lloyd_iteration():
    """With the (s - r)/dt form, chi = 1, fluid at rest and every cell over
    the threshold, moving the generators by w dt puts each on its cell's
    centre of mass: one Lloyd iteration. Cells under the threshold stay."""
    dim = 2
    rng = np.random.default_rng(41)
    pts = poisson_points(600, dim, rng)
    mesh = build_mesh(pts)
    W, g = state(mesh, dim, 42, still=True)
    dt = 0.01
    w = O.mesh_velocity(mesh, g, W, eta=1e-9, chi=1.0, dt_lloyd=dt)
    assert np.allclose(w * dt, mesh.centroid_off, rtol=1e-14, atol=1e-16)
    # a large eta leaves every generator where it is
    w0 = O.mesh_velocity(mesh, g, W, eta=1e9, chi=1.0, dt_lloyd=dt)
    assert np.all(w0 == 0.0)


def test_lloyd_iterations_relax_the_mesh():
    """Repeated Lloyd iterations (Section 4.1) drive a Poisson mesh towards
    a centroidal tessellation: the mean offset of the generators from their
    centres of mass, in units of the cell radius, falls several times over
    ten iterations."""
    dim = 2
    rng = np.random.default_rng(43)
    pts = poisson_points(800, dim, rng)

    def offset(mesh):
        d = np.sqrt(np.sum(mesh.centroid_off ** 2, axis=0))
        return float(np.mean(d / np.sqrt(mesh.volume / np.pi)))
    mesh = build_mesh(pts)
    first = offset(mesh)
    for _ in range(10):
        W, g = state(mesh, dim, 44, still=True)
        w = O.mesh_velocity(mesh, g, W, eta=1e-9, chi=1.0, dt_lloyd=1.0)
        pts = np.mod(mesh.positions + w.T, 1.0)
        mesh = build_mesh(pts)
    assert offset(mesh) < first / 3


@pytest.mark.parametrize("dim", [2, 3])
def test_sound_speed_correction_shape(dim):
    """The added velocity points from the generator to the centre of mass,
    vanishes below 0.9 eta R, has magnitude chi c_s above 1.1 eta R, and
    grows with the offset in between; a centroidal lattice gets none."""
    rng = np.random.default_rng(50 + dim)
    mesh = build_mesh(jittered_lattice(10 if dim == 3 else 24, dim, 0.25, rng))
    W, g = state(mesh, dim, 51)
    eta, chi = 0.08, 0.7
    w = O.mesh_velocity(mesh, g, W, eta=eta, chi=chi)
    extra = w - W[1:1 + dim]
    sr = mesh.centroid_off
    d = np.sqrt(np.sum(sr ** 2, axis=0))
    R = (3 * mesh.volume / (4 * np.pi)) ** (1 / 3) if dim == 3 else np.sqrt(mesh.volume / np.pi)
    x = d / (eta * R)
    c = np.sqrt(g * W[-1] / W[0])
    mag = np.sqrt(np.sum(extra ** 2, axis=0))
    lo, mid, hi = x < 0.9, (x >= 0.9) & (x < 1.1), x >= 1.1
    assert lo.any() and mid.any() and hi.any()
    assert np.all(mag[lo] == 0.0)
    assert np.allclose(mag[hi], chi * c[hi], rtol=1e-13)
    assert np.all((mag[mid] > 0) & (mag[mid] < chi * c[mid]))
    cosang = np.sum(extra[:, ~lo] * sr[:, ~lo], axis=0) / (mag[~lo] * d[~lo])
    assert np.allclose(cosang, 1.0, rtol=0, atol=1e-13)
    order = np.argsort(x[mid])                    # monotone in the offset
    assert np.all(np.diff((mag / (chi * c))[mid][order]) >= -1e-13)
    # a Cartesian lattice is centroidal: no correction
    n = 16
    xs = (np.arange(n) + 0.5) / n
    grid = np.stack(np.meshgrid(*([xs] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    lat = build_mesh(grid)
    Wl, _ = state(lat, dim, 52)
    assert np.array_equal(O.mesh_velocity(lat, g, Wl, eta=eta, chi=chi), Wl[1:1 + dim])
