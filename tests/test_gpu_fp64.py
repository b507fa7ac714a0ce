"""Parity of the double-precision HIP path (through the C ABI) with the CPU
oracle, element by element on seeded inputs: primitives, limited gradients,
face fluxes, the update and the full step, on the 2D Kelvin-Helmholtz
workload (64x64, 50 moving-mesh steps) and the 3D random-state workload
(several tiles with a ragged tail, and the full 64^3 size), plus
conservation, determinism, Galilean invariance and mesh validation."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_0901_4107_amd import mm
from paper_0901_4107_amd.inputs import build_mesh
from paper_0901_4107_amd.inputs.configs import kh2d, random3d, sedov3d, conserved_from_primitive, poisson_points
from tests.util import assert_cell_rel, boost, normwise_rel, update_condition

pytestmark = pytest.mark.gpu

TOL = 1e-12  # norm-wise relative, per conserved / primitive component
# per cell, mass and energy: |got - want| / |want| <= CELL_TOL K_i, K_i the
# condition of the cell's update (its terms' size against its result)
CELL_TOL = 1e-12


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Run:
    """A context with the mesh uploaded, plus device copies of Q."""

    def __init__(self, wl, mode=mm.MM_FP64, **kw):
        self.wl = wl
        m = wl.mesh
        self.ctx = mm.Context(m.dim, wl.gamma, wl.cfl, mode=mode, **kw)
        self.dm = mm.DeviceMesh.from_host(m)
        self.ctx.mm_mesh_upload(self.dm)
        self.Q = torch.from_numpy(np.ascontiguousarray(wl.Q)).cuda()
        self.rec = self.ctx.recon_buffer(m.n_cells)
        self.F = self.ctx.flux_buffer(m.n_faces)

    def gradients(self):
        self.ctx.mm_gradients(self.Q, self.rec)
        torch.cuda.synchronize()
        W, G, dl = mm.split_recon(self.rec.cpu().numpy(), self.wl.mesh.dim)
        assert np.array_equal(dl, self.wl.mesh.centroid_off)
        return W, G

    def fluxes(self, dt):
        self.ctx.mm_face_fluxes(dt, self.rec, self.F)
        torch.cuda.synchronize()
        return self.F.cpu().numpy().T


def assert_close(got, want, tol, what, floor=None):
    """Per row: max |got - want| <= tol * max(max |want|, floor)."""
    den = np.max(np.abs(want), axis=1)
    if floor is not None:
        den = np.maximum(den, floor)
    den = np.where(den > 0, den, 1.0)
    err = np.max(np.abs(got - want), axis=1) / den
    assert np.all(err <= tol), f"{what}: normwise errors {err}"
    return err


def gradient_floor(mesh, W):
    """Scale of a gradient row (c, k): max |W_c| / h with h the smallest cell
    size. A gradient that is analytically zero (a uniform field, or a cell
    limited to alpha = 0) is a sum of face terms of this size that cancel,
    so its round-off is measured against it."""
    h = np.min(mesh.volume) ** (1.0 / mesh.dim)
    return np.repeat(np.max(np.abs(W), axis=1) / h, mesh.dim)


def check_one_step(wl, tol=TOL):
    m = wl.mesh
    note(f"parity one step: {wl.name} N={m.n_cells} F={m.n_faces}")
    r = Run(wl)
    W, G = r.gradients()
    Wo = O.prim(m.dim, wl.gamma, m.volume, wl.Q)
    raw, Go, alpha = O.gradients(m, Wo)
    assert_close(W, Wo, tol, "primitives")
    assert_close(G, Go, tol, "limited gradients", floor=gradient_floor(m, Wo))
    dt = O.cfl_dt(m, wl.gamma, wl.cfl, Wo)
    F = r.fluxes(dt)
    Fo, fb, kase = O.face_fluxes(m, wl.gamma, dt, Wo, Go)
    assert_close(F, Fo, tol, "face fluxes")
    r.ctx.mm_apply_update(r.F, r.Q)
    Qo = O.apply_update(m, Fo, wl.Q)
    assert_close(r.Q.cpu().numpy(), Qo, tol, "updated Q")
    # the full step with the Courant timestep, from the original state
    r.Q.copy_(torch.from_numpy(wl.Q))
    r.ctx.mm_reset_diag()
    used = r.ctx.mm_hydro_step(r.Q)
    Qs, dto = O.hydro_step(m, wl.gamma, wl.cfl, wl.Q)
    assert abs(used - dto) <= 1e-14 * dto
    Qg = r.Q.cpu().numpy()
    err = assert_close(Qg, Qs, tol, "hydro step")
    # mass and energy cell by cell (the normwise bound above lets a light
    # cell hide in the scale of a heavy one)
    me = (0, m.dim + 1)
    K = update_condition(m, wl.Q, Fo, Qs, me)
    cell = assert_cell_rel(Qg, Qs, K, me, CELL_TOL, "hydro step, m and E per cell")
    diag = r.ctx.mm_get_diag()
    note(f"  max normwise error {err.max():.2e}; per-cell relative m {cell[0]:.2e} E {cell[1]:.2e} "
         f"(largest K {K.max():.3g}); vacuum faces {int(np.sum(kase != 0))}, "
         f"fallbacks {int(fb.sum())}; diag {diag}")
    assert diag["vacuum"] == int(np.sum(kase != 0))
    assert diag["positivity_fallback"] == int(fb.sum())
    assert diag["unconverged"] == 0
    return r, Qs


def test_kh2d_one_step():
    check_one_step(kh2d())


@pytest.mark.parametrize("side", [13, 24])
def test_random3d_small(side):
    """Several tiles and a ragged tail (13^3 = 2197 cells, ~17k faces)."""
    check_one_step(random3d(n_side=side, seed=500 + side))


def test_sedov3d_small():
    """The point explosion (pressure ratio 1e7 at the hot cells) on a
    20^3 jittered lattice."""
    check_one_step(sedov3d(n_side=20, seed=777))


def test_random3d_full_64():
    """The 64^3 random-state workload at full size, element by element."""
    wl = random3d()
    r, _ = check_one_step(wl)
    d = r.ctx.mm_get_diag()
    assert d["vacuum"] > 0 and d["positivity_fallback"] > 0


def test_kh2d_50_moving_steps():
    """50 steps with the mesh rebuilt after each (points moved with w = v).
    Each step starts both sides from the same state and mesh and must agree
    to the parity bound; the state then advances with the oracle's result."""
    wl = kh2d()
    m = wl.mesh
    g, cfl = wl.gamma, wl.cfl
    Q = wl.Q.copy()
    pts = m.positions.copy()
    ctx = mm.Context(2, g, cfl)
    worst = 0.0
    for step in range(50):
        W = O.prim(2, g, m.volume, Q)
        m.with_velocity(np.ascontiguousarray(W[1:3]))
        dm = mm.DeviceMesh.from_host(m)
        ctx.mm_mesh_upload(dm)
        Qd = torch.from_numpy(Q).cuda()
        used = ctx.mm_hydro_step(Qd)
        Qo, dto = O.hydro_step(m, g, cfl, Q)
        assert abs(used - dto) <= 1e-14 * dto
        err = assert_close(Qd.cpu().numpy(), Qo, TOL, f"step {step}")
        worst = max(worst, float(err.max()))
        Q = Qo
        pts = np.mod(pts + dto * W[1:3].T, 1.0)
        m = build_mesh(pts)
    note(f"kh2d 50 steps: worst normwise error {worst:.2e}")


def test_determinism_and_conservation():
    wl = random3d(n_side=20, seed=77)
    a = Run(wl); b = Run(wl)
    a.ctx.mm_hydro_step(a.Q, dt=1e-4)
    b.ctx.mm_hydro_step(b.Q, dt=1e-4)
    qa, qb = a.Q.cpu().numpy(), b.Q.cpu().numpy()
    assert np.array_equal(qa, qb)
    scale = np.abs(wl.Q).sum(axis=1)
    assert np.all(np.abs(qa.sum(axis=1) - wl.Q.sum(axis=1)) <= 1e-13 * scale)


def test_galilean_invariance_gpu():
    wl = kh2d(n_side=32)
    v0 = np.array([5.0, -3.0])
    a = Run(wl)
    a.ctx.mm_hydro_step(a.Q, dt=2e-3)
    wl.Q = boost(wl.Q, v0)
    wl.mesh.with_velocity(wl.mesh.mesh_vel + v0[:, None])
    b = Run(wl)
    b.ctx.mm_hydro_step(b.Q, dt=2e-3)
    back = boost(b.Q.cpu().numpy(), -v0)
    assert np.all(normwise_rel(back, a.Q.cpu().numpy()) < 1e-11)


def test_vacuum_cells():
    """Cells with zero mass are vacuum: W = 0, no timestep limit, and the
    faces around them follow the vacuum branches of the solver."""
    rng = np.random.default_rng(3)
    mesh = build_mesh(poisson_points(3000, 3, rng))
    g = 5.0 / 3.0
    rho = rng.uniform(0.5, 2, mesh.n_cells); P = rng.uniform(0.5, 2, mesh.n_cells)
    vel = rng.normal(size=(3, mesh.n_cells))
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, g)
    Q[:, rng.choice(mesh.n_cells, 40, replace=False)] = 0.0
    from paper_0901_4107_amd.inputs.configs import Workload
    wl = Workload("vacuum", mesh, Q, g, 0.4, np.zeros(3), 3)
    r, _ = check_one_step(wl)
    assert r.ctx.mm_get_diag()["vacuum"] > 0


@pytest.mark.parametrize("mode", [mm.MM_FP64, mm.MM_MIXED])
def test_nonfinite_step_is_reported(mode):
    """A NaN in one cell's energy: the step runs to its end (every loop of
    the kernels is bounded) and reports MM_E_NONFINITE; the next step, on a
    finite state, reports nothing, while the diagnostics keep the event
    until they are reset."""
    wl = random3d(n_side=13, seed=91)
    r = Run(wl, mode=mode)
    bad = r.Q.clone()
    bad[4, 100] = float("nan")
    with pytest.raises(mm.MMError) as e:
        r.ctx.mm_hydro_step(bad)
    assert e.value.status == mm.MM_E_NONFINITE
    used = r.ctx.mm_hydro_step(r.Q)
    assert used > 0 and bool(torch.isfinite(r.Q).all())
    assert r.ctx.mm_get_diag()["nonfinite"] == 1
    r.ctx.mm_reset_diag()
    assert r.ctx.mm_get_diag()["nonfinite"] == 0


def test_invalid_meshes_are_rejected():
    rng = np.random.default_rng(4)
    mesh = build_mesh(poisson_points(500, 3, rng))
    ctx = mm.Context(3, 1.4)
    good = mm.DeviceMesh.from_host(mesh)
    ctx.mm_mesh_upload(good)
    last = mesh.n_faces - 1
    assert mesh.face_L[last] > 0
    for field, idx, val in [("face_L", 3, -1), ("face_R", 5, mesh.n_cells), ("face_R", 7, int(mesh.face_L[7])),
                            ("volume", 2, 0.0), ("face_area", 1, -1.0), ("face_sep", 4, float("nan")),
                            # faces no longer sorted by their left cell
                            ("face_L", last, 0),
                            # two cells no longer closed (the closure check after the side lists)
                            ("face_area", 6, 2.0 * float(mesh.face_area[6]))]:
        bad = mm.DeviceMesh.from_host(mesh)
        t = getattr(bad, field)
        t.view(-1)[idx] = val
        with pytest.raises(mm.MMError) as e:
            ctx.mm_mesh_upload(bad)
        assert e.value.status == mm.MM_E_MESH, field
    ctx.mm_mesh_upload(good)  # the context recovers
