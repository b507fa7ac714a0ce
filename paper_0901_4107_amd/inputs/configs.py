"""Seeded synthetic workloads with the shapes of the paper's test problems.

Every workload is a periodic unit box tessellated by :func:`build_mesh`, with
cells in Morton order and faces sorted by their left cell. Fluid states are
set from primitive fields evaluated at each cell's centre of mass and turned
into cell totals ``Q = (m, p, E)`` with ``m = rho V``, ``p = m v`` and
``E = P V/(gamma-1) + m |v|^2/2`` (the definition of the state vector and the
ideal-gas law, Section 3). Nothing here evaluates any step of the scheme.

Workloads
  kh2d       2D Kelvin-Helmholtz (Section 8.7), 64x64 jittered lattice.
  random3d   3D random states on a 64^3 jittered lattice (log-uniform density
             and pressure, Gaussian velocities of three sound speeds), fixed
             mesh; stresses the Riemann solver.
  kh3d       3D Kelvin-Helmholtz shear layer on Poisson points with a uniform
             bulk boost and a comoving mesh (Galilean-invariance workload).
  sedov3d    3D Sedov-Taylor blast on a jittered lattice (Section 8.4).
  rt3d       3D single-mode Rayleigh-Taylor setup (Section 8.8) between two
             reflective walls in a static field, on a jittered lattice.
  riemann_problems
             independent 1D Riemann problems drawn from histograms of the
             problems that runs of random3d, kh3d and sedov3d pose (a data
             file produced offline), plus hard tails.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from .mesh import Mesh, build_mesh, morton_order


@dataclass
class Workload:
    name: str
    mesh: Mesh
    Q: np.ndarray          # [D+2][N] conserved cell totals
    gamma: float
    cfl: float
    boost: np.ndarray      # [D] uniform bulk velocity added to the flow (zeros if none)
    seed: int
    prim: tuple = None     # (rho [N], vel [D][N], P [N]) the initial primitive fields
    walls: "Walls" = None  # reflective walls (mirror cells), if any
    accel: np.ndarray = None   # [D][N] static field, if any

    @property
    def dim(self) -> int:
        return self.mesh.dim


def conserved_from_primitive(volume, rho, vel, P, gamma):
    """Cell totals from primitive values: m = rho V, p = m v, E = P V/(g-1) + m v^2/2."""
    m = rho * volume
    p = m[None, :] * vel
    E = P * volume / (gamma - 1.0) + 0.5 * m * np.sum(vel * vel, axis=0)
    return np.ascontiguousarray(np.concatenate([m[None], p, E[None]], axis=0))


def total_entropy(volume, rho, P, gamma):
    """Total entropy of a cell, S = M A with M = rho V and the entropic
    function A = P / rho^gamma (the definition of Section 3.5)."""
    return rho * volume * P / rho ** gamma


def with_entropy(wl: "Workload") -> np.ndarray:
    """The workload's conserved state with the total entropy appended as the
    last row, [D+3][N], from its initial primitive fields."""
    rho, _, P = wl.prim
    return np.ascontiguousarray(np.concatenate([wl.Q, total_entropy(wl.mesh.volume, rho, P, wl.gamma)[None]]))


def jittered_lattice(n_side: int, dim: int, jitter: float, rng) -> np.ndarray:
    """Lattice points (i+1/2)/n with each coordinate displaced by
    U(-jitter, +jitter) lattice spacings, in Morton order."""
    h = 1.0 / n_side
    axes = [(np.arange(n_side) + 0.5) * h] * dim
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, dim)
    grid = grid + rng.uniform(-jitter, jitter, size=grid.shape) * h
    grid = np.mod(grid, 1.0)
    return grid[morton_order(grid)]


def poisson_points(n: int, dim: int, rng) -> np.ndarray:
    pts = rng.random((n, dim))
    return pts[morton_order(pts)]


def _centres(mesh: Mesh) -> np.ndarray:
    return np.mod(mesh.positions.T + mesh.centroid_off, 1.0)   # [D][N]


def kh2d(n_side: int = 64, jitter: float = 0.05, seed: int = 1000, nthreads: int = 0) -> Workload:
    """2D KH: rho = 2 for |y-1/2| < 1/4 else 1, P = 2.5, v_x = +-0.5 (inside /
    outside), v_y = w0 sin(4 pi x)[exp(-(y-1/4)^2/(2 s^2)) + exp(-(y-3/4)^2/(2 s^2))]
    with w0 = 0.1, 2 s^2 = 0.005; gamma = 5/3. Mesh moves with the flow."""
    rng = np.random.default_rng(seed)
    gamma = 5.0 / 3.0
    mesh = build_mesh(jittered_lattice(n_side, 2, jitter, rng), nthreads)
    x, y = _centres(mesh)
    inside = np.abs(y - 0.5) < 0.25
    rho = np.where(inside, 2.0, 1.0)
    P = np.full_like(rho, 2.5)
    vx = np.where(inside, 0.5, -0.5)
    vy = 0.1 * np.sin(4 * np.pi * x) * (np.exp(-(y - 0.25) ** 2 / 0.005) + np.exp(-(y - 0.75) ** 2 / 0.005))
    vel = np.stack([vx, vy])
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, gamma)
    mesh.with_velocity(vel.copy())
    return Workload("kh2d_64x64", mesh, Q, gamma, 0.4, np.zeros(2), seed, (rho, vel, P))


def random_states(n: int, dim: int, gamma: float, rng):
    """log10 rho, log10 P ~ U(-2, 2); each velocity component ~ N(0, (3 c)^2)
    with c the cell's own sound speed sqrt(gamma P / rho)."""
    rho = 10.0 ** rng.uniform(-2.0, 2.0, n)
    P = 10.0 ** rng.uniform(-2.0, 2.0, n)
    c = np.sqrt(gamma * P / rho)
    vel = rng.normal(0.0, 1.0, (dim, n)) * (3.0 * c)[None, :]
    return rho, vel, P


def random3d(n_side: int = 64, jitter: float = 0.1, seed: int = 1001, nthreads: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    gamma = 5.0 / 3.0
    mesh = build_mesh(jittered_lattice(n_side, 3, jitter, rng), nthreads)
    rho, vel, P = random_states(mesh.n_cells, 3, gamma, rng)
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, gamma)
    return Workload(f"random3d_{n_side}^3", mesh, Q, gamma, 0.4, np.zeros(3), seed, (rho, vel, P))


def kh3d(n_points: int = 128 ** 3, seed: int = 1002, boost_mach: float = 10.0,
         nthreads: int = 0, points: np.ndarray | None = None) -> Workload:
    """3D KH: the 2D profile of the paper's KH test extended uniformly in z,
    on Poisson points, plus a bulk boost v0 = (boost_mach * c, 0, 0) with c
    the sound speed of the lighter phase (sqrt(gamma 2.5 / 1)); the mesh moves
    with the (boosted) flow."""
    rng = np.random.default_rng(seed)
    gamma = 5.0 / 3.0
    pts = poisson_points(n_points, 3, rng) if points is None else points
    mesh = build_mesh(pts, nthreads)
    x, y, _ = _centres(mesh)
    inside = np.abs(y - 0.5) < 0.25
    rho = np.where(inside, 2.0, 1.0)
    P = np.full_like(rho, 2.5)
    vx = np.where(inside, 0.5, -0.5)
    vy = 0.1 * np.sin(4 * np.pi * x) * (np.exp(-(y - 0.25) ** 2 / 0.005) + np.exp(-(y - 0.75) ** 2 / 0.005))
    c_light = np.sqrt(gamma * 2.5 / 1.0)
    boost = np.array([boost_mach * c_light, 0.0, 0.0])
    vel = np.stack([vx, vy, np.zeros_like(vx)]) + boost[:, None]
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, gamma)
    mesh.with_velocity(vel.copy())
    return Workload(f"kh3d_poisson_{n_points}", mesh, Q, gamma, 0.4, boost, seed, (rho, vel, P))


def sedov3d(n_side: int = 256, jitter: float = 0.1, seed: int = 1004, n_hot: int = 32,
            energy: float = 1.0, nthreads: int = 0) -> Workload:
    """Sedov blast: rho = 1, P = 1e-5, v = 0, with total energy `energy` added
    as thermal energy in equal parts to the n_hot cells whose generators lie
    nearest the box centre (ties to the lower index). Mesh moves with the
    flow (zero at the start)."""
    rng = np.random.default_rng(seed)
    gamma = 5.0 / 3.0
    mesh = build_mesh(jittered_lattice(n_side, 3, jitter, rng), nthreads)
    n = mesh.n_cells
    rho = np.ones(n)
    P = np.full(n, 1e-5)
    vel = np.zeros((3, n))
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, gamma)
    r2 = np.sum((mesh.positions - 0.5) ** 2, axis=1)
    hot = np.lexsort((np.arange(n), r2))[:n_hot]
    Q[4, hot] += energy / n_hot
    P[hot] += (gamma - 1.0) * (energy / n_hot) / mesh.volume[hot]   # the added thermal energy
    mesh.with_velocity(vel.copy())
    return Workload(f"sedov3d_{n_side}^3", mesh, Q, gamma, 0.4, np.zeros(3), seed, (rho, vel, P))


def riemann_tails(n: int, gamma: float, rng) -> np.ndarray:
    """Hard-tail Riemann problems [6][n] (rho_L, u_L, P_L, rho_R, u_R, P_R):
    half near vacuum (velocity jump 80-99.5% of the vacuum threshold
    2 (c_L + c_R)/(g-1)), half strong shocks (pressure ratios 1e2-1e6 in
    either order, colliding flows)."""
    h = n // 2
    rho = 10 ** rng.uniform(-2, 2, (2, n))
    P = 10 ** rng.uniform(-2, 2, (2, n))
    c = np.sqrt(gamma * P / rho)
    u = np.zeros((2, n))
    thr = 2 * (c[0] + c[1]) / (gamma - 1)
    jump = rng.uniform(0.8, 0.995, h) * thr[:h]
    u[0, :h] = -0.5 * jump
    u[1, :h] = 0.5 * jump
    ratio = 10 ** rng.uniform(2, 6, n - h) * rng.choice([-1, 1], n - h)
    P[1, h:] = np.where(ratio > 0, P[0, h:] * np.abs(ratio), P[0, h:] / np.abs(ratio))
    c = np.sqrt(gamma * P / rho)
    coll = rng.uniform(0, 3, n - h) * (c[0, h:] + c[1, h:])
    u[0, h:] = 0.5 * coll
    u[1, h:] = -0.5 * coll
    return np.stack([rho[0], u[0], P[0], rho[1], u[1], P[1]])


HARVEST = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "data", "riemann_harvest.npz")
HARVEST_SOURCES = ("random3d", "kh3d", "sedov3d")


def load_harvest(path: str = HARVEST) -> dict:
    """Histograms of the face-frame Riemann problems that runs of the
    random-state, boosted Kelvin-Helmholtz and point-explosion workloads pose
    (a data file of plain arrays; see its producer's description in the
    file's arrays: per source '<name>_joint' over (ln rho_R/rho_L,
    ln P_R/P_L, (u_R - u_L)/(c_L + c_R)), '<name>_scale' over
    (ln rho_L, ln P_L), '<name>_frame' over u_L / c_L, and 'edges_*')."""
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def sample_harvest(h: dict, source: str, n: int, gamma: float, rng) -> np.ndarray:
    """n problems [6][n] (rho_L, u_L, P_L, rho_R, u_R, P_R) drawn from one
    source's histograms: a joint bin by its count, a scale bin and a frame
    bin likewise, each value uniform inside its bin; then
    rho_R = rho_L e^x0, P_R = P_L e^x1, u_L = m c_L, u_R = u_L + x2 (c_L + c_R)
    with c = sqrt(gamma P / rho)."""
    def bins(counts, k):
        p = counts.ravel().astype(np.float64)
        return np.unravel_index(rng.choice(p.size, size=k, p=p / p.sum()), counts.shape)

    def inside(edges, i):
        return edges[i] + (edges[i + 1] - edges[i]) * rng.random(i.shape)

    i0, i1, i2 = bins(h[f"{source}_joint"], n)
    x0, x1, x2 = inside(h["edges_x0"], i0), inside(h["edges_x1"], i1), inside(h["edges_x2"], i2)
    a, b = bins(h[f"{source}_scale"], n)
    lr, lp = inside(h["edges_lr"], a), inside(h["edges_lp"], b)
    (im,) = bins(h[f"{source}_frame"], n)
    mach = inside(h["edges_m"], im)
    rhoL, PL = np.exp(lr), np.exp(lp)
    rhoR, PR = rhoL * np.exp(x0), PL * np.exp(x1)
    cL, cR = np.sqrt(gamma * PL / rhoL), np.sqrt(gamma * PR / rhoR)
    uL = mach * cL
    uR = uL + x2 * (cL + cR)
    return np.stack([rhoL, uL, PL, rhoR, uR, PR])


def riemann_problems(n: int = 1 << 24, seed: int = 1003, path: str = HARVEST) -> np.ndarray:
    """Batch of independent 1D Riemann problems [6][n]: 95% drawn in equal
    thirds from the histograms of the problems that runs of the
    random-state, boosted Kelvin-Helmholtz and point-explosion workloads pose
    (load_harvest; problems that generate vacuum are not among them), 5% hard
    tails (riemann_tails), in a seeded random order."""
    rng = np.random.default_rng(seed)
    h = load_harvest(path)
    gamma = float(h["gamma"])
    n_tail = n // 20
    n_body = n - n_tail
    per = [n_body // 3, n_body // 3, n_body - 2 * (n_body // 3)]
    body = [sample_harvest(h, src, k, gamma, rng) for src, k in zip(HARVEST_SOURCES, per)]
    out = np.concatenate(body + [riemann_tails(n_tail, gamma, rng)], axis=1)
    return np.ascontiguousarray(out[:, rng.permutation(n)])


# ---------------------------------------------------------------------------
# Reflective walls by mirrored generators.
#
# The domain is lo < y < hi (axis 1) inside the unit box, periodic in the
# other axes. Every generator within `layer` of a wall is mirrored across it
# into the band [0, lo) or (hi, 1]; the periodic tessellation of the whole
# set then clips each interior cell exactly at the wall planes (a point of
# the domain is nearer to an interior generator than to any mirror image),
# and an interior cell's only face with a mirror cell is the wall face
# shared with its own image. Before each step the mirror ("ghost") cells
# take their source cells' states with the normal momentum negated; the
# wall faces then carry symmetric Riemann problems: no mass or energy
# flux, the pressure's momentum flux. With layer >= 3 cell spacings the
# first rows of ghosts see mirrored neighbourhoods, so their gradients are
# the mirrored ones too.
# ---------------------------------------------------------------------------
@dataclass
class Walls:
    mesh: Mesh
    ghost: np.ndarray      # [G] int32 ghost cell indices
    src: np.ndarray        # [G] int32 their source cells
    axis: int              # the walls' normal axis
    interior: np.ndarray   # [N] bool


def mirrored_mesh(points: np.ndarray, lo: float, hi: float, layer: float, nthreads: int = 0,
                  axis: int = 1) -> Walls:
    """Tessellation of `points` (interior generators, lo < x_axis < hi, y by
    default) with their mirror images across the walls x_axis = lo and
    x_axis = hi (those within `layer` of a wall), cells in Morton order;
    lo - layer >= 0 and hi + layer <= 1."""
    assert lo - layer >= 0.0 and hi + layer <= 1.0
    p = np.asarray(points, dtype=np.float64)
    y = p[:, axis]
    assert np.all((y > lo) & (y < hi))
    low = np.nonzero(y - lo < layer)[0]
    high = np.nonzero(hi - y < layer)[0]
    ml, mh = p[low].copy(), p[high].copy()
    ml[:, axis] = 2.0 * lo - ml[:, axis]
    mh[:, axis] = 2.0 * hi - mh[:, axis]
    allp = np.concatenate([p, ml, mh])
    n = p.shape[0]
    src = np.concatenate([low, high])
    ghost = n + np.arange(src.shape[0])
    order = morton_order(allp)
    inv = np.empty_like(order)
    inv[order] = np.arange(order.shape[0])
    mesh = build_mesh(allp[order], nthreads)
    interior = np.zeros(allp.shape[0], bool)
    interior[inv[:n]] = True
    return Walls(mesh, inv[ghost].astype(np.int32), inv[src].astype(np.int32), axis, interior)


def walled_lattice(nx: int, lo: float = 0.125, hi: float = 0.875, jitter: float = 0.0, seed: int = 0) -> tuple:
    """2D Cartesian lattice of spacing 1/nx in the domain lo < y < hi
    (an integral number of rows), mirrored across the walls into the bands
    outside them (layer lo = 1 - hi). Returns (walls, x, y), the
    generators' coordinates."""
    h = 1.0 / nx
    rows = int(round((hi - lo) / h))
    assert abs(rows * h - (hi - lo)) < 1e-12
    xs = (np.arange(nx) + 0.5) * h
    ys = lo + (np.arange(rows) + 0.5) * h
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    if jitter:
        rng = np.random.default_rng(seed)
        pts = pts + rng.uniform(-jitter * h, jitter * h, pts.shape)
    walls = mirrored_mesh(pts, lo, hi, min(lo, 1.0 - hi))
    pos = walls.mesh.positions
    return walls, pos[:, 0], pos[:, 1]


def rt3d(n_side: int = 128, layer: int = 4, jitter: float = 0.1, seed: int = 1005, nthreads: int = 0) -> Workload:
    """Rayleigh-Taylor setup of Section 8.8 in the unit box: reflective walls
    at y = lo = layer h and y = hi = 1 - lo (h = 1/n_side; the generators in
    lo < y < hi a jittered lattice, their mirror images filling the `layer`
    rows beyond each wall), periodic in x and z. rho = 2 above the mid-plane
    y = 1/2, 1 below; gamma = 1.4; P = P0 + g (y - 1/2) rho with P0 = 2.5 and
    g = -0.1 (hydrostatic); v_y = w0 [1 - cos(2 pi x)][1 - cos(2 pi (y - lo)
    / (hi - lo))] with w0 = 0.0025, one mode vanishing at the walls (the
    paper's box is 0.5 x 1.5; this one is 1 x (hi - lo), uniform in z). The
    field at the mirror cells is mirrored (+0.1). Mesh at rest."""
    rng = np.random.default_rng(seed)
    gamma = 1.4
    h = 1.0 / n_side
    lo, hi = layer * h, 1.0 - layer * h
    rows = n_side - 2 * layer
    axes = [(np.arange(n_side) + 0.5) * h, lo + (np.arange(rows) + 0.5) * h, (np.arange(n_side) + 0.5) * h]
    pts = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    pts = pts + rng.uniform(-jitter, jitter, size=pts.shape) * h
    pts[:, 0] = np.mod(pts[:, 0], 1.0)
    pts[:, 2] = np.mod(pts[:, 2], 1.0)
    walls = mirrored_mesh(pts, lo, hi, lo, nthreads)
    mesh = walls.mesh
    n = mesh.n_cells
    x, y = mesh.positions[:, 0], mesh.positions[:, 1]
    rho = np.where(y > 0.5, 2.0, 1.0)
    P = 2.5 - 0.1 * (y - 0.5) * rho
    vy = 0.0025 * (1.0 - np.cos(2 * np.pi * x)) * (1.0 - np.cos(2 * np.pi * (y - lo) / (hi - lo)))
    vel = np.stack([np.zeros(n), vy, np.zeros(n)])
    Q = conserved_from_primitive(mesh.volume, rho, vel, P, gamma)
    accel = np.zeros((3, n))
    accel[1] = -0.1
    accel[1, walls.ghost] = 0.1
    return Workload(f"rt3d_{n_side}^3", mesh, Q, gamma, 0.4, np.zeros(3), seed, (rho, vel, P), walls, accel)
