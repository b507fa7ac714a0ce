"""The input generator's periodic Voronoi builder against scipy's Qhull
(an independent construction) on small point sets."""
import itertools

import numpy as np
import pytest
from scipy.spatial import ConvexHull, Voronoi

from paper_0901_4107_amd.inputs import build_mesh, morton_order
from paper_0901_4107_amd.inputs.configs import jittered_lattice, poisson_points


def qhull_periodic(pts):
    n, dim = pts.shape
    shifts = np.array(list(itertools.product([-1, 0, 1], repeat=dim)), dtype=float)
    allp = np.concatenate([pts + s for s in shifts])
    vor = Voronoi(allp)
    centre = int(np.where(np.all(shifts == 0, axis=1))[0][0])
    vols = np.empty(n)
    nbrs = [set() for _ in range(n)]
    for i in range(n):
        reg = vor.regions[vor.point_region[centre * n + i]]
        hull = ConvexHull(vor.vertices[reg])
        vols[i] = hull.volume
    for (a, b) in vor.ridge_points:
        ia, ib = a % n, b % n
        if a // n == centre:
            nbrs[ia].add(ib)
        if b // n == centre:
            nbrs[ib].add(ia)
    return vols, nbrs


@pytest.mark.parametrize("dim,kind", [(2, "poisson"), (3, "poisson"), (3, "lattice")])
def test_against_qhull(dim, kind):
    rng = np.random.default_rng(17)
    if kind == "poisson":
        pts = poisson_points(300 if dim == 2 else 400, dim, rng)
    else:
        pts = jittered_lattice(7, dim, 0.1, rng)
    m = build_mesh(pts)
    vols, nbrs = qhull_periodic(m.positions)
    assert np.allclose(m.volume, vols, rtol=1e-9, atol=0)
    mine = [set() for _ in range(m.n_cells)]
    big = m.face_area > 1e-9 * np.median(m.face_area)
    for l, r in zip(m.face_L[big], m.face_R[big]):
        mine[l].add(r); mine[r].add(l)
    # every non-degenerate face is a Qhull ridge
    for i in range(m.n_cells):
        assert mine[i] <= nbrs[i]


@pytest.mark.parametrize("dim", [2, 3])
def test_closure_and_layout(dim):
    rng = np.random.default_rng(5)
    m = build_mesh(poisson_points(500, dim, rng))
    assert np.all(m.face_L < m.face_R) and np.all(np.diff(m.face_L) >= 0)
    ell = np.sqrt(np.sum(m.face_sep ** 2, axis=0))
    An = m.face_area * m.face_sep / ell
    tot = np.zeros((dim, m.n_cells))
    for k in range(dim):
        np.add.at(tot[k], m.face_L, An[k]); np.add.at(tot[k], m.face_R, -An[k])
    assert np.abs(tot).max() < 1e-12
    # face centroids lie on the bisector planes
    d = m.face_sep
    assert np.abs(np.sum((m.face_ctr - 0.5 * d) * d, axis=0)).max() < 1e-12
    # centres of mass: sum V (r + delta) over the box equals the box centroid
    # modulo wrapping, so check |delta| is bounded by the cell size instead
    assert np.all(np.sqrt(np.sum(m.centroid_off ** 2, axis=0)) < m.volume ** (1 / dim) * 2)
    assert np.all(np.diff(morton_order(m.positions)) > 0)  # Morton order kept
