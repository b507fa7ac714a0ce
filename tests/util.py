"""Helpers shared by the tests (no step of the scheme lives here)."""
import numpy as np


def boost(Q, v0):
    """Galilean boost of cell totals by v0, Section 3.4's G(Q, v):
    (m, p, E) -> (m, p + m v0, E + p.v0 + m |v0|^2 / 2)."""
    D = Q.shape[0] - 2
    v0 = np.asarray(v0, dtype=np.float64)
    out = Q.copy()
    out[1:1 + D] = Q[1:1 + D] + Q[0][None, :] * v0[:, None]
    out[D + 1] = Q[D + 1] + np.sum(Q[1:1 + D] * v0[:, None], axis=0) + 0.5 * Q[0] * float(v0 @ v0)
    return out


def normwise_rel(a, b):
    """Per component k: max_i |a_ki - b_ki| / max_i |b_ki|."""
    a = np.asarray(a); b = np.asarray(b)
    den = np.max(np.abs(b), axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.max(np.abs(a - b), axis=1) / den


def l1_rel(a, b):
    """Per component k: sum_i |a_ki - b_ki| / sum_i |b_ki|."""
    a = np.asarray(a); b = np.asarray(b)
    den = np.sum(np.abs(b), axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.sum(np.abs(a - b), axis=1) / den


def l1_state(a, b):
    """L1 error of conserved states [D+2][N] per component: mass and energy as
    sum_i |a - b| / sum_i |b|; each momentum component against the L1 norm of
    the momentum vector, sum_i |a_k - b_k| / sum_i ||p_i||, so that a
    component that is analytically ~0 (p_z of a 2D flow in 3D) is measured
    against the momentum scale, not against its own round-off."""
    a = np.asarray(a); b = np.asarray(b)
    D = b.shape[0] - 2
    num = np.sum(np.abs(a - b), axis=1)
    den = np.sum(np.abs(b), axis=1)
    pmag = np.sum(np.sqrt(np.sum(b[1:1 + D] ** 2, axis=0)))
    den[1:1 + D] = pmag
    den = np.where(den > 0, den, 1.0)
    return num / den


def blast_radius(mesh, rho, centre=0.5):
    """Shock radius of a spherical blast about `centre`: cell densities
    averaged over radial shells half a mean cell spacing thick (radii of
    the cell centroids), then the densest shell's radius refined by the
    vertex of the parabola through it and its two neighbours. Returns
    (radius, density of the densest shell)."""
    D = mesh.dim
    cen = np.mod(mesh.positions.T + mesh.centroid_off, 1.0)
    r = np.sqrt(np.sum((cen - centre) ** 2, axis=0))
    h = 0.5 * (1.0 / mesh.n_cells) ** (1.0 / D)
    nb = int(0.5 / h)
    idx = np.minimum((r / h).astype(np.int64), nb)
    cnt = np.bincount(idx, minlength=nb + 1)[:nb]
    prof = np.bincount(idx, weights=rho, minlength=nb + 1)[:nb] / np.maximum(cnt, 1)
    i = int(np.clip(np.argmax(prof), 1, nb - 2))
    y0, y1, y2 = prof[i - 1:i + 2]
    curv = y0 - 2.0 * y1 + y2
    off = 0.5 * (y0 - y2) / curv if curv < 0 else 0.0
    return (i + 0.5 + off) * h, float(y1)


def update_condition(mesh, Q0, F, Q1, rows):
    """Condition of each cell's update for the given rows of Q:
    K_i = (|Q0_i| + sum over the cell's faces |F_f|) / |Q1_i| (at least 1),
    the size of the terms the update sums against the result. Rounding of
    relative size eps in those terms moves Q1_i by up to about eps K_i |Q1_i|.
    F [D+2][F] are the face fluxes (dt A Fhat) of the step."""
    K = np.empty((len(rows), mesh.n_cells))
    for a, row in enumerate(rows):
        aF = np.abs(F[row])
        s = (np.abs(Q0[row]) + np.bincount(mesh.face_L, weights=aF, minlength=mesh.n_cells)
             + np.bincount(mesh.face_R, weights=aF, minlength=mesh.n_cells))
        K[a] = np.maximum(s / np.maximum(np.abs(Q1[row]), 1e-300), 1.0)
    return K


def cell_rel(got, want, rows, floor=1e-12):
    """Per-cell relative error of the given rows: |got - want| / |want| per
    cell, against floor * max |want| where a cell's value is near zero."""
    out = []
    for row in rows:
        w = np.abs(want[row])
        out.append(np.abs(got[row] - want[row]) / np.maximum(w, floor * w.max()))
    return np.array(out)


def assert_cell_rel(got, want, K, rows, tol, what):
    """Per cell and row: |got - want| / |want| <= tol * K_i (K from
    update_condition). Returns the largest plain per-cell relative error of
    each row."""
    rel = cell_rel(got, want, rows)
    worst = np.max(rel / K, axis=1)
    assert np.all(worst <= tol), f"{what}: per-cell relative error / K {worst}, rows {rows}"
    return np.max(rel, axis=1)
