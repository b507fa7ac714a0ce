"""Periodic Voronoi meshes for the unit box, built by the C++ clipper in
``voronoi.cpp`` (compiled to ``libvoronoi.so`` next to this file).

Arrays follow the hydro library's layouts: per-cell vectors are ``[D][N]``,
per-face vectors ``[D][F]``, every face appears once with ``L < R`` and faces
are sorted by ``L``. ``face_ctr`` is the face centroid relative to the left
generator and ``face_sep`` the separation from the left generator to the
(periodic image of the) right one, so the face normal points from L to R.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libvoronoi.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        lib.vor_build.restype = ctypes.c_void_p
        lib.vor_build.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32]
        lib.vor_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.vor_fetch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 7
        lib.vor_free.argtypes = [ctypes.c_void_p]
        _LIB = lib
    return _LIB


@dataclass
class Mesh:
    dim: int
    positions: np.ndarray          # [N][D] generators in [0,1)
    volume: np.ndarray             # [N]
    centroid_off: np.ndarray       # [D][N]  s_i - r_i
    face_L: np.ndarray             # [F] int32
    face_R: np.ndarray             # [F] int32
    face_area: np.ndarray          # [F]
    face_ctr: np.ndarray           # [D][F]  f - r_L
    face_sep: np.ndarray           # [D][F]  r_R - r_L
    mesh_vel: np.ndarray = field(default=None)  # [D][N] generator velocities w_i
    n_bad: int = 0                 # cells whose neighbour search did not close
    n_asym: int = 0                # faces seen from one side only

    @property
    def n_cells(self) -> int:
        return int(self.volume.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_area.shape[0])

    def with_velocity(self, w: np.ndarray) -> "Mesh":
        w = np.ascontiguousarray(w, dtype=np.float64)
        assert w.shape == (self.dim, self.n_cells)
        self.mesh_vel = w
        return self


def build_mesh(points: np.ndarray, nthreads: int = 0) -> Mesh:
    """Tessellate ``points`` ([N][D], wrapped into [0,1)) periodically."""
    pts = np.ascontiguousarray(np.mod(points, 1.0), dtype=np.float64)
    n, dim = pts.shape
    lib = _lib()
    h = lib.vor_build(dim, n, pts.ctypes.data, nthreads)
    if not h:
        raise RuntimeError("voronoi build failed")
    try:
        counts = np.zeros(3, dtype=np.int64)
        lib.vor_counts(h, counts.ctypes.data)
        nf = int(counts[0])
        vol = np.empty(n)
        coff = np.empty((dim, n))
        L = np.empty(nf, dtype=np.int32)
        R = np.empty(nf, dtype=np.int32)
        area = np.empty(nf)
        ctr = np.empty((dim, nf))
        sep = np.empty((dim, nf))
        lib.vor_fetch(h, vol.ctypes.data, coff.ctypes.data, L.ctypes.data, R.ctypes.data,
                      area.ctypes.data, ctr.ctypes.data, sep.ctypes.data)
    finally:
        lib.vor_free(h)
    m = Mesh(dim, pts, vol, coff, L, R, area, ctr, sep,
             mesh_vel=np.zeros((dim, n)), n_bad=int(counts[1]), n_asym=int(counts[2]))
    if m.n_bad:
        raise RuntimeError(f"{m.n_bad} Voronoi cells did not close; too few points for the box")
    if m.n_asym:
        # A face seen from one side only leaves a cell open unless it is of
        # round-off size: every cell's sum of A n must vanish.
        nrm = sep / np.sqrt(np.sum(sep * sep, axis=0))
        acc = np.zeros((dim, n))
        for k in range(dim):
            np.add.at(acc[k], L, area * nrm[k])
            np.add.at(acc[k], R, -area * nrm[k])
        scale = vol ** ((dim - 1.0) / dim)
        worst = float(np.max(np.sqrt(np.sum(acc * acc, axis=0)) / scale))
        if worst > 1e-9:
            raise RuntimeError(f"{m.n_asym} faces seen from one side only leave cells open "
                               f"(largest |sum A n| {worst:.1e} of the cell's face scale)")
    return m


def _spread_bits(x: np.ndarray, dim: int, bits: int) -> np.ndarray:
    x = x.astype(np.uint64)
    out = np.zeros_like(x)
    for b in range(bits):
        out |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * dim)
    return out


def morton_order(points: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation that sorts points along a Morton (Z-order) curve, the
    space-filling-curve ordering used for memory locality of cells."""
    pts = np.mod(points, 1.0)
    n, dim = pts.shape
    q = np.minimum((pts * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    code = np.zeros(n, dtype=np.uint64)
    for k in range(dim):
        code |= _spread_bits(q[:, k], dim, bits) << np.uint64(dim - 1 - k)
    return np.argsort(code, kind="stable")
