"""Python binding of libmm (include/mm.h): argument marshalling only.

Every entry point of the C ABI has a method of the same name on
:class:`Context`. Device memory and streams come from PyTorch; every step of
the hydro path runs in the HIP kernels of ``libmm.so``. There is no CPU
fallback: a missing library or a missing GPU raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBMM_PATH = os.path.join(_HERE, "libmm.so")

MM_OK, MM_E_ARG, MM_E_MESH, MM_E_DEVICE, MM_E_STATE, MM_E_WORKSPACE, MM_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
MM_E_RANGE = -7
MM_FP64, MM_MIXED = 0, 1
MM_GUESS_STANDARD, MM_GUESS_LEARNED = 0, 1
MM_ENTROPY_OFF, MM_ENTROPY_MACH, MM_ENTROPY_ENERGY = 0, 1, 2
MM_STEPS_GLOBAL, MM_STEPS_INDIVIDUAL = 0, 1

_vp = ctypes.c_void_p


class mm_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("mode", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("newton_max_iter", ctypes.c_int32), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("newton_tol64", ctypes.c_double), ("newton_tol32", ctypes.c_double), ("stream", _vp),
                ("entropy", ctypes.c_int32), ("steps", ctypes.c_int32), ("mach_thresh", ctypes.c_double),
                ("alpha_s", ctypes.c_double), ("beta_s", ctypes.c_double)]


class mm_mesh(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64), ("volume", _vp),
                ("centroid_off", _vp), ("mesh_vel", _vp), ("face_L", _vp), ("face_R", _vp),
                ("face_area", _vp), ("face_ctr", _vp), ("face_sep", _vp)]


class mm_diag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("faces", "newton_iters", "newton_max", "unconverged", "vacuum", "positivity_fallback",
                 "fp64_fallback", "guess_fallback", "wave_iter_max_sum", "waves", "entropy_kept")] + \
               [("nonfinite", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mm_tb_info(ctypes.Structure):
    _fields_ = [("tick", ctypes.c_int64), ("next_tick", ctypes.c_int64), ("active_cells", ctypes.c_int64),
                ("active_faces", ctypes.c_int64), ("min_bin", ctypes.c_int32), ("max_bin", ctypes.c_int32),
                ("sparse", ctypes.c_int32), ("points", ctypes.c_int32), ("sparse_points", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("total_cells", ctypes.c_int64), ("total_faces", ctypes.c_int64),
                ("next_time", ctypes.c_double)]


class MMError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        super().__init__(f"{call} failed: {status} ({lib().mm_status_str(status).decode()})")


_LIB = None

# name -> (restype, argtypes); the exported symbols of include/mm.h
SIGNATURES = {
    "mm_create": (ctypes.c_int32, [ctypes.POINTER(mm_params), ctypes.POINTER(_vp)]),
    "mm_destroy": (ctypes.c_int32, [_vp]),
    "mm_workspace_bytes": (ctypes.c_int64, [_vp, ctypes.c_int64, ctypes.c_int64]),
    "mm_set_workspace": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64]),
    "mm_mesh_upload": (ctypes.c_int32, [_vp, ctypes.POINTER(mm_mesh)]),
    "mm_gradients": (ctypes.c_int32, [_vp, _vp, _vp]),
    "mm_face_fluxes": (ctypes.c_int32, [_vp, ctypes.c_double, _vp, _vp]),
    "mm_apply_update": (ctypes.c_int32, [_vp, _vp, _vp]),
    "mm_hydro_step": (ctypes.c_int32, [_vp, _vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "mm_get_diag": (ctypes.c_int32, [_vp, ctypes.POINTER(mm_diag)]),
    "mm_reset_diag": (ctypes.c_int32, [_vp]),
    "mm_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "mm_mlp_load": (ctypes.c_int32, [_vp, _vp]),
    "mm_mlp_infer": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp]),
    "mm_mlp_forward": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mm_mlp_grad_scratch_bytes": (ctypes.c_int64, [ctypes.c_int64]),
    "mm_mlp_grad": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]),
    "mm_mlp_adam": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_int32, _vp]),
    "mm_riemann_batch": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mm_riemann_batch_noalloc": (ctypes.c_int32, [ctypes.POINTER(mm_params), ctypes.c_int64, _vp, _vp, _vp, _vp]),
    "mm_face_states": (ctypes.c_int32, [_vp, ctypes.c_double, _vp, _vp]),
    "mm_entropy_init": (ctypes.c_int32, [_vp, _vp]),
    "mm_mesh_velocity": (ctypes.c_int32, [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp]),
    "mm_volume_rate": (ctypes.c_int32, [_vp, _vp]),
    "mm_mesh_set_velocity": (ctypes.c_int32, [_vp, _vp]),
    "mm_set_gravity": (ctypes.c_int32, [_vp, _vp]),
    "mm_set_walls": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int32]),
    "mm_reflect": (ctypes.c_int32, [_vp, _vp]),
    "mm_tb_begin": (ctypes.c_int32, [_vp, ctypes.c_double, ctypes.c_int32]),
    "mm_tb_step": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(mm_tb_info)]),
    "mm_tb_advance": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(mm_tb_info)]),
    "mm_tb_state": (ctypes.c_int32, [_vp, _vp, _vp]),
}

MM_MLP_PARAMS = 4481


def lib():
    """Load libmm.so (built in-tree by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBMM_PATH):
            raise RuntimeError(f"{LIBMM_PATH} is missing: build it with __graft_entry__.build()")
        so = ctypes.CDLL(LIBMM_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(so, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = so
    return _LIB


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libmm takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("libmm takes contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _check(call, status):
    if status != MM_OK:
        raise MMError(call, status)


def _need(t: torch.Tensor | None, name: str, dtype: torch.dtype, numel: int, optional: bool = False):
    """Refuse a tensor the library would read or write out of bounds: it must
    have the element type the entry point takes and at least `numel`
    elements (device residence and contiguity are checked by _ptr)."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name}: a tensor is required")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, the library takes {dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, the library needs at least {numel}")


@dataclass
class DeviceMesh:
    """Device copies of a tessellation in the layouts of ``mm_mesh``."""
    dim: int
    volume: torch.Tensor
    centroid_off: torch.Tensor
    mesh_vel: torch.Tensor
    face_L: torch.Tensor
    face_R: torch.Tensor
    face_area: torch.Tensor
    face_ctr: torch.Tensor
    face_sep: torch.Tensor

    @property
    def n_cells(self):
        return int(self.volume.shape[0])

    @property
    def n_faces(self):
        return int(self.face_area.shape[0])

    @classmethod
    def from_host(cls, mesh, device="cuda"):
        f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
        i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
        mv = mesh.mesh_vel if mesh.mesh_vel is not None else np.zeros_like(mesh.centroid_off)
        return cls(int(mesh.dim), f64(mesh.volume), f64(mesh.centroid_off), f64(mv), i32(mesh.face_L),
                   i32(mesh.face_R), f64(mesh.face_area), f64(mesh.face_ctr), f64(mesh.face_sep))

    def as_struct(self) -> mm_mesh:
        n, nf, D = self.n_cells, self.n_faces, self.dim
        for name, dt, size in (("volume", torch.float64, n), ("centroid_off", torch.float64, D * n),
                               ("mesh_vel", torch.float64, D * n), ("face_L", torch.int32, nf),
                               ("face_R", torch.int32, nf), ("face_area", torch.float64, nf),
                               ("face_ctr", torch.float64, D * nf), ("face_sep", torch.float64, D * nf)):
            _need(getattr(self, name), f"mm_mesh.{name}", dt, size)
        return mm_mesh(self.n_cells, self.n_faces, _ptr(self.volume), _ptr(self.centroid_off), _ptr(self.mesh_vel),
                       _ptr(self.face_L), _ptr(self.face_R), _ptr(self.face_area), _ptr(self.face_ctr),
                       _ptr(self.face_sep))


class Context:
    """An ``mm_ctx`` with its workspace held as a torch byte tensor."""

    def __init__(self, dim: int, gamma: float, cfl: float = 0.4, mode: int = MM_FP64,
                 guess: int = MM_GUESS_STANDARD, newton_max_iter: int = 0, newton_tol64: float = 0.0,
                 newton_tol32: float = 0.0, device="cuda", stream: torch.cuda.Stream | None = None,
                 entropy: int = MM_ENTROPY_OFF, mach_thresh: float = 1.1, steps: int = MM_STEPS_GLOBAL,
                 alpha_s: float = 0.01, beta_s: float = 0.0):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = mm_params(dim, mode, guess, newton_max_iter, gamma, cfl, newton_tol64, newton_tol32,
                                ctypes.c_void_p(self.stream.cuda_stream), entropy, steps, mach_thresh, alpha_s,
                                beta_s)
        self.dim = dim
        self.mode = mode
        self.entropy = entropy
        self._ctx = ctypes.c_void_p()
        _check("mm_create", lib().mm_create(ctypes.byref(self.params), ctypes.byref(self._ctx)))
        self._ws = None
        self._mesh = None
        self._mlp = None

    def __del__(self):
        if getattr(self, "_ctx", None) and _LIB is not None:
            _LIB.mm_destroy(self._ctx)
            self._ctx = None

    # --- sizes the library derives from the uploaded mesh --------------------
    def _cells(self, call: str) -> int:
        if self._mesh is None:
            raise MMError(call, MM_E_STATE)
        return self._mesh.n_cells

    def _faces(self, call: str) -> int:
        if self._mesh is None:
            raise MMError(call, MM_E_STATE)
        return self._mesh.n_faces

    def _rows(self) -> int:
        """Rows of Q: D + 2 conserved totals, plus the entropy row."""
        return self.dim + 2 + (1 if self.entropy else 0)

    def _recon_dtype(self):
        return torch.float64 if self.mode == MM_FP64 else torch.float32

    def _need_Q(self, Q, call):
        _need(Q, f"{call}: Q", torch.float64, self._rows() * self._cells(call))

    def _need_recon(self, recon, call):
        _need(recon, f"{call}: recon", self._recon_dtype(), self._cells(call) * recon_stride(self.dim))

    def _need_flux(self, flux, call):
        _need(flux, f"{call}: face_flux", torch.float64, self._faces(call) * flux_stride(self.dim, self.entropy))

    # --- C ABI, one method per entry point ----------------------------------
    def mm_workspace_bytes(self, n_cells: int, n_faces: int) -> int:
        return int(lib().mm_workspace_bytes(self._ctx, n_cells, n_faces))

    def mm_set_workspace(self, ws: torch.Tensor):
        _check("mm_set_workspace", lib().mm_set_workspace(self._ctx, _ptr(ws), ws.numel() * ws.element_size()))
        self._ws = ws

    def mm_mesh_upload(self, mesh: DeviceMesh):
        need = self.mm_workspace_bytes(mesh.n_cells, mesh.n_faces)
        if need < 0:
            raise MMError("mm_workspace_bytes", MM_E_ARG)
        if self._ws is None or self._ws.numel() < need:
            self.mm_set_workspace(torch.empty(need + 256, dtype=torch.uint8, device=self.device))
            if self._mlp is not None:  # a new workspace holds no packed network yet
                _check("mm_mlp_load", lib().mm_mlp_load(self._ctx, _ptr(self._mlp)))
        self._mesh = mesh  # keep the arrays alive while the library refers to them
        _check("mm_mesh_upload", lib().mm_mesh_upload(self._ctx, ctypes.byref(mesh.as_struct())))

    def mm_gradients(self, Q: torch.Tensor, recon: torch.Tensor):
        self._need_Q(Q, "mm_gradients")
        self._need_recon(recon, "mm_gradients")
        _check("mm_gradients", lib().mm_gradients(self._ctx, _ptr(Q), _ptr(recon)))

    def mm_face_fluxes(self, dt: float, recon: torch.Tensor, face_flux: torch.Tensor):
        self._need_recon(recon, "mm_face_fluxes")
        self._need_flux(face_flux, "mm_face_fluxes")
        _check("mm_face_fluxes", lib().mm_face_fluxes(self._ctx, float(dt), _ptr(recon), _ptr(face_flux)))

    def mm_apply_update(self, face_flux: torch.Tensor, Q: torch.Tensor):
        self._need_flux(face_flux, "mm_apply_update")
        self._need_Q(Q, "mm_apply_update")
        _check("mm_apply_update", lib().mm_apply_update(self._ctx, _ptr(face_flux), _ptr(Q)))

    def mm_hydro_step(self, Q: torch.Tensor, dt: float = 0.0, sync: bool = True):
        """One step on Q in place; returns the timestep used (None if sync=False)."""
        self._need_Q(Q, "mm_hydro_step")
        if sync:
            used = ctypes.c_double(0.0)
            _check("mm_hydro_step", lib().mm_hydro_step(self._ctx, _ptr(Q), float(dt), ctypes.byref(used)))
            return used.value
        _check("mm_hydro_step", lib().mm_hydro_step(self._ctx, _ptr(Q), float(dt), None))
        return None

    def mm_get_diag(self) -> dict:
        d = mm_diag()
        _check("mm_get_diag", lib().mm_get_diag(self._ctx, ctypes.byref(d)))
        return {name: getattr(d, name) for name, _ in mm_diag._fields_ if name != "reserved"}

    def mm_reset_diag(self):
        _check("mm_reset_diag", lib().mm_reset_diag(self._ctx))

    def ensure_workspace(self):
        """A workspace large enough for the mesh-free entry points."""
        if self._ws is None:
            need = self.mm_workspace_bytes(2, 1)
            self.mm_set_workspace(torch.empty(need + 256, dtype=torch.uint8, device=self.device))

    def mm_mlp_load(self, params: torch.Tensor):
        _need(params, "mm_mlp_load: params", torch.float32, MM_MLP_PARAMS)
        self.ensure_workspace()
        _check("mm_mlp_load", lib().mm_mlp_load(self._ctx, _ptr(params)))
        self._mlp = params

    def mm_mlp_infer(self, X: torch.Tensor, Y: torch.Tensor):
        n = X.shape[0]
        _need(X, "mm_mlp_infer: X", torch.float32, 3 * n)
        _need(Y, "mm_mlp_infer: Y", torch.float32, n)
        _check("mm_mlp_infer", lib().mm_mlp_infer(self._ctx, X.shape[0], _ptr(X), _ptr(Y)))

    def mm_riemann_batch(self, states: torch.Tensor, out: torch.Tensor, iters: torch.Tensor | None = None):
        """states [6][n] double -> out [n][5] double (rho_F, u_F, P_F, p*,
        p_std), iters [n] int32 (optional)."""
        if states.dim() != 2 or states.shape[0] != 6:
            raise ValueError("mm_riemann_batch: states must be [6][n]")
        n = states.shape[1]
        _need(states, "mm_riemann_batch: states", torch.float64, 6 * n)
        _need(out, "mm_riemann_batch: out", torch.float64, 5 * n)
        _need(iters, "mm_riemann_batch: iters", torch.int32, n, optional=True)
        self.ensure_workspace()
        _check("mm_riemann_batch", lib().mm_riemann_batch(self._ctx, states.shape[1], _ptr(states), _ptr(out),
                                                          _ptr(iters)))

    def mm_face_states(self, dt: float, recon: torch.Tensor, out: torch.Tensor):
        self._need_recon(recon, "mm_face_states")
        _need(out, "mm_face_states: out", torch.float32, 6 * self._faces("mm_face_states"))
        _check("mm_face_states", lib().mm_face_states(self._ctx, float(dt), _ptr(recon), _ptr(out)))

    def mm_mesh_velocity(self, Q: torch.Tensor, w_out: torch.Tensor, eta: float = 0.25, chi: float = 1.0,
                         dt_lloyd: float = 0.0):
        n = self._cells("mm_mesh_velocity")
        _need(Q, "mm_mesh_velocity: Q", torch.float64, (self.dim + 2) * n)
        _need(w_out, "mm_mesh_velocity: w_out", torch.float64, self.dim * n)
        _check("mm_mesh_velocity", lib().mm_mesh_velocity(self._ctx, _ptr(Q), float(eta), float(chi),
                                                          float(dt_lloyd), _ptr(w_out)))

    def mm_mesh_set_velocity(self, w: torch.Tensor):
        _need(w, "mm_mesh_set_velocity: w", torch.float64, self.dim * self._cells("mm_mesh_set_velocity"))
        _check("mm_mesh_set_velocity", lib().mm_mesh_set_velocity(self._ctx, _ptr(w)))
        self._mesh_vel = w  # kept alive while the library refers to it

    def mm_set_gravity(self, accel: torch.Tensor | None):
        _need(accel, "mm_set_gravity: accel", torch.float64, self.dim * self._cells("mm_set_gravity"), optional=True)
        _check("mm_set_gravity", lib().mm_set_gravity(self._ctx, _ptr(accel)))
        self._accel = accel  # kept alive while the library refers to it

    def mm_set_walls(self, ghost: torch.Tensor | None, src: torch.Tensor | None, axis: int = 1):
        """Mirror cells ghost [k] of src [k] (int32 device); None removes the walls."""
        n = 0 if ghost is None else int(ghost.numel())
        if n:
            _need(ghost, "mm_set_walls: ghost", torch.int32, n)
            _need(src, "mm_set_walls: src", torch.int32, n)
        self._walls = None
        _check("mm_set_walls", lib().mm_set_walls(self._ctx, n, _ptr(ghost), _ptr(src), int(axis)))
        self._walls = (ghost, src)  # kept alive while the library refers to them

    def mm_reflect(self, Q: torch.Tensor):
        self._need_Q(Q, "mm_reflect")
        _check("mm_reflect", lib().mm_reflect(self._ctx, _ptr(Q)))

    def mm_volume_rate(self, rate: torch.Tensor):
        _need(rate, "mm_volume_rate: rate", torch.float64, self._cells("mm_volume_rate"))
        _check("mm_volume_rate", lib().mm_volume_rate(self._ctx, _ptr(rate)))

    def mm_entropy_init(self, Q: torch.Tensor):
        self._need_Q(Q, "mm_entropy_init")
        _check("mm_entropy_init", lib().mm_entropy_init(self._ctx, _ptr(Q)))


    def mm_tb_begin(self, dt_max: float, levels: int):
        _check("mm_tb_begin", lib().mm_tb_begin(self._ctx, float(dt_max), int(levels)))

    def mm_tb_step(self, Q: torch.Tensor) -> dict:
        """One synchronisation point on Q in place; returns the point's
        summary (tick, next_tick, active_cells, active_faces, min_bin,
        max_bin, sparse, points, sparse_points, total_cells, total_faces,
        next_time)."""
        self._need_Q(Q, "mm_tb_step")
        info = mm_tb_info()
        _check("mm_tb_step", lib().mm_tb_step(self._ctx, _ptr(Q), ctypes.byref(info)))
        return {name: getattr(info, name) for name, _ in mm_tb_info._fields_ if name != "reserved"}

    def mm_tb_advance(self, Q: torch.Tensor, until_tick: int, max_points: int) -> dict:
        """Up to max_points points, stopping at until_tick, synchronising
        once; returns the last point's summary and the call's totals."""
        self._need_Q(Q, "mm_tb_advance")
        info = mm_tb_info()
        _check("mm_tb_advance", lib().mm_tb_advance(self._ctx, _ptr(Q), int(until_tick), int(max_points),
                                                    ctypes.byref(info)))
        return {name: getattr(info, name) for name, _ in mm_tb_info._fields_ if name != "reserved"}

    def mm_tb_state(self, bins: torch.Tensor | None = None, trec: torch.Tensor | None = None):
        """Copies of the bins (int8 [N]) and step start ticks (int64 [N])."""
        n = self._cells("mm_tb_state")
        _need(bins, "mm_tb_state: bins", torch.int8, n, optional=True)
        _need(trec, "mm_tb_state: trec", torch.int64, n, optional=True)
        _check("mm_tb_state", lib().mm_tb_state(self._ctx, _ptr(bins), _ptr(trec)))

    def recon_buffer(self, n_cells: int):
        """Reconstruction buffer for mm_gradients in this context's mode
        (double in MM_FP64, float in MM_MIXED): N * MM_RECON_STRIDE elements,
        the primitive block [N][8] then the gradient block [N][16 or 8]."""
        dt = torch.float64 if self.mode == MM_FP64 else torch.float32
        return torch.empty(n_cells * recon_stride(self.dim), dtype=dt, device=self.device)

    def flux_buffer(self, n_faces: int):
        """Face fluxes [F][MM_FLUX_STRIDE] (double): D+2 fluxes, then with the
        entropy row the entropy flux, and with the Mach switch the face's shock
        Mach number."""
        return torch.empty((n_faces, flux_stride(self.dim, self.entropy)), dtype=torch.float64, device=self.device)



def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mm_mlp_forward(params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, stream=None):
    n = X.shape[0]
    _need(params, "mm_mlp_forward: params", torch.float32, MM_MLP_PARAMS)
    _need(X, "mm_mlp_forward: X", torch.float32, 3 * n)
    _need(Y, "mm_mlp_forward: Y", torch.float32, n)
    _check("mm_mlp_forward", lib().mm_mlp_forward(_ptr(params), X.shape[0], _ptr(X), _ptr(Y), _stream_ptr(stream)))


def mm_mlp_grad_scratch_bytes(n: int) -> int:
    return int(lib().mm_mlp_grad_scratch_bytes(n))


def mm_mlp_grad(params, X, T, scratch, grad, n_total=None, stream=None):
    n = X.shape[0]
    _need(params, "mm_mlp_grad: params", torch.float32, MM_MLP_PARAMS)
    _need(X, "mm_mlp_grad: X", torch.float32, 3 * n)
    _need(T, "mm_mlp_grad: T", torch.float32, n)
    if scratch is None or scratch.numel() * scratch.element_size() < mm_mlp_grad_scratch_bytes(n):
        raise ValueError("mm_mlp_grad: scratch smaller than mm_mlp_grad_scratch_bytes(n)")
    _need(grad, "mm_mlp_grad: grad", torch.float32, MM_MLP_PARAMS)
    _check("mm_mlp_grad", lib().mm_mlp_grad(_ptr(params), n, n if n_total is None else n_total, _ptr(X), _ptr(T),
                                            _ptr(scratch), _ptr(grad), _stream_ptr(stream)))


def mm_mlp_adam(params, grad, m1, m2, lr, beta1, beta2, eps, step, stream=None):
    for name, t in (("params", params), ("grad", grad), ("m1", m1), ("m2", m2)):
        _need(t, f"mm_mlp_adam: {name}", torch.float32, MM_MLP_PARAMS)
    _check("mm_mlp_adam", lib().mm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), lr, beta1, beta2, eps,
                                            step, _stream_ptr(stream)))

MM_NOALLOC_CHUNK = 1 << 20
MM_NOALLOC_MAX_BATCH = 1 << 32


def mm_riemann_batch_noalloc(states: torch.Tensor, out: torch.Tensor, iters: torch.Tensor | None = None,
                             gamma: float = 5.0 / 3.0, mode: int = MM_FP64, guess: int = MM_GUESS_STANDARD,
                             mlp_params: torch.Tensor | None = None, newton_max_iter: int = 0,
                             newton_tol64: float = 0.0, newton_tol32: float = 0.0, stream=None):
    """The batch of mm_riemann_batch without a context or workspace: the
    library's fixed per-GPU scratch serves instead, and nothing is
    allocated. states [6][n] double -> out [n][5] double, iters [n] int32
    (optional); mlp_params (float [MM_MLP_PARAMS]) with the learned guess."""
    if states.dim() != 2 or states.shape[0] != 6:
        raise ValueError("mm_riemann_batch_noalloc: states must be [6][n]")
    n = states.shape[1]
    _need(states, "mm_riemann_batch_noalloc: states", torch.float64, 6 * n)
    _need(out, "mm_riemann_batch_noalloc: out", torch.float64, 5 * n)
    _need(iters, "mm_riemann_batch_noalloc: iters", torch.int32, n, optional=True)
    _need(mlp_params, "mm_riemann_batch_noalloc: mlp_params", torch.float32, MM_MLP_PARAMS,
          optional=guess != MM_GUESS_LEARNED)
    p = mm_params(3, mode, guess, newton_max_iter, gamma, 0.4, newton_tol64, newton_tol32, _stream_ptr(stream),
                  MM_ENTROPY_OFF, MM_STEPS_GLOBAL, 1.1, 0.0, 0.0)
    _check("mm_riemann_batch_noalloc", lib().mm_riemann_batch_noalloc(ctypes.byref(p), n, _ptr(states), _ptr(out),
                                                                      _ptr(iters), _ptr(mlp_params)))


def flux_stride(dim: int, entropy: int = MM_ENTROPY_OFF) -> int:
    """MM_FLUX_STRIDE: doubles per face record of the face-flux array."""
    return dim + 2 + {MM_ENTROPY_MACH: 2, MM_ENTROPY_ENERGY: 1}.get(entropy, 0)


def recon_stride(dim: int) -> int:
    """MM_RECON_STRIDE: elements per cell of the reconstruction buffer."""
    return 24 if dim == 3 else 16


def split_recon(rec, dim: int):
    """(W [D+2][N], G [(D+2)*D][N], s - r [D][N]) views of a reconstruction
    buffer in the oracle's structure-of-arrays layout (numpy or torch)."""
    nv = dim + 2
    n = rec.shape[0] // recon_stride(dim)
    grec = 16 if dim == 3 else 8
    prim = rec[:n * 8].reshape(n, 8)
    grad = rec[n * 8:].reshape(n, grec)
    return prim[:, :nv].T, grad[:, :nv * dim].T, prim[:, nv:nv + dim].T
