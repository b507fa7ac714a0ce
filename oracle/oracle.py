"""ctypes binding of ``oracle.c`` (test infrastructure only; see the header of
``oracle.c``). Mesh arguments are any object with the attributes ``dim,
volume, centroid_off, mesh_vel, face_L, face_R, face_area, face_ctr,
face_sep`` as numpy arrays in the layouts documented there."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.environ.get("ORACLE_SO") or os.path.join(_HERE, "liboracle.so")
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA; OpenMP
    over independent faces and cells, bitwise the same for any thread
    count)."""
    src = os.path.join(_HERE, "oracle.c")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-fopenmp",
                           "-ffp-contract=off", "-o", _SO + ".tmp", src, "-lm"])
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _OMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64),
                ("volume", _dp), ("centroid_off", _dp), ("mesh_vel", _dp),
                ("face_L", _ip), ("face_R", _ip), ("face_area", _dp),
                ("face_ctr", _dp), ("face_sep", _dp)]


class _OParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double)]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_set_threads.argtypes = [ctypes.c_int32]
        lib.oracle_threads.restype = ctypes.c_int32
        lib.oracle_riemann_batch.argtypes = [ctypes.c_int64, ctypes.c_double] + [_dp] * 12 + [_ip, _ip]
        lib.oracle_pressure_function.restype = ctypes.c_double
        lib.oracle_pressure_function.argtypes = [ctypes.c_double, _dp, _dp, ctypes.c_double]
        lib.oracle_prim.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp]
        lib.oracle_gradients.argtypes = [ctypes.POINTER(_OMesh), _dp, _dp, _dp, _dp]
        lib.oracle_face_velocity.argtypes = [ctypes.POINTER(_OMesh), _dp]
        lib.oracle_face_fluxes.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                           _dp, _dp, _dp, _ip, _ip]
        lib.oracle_face_states.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                           _dp, _dp, _dp]
        lib.oracle_apply_update.argtypes = [ctypes.POINTER(_OMesh), _dp, _dp]
        lib.oracle_cfl_dt.restype = ctypes.c_double
        lib.oracle_cfl_dt.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), _dp]
        lib.oracle_hydro_step.restype = ctypes.c_double
        lib.oracle_hydro_step.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double, _dp]
        lib.oracle_face_fluxes_ex.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                              _dp, _dp, _dp, _ip, _ip, _dp, _dp]
        lib.oracle_apply_update_entropy.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), _dp, _dp, _dp,
                                                    ctypes.c_double, _dp, _ip]
        lib.oracle_hydro_step_entropy.restype = ctypes.c_double
        lib.oracle_hydro_step_entropy.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                                  ctypes.c_double, _dp, _ip]
        lib.oracle_mesh_velocity.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), _dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_volume_rate.argtypes = [ctypes.POINTER(_OMesh), _dp]
        lib.oracle_face_fluxes_full.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                                _dp, _dp, _dp, _dp, _ip, _ip, _dp, _dp]
        lib.oracle_hydro_step_full.restype = ctypes.c_double
        lib.oracle_hydro_step_full.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                               _dp, ctypes.c_int32, ctypes.c_double, _dp, _ip]
        lib.oracle_shock_mach.restype = ctypes.c_double
        lib.oracle_shock_mach.argtypes = [ctypes.c_double, _dp, _dp]
        lib.oracle_hydro_step_energy.restype = ctypes.c_double
        lib.oracle_hydro_step_energy.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                                 _dp, ctypes.c_double, ctypes.c_double, _dp, _ip]
        lib.oracle_reflect.argtypes = [ctypes.c_int32, ctypes.c_int64, _dp, ctypes.c_int64, _ip, _ip, ctypes.c_int32]
        lib.oracle_tb_criterion.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), _dp, _dp]
        lib.oracle_tb_step.restype = ctypes.c_int
        lib.oracle_tb_step.argtypes = [ctypes.POINTER(_OMesh), ctypes.POINTER(_OParams), ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, _dp, _dp,
                                       _dp, _dp, _dp, _ip, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]
        _LIB = lib
    return _LIB


def set_threads(n: int) -> None:
    """Host threads of the oracle's loops (results do not depend on it)."""
    _lib().oracle_set_threads(int(n))


def threads() -> int:
    return int(_lib().oracle_threads())


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Held:
    """Keeps the numpy arrays behind an _OMesh alive."""

    def __init__(self, mesh):
        self.arrs = dict(
            volume=_f64(mesh.volume), centroid_off=_f64(mesh.centroid_off),
            mesh_vel=_f64(mesh.mesh_vel if mesh.mesh_vel is not None else np.zeros_like(mesh.centroid_off)),
            face_L=np.ascontiguousarray(mesh.face_L, dtype=np.int32),
            face_R=np.ascontiguousarray(mesh.face_R, dtype=np.int32),
            face_area=_f64(mesh.face_area), face_ctr=_f64(mesh.face_ctr), face_sep=_f64(mesh.face_sep))
        a = self.arrs
        self.s = _OMesh(int(mesh.dim), a["volume"].shape[0], a["face_area"].shape[0],
                        _d(a["volume"]), _d(a["centroid_off"]), _d(a["mesh_vel"]),
                        _i(a["face_L"]), _i(a["face_R"]), _d(a["face_area"]),
                        _d(a["face_ctr"]), _d(a["face_sep"]))
        self.dim = int(mesh.dim)
        self.n = a["volume"].shape[0]
        self.nf = a["face_area"].shape[0]


def riemann(gamma, rhoL, uL, PL, rhoR, uR, PR):
    """Exact Riemann problems sampled at x/t=0. Returns a dict of arrays:
    rho, u, P (sampled state), side (0 left / 1 right of the contact),
    pstar, ustar (NaN where undefined), case, iters."""
    arrs = [_f64(np.atleast_1d(x)) for x in (rhoL, uL, PL, rhoR, uR, PR)]
    n = max(a.shape[0] for a in arrs)
    arrs = [np.ascontiguousarray(np.broadcast_to(a, (n,))) for a in arrs]
    out = {k: np.empty(n) for k in ("rho", "u", "P", "side", "pstar", "ustar")}
    kase = np.empty(n, dtype=np.int32)
    iters = np.empty(n, dtype=np.int32)
    _lib().oracle_riemann_batch(n, float(gamma), *[_d(a) for a in arrs],
                                _d(out["rho"]), _d(out["u"]), _d(out["P"]), _d(out["side"]),
                                _d(out["pstar"]), _d(out["ustar"]), _i(kase), _i(iters))
    out["case"] = kase
    out["iters"] = iters
    return out


def pressure_function(gamma, L, R, p):
    L = _f64(L); R = _f64(R)
    return _lib().oracle_pressure_function(float(gamma), _d(L), _d(R), float(p))


def prim(dim, gamma, volume, Q):
    Q = _f64(Q); V = _f64(volume)
    W = np.empty_like(Q)
    _lib().oracle_prim(int(dim), V.shape[0], float(gamma), _d(V), _d(Q), _d(W))
    return W


def gradients(mesh, W):
    h = _Held(mesh)
    W = _f64(W)
    nv = h.dim + 2
    raw = np.empty((nv * h.dim, h.n)); lim = np.empty_like(raw); alpha = np.empty((nv, h.n))
    _lib().oracle_gradients(ctypes.byref(h.s), _d(W), _d(raw), _d(lim), _d(alpha))
    return raw, lim, alpha


def face_velocity(mesh):
    h = _Held(mesh)
    wf = np.empty((h.dim, h.nf))
    _lib().oracle_face_velocity(ctypes.byref(h.s), _d(wf))
    return wf


def face_fluxes(mesh, gamma, dt, W, grad):
    h = _Held(mesh)
    W = _f64(W); grad = _f64(grad)
    fl = np.empty((h.dim + 2, h.nf))
    fb = np.empty(h.nf, dtype=np.int32)
    kase = np.empty(h.nf, dtype=np.int32)
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_face_fluxes(ctypes.byref(h.s), ctypes.byref(p), float(dt), _d(W), _d(grad),
                              _d(fl), _i(fb), _i(kase))
    return fl, fb, kase


def face_fluxes_entropy(mesh, gamma, dt, W, grad):
    """face_fluxes plus, per face, the entropy flux dt A m_F A_U and the
    largest shock Mach number of the face's Riemann solution (Section 3.5)."""
    h = _Held(mesh)
    W = _f64(W); grad = _f64(grad)
    fl = np.empty((h.dim + 2, h.nf))
    sf = np.empty(h.nf)
    mach = np.empty(h.nf)
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_face_fluxes_ex(ctypes.byref(h.s), ctypes.byref(p), float(dt), _d(W), _d(grad),
                                 _d(fl), None, None, _d(sf), _d(mach))
    return fl, sf, mach


def apply_update_entropy(mesh, gamma, face_flux, s_flux, mach, mach_thresh, Q):
    """Conservative update of Q [D+3][N] (entropy last) with the Mach
    switch; returns (Q_new, kept [N])."""
    h = _Held(mesh)
    Q = _f64(Q).copy()
    kept = np.empty(h.n, dtype=np.int32)
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_apply_update_entropy(ctypes.byref(h.s), ctypes.byref(p), _d(_f64(face_flux)), _d(_f64(s_flux)),
                                       _d(_f64(mach)), float(mach_thresh), _d(Q), _i(kept))
    return Q, kept


def hydro_step_entropy(mesh, gamma, cfl, Q, mach_thresh, dt=0.0):
    """One step with the entropy row (Q [D+3][N]); returns (Q_new, dt_used, kept)."""
    h = _Held(mesh)
    Q = _f64(Q).copy()
    kept = np.empty(h.n, dtype=np.int32)
    p = _OParams(float(gamma), float(cfl))
    used = _lib().oracle_hydro_step_entropy(ctypes.byref(h.s), ctypes.byref(p), float(dt), float(mach_thresh),
                                            _d(Q), _i(kept))
    return Q, used, kept


def face_fluxes_gravity(mesh, gamma, dt, W, grad, accel):
    """face_fluxes with the half-step kick of a static field accel [D][N]
    (Section 5.2)."""
    h = _Held(mesh)
    fl = np.empty((h.dim + 2, h.nf))
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_face_fluxes_full(ctypes.byref(h.s), ctypes.byref(p), float(dt), _d(_f64(accel)), _d(_f64(W)),
                                   _d(_f64(grad)), _d(fl), None, None, None, None)
    return fl


def hydro_step_full(mesh, gamma, cfl, Q, dt=0.0, accel=None, mach_thresh=None):
    """One step with the options: a static field accel [D][N] (Section 5.2)
    and, with mach_thresh, the entropy row (Q [D+3][N], Section 3.5).
    Returns (Q_new, dt_used, kept or None)."""
    h = _Held(mesh)
    Q = _f64(Q).copy()
    ent = mach_thresh is not None
    kept = np.empty(h.n, dtype=np.int32)
    p = _OParams(float(gamma), float(cfl))
    acc = _f64(accel) if accel is not None else None
    used = _lib().oracle_hydro_step_full(ctypes.byref(h.s), ctypes.byref(p), float(dt),
                                         _d(acc) if acc is not None else None, int(ent),
                                         float(mach_thresh) if ent else 0.0, _d(Q), _i(kept))
    return Q, used, (kept if ent else None)


def hydro_step_energy(mesh, gamma, cfl, Q, alpha_s, beta_s=0.0, dt=0.0, accel=None):
    """One step with the entropy row (Q [D+3][N]) and the energy switch of
    Section 3.5 (eqs. eqnScrit1-eqnScrit2), optionally with a static field.
    Returns (Q_new, dt_used, kept)."""
    h = _Held(mesh)
    Q = _f64(Q).copy()
    kept = np.empty(h.n, dtype=np.int32)
    p = _OParams(float(gamma), float(cfl))
    acc = _f64(accel) if accel is not None else None
    used = _lib().oracle_hydro_step_energy(ctypes.byref(h.s), ctypes.byref(p), float(dt),
                                           _d(acc) if acc is not None else None, float(alpha_s), float(beta_s),
                                           _d(Q), _i(kept))
    return Q, used, kept


def mesh_velocity(mesh, gamma, W, eta=0.25, chi=1.0, dt_lloyd=0.0):
    """Generator velocities [D][N]: w = v plus the roundness correction of
    Section 4.1 (sound-speed form, or (s - r)/dt_lloyd when dt_lloyd > 0)."""
    h = _Held(mesh)
    w = np.empty((h.dim, h.n))
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_mesh_velocity(ctypes.byref(h.s), ctypes.byref(p), _d(_f64(W)), float(eta), float(chi),
                                float(dt_lloyd), _d(w))
    return w


def volume_rate(mesh):
    """dV_i/dt from the generator velocities (eq. eqnvolchange) [N]."""
    h = _Held(mesh)
    out = np.empty(h.n)
    _lib().oracle_volume_rate(ctypes.byref(h.s), _d(out))
    return out


def shock_mach(gamma, L, R):
    return _lib().oracle_shock_mach(float(gamma), _d(_f64(L)), _d(_f64(R)))


def face_states(mesh, gamma, dt, W, grad):
    """Face-frame Riemann inputs [6][F]: rho_L, u_L, P_L, rho_R, u_R, P_R."""
    h = _Held(mesh)
    out = np.empty((6, h.nf))
    p = _OParams(float(gamma), 0.0)
    _lib().oracle_face_states(ctypes.byref(h.s), ctypes.byref(p), float(dt), _d(_f64(W)), _d(_f64(grad)), _d(out))
    return out


def apply_update(mesh, face_flux, Q):
    h = _Held(mesh)
    Q = _f64(Q).copy()
    _lib().oracle_apply_update(ctypes.byref(h.s), _d(_f64(face_flux)), _d(Q))
    return Q


def cfl_dt(mesh, gamma, cfl, W):
    h = _Held(mesh)
    p = _OParams(float(gamma), float(cfl))
    return _lib().oracle_cfl_dt(ctypes.byref(h.s), ctypes.byref(p), _d(_f64(W)))


def hydro_step(mesh, gamma, cfl, Q, dt=0.0):
    """One full step; returns (Q_new, dt_used). dt <= 0 uses the CFL step."""
    h = _Held(mesh)
    Q = _f64(Q).copy()
    p = _OParams(float(gamma), float(cfl))
    used = _lib().oracle_hydro_step(ctypes.byref(h.s), ctypes.byref(p), float(dt), _d(Q))
    return Q, used


def tb_criterion(mesh, gamma, cfl, W):
    """Per-cell individual timestep bound [N] (Section 7.2,
    eq. EqnTiStepIndividual over the Voronoi neighbours)."""
    h = _Held(mesh)
    out = np.empty(h.n)
    p = _OParams(float(gamma), float(cfl))
    _lib().oracle_tb_criterion(ctypes.byref(h.s), ctypes.byref(p), _d(_f64(W)), _d(out))
    return out


class Timeline:
    """Individual power-of-two timesteps (Section 7.2) on a fixed mesh:
    ticks of dt_max / 2^levels, per-cell bins, record times and stored
    primitive and gradient records, advanced one synchronisation point per
    call of ``step`` (see ``oracle_tb_step``)."""

    def __init__(self, mesh, gamma, cfl, dt_max, levels):
        self.h = _Held(mesh)
        self.p = _OParams(float(gamma), float(cfl))
        self.dt_max = float(dt_max)
        self.levels = int(levels)
        n, D = self.h.n, self.h.dim
        self.bin = np.full(n, self.levels, dtype=np.int8)
        self.trec = np.zeros(n, dtype=np.int64)
        self.W = np.zeros((D + 2, n))
        self.G = np.zeros(((D + 2) * D, n))
        self.ti = 0

    @property
    def tick(self):
        return np.ldexp(self.dt_max, -self.levels)

    @property
    def time(self):
        return self.ti * self.tick

    def step(self, Q):
        """One synchronisation point on Q ([D+2][N], updated in place).
        Returns a dict: status (0, or 1 when a criterion is below one tick),
        ti (the tick of this point), next (the next point), active [N],
        face_dt [F], pred [2][F] (each side's prediction interval),
        n_faces (active faces)."""
        assert Q.dtype == np.float64 and Q.flags.c_contiguous
        h = self.h
        face_dt = np.empty(h.nf)
        pred = np.empty((2, h.nf))
        active = np.empty(h.n, dtype=np.int32)
        nxt = ctypes.c_int64(0)
        na = ctypes.c_int64(0)
        ti = self.ti
        st = _lib().oracle_tb_step(ctypes.byref(h.s), ctypes.byref(self.p), self.dt_max, self.levels, ti,
                                   self.bin.ctypes.data, self.trec.ctypes.data, _d(self.W), _d(self.G), _d(Q),
                                   _d(face_dt), _d(pred), _i(active), ctypes.byref(nxt), ctypes.byref(na))
        if st == 0:
            self.ti = nxt.value
        return dict(status=st, ti=ti, next=nxt.value if st == 0 else ti, active=active.astype(bool),
                    face_dt=face_dt, pred=pred, n_faces=na.value)


def reflect(Q, ghost, src, axis):
    """Ghost cells' states from their sources with the normal momentum
    (row 1 + axis) negated; returns a copy of Q [rows][N]."""
    Q = _f64(Q).copy()
    g = np.ascontiguousarray(ghost, dtype=np.int32)
    s = np.ascontiguousarray(src, dtype=np.int32)
    _lib().oracle_reflect(Q.shape[0], Q.shape[1], _d(Q), g.shape[0], _i(g), _i(s), int(axis))
    return Q
