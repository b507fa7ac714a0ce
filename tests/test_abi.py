"""The C ABI library loads, exports every entry point include/mm.h declares,
and validates arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_0901_4107_amd import mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:mm_status|int64_t|const char \*)\s*(mm_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for want in ("mm_mesh_upload", "mm_gradients", "mm_face_fluxes", "mm_apply_update", "mm_hydro_step"):
        assert want in names


def test_library_exports_every_declared_symbol():
    so = mm.lib()
    for name in declared_symbols():
        assert hasattr(so, name), name
        assert name in mm.SIGNATURES, name


def _params(**kw):
    p = dict(dim=3, mode=mm.MM_FP64, guess=mm.MM_GUESS_STANDARD, newton_max_iter=0, gamma=5 / 3, cfl=0.4,
             newton_tol64=0.0, newton_tol32=0.0, stream=None, entropy=mm.MM_ENTROPY_OFF, mach_thresh=1.1,
             steps=mm.MM_STEPS_GLOBAL, alpha_s=0.01, beta_s=0.0)
    p.update(kw)
    return mm.mm_params(p["dim"], p["mode"], p["guess"], p["newton_max_iter"], p["gamma"], p["cfl"],
                        p["newton_tol64"], p["newton_tol32"], p["stream"], p["entropy"], p["steps"],
                        p["mach_thresh"], p["alpha_s"], p["beta_s"])


def _create(**kw):
    ctx = ctypes.c_void_p()
    st = mm.lib().mm_create(ctypes.byref(_params(**kw)), ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("kw", [dict(dim=1), dict(dim=4), dict(mode=7), dict(guess=3), dict(gamma=1.0),
                                dict(gamma=float("nan")), dict(cfl=0.0), dict(entropy=-1),
                                dict(entropy=mm.MM_ENTROPY_MACH, mach_thresh=float("nan")), dict(steps=2),
                                dict(steps=-1), dict(steps=mm.MM_STEPS_INDIVIDUAL, entropy=mm.MM_ENTROPY_MACH),
                                dict(entropy=3), dict(entropy=mm.MM_ENTROPY_ENERGY, alpha_s=-0.1),
                                dict(entropy=mm.MM_ENTROPY_ENERGY, alpha_s=float("nan")),
                                dict(entropy=mm.MM_ENTROPY_ENERGY, beta_s=float("inf")),
                                dict(steps=mm.MM_STEPS_INDIVIDUAL, entropy=mm.MM_ENTROPY_ENERGY)])
def test_create_rejects_bad_params(kw):
    st, ctx = _create(**kw)
    assert st == mm.MM_E_ARG and not ctx.value


def test_workspace_and_state_errors_without_device():
    L = mm.lib()
    st, ctx = _create()
    assert st == mm.MM_OK
    try:
        assert L.mm_workspace_bytes(ctx, 1, 10) < 0
        assert L.mm_workspace_bytes(ctx, 100, 0) < 0
        a = L.mm_workspace_bytes(ctx, 1000, 8000)
        b = L.mm_workspace_bytes(ctx, 2000, 16000)
        assert 0 < a < b
        assert L.mm_set_workspace(ctx, None, 1024) == mm.MM_E_ARG
        assert L.mm_set_workspace(ctx, ctypes.c_void_p(0x1001), 1024) == mm.MM_E_ARG  # misaligned
        m = mm.mm_mesh()
        assert L.mm_mesh_upload(ctx, ctypes.byref(m)) == mm.MM_E_STATE          # no workspace yet
        assert L.mm_hydro_step(ctx, ctypes.c_void_p(256), 0.0, None) == mm.MM_E_STATE  # no mesh
        assert L.mm_gradients(ctx, None, None, None) == mm.MM_E_ARG
        assert L.mm_face_fluxes(ctx, -1.0, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256)) == mm.MM_E_ARG
        assert L.mm_get_diag(ctx, None) == mm.MM_E_ARG
        # the largest accepted mesh, and the first refused sizes
        assert L.mm_workspace_bytes(ctx, (1 << 31) - 2, (1 << 30) - 1) > 0
        assert L.mm_workspace_bytes(ctx, (1 << 31) - 1, 100) < 0
        assert L.mm_workspace_bytes(ctx, 100, 1 << 30) < 0
        # sizes and pointers are checked before anything reaches the device
        # (the workspace pointer is only recorded, never dereferenced here)
        assert L.mm_set_workspace(ctx, ctypes.c_void_p(1 << 20), a) == mm.MM_OK
        def mesh(n, nf, ptr=1 << 21, idx=1 << 22):
            return mm.mm_mesh(n, nf, ptr, ptr, ptr, idx, idx, ptr, ptr, ptr)
        for n, nf in [(1, 10), (1000, 0), (0, 0), (1000, 1 << 30), (-5, 10)]:
            assert L.mm_mesh_upload(ctx, ctypes.byref(mesh(n, nf))) == mm.MM_E_ARG, (n, nf)
        assert L.mm_mesh_upload(ctx, ctypes.byref(mesh(1000, 8000, idx=None))) == mm.MM_E_ARG
        assert L.mm_mesh_upload(ctx, ctypes.byref(mesh(2000, 16000))) == mm.MM_E_WORKSPACE
        assert L.mm_hydro_step(ctx, ctypes.c_void_p(256), 0.0, None) == mm.MM_E_STATE  # still no mesh
        # mesh motion: arguments first, then the missing mesh
        P = ctypes.c_void_p(1 << 21)
        for eta, chi, dtl in [(0.0, 1.0, 0.0), (0.25, -1.0, 0.0), (0.25, 1.0, -1.0), (float("nan"), 1.0, 0.0),
                              (0.25, float("inf"), 0.0)]:
            assert L.mm_mesh_velocity(ctx, P, eta, chi, dtl, P) == mm.MM_E_ARG, (eta, chi, dtl)
        assert L.mm_mesh_velocity(ctx, P, 0.25, 1.0, 0.0, P) == mm.MM_E_STATE
        assert L.mm_volume_rate(ctx, P) == mm.MM_E_STATE
        assert L.mm_mesh_set_velocity(ctx, P) == mm.MM_E_STATE
        assert L.mm_set_gravity(ctx, P) == mm.MM_E_STATE
        assert L.mm_volume_rate(ctx, None) == mm.MM_E_ARG
        # walls: no context, then the missing mesh (lists are checked on the device after that)
        assert L.mm_set_walls(None, 4, P, P, 1) == mm.MM_E_ARG
        assert L.mm_set_walls(ctx, 4, P, P, 1) == mm.MM_E_STATE
        assert L.mm_reflect(ctx, None) == mm.MM_E_ARG
        assert L.mm_reflect(ctx, P) == mm.MM_E_STATE
    finally:
        L.mm_destroy(ctx)
    assert L.mm_destroy(None) == mm.MM_OK
    assert L.mm_status_str(mm.MM_E_MESH) == b"invalid mesh"


def test_entropy_mode_widens_the_flux_records():
    """The face-flux array of the entropy mode holds two more doubles per
    face (entropy flux, Mach number); its entry point needs the mode."""
    L = mm.lib()
    _, c0 = _create()
    _, c1 = _create(entropy=mm.MM_ENTROPY_MACH)
    try:
        n, nf = 100000, 800000
        assert L.mm_workspace_bytes(c1, n, nf) - L.mm_workspace_bytes(c0, n, nf) >= 2 * 8 * nf
        assert mm.flux_stride(3, mm.MM_ENTROPY_MACH) == 7 and mm.flux_stride(2) == 4
        assert L.mm_entropy_init(c0, ctypes.c_void_p(256)) == mm.MM_E_ARG    # not in entropy mode
        assert L.mm_entropy_init(c1, ctypes.c_void_p(256)) == mm.MM_E_STATE  # no mesh
    finally:
        L.mm_destroy(c0); L.mm_destroy(c1)


def test_individual_steps_widen_the_workspace():
    """A context for individual timesteps holds per-cell bins, step starts,
    signal records and touch stamps, and two split lists; its timeline entry
    points check their arguments and state before touching the device."""
    L = mm.lib()
    _, c0 = _create()
    _, c1 = _create(steps=mm.MM_STEPS_INDIVIDUAL)
    try:
        n, nf = 100000, 800000
        assert L.mm_workspace_bytes(c1, n, nf) - L.mm_workspace_bytes(c0, n, nf) >= (1 + 8 + 5 * 8 + 4) * n + 4 * nf
        assert L.mm_tb_begin(c0, 1e-3, 3) == mm.MM_E_STATE     # not an individual-timestep context
        for dt, lv in ((1e-3, 31), (1e-3, -1), (0.0, 3), (float("inf"), 3), (float("nan"), 3)):
            assert L.mm_tb_begin(c1, dt, lv) == mm.MM_E_ARG, (dt, lv)
        assert L.mm_tb_begin(c1, 1e-3, 3) == mm.MM_E_STATE     # no mesh
        assert L.mm_tb_step(c1, ctypes.c_void_p(256), None) == mm.MM_E_STATE
        assert L.mm_tb_step(c1, None, None) == mm.MM_E_ARG
        assert L.mm_tb_state(c1, None, None) == mm.MM_E_STATE
        assert L.mm_status_str(mm.MM_E_RANGE) == b"timestep criterion below the smallest step"
    finally:
        L.mm_destroy(c0); L.mm_destroy(c1)


def test_mixed_workspace_is_smaller_per_cell():
    L = mm.lib()
    _, c64 = _create(mode=mm.MM_FP64)
    _, c32 = _create(mode=mm.MM_MIXED)
    try:
        assert L.mm_workspace_bytes(c32, 10 ** 6, 8 * 10 ** 6) > 0
        assert L.mm_workspace_bytes(c64, 10 ** 6, 8 * 10 ** 6) > 0
    finally:
        L.mm_destroy(c64); L.mm_destroy(c32)


def test_binding_refuses_tensors_the_library_would_overrun():
    """The binding checks element type and size before a call reaches the
    library (the C ABI takes bare pointers): a batch output of 4 instead of
    5 doubles per problem, a float state array or missing rows raise."""
    import torch
    need = mm._need
    need(torch.empty(10, dtype=torch.float64), "x", torch.float64, 10)
    need(None, "x", torch.float64, 10, optional=True)
    with pytest.raises(ValueError, match="dtype"):
        need(torch.empty(10, dtype=torch.float32), "x", torch.float64, 10)
    with pytest.raises(ValueError, match="at least 50"):
        need(torch.empty((10, 4), dtype=torch.float64), "out", torch.float64, 5 * 10)
    with pytest.raises(ValueError, match="required"):
        need(None, "x", torch.float64, 1)
    # sizes of the entry points' arrays follow the header's strides
    assert mm.recon_stride(3) == 24 and mm.recon_stride(2) == 16
    assert mm.flux_stride(3) == 5 and mm.flux_stride(3, mm.MM_ENTROPY_MACH) == 7
    assert mm.flux_stride(3, mm.MM_ENTROPY_ENERGY) == 6 and mm.flux_stride(2, mm.MM_ENTROPY_ENERGY) == 5
