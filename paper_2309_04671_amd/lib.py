"""ctypes binding of libstencil (include/stencil.h): same names, same structs.

Argument marshalling only.  The shared library must have been built
(``python -m paper_2309_04671_amd.build`` or ``__graft_entry__.build()``);
loading fails loudly otherwise -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstencil.so")

SP_OK, SP_EINVAL, SP_EUNSUPPORTED, SP_EDEVICE, SP_ENOMEM, SP_EBUDGET, SP_EPENDING, SP_ENUMERIC = range(8)
SP_F32, SP_F16, SP_BF16 = 0, 1, 2
SP_HALO = 4
SP_MAX_SOURCES = 16
SP_SLAB = 16

ERROR_NAMES = {0: "SP_OK", 1: "SP_EINVAL", 2: "SP_EUNSUPPORTED", 3: "SP_EDEVICE",
               4: "SP_ENOMEM", 5: "SP_EBUDGET", 6: "SP_EPENDING", 7: "SP_ENUMERIC"}

# Every symbol include/stencil.h declares (checked by the ABI tests).
EXPORTS = [
    "sp_grid_init", "sp_grid_init_2d", "sp_stencil_apply", "sp_apply", "sp_wave_meta_bytes", "sp_wave_step",
    "sp_wave_step_fused", "sp_wave_run_states", "sp_wave_adjoint_step", "sp_grad_finish", "sp_decode", "sp_energy_ws_bytes",
    "sp_energy", "sp_energy_noalloc_max_partials", "sp_energy_noalloc", "sp_pml_profile", "sp_wave_step_pml", "sp_shot_bytes", "sp_queue_create", "sp_submit", "sp_poll", "sp_queue_drain",
    "sp_queue_destroy", "sp_last_error", "sp_version",
]

SP_QUEUE_EAGER, SP_QUEUE_FAKE = 1, 2
SP_SHOT_QUEUED, SP_SHOT_RUNNING, SP_SHOT_DONE, SP_SHOT_FAILED = range(4)


class SpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, str(code)), msg))
        self.code = code


class sp_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("dtype", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("pitch_x", ctypes.c_int64), ("pitch_y", ctypes.c_int64), ("planes", ctypes.c_int64),
                ("origin", ctypes.c_int64), ("elems", ctypes.c_int64), ("bytes", ctypes.c_int64)]


class sp_coeffs(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double), ("ax", ctypes.c_double * 4),
                ("ay", ctypes.c_double * 4), ("az", ctypes.c_double * 4)]


class sp_stencil(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("ndim", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("w", ctypes.POINTER(ctypes.c_double))]


SP_STAR, SP_BOX = 0, 1


class sp_pml(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("decomposition", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eta", ctypes.c_void_p), ("psi", ctypes.c_void_p)]


SP_PML_UNIFIED, SP_PML_SEVEN, SP_PML_TWO = 0, 1, 2


class sp_wave_state(ctypes.Structure):
    _fields_ = [("cur", ctypes.c_void_p), ("prev", ctypes.c_void_p), ("meta", ctypes.c_void_p),
                ("step", ctypes.c_int64)]


class sp_sources(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xyz", (ctypes.c_int32 * 3) * SP_MAX_SOURCES),
                ("amp", ctypes.c_void_p), ("amp_stride", ctypes.c_int64)]


class sp_receivers(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("traces", ctypes.c_void_p),
                ("trace_stride", ctypes.c_int64)]


class sp_queue_cfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("chunk_steps", ctypes.c_int32), ("flags", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class sp_shot_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("nsteps", ctypes.c_int32), ("dt", ctypes.c_double),
                ("dx", ctypes.c_double), ("coeffs", sp_coeffs), ("v", ctypes.c_void_p),
                ("nsrc", ctypes.c_int32), ("src_xyz", (ctypes.c_int32 * 3) * SP_MAX_SOURCES),
                ("src_amp", ctypes.c_void_p), ("nrec", ctypes.c_int32), ("rec_xyz", ctypes.c_void_p),
                ("traces", ctypes.c_void_p), ("final_out", ctypes.c_void_p)]


class sp_shot_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32), ("steps_done", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def load():
    """Load libstencil.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libstencil.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    lib.sp_grid_init.argtypes = [i, i, i, i, i, P(sp_grid)]
    lib.sp_stencil_apply.argtypes = [P(sp_grid), P(sp_coeffs), i, vp, vp, P(ctypes.c_int), vp]
    lib.sp_grid_init_2d.argtypes = [i, i, i, i, P(sp_grid)]
    lib.sp_apply.argtypes = [P(sp_grid), P(sp_stencil), i, vp, vp, P(ctypes.c_int), vp]
    lib.sp_wave_meta_bytes.argtypes = [P(sp_grid)]
    lib.sp_wave_meta_bytes.restype = i64
    lib.sp_wave_step.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, P(sp_wave_state), i,
                                 P(sp_sources), P(sp_receivers), vp]
    lib.sp_wave_step_fused.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, P(sp_wave_state),
                                       i, P(vp), P(sp_sources), P(sp_receivers), vp]
    lib.sp_wave_run_states.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, P(vp), i64,
                                       i, P(sp_sources), P(sp_receivers), vp]
    lib.sp_wave_adjoint_step.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp,
                                         P(sp_wave_state), P(vp), i, P(sp_sources),
                                         P(sp_receivers), vp, vp]
    lib.sp_grad_finish.argtypes = [P(sp_grid), vp, vp, vp, vp]
    lib.sp_decode.argtypes = [P(sp_grid), vp, vp, i64, vp, vp]
    lib.sp_energy_ws_bytes.argtypes = [P(sp_grid)]
    lib.sp_energy_ws_bytes.restype = i64
    lib.sp_energy.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, vp, vp, vp, vp, vp]
    lib.sp_energy_noalloc_max_partials.argtypes = []
    lib.sp_energy_noalloc_max_partials.restype = i64
    lib.sp_energy_noalloc.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, vp, vp, vp, vp]
    lib.sp_pml_profile.argtypes = [P(sp_grid), i, d, vp, vp]
    lib.sp_wave_step_pml.argtypes = [P(sp_grid), P(sp_coeffs), d, d, P(sp_grid), vp, P(sp_wave_state), i,
                                     P(sp_pml), P(sp_sources), P(sp_receivers), vp]
    lib.sp_shot_bytes.argtypes = [P(sp_shot_desc)]
    lib.sp_shot_bytes.restype = i64
    lib.sp_queue_create.argtypes = [P(sp_queue_cfg), P(vp)]
    lib.sp_submit.argtypes = [vp, P(sp_shot_desc), P(ctypes.c_uint64)]
    lib.sp_poll.argtypes = [vp, ctypes.c_uint64, P(sp_shot_status)]
    lib.sp_queue_drain.argtypes = [vp]
    lib.sp_queue_destroy.argtypes = [vp]
    lib.sp_last_error.restype = ctypes.c_char_p
    lib.sp_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("sp_wave_meta_bytes", "sp_energy_ws_bytes", "sp_energy_noalloc_max_partials",
                        "sp_shot_bytes", "sp_last_error", "sp_version"):
            fn.restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc):
    if rc != SP_OK:
        raise SpError(rc, load().sp_last_error().decode())
    return rc


def last_error() -> str:
    return load().sp_last_error().decode()


def grid_init(nx, ny, nz, dtype=SP_F32, halo=SP_HALO) -> sp_grid:
    g = sp_grid()
    check(load().sp_grid_init(nx, ny, nz, halo, dtype, ctypes.byref(g)))
    return g


def grid_init_2d(nx, ny, dtype=SP_F32, halo=SP_HALO) -> sp_grid:
    g = sp_grid()
    check(load().sp_grid_init_2d(nx, ny, halo, dtype, ctypes.byref(g)))
    return g


def coeffs(d) -> sp_coeffs:
    """Build sp_coeffs from {'center', 'ax', 'ay', 'az'}."""
    c = sp_coeffs()
    c.center = float(d["center"])
    for k in ("ax", "ay", "az"):
        arr = getattr(c, k)
        for j in range(4):
            arr[j] = float(d[k][j])
    return c


def stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def sp_stencil_apply(g, c, sweeps, u, v, stream=None) -> int:
    """u, v: device pointers (int).  Returns result_in."""
    out = ctypes.c_int(-1)
    check(load().sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), int(sweeps), ctypes.c_void_p(u),
                                  ctypes.c_void_p(v), ctypes.byref(out), stream_ptr(stream)))
    return out.value


def sp_apply(g, shape, w, u, v, sweeps=1, stream=None) -> int:
    """Suite stencil: shape "star"/"box" (or SP_STAR/SP_BOX); w: array of
    shape (2r+1,)*ndim, x offset last.  u, v: device pointers (int).
    Returns result_in."""
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float64)
    st = sp_stencil()
    st.shape = {"star": SP_STAR, "box": SP_BOX}.get(shape, shape)
    st.ndim = w.ndim
    st.radius = (w.shape[0] - 1) // 2
    st.w = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_int(-1)
    check(load().sp_apply(ctypes.byref(g), ctypes.byref(st), int(sweeps), ctypes.c_void_p(u),
                          ctypes.c_void_p(v), ctypes.byref(out), stream_ptr(stream)))
    return out.value


def sp_pml_profile(gv, width, eta_max, eta_ptr, stream=None):
    check(load().sp_pml_profile(ctypes.byref(gv), int(width), float(eta_max), ctypes.c_void_p(eta_ptr),
                                stream_ptr(stream)))


def make_pml(width, eta_ptr, psi_ptr, alpha=0.0, decomposition=SP_PML_SEVEN) -> sp_pml:
    return sp_pml(int(width), int(decomposition), float(alpha), eta_ptr, psi_ptr)


def sp_wave_step_pml(g, c, dt, dx, gv, v_ptr, st, nsteps, pml, src=None, rec=None, stream=None):
    check(load().sp_wave_step_pml(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx), ctypes.byref(gv),
                                  ctypes.c_void_p(v_ptr), ctypes.byref(st), int(nsteps), ctypes.byref(pml),
                                  ctypes.byref(src) if src is not None else None,
                                  ctypes.byref(rec) if rec is not None else None, stream_ptr(stream)))


def make_sources(xyz, amp_ptr, amp_stride) -> sp_sources:
    s = sp_sources()
    s.n = len(xyz)
    if s.n > SP_MAX_SOURCES:
        raise ValueError("at most %d sources" % SP_MAX_SOURCES)
    for k, p in enumerate(xyz):
        for j in range(3):
            s.xyz[k][j] = int(p[j])
    s.amp = amp_ptr
    s.amp_stride = int(amp_stride)
    return s


def make_receivers(n, xyz_ptr, traces_ptr, trace_stride) -> sp_receivers:
    r = sp_receivers()
    r.n = int(n)
    r.xyz = xyz_ptr
    r.traces = traces_ptr
    r.trace_stride = int(trace_stride)
    return r


def sp_wave_step(g, c, dt, dx, gv, v_ptr, state, nsteps, src=None, rec=None, stream=None):
    check(load().sp_wave_step(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx), ctypes.byref(gv),
                              ctypes.c_void_p(v_ptr), ctypes.byref(state), int(nsteps),
                              ctypes.byref(src) if src is not None else None,
                              ctypes.byref(rec) if rec is not None else None, stream_ptr(stream)))


def _ptrs(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[int(p) for p in ptrs])
    return arr


def sp_wave_step_fused(g, c, dt, dx, gv, v_ptr, state, nsteps, spare, src=None, rec=None,
                       stream=None):
    """Two leapfrog steps per sweep.  ``spare`` is a list of two device
    pointers (zero-halo fields on g); like the state, it is rotated in place."""
    arr = _ptrs(spare)
    check(load().sp_wave_step_fused(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx),
                                    ctypes.byref(gv), ctypes.c_void_p(v_ptr), ctypes.byref(state),
                                    int(nsteps), arr,
                                    ctypes.byref(src) if src is not None else None,
                                    ctypes.byref(rec) if rec is not None else None, stream_ptr(stream)))
    spare[0], spare[1] = arr[0], arr[1]


def sp_wave_run_states(g, c, dt, dx, gv, v_ptr, states, n0, nsteps, src=None, rec=None, stream=None):
    arr = _ptrs(states)
    check(load().sp_wave_run_states(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx),
                                    ctypes.byref(gv), ctypes.c_void_p(v_ptr), arr, int(n0), int(nsteps),
                                    ctypes.byref(src) if src is not None else None,
                                    ctypes.byref(rec) if rec is not None else None, stream_ptr(stream)))


def sp_wave_adjoint_step(g, c, dt, dx, gv, v_ptr, adj, u_hist, nsteps, src, rec, G_ptr, stream=None):
    arr = _ptrs(u_hist)
    check(load().sp_wave_adjoint_step(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx),
                                      ctypes.byref(gv), ctypes.c_void_p(v_ptr), ctypes.byref(adj), arr,
                                      int(nsteps), ctypes.byref(src) if src is not None else None,
                                      ctypes.byref(rec) if rec is not None else None,
                                      ctypes.c_void_p(G_ptr), stream_ptr(stream)))


def sp_grad_finish(gv, v_ptr, G_ptr, out_ptr, stream=None):
    check(load().sp_grad_finish(ctypes.byref(gv), ctypes.c_void_p(v_ptr), ctypes.c_void_p(G_ptr),
                                ctypes.c_void_p(out_ptr), stream_ptr(stream)))


def sp_decode(g, field_ptr, meta_ptr, k, out_ptr, stream=None):
    check(load().sp_decode(ctypes.byref(g), ctypes.c_void_p(field_ptr), ctypes.c_void_p(meta_ptr),
                           int(k), ctypes.c_void_p(out_ptr), stream_ptr(stream)))


def sp_energy(g, c, dt, dx, gv, v_ptr, u0_ptr, u1_ptr, out_ptr, ws_ptr, stream=None):
    check(load().sp_energy(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx), ctypes.byref(gv),
                           ctypes.c_void_p(v_ptr), ctypes.c_void_p(u0_ptr), ctypes.c_void_p(u1_ptr),
                           ctypes.c_void_p(out_ptr), ctypes.c_void_p(ws_ptr), stream_ptr(stream)))


def sp_energy_noalloc(g, c, dt, dx, gv, v_ptr, u0_ptr, u1_ptr, out_ptr, stream=None):
    check(load().sp_energy_noalloc(ctypes.byref(g), ctypes.byref(c), float(dt), float(dx),
                                   ctypes.byref(gv), ctypes.c_void_p(v_ptr), ctypes.c_void_p(u0_ptr),
                                   ctypes.c_void_p(u1_ptr), ctypes.c_void_p(out_ptr), stream_ptr(stream)))
