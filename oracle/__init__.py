"""FP64 CPU oracle for the star-stencil wave path.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the library itself never does.  It shares no code with the
GPU path (it reads inputs from the seeded generators in ``synth`` only).

The arithmetic lives in ``ref.c`` (plain C loop nests, FP64) and, for the
low-precision storage emulation, in ``lowp.py`` (numpy).  ``brute.py`` is an
independent pure-Python exact-rational stencil used to pin ``ref.c``.

Parity pins: see tests/test_oracle_*.py.  Every function here is pinned by at
least one property fixed by the mathematics (polynomial exactness, impulse
response, symmetry, energy conservation, Fourier-mode recursion, exact
rational brute force, finite differences); the FP16/BF16 emulation is pinned
by exact small cases of its scale rule and rounding.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build_oracle, LIB_PATH

HALO = 4
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build_oracle()
    lib = ctypes.CDLL(LIB_PATH)
    i, d = ctypes.c_int, ctypes.c_double
    lib.ref_laplacian.argtypes = [i, i, i, _dp, _dp, _dp]
    lib.ref_laplacian.restype = None
    lib.ref_stencil_apply.argtypes = [i, i, i, _dp, i, _dp, _dp]
    lib.ref_stencil_apply.restype = i
    lib.ref_wave_run.argtypes = [i, i, i, _dp, d, d, _dp, i, i, _ip, _dp, i, _ip, _dp, _dp, _dp]
    lib.ref_wave_run.restype = None
    lib.ref_energy.argtypes = [i, i, i, _dp, d, d, _dp, _dp, _dp]
    lib.ref_energy.restype = d
    lib.ref_adjoint_grad.argtypes = [i, i, i, _dp, d, d, _dp, i, i, _ip, _dp, i, _ip, _dp, _dp]
    lib.ref_adjoint_grad.restype = d
    lib.ref_adjoint_grad_ckpt.argtypes = [i, i, i, _dp, d, d, _dp, i, i, _ip, _dp, i, _ip, _dp, i,
                                          _dp, _dp]
    lib.ref_adjoint_grad_ckpt.restype = d
    lib.ref_pml_profile.argtypes = [i, i, i, i, d, _dp]
    lib.ref_pml_profile.restype = None
    lib.ref_stencil_general.argtypes = [i, i, i, i, i, _dp, _dp, _dp]
    lib.ref_stencil_general.restype = None
    lib.ref_wave_pml_run.argtypes = [i, i, i, _dp, d, d, _dp, _dp, d, i, i, _ip, _dp, i, _ip, _dp,
                                     _dp, _dp, _dp]
    lib.ref_wave_pml_run.restype = None
    lib.ref_num_threads.argtypes = []
    lib.ref_num_threads.restype = i
    lib.ref_set_num_threads.argtypes = [i]
    lib.ref_set_num_threads.restype = None
    lib.ref_set_progress.argtypes = [i]
    lib.ref_set_progress.restype = None
    _lib = lib
    return lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def coeff_vector(coeffs) -> np.ndarray:
    """[c_xyz, c_x1..4, c_y1..4, c_z1..4] as FP64."""
    c = np.empty(13, dtype=np.float64)
    c[0] = coeffs["center"]
    c[1:5] = coeffs["ax"]
    c[5:9] = coeffs["ay"]
    c[9:13] = coeffs["az"]
    return c


def padded(a, halo_value=0.0) -> np.ndarray:
    """Interior (nz, ny, nx) -> FP64 padded array with a constant halo."""
    a = np.asarray(a, dtype=np.float64)
    out = np.full(tuple(s + 2 * HALO for s in a.shape), halo_value, dtype=np.float64)
    out[HALO:-HALO, HALO:-HALO, HALO:-HALO] = a
    return out


def interior(p) -> np.ndarray:
    return p[HALO:-HALO, HALO:-HALO, HALO:-HALO]


def num_threads() -> int:
    return _load().ref_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    _load().ref_set_num_threads(int(n))


def set_progress(every: int) -> None:
    """Print a line on stderr every ``every`` time steps of the long runs
    (leapfrog and checkpointed adjoint); 0 turns it off."""
    _load().ref_set_progress(int(every))


def laplacian(u_pad, coeffs) -> np.ndarray:
    """L u on the interior (Eq. 3), reading the halo of the padded input.
    Returns an interior (nz, ny, nx) FP64 array."""
    u_pad = np.ascontiguousarray(u_pad, dtype=np.float64)
    nz, ny, nx = (s - 2 * HALO for s in u_pad.shape)
    out = np.zeros_like(u_pad)
    _load().ref_laplacian(nx, ny, nz, _p(coeff_vector(coeffs)), _p(u_pad), _p(out))
    return interior(out).copy()


def stencil_apply(u_pad, v_pad, coeffs, sweeps: int):
    """Ping-pong sweeps (paper's star2d4r listing).  Returns (u, v, in_v) as
    padded FP64 arrays, in_v = 1 when the last result is in v."""
    u = np.array(u_pad, dtype=np.float64, order="C")
    v = np.array(v_pad, dtype=np.float64, order="C")
    nz, ny, nx = (s - 2 * HALO for s in u.shape)
    in_v = _load().ref_stencil_apply(nx, ny, nz, _p(coeff_vector(coeffs)), sweeps, _p(u), _p(v))
    return u, v, in_v


def wave_run(coeffs, v, dt, dx, nsteps, src=None, amp=None, rec=None, prev=None, cur=None):
    """FP64 leapfrog run (Eq. 2, Algorithm 1).

    v: interior (nz, ny, nx).  src (ns,3) int, amp (nsteps, ns); rec (nr,3).
    prev/cur: optional padded initial states u^{-1}, u^0 (default zero).
    Returns dict(prev=u^{N-1}, cur=u^N (padded FP64), traces (nsteps, nr)).
    """
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = v.shape
    shp = (nz + 2 * HALO, ny + 2 * HALO, nx + 2 * HALO)
    prev = np.zeros(shp) if prev is None else np.array(prev, dtype=np.float64, order="C")
    cur = np.zeros(shp) if cur is None else np.array(cur, dtype=np.float64, order="C")
    src = np.zeros((0, 3), np.int32) if src is None else np.ascontiguousarray(src, np.int32)
    rec = np.zeros((0, 3), np.int32) if rec is None else np.ascontiguousarray(rec, np.int32)
    ns, nr = len(src), len(rec)
    amp = np.zeros((nsteps, max(ns, 1))) if amp is None else np.ascontiguousarray(amp, np.float64)
    traces = np.zeros((nsteps, max(nr, 1)), dtype=np.float64)
    _load().ref_wave_run(nx, ny, nz, _p(coeff_vector(coeffs)), float(dt), float(dx), _p(v),
                         int(nsteps), ns, _p(src, _ip), _p(amp), nr, _p(rec, _ip), _p(traces),
                         _p(prev), _p(cur))
    return {"prev": prev, "cur": cur, "traces": traces[:, :nr]}


def energy(coeffs, v, dt, dx, u0_pad, u1_pad) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = v.shape
    u0 = np.ascontiguousarray(u0_pad, dtype=np.float64)
    u1 = np.ascontiguousarray(u1_pad, dtype=np.float64)
    return _load().ref_energy(nx, ny, nz, _p(coeff_vector(coeffs)), float(dt), float(dx),
                              _p(v), _p(u0), _p(u1))


def adjoint_grad(coeffs, v, dt, dx, nsteps, src, amp, rec, obs):
    """Misfit J and dJ/dv (interior FP64) by the discrete adjoint."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = v.shape
    src = np.ascontiguousarray(src, np.int32)
    rec = np.ascontiguousarray(rec, np.int32)
    amp = np.ascontiguousarray(amp, np.float64)
    obs = np.ascontiguousarray(obs, np.float64)
    g = np.zeros((nz, ny, nx), dtype=np.float64)
    J = _load().ref_adjoint_grad(nx, ny, nz, _p(coeff_vector(coeffs)), float(dt), float(dx),
                                 _p(v), int(nsteps), len(src), _p(src, _ip), _p(amp),
                                 len(rec), _p(rec, _ip), _p(obs), _p(g))
    return J, g


def adjoint_grad_ckpt(coeffs, v, dt, dx, nsteps, src, amp, rec, obs, ckpt, traces=False):
    """The same J and dJ/dv with checkpointing (ref.c ``ref_adjoint_grad_ckpt``):
    the pair (u^{n0-1}, u^{n0}) is kept every ``ckpt`` steps and each segment
    recomputed, so memory is about 2 N/ckpt + ckpt fields.  Bit-identical to
    ``adjoint_grad``.  With traces=True also returns the forward traces
    R u^{n+1}, shape (nsteps, nrec)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = v.shape
    src = np.ascontiguousarray(src, np.int32).reshape(-1, 3)
    rec = np.ascontiguousarray(rec, np.int32).reshape(-1, 3)
    amp = np.ascontiguousarray(amp, np.float64).reshape(int(nsteps), max(len(src), 1))
    obs = np.ascontiguousarray(obs, np.float64)
    g = np.zeros((nz, ny, nx), dtype=np.float64)
    tr = np.zeros((int(nsteps), max(len(rec), 1)), dtype=np.float64)
    J = _load().ref_adjoint_grad_ckpt(nx, ny, nz, _p(coeff_vector(coeffs)), float(dt), float(dx),
                                      _p(v), int(nsteps), len(src), _p(src, _ip), _p(amp),
                                      len(rec), _p(rec, _ip), _p(obs), int(ckpt), _p(tr), _p(g))
    if traces:
        return J, g, tr[:, :len(rec)]
    return J, g


def pml_profile(nx, ny, nz, width, eta_max) -> np.ndarray:
    """Damping of the absorbing layer on the padded (nz+8, ny+8, nx+8) array
    (ref.c ``ref_pml_profile``): eta_max * sum over axes (d_a / W)^2."""
    out = np.zeros((nz + 2 * HALO, ny + 2 * HALO, nx + 2 * HALO))
    _load().ref_pml_profile(int(nx), int(ny), int(nz), int(width), float(eta_max), _p(out))
    return out


def stencil_general(u, w, ndim: int, sweeps: int = 1, frame=None) -> np.ndarray:
    """Stencil-suite kernel (Sec. 6 accuracy study; Eq. 3 generalised to
    star/box shapes of radius r in 2D or 3D): ``sweeps`` applications of
        out(p) = sum_k w[k] * in(p + k),  k over [-r, r]^ndim,
    each reading a zero frame around the interior (a fresh zero frame per
    sweep, as the ping-pong grids of the paper's listing keep their halo).

    u: interior array (nz, ny, nx) (or (ny, nx) for ndim 2; a 3D array with
    ndim 2 holds independent planes).  w: (2r+1,)*ndim weights, x fastest,
    w[..., r + dy, r + dx] the weight of offset (dx, dy).  Returns the
    interior FP64 result of the last sweep.  frame: optional padded array
    (nz + 2*hz, ny + 8, nx + 8) (hz = 4 for ndim 3, else 0) whose frame the
    first sweep reads instead of zeros.
    """
    lib = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    r = (w.shape[0] - 1) // 2
    assert w.shape == (2 * r + 1,) * ndim and 1 <= r <= HALO and ndim in (2, 3)
    a = np.asarray(u, dtype=np.float64)
    flat2d = a.ndim == 2
    if flat2d:
        a = a[None]
    assert a.ndim == 3
    nz, ny, nx = a.shape
    hz = HALO if ndim == 3 else 0
    shp = (nz + 2 * hz, ny + 2 * HALO, nx + 2 * HALO)
    cur = np.zeros(shp)
    if frame is not None:
        cur[...] = np.asarray(frame, dtype=np.float64).reshape(shp)
    cur[hz:hz + nz, HALO:-HALO, HALO:-HALO] = a
    for _ in range(sweeps):
        nxt = np.zeros(shp)
        lib.ref_stencil_general(nx, ny, nz, ndim, r, _p(w), _p(cur), _p(nxt))
        cur = nxt
    out = cur[hz:hz + nz, HALO:-HALO, HALO:-HALO].copy()
    return out[0] if flat2d else out


def wave_pml_run(coeffs, v, eta_pad, dt, dx, nsteps, src=None, amp=None, rec=None, prev=None,
                 cur=None, psi=None, alpha=0.0):
    """Leapfrog with the absorbing layer (ref.c ``ref_wave_pml_run``).
    eta_pad: padded (nz+8, ny+8, nx+8) damping field in 1/s, frame read.
    Returns dict(prev, cur, psi (padded), traces)."""
    lib = _load()
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = v.shape
    eta = np.ascontiguousarray(eta_pad, dtype=np.float64)
    assert eta.shape == (nz + 8, ny + 8, nx + 8)
    prev = np.zeros((nz + 8, ny + 8, nx + 8)) if prev is None else np.array(prev, dtype=np.float64)
    cur = np.zeros_like(prev) if cur is None else np.array(cur, dtype=np.float64)
    psi = np.zeros_like(prev) if psi is None else np.array(psi, dtype=np.float64)
    src = np.zeros((0, 3), np.int32) if src is None else np.ascontiguousarray(src, dtype=np.int32)
    nsrc = len(src)
    amp = np.zeros((nsteps, max(nsrc, 1))) if amp is None else np.ascontiguousarray(amp, dtype=np.float64)
    rec = np.zeros((0, 3), np.int32) if rec is None else np.ascontiguousarray(rec, dtype=np.int32)
    traces = np.zeros((nsteps, max(len(rec), 1)))
    lib.ref_wave_pml_run(nx, ny, nz, _p(coeff_vector(coeffs)), float(dt), float(dx), _p(v), _p(eta),
                         float(alpha), int(nsteps), nsrc, _p(src, _ip), _p(amp), len(rec), _p(rec, _ip),
                         _p(traces), _p(prev), _p(cur), _p(psi))
    return {"prev": prev, "cur": cur, "psi": psi, "traces": traces[:, :len(rec)]}
