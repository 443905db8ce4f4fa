"""Seeded synthetic inputs for the star-stencil wave workloads.

This module is shared by the tests, the benchmark and the oracle.  It only
draws and arranges input data (fields, velocity models, wavelets, point sets,
coefficient sets); it performs none of the stencil, leapfrog, adjoint or
storage-encoding arithmetic.

Array convention: fields are numpy arrays of shape (nz, ny, nx) holding the
interior only, x fastest (i <-> x, j <-> y, k <-> z in the paper's Eq. 3).
Point sets are int32 arrays of shape (n, 3) holding (x, y, z) interior indices.
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

HALO = 4

# Eighth-order central second-derivative weights for unit spacing, offsets
# 0..4 (the discretisation parameters of the paper's Eq. 3 are left open; this
# is the standard radius-4 set).  Exact rationals; callers round as needed.
FD8_WEIGHTS = (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
               Fraction(8, 315), Fraction(-1, 560))


def star25_coeffs(scale: float = 1.0) -> dict:
    """Coefficient set for the 25-point star: centre and per-axis arrays.

    The centre weight is the sum of the three axes' offset-0 weights.  Each
    value is exact in FP64 up to one rounding of the rational.
    """
    w = [float(f) * scale for f in FD8_WEIGHTS]
    return {
        "center": 3.0 * float(FD8_WEIGHTS[0]) * scale,
        "ax": w[1:], "ay": w[1:], "az": w[1:],
    }


def integer_coeffs() -> dict:
    """5040 x the eighth-order set: integer weights (centre -43050)."""
    w = [int(f * 5040) for f in FD8_WEIGHTS]
    return {"center": float(3 * w[0]), "ax": [float(a) for a in w[1:]],
            "ay": [float(a) for a in w[1:]], "az": [float(a) for a in w[1:]]}


def random_coeffs(seed: int) -> dict:
    """Anisotropic random coefficient set (distinct per axis) for parity tests."""
    rng = np.random.default_rng(seed)
    return {"center": float(rng.uniform(-3, -1)),
            "ax": [float(a) for a in rng.uniform(-1, 1, 4)],
            "ay": [float(a) for a in rng.uniform(-1, 1, 4)],
            "az": [float(a) for a in rng.uniform(-1, 1, 4)]}


def uniform_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0,
                  dtype=np.float32) -> np.ndarray:
    """u ~ U[lo, hi] i.i.d. over the interior, shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def integer_field(shape, seed: int, bound: int = 170) -> np.ndarray:
    """Integers in [-bound, bound] (as float32, exactly representable)."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=shape).astype(np.float32)


def layered_velocity(nx: int, ny: int, nz: int, seed: int, nlayers: int = 8,
                     vmin: float = 1500.0, vmax: float = 4500.0) -> np.ndarray:
    """Horizontal layers of equal thickness nz // nlayers (the last layer takes
    the remainder); per-layer speeds i.i.d. U[vmin, vmax], unsorted.  FP32."""
    rng = np.random.default_rng(seed)
    speeds = rng.uniform(vmin, vmax, size=nlayers)
    thick = max(nz // nlayers, 1)
    v = np.empty((nz, ny, nx), dtype=np.float32)
    for k in range(nz):
        v[k] = speeds[min(k // thick, nlayers - 1)]
    return v


def gaussian_bump(v: np.ndarray, center, sigma: float, frac: float) -> np.ndarray:
    """v * (1 + frac * exp(-|x - c|^2 / (2 sigma^2))), c = (x, y, z); FP32."""
    nz, ny, nx = v.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = center
    r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
    return (v.astype(np.float64) * (1.0 + frac * np.exp(-r2 / (2.0 * sigma ** 2)))
            ).astype(np.float32)


def adjoint_models(n: int, seed: int = 0):
    """Velocity models of the n^3 misfit-gradient workload: the model v0 is
    the layered model (seed) with a 10 % Gaussian anomaly at (n/2, n/2,
    3n/16), sigma 10n/256 cells; the data come from v_obs, v0 with a further
    5 % Gaussian at (3n/8, 5n/8, n/4), sigma 12n/256.  Both anomalies lie
    within the depth whose reflections reach the receiver plane z = 8 within
    1000 steps at n = 256 (two-way vertical time about 0.28 s and 0.42 s of
    the 0.92 s simulated).  Returns (v0, v_obs), FP32 (nz, ny, nx)."""
    v = layered_velocity(n, n, n, seed)
    v0 = gaussian_bump(v, (n // 2, n // 2, 3 * n // 16), 10.0 * n / 256, 0.10)
    v_obs = gaussian_bump(v0, (3 * n // 8, 5 * n // 8, n // 4), 12.0 * n / 256, 0.05)
    return v0, v_obs


def cfl_dt(v: np.ndarray, dx: float, cfl: float = 0.4) -> float:
    """Time step at a given Courant number: dt = cfl * dx / max(v) (FP64)."""
    return cfl * dx / float(np.max(v))


def ricker(nsteps: int, dt: float, f0: float = 15.0, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet samples w(n dt), n = 0..nsteps-1, FP64.

    w(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0,
    t0 = 1.5 / f0 by default.
    """
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nsteps, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def center_point(nx: int, ny: int, nz: int) -> np.ndarray:
    return np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32)


def receiver_plane(nx: int, ny: int, z: int, stride: int) -> np.ndarray:
    """Receivers on the plane z at every stride-th cell in x and y."""
    ys, xs = np.meshgrid(np.arange(0, ny, stride), np.arange(0, nx, stride), indexing="ij")
    n = xs.size
    pts = np.empty((n, 3), dtype=np.int32)
    pts[:, 0] = xs.ravel()
    pts[:, 1] = ys.ravel()
    pts[:, 2] = z
    return pts


def random_points(nx: int, ny: int, nz: int, n: int, seed: int, margin: int = 0) -> np.ndarray:
    """n distinct random interior points at least `margin` cells from faces."""
    rng = np.random.default_rng(seed)
    seen = set()
    out = []
    while len(out) < n:
        p = (int(rng.integers(margin, nx - margin)), int(rng.integers(margin, ny - margin)),
             int(rng.integers(margin, nz - margin)))
        if p not in seen:
            seen.add(p)
            out.append(p)
    return np.array(out, dtype=np.int32).reshape(n, 3)


def pad(a: np.ndarray, value: float = 0.0, dtype=None) -> np.ndarray:
    """Embed an interior (nz, ny, nx) array in a HALO-wide frame."""
    dt = a.dtype if dtype is None else dtype
    out = np.full(tuple(s + 2 * HALO for s in a.shape), value, dtype=dt)
    out[HALO:-HALO, HALO:-HALO, HALO:-HALO] = a
    return out


def wave_problem(nx: int, ny: int, nz: int, nsteps: int, seed: int = 0,
                 dx: float = 10.0, cfl: float = 0.4, f0: float = 15.0,
                 src=None, rec=None) -> dict:
    """A complete forward-modelling input: layered v, dt, Ricker at a point.

    Returns a dict with v (FP32 interior), dt, dx, src (n,3), wavelet
    (nsteps, nsrc) FP64 source samples, rec (m,3).
    """
    v = layered_velocity(nx, ny, nz, seed)
    dt = cfl_dt(v, dx, cfl)
    if src is None:
        src = center_point(nx, ny, nz)
    w = ricker(nsteps, dt, f0)
    amp = np.repeat(w[:, None], len(src), axis=1)
    if rec is None:
        rec = np.zeros((0, 3), dtype=np.int32)
    return {"v": v, "dt": dt, "dx": dx, "src": np.asarray(src, np.int32),
            "amp": amp, "rec": np.asarray(rec, np.int32), "nsteps": nsteps}


# ---------------------------------------------------------------------------
# Stencil suite of the paper's accuracy study (Sec. 6 table of kernels): star
# and box shapes of radius 1..4 in 2D and 3D, plus four classic Jacobi
# kernels.  name -> (shape, ndim, radius).  The paper does not print their
# weights; suite_weights draws seeded ones.
SUITE = {}
for _d in (2, 3):
    for _r in (1, 2, 3, 4):
        SUITE["star%dd%dr" % (_d, _r)] = ("star", _d, _r)
for _d in (2, 3):
    for _r in (1, 2, 3, 4):
        SUITE["box%dd%dr" % (_d, _r)] = ("box", _d, _r)
SUITE.update({"j2d5pt": ("star", 2, 1), "j2d9pt-gol": ("box", 2, 1),
              "j2d9pt": ("star", 2, 2), "j3d27pt": ("box", 3, 1)})


def stencil_support(shape: str, ndim: int, r: int) -> np.ndarray:
    """Boolean (2r+1,)*ndim mask of the offsets a kernel of this shape uses:
    every offset for a box, the centre and the axis lines for a star."""
    if shape == "box":
        return np.ones((2 * r + 1,) * ndim, dtype=bool)
    m = np.zeros((2 * r + 1,) * ndim, dtype=bool)
    for ax in range(ndim):
        idx = [r] * ndim
        idx[ax] = slice(None)
        m[tuple(idx)] = True
    return m


def suite_weights(name: str, seed: int, signed: bool = False) -> np.ndarray:
    """Seeded weights for a suite kernel: dense (2r+1,)*ndim FP64 array,
    index [dz][dy][dx] (x fastest), zero off the kernel's support.  Default:
    positive weights U[0.05, 1] scaled to sum 1 (an averaging kernel, so
    repeated sweeps keep values in range); signed=True: U[-1, 1]."""
    shape, ndim, r = SUITE[name]
    rng = np.random.default_rng(seed)
    m = stencil_support(shape, ndim, r)
    if signed:
        w = rng.uniform(-1.0, 1.0, m.shape)
    else:
        w = rng.uniform(0.05, 1.0, m.shape)
    w = np.where(m, w, 0.0)
    if not signed:
        w /= w.sum()
    return w


def listing_star2d4r_weights() -> np.ndarray:
    """The star2d4r weights of the paper's example kernel (Sec. 5 listing),
    as a 9x9 array [dy + 4][dx + 4]; the first offset of the listing's
    ``at(., .)`` is read as x."""
    w = np.zeros((9, 9))
    w[4, 4] = 0.25005
    for d, c in zip((1, 2, 3, 4), (0.06245, 0.06255, 0.06251, 0.11111)):
        w[4, 4 - d] = w[4, 4 + d] = c
    for d, c in zip((1, 2, 3, 4), (0.06248, 0.06243, 0.06253, -0.22220)):
        w[4 - d, 4] = w[4 + d, 4] = c
    return w


def suite_field(shape, seed: int, lo: float = 1e-4, hi: float = 1e5) -> np.ndarray:
    """Positive values log-uniform in [lo, hi] (the accuracy study's inputs
    span 1e-4 .. 1e5), FP32-representable."""
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(np.log(lo), np.log(hi), shape))
    return a.astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Absorbing layer (the paper's PML region).  Damping profile of a layer of
# `width` cells on every face: eta = eta_max * sum over axes (d_a / width)^2,
# d_a = max(0, width - 1 - a, a - (n_a - width)) the depth of index a into
# the layer (0 on the layer's inner face, growing into the halo frame).  The
# cells next to the inner box have eta = 0 on both sides, so grad eta
# vanishes on the inner box.

def pml_eta_max(v_max: float, width: int, dx: float, reflection: float = 1e-3) -> float:
    """Peak damping (1/s) of a quadratic profile with the given nominal
    reflection coefficient: 3 v ln(1/R) / (2 W dx) (Collino and Tsogka)."""
    return 3.0 * v_max * math.log(1.0 / reflection) / (2.0 * width * dx)


def pml_profile(nx: int, ny: int, nz: int, width: int, eta_max: float) -> np.ndarray:
    """Damping on the padded (nz+8, ny+8, nx+8) array (frame included), FP64."""
    def depth(n):
        a = np.arange(-HALO, n + HALO)
        return np.maximum(0, np.maximum(width - 1 - a, a - (n - width))) / width
    dz, dy, dx_ = depth(nz), depth(ny), depth(nx)
    return eta_max * (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx_[None, None, :] ** 2)
