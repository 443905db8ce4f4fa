"""Helpers for the GPU parity tests: error metrics and oracle sampling.

Inputs come from ``synth``; expected values come from ``oracle`` only.
"""

from __future__ import annotations

import contextlib

import numpy as np

import oracle


def errors(got, ref) -> dict:
    """rel-L2 (FP64 sums), max abs and RMSD (the paper's Sec. 13.1 metrics)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    nref = float(np.sqrt(np.sum(ref * ref)))
    return {"rel_l2": float(np.sqrt(np.sum(d * d))) / (nref if nref > 0 else 1.0),
            "max_abs": float(np.max(np.abs(d))) if d.size else 0.0,
            "rmsd": float(np.sqrt(np.mean(d * d))) if d.size else 0.0}


def sample_points(nx, ny, nz, n, seed) -> np.ndarray:
    """Random interior points plus every corner and face-centre point."""
    rng = np.random.default_rng(seed)
    pts = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)))
           for _ in range(n)]
    for x in (0, nx - 1):
        for y in (0, ny - 1):
            for z in (0, nz - 1):
                pts.append((x, y, z))
    pts += [(0, ny // 2, nz // 2), (nx - 1, ny // 2, nz // 2), (nx // 2, 0, nz // 2),
            (nx // 2, ny - 1, nz // 2), (nx // 2, ny // 2, 0), (nx // 2, ny // 2, nz - 1)]
    return np.array(pts, dtype=np.int32)


def patch(padded, x, y, z) -> np.ndarray:
    """9x9x9 FP64 neighbourhood of interior point (x, y, z) of a padded array
    (the 1x1x1 interior of a padded block whose halo is the neighbourhood)."""
    return np.asarray(padded[z:z + 9, y:y + 9, x:x + 9], dtype=np.float64)


def oracle_star_at(padded, coeffs, pts) -> np.ndarray:
    """L u at each point, computed by the oracle on the point's neighbourhood."""
    out = np.empty(len(pts))
    for k, (x, y, z) in enumerate(pts):
        out[k] = oracle.laplacian(patch(padded, x, y, z), coeffs)[0, 0, 0]
    return out


def oracle_wave_at(prev_pad, cur_pad, v, coeffs, dt, dx, pts, src=None, amp_row=None) -> np.ndarray:
    """One leapfrog step at each point (oracle.wave_run on the neighbourhood)."""
    out = np.empty(len(pts))
    for k, (x, y, z) in enumerate(pts):
        s, a = None, None
        if src is not None:
            hit = [j for j, p in enumerate(src) if tuple(int(q) for q in p) == (x, y, z)]
            if hit:
                s = np.array([[0, 0, 0]] * len(hit), np.int32)
                a = np.array([[float(amp_row[j]) for j in hit]])
        r = oracle.wave_run(coeffs, np.array([[[v[z, y, x]]]], dtype=np.float64), dt, dx, 1,
                            src=s, amp=a, prev=patch(prev_pad, x, y, z), cur=patch(cur_pad, x, y, z))
        out[k] = r["cur"][4, 4, 4]
    return out


def errors_chunked(got, ref, chunk=32) -> dict:
    """errors() of two (nz, ny, nx) arrays, accumulated over z-chunks so that
    full-size fields need no full-size FP64 temporaries.  The sums are FP64."""
    nz = got.shape[0]
    sd = sr = 0.0
    mx = 0.0
    for z0 in range(0, nz, chunk):
        a = np.asarray(got[z0:z0 + chunk], dtype=np.float64)
        b = np.asarray(ref[z0:z0 + chunk], dtype=np.float64)
        d = a - b
        sd += float(np.sum(d * d))
        sr += float(np.sum(b * b))
        if d.size:
            mx = max(mx, float(np.max(np.abs(d))))
    n = got.size
    return {"rel_l2": float(np.sqrt(sd)) / (float(np.sqrt(sr)) if sr > 0 else 1.0),
            "max_abs": mx, "rmsd": float(np.sqrt(sd / n)) if n else 0.0}


@contextlib.contextmanager
def oracle_progress(capsys, every=100):
    """Let the oracle's own progress lines (one per ``every`` steps of a long
    run) reach the terminal past pytest's output capture."""
    oracle.set_progress(every)
    try:
        with capsys.disabled():
            yield
    finally:
        oracle.set_progress(0)
