"""Emulation of the leapfrog with FP16/BF16 wavefield storage.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Storage rule (an extension of the paper's FP32 method, Eq. 2): a stored field
value is q * s_k, where q is an FP16 or BF16 number and s_k = 2^e_k is the
scale of the 16-plane z-slab k holding the point.  One step computes u^{n+1}
exactly (here in FP64, the oracle's precision) from the decoded inputs, then
stores q = RNE(u^{n+1} / s_k) with the slab exponent chosen before the step:

    B_k = 8 * max(amax(u^n) on slabs k-1..k+1, amax(u^{n-1}) on slab k)
          + sum over sources s in slab k of |dt^2 v_s^2 a_s|,
    e_k = ceil(log2 B_k) - 15   (s_k = 1 when B_k = 0),

so that |q| <= 2^15 whatever the step does inside the stability limit.  The
exponent is an integer decided by floating point, so it is taken here in the
kernel's precision (IEEE FP32, same operation order); everything else is FP64.
amax(field)[k] = max |q| * s_k over slab k.

Rounding: RNE to the format's significand width (11 bits FP16, 8 bits BF16)
with gradual underflow (FP16 subnormal spacing 2^-24, BF16 2^-133), written
from the format definitions.
"""

from __future__ import annotations

import numpy as np

import oracle

SLAB = 16
FORMATS = {"f16": (11, -24), "bf16": (8, -133)}   # significant bits, log2(min spacing)


def round_to(x, fmt: str) -> np.ndarray:
    """Round FP64 values to the nearest FP16/BF16 value, ties to even."""
    bits, emin = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                       # |x| in [2^(e-1), 2^e)
    spacing = np.ldexp(1.0, np.maximum(e - bits, emin))
    return np.rint(x / spacing) * spacing    # np.rint rounds half to even


def ulp(x, fmt: str) -> np.ndarray:
    """Spacing of the format at |x| (at the larger side of a binade edge)."""
    bits, emin = FORMATS[fmt]
    a = np.abs(np.asarray(x, dtype=np.float64))
    _, e = np.frexp(a)
    e = np.where(a == 0, emin + bits, e)      # zero: the subnormal spacing
    return np.ldexp(1.0, np.maximum(e - bits, emin))


def nslab(nz: int) -> int:
    return (nz + SLAB - 1) // SLAB


def plane_scales(s, nz: int) -> np.ndarray:
    """Per-plane scale for planes 0..nz-1."""
    return np.asarray(s, np.float64)[np.arange(nz) // SLAB]


def slab_amax(q, s) -> np.ndarray:
    """max |q| * s_k per slab (exact)."""
    nz = q.shape[0]
    out = np.zeros(nslab(nz), np.float32)
    for k in range(nslab(nz)):
        out[k] = np.float32(np.max(np.abs(q[k * SLAB:(k + 1) * SLAB])) * s[k])
    return out


def _ceil_log2_f32(B: np.float32) -> int:
    m, E = np.frexp(np.float32(B))
    return int(E) - 1 if m == 0.5 else int(E)


def next_scales(amax_cur, amax_prev, nz, dt, src, amp_row, v) -> np.ndarray:
    """Slab scales of u^{n+1} by the rule above, decided in IEEE FP32."""
    f = np.float32
    n = nslab(nz)
    dt2 = f(dt * dt)
    s = np.ones(n, np.float32)
    for k in range(n):
        M = f(amax_cur[k])
        if k > 0:
            M = max(M, f(amax_cur[k - 1]))
        if k + 1 < n:
            M = max(M, f(amax_cur[k + 1]))
        M = max(M, f(amax_prev[k]))
        B = f(8.0) * M
        if src is not None:
            for j, (x, y, z) in enumerate(src):
                if int(z) // SLAB == k:
                    vs = f(v[int(z), int(y), int(x)])
                    inj = f(f(dt2 * f(vs * vs)) * f(amp_row[j]))
                    B = f(B + f(abs(inj)))
        if not B > 0:
            continue
        e = min(max(_ceil_log2_f32(B) - 15, -110), 110)
        s[k] = f(2.0 ** e)
    return s


def step(coeffs, v, dt, dx, fmt, q_prev, s_prev, a_prev, q_cur, s_cur, a_cur,
         src=None, amp_row=None):
    """One storage-rounded leapfrog step.

    q_*: stored values (interior (nz, ny, nx), as FP64); s_*: per-slab scales;
    a_*: per-slab maxima.  Returns (q_next, s_next, a_next, u_next_exact) where
    u_next_exact is the FP64 value before storage rounding.
    """
    nz = q_cur.shape[0]
    cur = np.asarray(q_cur, np.float64) * plane_scales(s_cur, nz)[:, None, None]
    prev = np.asarray(q_prev, np.float64) * plane_scales(s_prev, nz)[:, None, None]
    amp = None if src is None else np.asarray(amp_row, np.float64)[None, :]
    r = oracle.wave_run(coeffs, v, dt, dx, 1, src=src, amp=amp,
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    u_next = oracle.interior(r["cur"]).copy()
    s_next = next_scales(a_cur, a_prev, nz, dt, src, amp_row, v)
    q_next = round_to(u_next / plane_scales(s_next, nz)[:, None, None], fmt)
    return q_next, s_next, slab_amax(q_next, s_next), u_next


def run(coeffs, v, dt, dx, fmt, nsteps, src=None, amp=None, rec=None):
    """nsteps storage-rounded steps from zero fields.  Returns the final
    decoded field u^N (FP64 interior) and the traces (decoded stored values
    at the receivers after each step)."""
    nz, ny, nx = v.shape
    n = nslab(nz)
    q_prev = np.zeros((nz, ny, nx))
    q_cur = np.zeros((nz, ny, nx))
    s_prev = np.zeros(n, np.float32)
    s_cur = np.zeros(n, np.float32)
    a_prev = np.zeros(n, np.float32)
    a_cur = np.zeros(n, np.float32)
    traces = []
    for k in range(nsteps):
        q_next, s_next, a_next, _ = step(coeffs, v, dt, dx, fmt, q_prev, s_prev, a_prev,
                                         q_cur, s_cur, a_cur, src=src,
                                         amp_row=None if amp is None else amp[k])
        q_prev, s_prev, a_prev = q_cur, s_cur, a_cur
        q_cur, s_cur, a_cur = q_next, s_next, a_next
        if rec is not None:
            dec = q_cur * plane_scales(s_cur, nz)[:, None, None]
            traces.append([dec[int(z), int(y), int(x)] for (x, y, z) in rec])
    return q_cur * plane_scales(s_cur, nz)[:, None, None], np.array(traces)
