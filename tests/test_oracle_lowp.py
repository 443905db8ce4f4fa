"""Pins for the FP16/BF16 storage emulation (oracle/lowp.py).

Rounding is checked against exact ties and numpy's own FP16 conversion; the
scale rule against hand-computed exponents and its guarantee |q| <= 2^15.
"""

import numpy as np
import pytest

import oracle
from oracle import lowp
import synth


def test_fp16_rounding_exact_cases():
    r = lambda x: float(lowp.round_to(x, "f16"))     # noqa: E731
    assert r(1 + 2 ** -11) == 1.0                    # tie -> even
    assert r(1 + 3 * 2 ** -11) == 1 + 2 ** -9        # tie -> even (up)
    assert r(1 + 2 ** -11 + 2 ** -30) == 1 + 2 ** -10
    assert r(2 ** -25) == 0.0                        # half the min subnormal -> 0 (even)
    assert r(3 * 2 ** -25) == 2 ** -23               # tie between 2^-24 and 2^-23 -> even
    assert r(-1.5 * 2 ** -24) == -2 ** -23
    assert r(65504.0) == 65504.0
    assert r(2 ** 15 + 15) == 2 ** 15                # spacing 32 above 2^15
    assert r(2 ** 15 + 17) == 2 ** 15 + 32
    assert r(2 ** 15 + 16) == 2 ** 15                # tie -> even


def test_fp16_rounding_matches_numpy():
    x = np.random.default_rng(0).standard_normal(200000) * np.exp(
        np.random.default_rng(1).uniform(-25, 10, 200000))
    x = x[np.abs(x) < 65000]                 # the finite range (no overflow handling needed)
    ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(lowp.round_to(x, "f16"), ref)


def test_bf16_rounding_exact_cases():
    r = lambda x: float(lowp.round_to(x, "bf16"))    # noqa: E731
    assert r(1 + 2 ** -8) == 1.0                     # tie -> even
    assert r(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert r(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert r(3.0 * 2 ** -134) == 2 ** -132           # subnormal tie -> even
    # against truncation of FP32 bits with the round-half-even increment
    x = np.random.default_rng(2).standard_normal(100000).astype(np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    ref = b.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(lowp.round_to(x.astype(np.float64), "bf16"), ref)


def test_ulp():
    assert lowp.ulp(1.0, "f16") == 2 ** -10
    assert lowp.ulp(1.0, "bf16") == 2 ** -7
    assert lowp.ulp(0.0, "f16") == 2 ** -24
    assert lowp.ulp(40000.0, "f16") == 32.0


def test_scale_rule_exponents():
    # B = 8 * max(...) + |inj|; e = ceil(log2 B) - 15
    nz = 48
    a_cur = np.array([0.0, 1.0, 0.0], np.float32)
    a_prev = np.array([0.0, 0.0, 3.0], np.float32)
    s = lowp.next_scales(a_cur, a_prev, nz, 1.0, None, None, None)
    # slab 0: B = 8*1 = 8 = 2^3 -> e = -12; slab 1: 8 -> -12; slab 2: 8*3 = 24 -> ceil = 5 -> -10
    assert list(s) == [2.0 ** -12, 2.0 ** -12, 2.0 ** -10]
    s = lowp.next_scales(np.zeros(3, np.float32), np.zeros(3, np.float32), nz, 1.0, None, None, None)
    assert list(s) == [1.0, 1.0, 1.0]
    # an injection alone sets the scale of its slab only
    v = np.full((nz, 4, 4), 2.0, np.float32)
    s = lowp.next_scales(np.zeros(3, np.float32), np.zeros(3, np.float32), nz, 0.5,
                         np.array([[1, 1, 20]]), np.array([3.0], np.float32), v)
    # inj = 0.25 * 4 * 3 = 3 -> ceil(log2 3) = 2 -> e = -13
    assert list(s) == [1.0, 2.0 ** -13, 1.0]


def test_scale_rule_exponent_is_clamped():
    # tiny and huge slab maxima: e = ceil(log2 B) - 15 is clamped to
    # [-110, 110], so the scale and its reciprocal stay normal FP32 numbers
    a_cur = np.array([2.0 ** -100, 2.0 ** -98, 2.0 ** 100, 2.0 ** 124], np.float32)
    s = lowp.next_scales(a_cur, np.zeros(4, np.float32), 64, 1.0, None, None, None)
    # slab 0: B = 8 max(2^-100, 2^-98) = 2^-95 -> e = -110 (exactly the bound)
    # slab 1: B = 8 * 2^100 = 2^103 -> e = 88
    # slabs 2, 3: B = 8 * 2^124 = 2^127 -> e = 112, clamped to 110
    assert list(s) == [2.0 ** -110, 2.0 ** 88, 2.0 ** 110, 2.0 ** 110]
    s = lowp.next_scales(np.array([2.0 ** -120], np.float32), np.zeros(1, np.float32), 16, 1.0,
                         None, None, None)
    assert list(s) == [2.0 ** -110]          # 2^-117 - 15 = -132 -> -110
    assert np.isfinite(1.0 / s).all() and (s >= np.finfo(np.float32).tiny).all()


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_step_keeps_stored_values_in_range(fmt):
    # Worst-case growth inside the stability limit: |q_next| <= 2^15.
    co = synth.star25_coeffs()
    nz, ny, nx = 40, 12, 12
    rng = np.random.default_rng(5)
    v = np.full((nz, ny, nx), 3000.0, np.float32)
    dx = 10.0
    dt = 0.45 * dx / 3000.0                    # just inside sqrt(105/512)
    n = lowp.nslab(nz)
    s = np.float32(2.0 ** -5) * np.ones(n, np.float32)
    # alternating signs: the Nyquist pattern maximises |L u|
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sign = (-1.0) ** (x + y + z)
    q_cur = lowp.round_to(sign * 2 ** 12 * rng.uniform(0.99, 1.0, (nz, ny, nx)), fmt)
    q_prev = q_cur.copy()                      # -u^{n-1} adds to m L u^n here
    a = lowp.slab_amax(q_cur, s)
    qn, sn, an, un = lowp.step(co, v, dt, dx, fmt, q_prev, s, a, q_cur, s, a)
    assert np.max(np.abs(qn)) <= 2 ** 15
    assert np.max(np.abs(qn)) > 2 ** 13        # the bound is not vacuous here
    dec = qn * lowp.plane_scales(sn, nz)[:, None, None]
    assert np.all(np.abs(dec - un) <= 0.5 * lowp.ulp(qn, fmt) * lowp.plane_scales(sn, nz)[:, None, None])


def test_run_converges_to_fp64_for_fp16():
    # FP16 storage error after 30 steps is small but nonzero, BF16 larger.
    p = synth.wave_problem(24, 20, 36, 30)
    co = synth.star25_coeffs()
    ref = oracle.wave_run(co, p["v"], p["dt"], p["dx"], 30, src=p["src"], amp=p["amp"])
    ref = oracle.interior(ref["cur"])
    e16 = np.linalg.norm(lowp.run(co, p["v"], p["dt"], p["dx"], "f16", 30, p["src"], p["amp"])[0] - ref)
    e8 = np.linalg.norm(lowp.run(co, p["v"], p["dt"], p["dx"], "bf16", 30, p["src"], p["amp"])[0] - ref)
    n = np.linalg.norm(ref)
    assert 0 < e16 / n < 5e-3
    assert e16 < e8 < 5e-2 * n
