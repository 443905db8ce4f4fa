"""Pins for the oracle's 25-point star (paper Sec. 2.2, Eq. 3).

Each test checks the C oracle against something fixed by the mathematics, not
against a retyped copy of its own loop: exact polynomial reproduction, the
impulse response, symmetries, exact-rational brute force, and the
ping-pong semantics of the paper's star2d4r listing.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

INT_W = [-14350, 8064, -1008, 128, -9]          # 5040 x FD8 weights, offsets 0..4


def test_fd8_weights_are_the_integer_set():
    # 5040 * (-205/72, 8/5, -1/5, 8/315, -1/560) are integers; 1D sum is 0.
    w = [f * 5040 for f in synth.FD8_WEIGHTS]
    assert all(x.denominator == 1 for x in w)
    assert [int(x) for x in w] == INT_W
    assert INT_W[0] + 2 * sum(INT_W[1:]) == 0


def _poly_values(terms, shape):
    """Evaluate sum a * x^i y^j z^k on the padded grid, coordinates centred so
    that |x|,|y|,|z| stay small.  Returns (padded values, exact 5040*lap on the
    interior) as Python-int-exact float64 arrays."""
    nz, ny, nx = shape
    H = 4
    off = [nx // 2, ny // 2, nz // 2]
    P = np.zeros((nz + 2 * H, ny + 2 * H, nx + 2 * H))
    LAP = np.zeros(shape)
    for z in range(-H, nz + H):
        for y in range(-H, ny + H):
            for x in range(-H, nx + H):
                X, Y, Z = x - off[0], y - off[1], z - off[2]
                val = 0
                lap = 0
                for (a, i, j, k) in terms:
                    val += a * X ** i * Y ** j * Z ** k
                    if i >= 2:
                        lap += a * i * (i - 1) * X ** (i - 2) * Y ** j * Z ** k
                    if j >= 2:
                        lap += a * j * (j - 1) * X ** i * Y ** (j - 2) * Z ** k
                    if k >= 2:
                        lap += a * k * (k - 1) * X ** i * Y ** j * Z ** (k - 2)
                assert abs(val) < 2 ** 53 // 98304
                P[z + H, y + H, x + H] = val
                if 0 <= x < nx and 0 <= y < ny and 0 <= z < nz:
                    LAP[z, y, x] = 5040 * lap
    return P, LAP


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_on_polynomials_up_to_degree_9(seed):
    # The radius-4 eighth-order weights differentiate x^d exactly for d <= 9,
    # so 5040*L P equals 5040*lap(P) exactly in int64 (FP64 here: every value
    # stays below 2^53 / sum|w| so every partial sum is exact).
    rng = np.random.default_rng(seed)
    terms = [(3, 9, 0, 0), (-2, 0, 9, 0), (1, 0, 0, 9), (2, 8, 2, 0)]
    for _ in range(4):
        i, j, k = (int(a) for a in rng.integers(0, 10, 3))
        while i + j + k > 11:
            i, j, k = (int(a) for a in rng.integers(0, 10, 3))
        terms.append((int(rng.integers(-3, 4)), i, j, k))
    shape = (5, 6, 7)
    P, LAP = _poly_values(terms, shape)
    out = oracle.laplacian(P, synth.integer_coeffs())
    assert np.array_equal(out, LAP)


def test_degree_10_is_not_exact():
    # The pin above must be able to fail: x^10 is outside the exact range.
    P, LAP = _poly_values([(1, 10, 0, 0)], (3, 3, 5))
    out = oracle.laplacian(P, synth.integer_coeffs())
    assert not np.array_equal(out, LAP)


def test_constant_maps_to_zero():
    c = np.full((6, 7, 8), 3.0)
    out = oracle.laplacian(oracle.padded(c, halo_value=3.0), synth.integer_coeffs())
    assert np.all(out == 0.0)
    out = oracle.laplacian(oracle.padded(c, halo_value=3.0), synth.star25_coeffs())
    assert np.max(np.abs(out)) < 1e-13


def test_impulse_returns_the_coefficient_table():
    co = synth.random_coeffs(7)          # anisotropic: a transposed axis fails
    nz, ny, nx = 11, 12, 13
    u = np.zeros((nz, ny, nx))
    px, py, pz = 6, 5, 4
    u[pz, py, px] = 1.0
    out = oracle.laplacian(oracle.padded(u), co)
    expect = np.zeros_like(out)
    expect[pz, py, px] = co["center"]
    for m in range(1, 5):
        for s in (-1, 1):
            expect[pz, py, px + s * m] = co["ax"][m - 1]
            expect[pz, py + s * m, px] = co["ay"][m - 1]
            expect[pz + s * m, py, px] = co["az"][m - 1]
    assert np.array_equal(out, expect)


def test_star_has_25_points_and_49_flops():
    # Paper Table "Kernels for numerical correctness evaluation": star3d4r has
    # 49 FLOPs = 2 * points - 1, i.e. 25 points.
    co = {"center": 1.0, "ax": [1.0] * 4, "ay": [1.0] * 4, "az": [1.0] * 4}
    u = np.zeros((9, 9, 9))
    u[4, 4, 4] = 1.0
    out = oracle.laplacian(oracle.padded(u), co)
    npts = int(np.count_nonzero(out))
    assert npts == 25 and 2 * npts - 1 == 49


def test_mirror_and_permutation_symmetry():
    co = synth.star25_coeffs()
    u = synth.uniform_field((9, 10, 11), 3).astype(np.float64)
    base = oracle.laplacian(oracle.padded(u), co)
    for ax in range(3):
        flipped = oracle.laplacian(oracle.padded(np.flip(u, axis=ax).copy()), co)
        assert np.allclose(flipped, np.flip(base, axis=ax), rtol=0, atol=1e-12)
    # swap x and y with anisotropic coefficients swapped accordingly
    ca = synth.random_coeffs(11)
    cs = dict(ca, ax=ca["ay"], ay=ca["ax"])
    a = oracle.laplacian(oracle.padded(u), ca)
    b = oracle.laplacian(oracle.padded(np.swapaxes(u, 1, 2).copy()), cs)
    assert np.allclose(np.swapaxes(b, 1, 2), a, rtol=0, atol=1e-12)


def test_linearity():
    co = synth.random_coeffs(5)
    u = synth.uniform_field((6, 7, 8), 1).astype(np.float64)
    w = synth.uniform_field((6, 7, 8), 2).astype(np.float64)
    lu = oracle.laplacian(oracle.padded(u), co)
    lw = oracle.laplacian(oracle.padded(w), co)
    luw = oracle.laplacian(oracle.padded(2.5 * u - 0.75 * w), co)
    assert np.allclose(luw, 2.5 * lu - 0.75 * lw, rtol=0, atol=1e-12)


def _nested(a):
    return [[[int(v) for v in row] for row in plane] for plane in a]


@pytest.mark.parametrize("shape", [(3, 4, 5), (7, 5, 6), (1, 2, 9)])
def test_matches_exact_brute_force(shape):
    # Integer field, integer weights, non-zero halo: the C oracle (FP64) must
    # equal the exact rational brute force bit for bit.
    rng = np.random.default_rng(sum(shape))
    u = rng.integers(-170, 171, size=shape)
    halo_fn = lambda x, y, z: (7 * x - 3 * y + 5 * z) % 11 - 5    # noqa: E731
    nz, ny, nx = shape
    up = np.zeros((nz + 8, ny + 8, nx + 8))
    for z in range(-4, nz + 4):
        for y in range(-4, ny + 4):
            for x in range(-4, nx + 4):
                inside = 0 <= x < nx and 0 <= y < ny and 0 <= z < nz
                up[z + 4, y + 4, x + 4] = u[z, y, x] if inside else halo_fn(x, y, z)
    ci = synth.integer_coeffs()
    ref = brute.star25(_nested(u), {k: ([int(a) for a in v] if isinstance(v, list) else int(v))
                                    for k, v in ci.items()}, boundary=halo_fn)
    out = oracle.laplacian(up, ci)
    assert np.array_equal(out, np.array(ref, dtype=np.float64))


def test_rational_brute_force_fd8_on_tiny_grid():
    # Exact FD8 rationals vs FP64-rounded weights: agreement to rounding.
    shape = (4, 5, 6)
    u = synth.integer_field(shape, 9, bound=50)
    co = {"center": 3 * synth.FD8_WEIGHTS[0], "ax": list(synth.FD8_WEIGHTS[1:]),
          "ay": list(synth.FD8_WEIGHTS[1:]), "az": list(synth.FD8_WEIGHTS[1:])}
    ref = brute.star25(_nested(u), co)
    out = oracle.laplacian(oracle.padded(u), synth.star25_coeffs())
    exact = np.array([[[float(Fraction(v)) for v in row] for row in plane] for plane in ref])
    assert np.allclose(out, exact, rtol=0, atol=1e-12)


def test_symmetric_operator_with_zero_halo():
    co = synth.star25_coeffs()
    x = synth.uniform_field((7, 8, 9), 21).astype(np.float64)
    y = synth.uniform_field((7, 8, 9), 22).astype(np.float64)
    lx = oracle.laplacian(oracle.padded(x), co)
    ly = oracle.laplacian(oracle.padded(y), co)
    a, b = float(np.sum(lx * y)), float(np.sum(x * ly))
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0)


def test_pingpong_sweeps_follow_the_listing():
    # Listing 1 swaps the two grids after every sweep: an odd number of sweeps
    # leaves the result in v, an even number in u; v's halo feeds sweep 2.
    co = synth.random_coeffs(3)
    u = synth.uniform_field((5, 6, 7), 4).astype(np.float64)
    up = oracle.padded(u, halo_value=0.5)
    vp = oracle.padded(np.zeros_like(u), halo_value=-0.25)
    uu, vv, in_v = oracle.stencil_apply(up, vp, co, 1)
    assert in_v == 1
    assert np.allclose(oracle.interior(vv), oracle.laplacian(up, co), rtol=0, atol=0)
    uu, vv, in_v = oracle.stencil_apply(up, vp, co, 2)
    assert in_v == 0
    first = vp.copy()
    first[4:-4, 4:-4, 4:-4] = oracle.laplacian(up, co)
    assert np.array_equal(oracle.interior(uu), oracle.laplacian(first, co))
    assert np.array_equal(uu[:4], up[:4])          # halo of u untouched
