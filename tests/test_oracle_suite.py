"""Pins of the oracle's stencil-suite kernel (star/box, radius 1..4, 2D/3D;
the accuracy study of Sec. 6, with Eq. 3's star as one member).

Pins, each independent of the oracle's own loop nest:
 * scipy.ndimage.correlate with a zero constant boundary (a library routine
   computing the same definition) on every suite kernel, ragged shapes,
   signed and positive weights, one and two sweeps;
 * impulse response: a unit impulse at p yields w[k] at p - k (orientation
   of every axis; a transposed or mirrored weight array fails);
 * closed forms: separable products of 1D second-difference weights applied
   to polynomials give the exact mixed derivatives; a radius-1 star with
   [1, -2, 1] per axis gives the exact Laplacian of a cubic;
 * Eq. 3: the symmetric eighth-order star3d4r equals the pinned 25-point
   oracle.
"""

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth


def _field(name, shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("name", sorted(synth.SUITE))
@pytest.mark.parametrize("signed", [False, True])
def test_matches_scipy_correlate(name, signed):
    kind, ndim, r = synth.SUITE[name]
    w = synth.suite_weights(name, seed=7, signed=signed)
    shape = (11, 13, 17) if ndim == 3 else (13, 19)
    u = _field(name, shape, 3)
    got = oracle.stencil_general(u, w, ndim)
    ref = ndi.correlate(u, w, mode="constant", cval=0.0)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    got2 = oracle.stencil_general(u, w, ndim, sweeps=2)
    ref2 = ndi.correlate(ref, w, mode="constant", cval=0.0)
    assert np.allclose(got2, ref2, rtol=1e-12, atol=1e-12)


def test_2d_kernel_on_a_stack_of_planes():
    w = synth.suite_weights("box2d3r", seed=1, signed=True)
    u = _field("x", (5, 12, 14), 4)
    got = oracle.stencil_general(u, w, 2)
    for z in range(5):
        ref = ndi.correlate(u[z], w, mode="constant", cval=0.0)
        assert np.allclose(got[z], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("ndim,r", [(2, 1), (2, 4), (3, 2), (3, 4)])
def test_impulse_response(ndim, r):
    w = np.random.default_rng(r).uniform(1, 2, (2 * r + 1,) * ndim)
    n = 2 * r + 5
    shape = (n,) * ndim
    p = (n // 2,) * ndim
    u = np.zeros(shape)
    u[p] = 1.0
    out = oracle.stencil_general(u, w, ndim)
    exp = np.zeros(shape)
    for k in np.ndindex(*w.shape):
        off = tuple(ki - r for ki in k)
        exp[tuple(pi - oi for pi, oi in zip(p, off))] = w[k]
    assert np.array_equal(out, exp)


def test_separable_box_gives_exact_mixed_derivatives():
    # 12 * (4th-order 1D second difference), exact for degree <= 5
    a = np.array([-1.0, 16.0, -30.0, 16.0, -1.0])
    n = 16
    c = np.arange(n) - n / 2.0
    # 2D: P = x^5 y^3  ->  144 * d2x d2y P = 144 * 20 x^3 * 6 y
    w2 = np.outer(a, a)
    Y, X = np.meshgrid(c, c, indexing="ij")
    out = oracle.stencil_general(X ** 5 * Y ** 3, w2, 2)
    exp = 144.0 * (20 * X ** 3) * (6 * Y)
    s = (slice(2, -2),) * 2
    assert np.array_equal(out[s], exp[s])
    # 3D: P = x^4 y^2 z^5  ->  1728 * 12 x^2 * 2 * 20 z^3
    w3 = a[:, None, None] * a[None, :, None] * a[None, None, :]
    Z, Y, X = np.meshgrid(c[:12], c[:12], c[:12], indexing="ij")
    out = oracle.stencil_general(X ** 4 * Y ** 2 * Z ** 5, w3, 3)
    exp = 1728.0 * (12 * X ** 2) * 2.0 * (20 * Z ** 3)
    s = (slice(2, -2),) * 3
    assert np.array_equal(out[s], exp[s])


def test_radius1_star_gives_exact_laplacian_of_cubic():
    w = np.zeros((3, 3, 3))
    w[1, 1, 1] = -6.0
    for ax in range(3):
        for d in (0, 2):
            idx = [1, 1, 1]
            idx[ax] = d
            w[tuple(idx)] = 1.0
    c = np.arange(10) - 5.0
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    u = X ** 3 - 2 * X * Y ** 2 + Z ** 3 * Y + 7
    out = oracle.stencil_general(u, w, 3)
    exp = 6 * X - 4 * X + 6 * Z * Y
    s = (slice(1, -1),) * 3
    assert np.array_equal(out[s], exp[s])


def test_eighth_order_star3d4r_is_eq3():
    co = synth.star25_coeffs()
    w = np.zeros((9, 9, 9))
    w[4, 4, 4] = co["center"]
    for m in range(1, 5):
        w[4, 4, 4 - m] = w[4, 4, 4 + m] = co["ax"][m - 1]
        w[4, 4 - m, 4] = w[4, 4 + m, 4] = co["ay"][m - 1]
        w[4 - m, 4, 4] = w[4 + m, 4, 4] = co["az"][m - 1]
    u = synth.uniform_field((9, 10, 12), seed=5)
    got = oracle.stencil_general(u, w, 3)
    ref = oracle.laplacian(oracle.padded(u), co)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-13)


def test_suite_inputs_have_the_stated_support_and_range():
    for name, (kind, ndim, r) in synth.SUITE.items():
        w = synth.suite_weights(name, 0)
        assert w.shape == (2 * r + 1,) * ndim and abs(w.sum() - 1) < 1e-12
        nz = np.count_nonzero(w)
        assert nz == ((2 * r + 1) ** ndim if kind == "box" else 2 * ndim * r + 1)
    f = synth.suite_field((1000,), 0)
    assert f.min() >= 1e-4 * (1 - 1e-7) and f.max() <= 1e5 * (1 + 1e-7)
    L = synth.listing_star2d4r_weights()
    assert np.count_nonzero(L) == 17 and L[4, 0] == L[4, 8] == 0.11111 and L[0, 4] == -0.22220


def test_frame_values_enter_like_interior_values():
    # a field whose frame is read: same as correlating the whole padded array
    w = synth.suite_weights("box3d2r", seed=2, signed=True)
    rng = np.random.default_rng(9)
    full = rng.standard_normal((6 + 8, 7 + 8, 9 + 8))
    got = oracle.stencil_general(full[4:-4, 4:-4, 4:-4], w, 3, frame=full)
    ref = ndi.correlate(full, w, mode="constant", cval=0.0)[4:-4, 4:-4, 4:-4]
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    full2 = rng.standard_normal((3, 5 + 8, 11 + 8))
    got = oracle.stencil_general(full2[:, 4:-4, 4:-4], synth.suite_weights("star2d4r", 1), 2, frame=full2)
    for z in range(3):
        ref = ndi.correlate(full2[z], synth.suite_weights("star2d4r", 1), mode="constant")[4:-4, 4:-4]
        assert np.allclose(got[z], ref, rtol=1e-13, atol=1e-13)
