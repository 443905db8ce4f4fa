"""Pins of the oracle's absorbing-layer leapfrog (the paper's PML region,
formulation read as the isotropic complex-stretching layer with a frequency
shift alpha in the auxiliary equation; Sec. 2.2).

 * eta = 0: identical to the plain leapfrog oracle;
 * uniform eta (no gradient): the damped recurrence's closed form
   u^n = A (1 + a)^-n + B (1 - a)^n, a = eta dt, at points the boundary has
   not reached;
 * linear eta and u: the 7-point gradient product equals grad eta . grad u
   exactly, so one step gives psi^1 = -dt (grad eta . grad u) / (1 + b/2),
   b = (eta + alpha) dt, and u^1 takes half of it;
 * absorption: a pulse leaving a box with the layer leaves < 1e-4 of the
   energy a reflecting (Dirichlet) box keeps;
 * long runs decay once the source has stopped (alpha = pi f0), while the
   unshifted form (alpha = 0) grows: the reason for the shift;
 * the damping profile vanishes on the inner box and on its neighbours.
"""

import numpy as np
import pytest

import oracle
import synth


def test_zero_damping_is_the_plain_leapfrog():
    n = 24
    v = synth.layered_velocity(n, n, n, 2)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.random_coeffs(3)
    src = np.array([[5, 17, 9]], np.int32)
    amp = synth.ricker(40, dt)[:, None]
    rec = synth.random_points(n, n, n, 7, 1)
    a = oracle.wave_pml_run(co, v, np.zeros((n + 8,) * 3), dt, dx, 40, src=src, amp=amp, rec=rec)
    b = oracle.wave_run(co, v, dt, dx, 40, src=src, amp=amp, rec=rec)
    assert np.array_equal(a["cur"], b["cur"]) and np.array_equal(a["prev"], b["prev"])
    assert np.array_equal(a["traces"], b["traces"]) and not a["psi"].any()


@pytest.mark.parametrize("a", [0.05, 0.3, 0.9])
def test_uniform_damping_closed_form(a):
    n, steps = 96, 10
    v = np.full((n, n, n), 3000.0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    eta = np.full((n + 8,) * 3, a / dt)
    one = oracle.padded(np.ones((n, n, n)))
    c = n // 2 + 4
    for k in range(1, steps + 1):
        r = oracle.wave_pml_run(synth.star25_coeffs(), v, eta, dt, dx, k, prev=one, cur=one)
        # roots of (1 + a) r^2 - (2 - a^2) r + (1 - a) = 0 are 1/(1 + a) and
        # 1 - a; u^-1 = u^0 = 1 fixes A = 1/a, B = 1 - 1/a
        exact = (1.0 / a) * (1.0 + a) ** -k + (1.0 - 1.0 / a) * (1.0 - a) ** k
        assert abs(r["cur"][c, c, c] - exact) <= 1e-12 * max(1.0, abs(exact)), k
        assert abs(r["psi"][c, c, c]) == 0.0


def test_gradient_product_of_linear_fields_is_exact():
    n = 20
    v = np.full((n, n, n), 2500.0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    Z, Y, X = np.meshgrid(*(np.arange(-4, n + 4, dtype=float),) * 3, indexing="ij")
    g = (3.0, -2.0, 0.5)               # d eta / d(x, y, z) per cell, 1/s
    al = (0.25, 1.5, -0.75)            # d u / d(x, y, z) per cell
    eta = 40.0 + g[0] * X + g[1] * Y + g[2] * Z
    u = 2.0 + al[0] * X + al[1] * Y + al[2] * Z
    alpha = 47.0
    r = oracle.wave_pml_run(synth.star25_coeffs(), v, eta, dt, dx, 1, prev=u, cur=u, alpha=alpha)
    dot = g[0] * al[0] + g[1] * al[1] + g[2] * al[2]
    ex = -dt * dot / (1.0 + 0.5 * (eta + alpha) * dt)
    s = (slice(4, -4),) * 3
    assert np.allclose(r["psi"][s], ex[s], rtol=1e-13, atol=0)
    # the u update sees L u = 0 and the mean of psi^{-1/2} = 0 and psi^{1/2}
    a = eta * dt
    m = (2500.0 * dt / dx) ** 2
    uex = ((2.0 - a * a) * u - (1.0 - a) * u + m * 0.5 * ex) / (1.0 + a)
    inner = (slice(8, -8),) * 3               # away from the zero halo of u
    assert np.allclose(r["cur"][inner], uex[inner], rtol=1e-13, atol=1e-13)


def _pulse(width, eta_on, steps=500, n=48):
    v = np.full((n, n, n), 2000.0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    src = np.array([[n // 2] * 3], np.int32)
    amp = synth.ricker(steps, dt)[:, None] * 1e3
    eta = synth.pml_profile(n, n, n, width, synth.pml_eta_max(2000.0, width, dx))
    if not eta_on:
        eta = np.zeros_like(eta)
    r = oracle.wave_pml_run(synth.star25_coeffs(), v, eta, dt, dx, steps, src=src, amp=amp,
                            alpha=np.pi * 15.0)
    u = oracle.interior(r["cur"])[width:-width, width:-width, width:-width]
    return float((u ** 2).sum()), r


def test_layer_absorbs_the_outgoing_pulse():
    e_pml, _ = _pulse(10, True)
    e_rigid, _ = _pulse(10, False)
    assert e_rigid > 1e6 and e_pml < 1e-4 * e_rigid


def _long_run(alpha, chunks=30):
    n, W = 40, 8
    v = np.full((n, n, n), 3000.0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    eta = synth.pml_profile(n, n, n, W, synth.pml_eta_max(3000.0, W, dx))
    src = np.array([[20, 20, 20]], np.int32)
    amp = np.zeros((chunks * 100, 1))
    amp[:200, 0] = synth.ricker(200, dt) * 1e3
    peaks, st = [], None
    for c in range(chunks):
        st = oracle.wave_pml_run(synth.star25_coeffs(), v, eta, dt, dx, 100, src=src,
                                 amp=amp[c * 100:(c + 1) * 100], alpha=alpha,
                                 prev=None if st is None else st["prev"],
                                 cur=None if st is None else st["cur"],
                                 psi=None if st is None else st["psi"])
        peaks.append(float(np.abs(st["cur"]).max()))
    return peaks


def test_frequency_shift_makes_long_runs_decay():
    shifted = _long_run(np.pi * 15.0)
    assert all(np.isfinite(shifted)) and shifted[-1] < 1e-6 * shifted[0]
    assert max(shifted[10:]) < 1e-3 * shifted[0]
    unshifted = _long_run(0.0)
    assert unshifted[-1] > 100 * min(unshifted)          # the zero-frequency mode grows


@pytest.mark.parametrize("profile", ["oracle", "synth"])
def test_profile_vanishes_on_the_inner_box_and_its_neighbours(profile):
    n, W = 30, 6
    e = (oracle.pml_profile if profile == "oracle" else synth.pml_profile)(n, n, n, W, 100.0)
    inner = e[4 + W - 1:4 + n - W + 1, 4 + W - 1:4 + n - W + 1, 4 + W - 1:4 + n - W + 1]
    assert not inner.any()
    # outermost interior cell of a face centre: depth W-1 on one axis
    assert e[4 + 0, 4 + n // 2, 4 + n // 2] == pytest.approx(100.0 * ((W - 1) / W) ** 2)
    assert synth.pml_eta_max(2000.0, 10, 10.0) == pytest.approx(3 * 2000.0 * np.log(1e3) / 200.0)


def test_oracle_profile_closed_forms():
    # eta = eta_max * sum over axes (d_a / W)^2 with d_a the depth into the
    # layer, checked cell by cell against values worked out by hand on a
    # ragged grid (a wrong axis, offset or square fails one of them).
    nx, ny, nz, W, emax = 20, 13, 17, 4, 8.0
    e = oracle.pml_profile(nx, ny, nz, W, emax)
    assert e.shape == (nz + 8, ny + 8, nx + 8)

    def at(x, y, z):
        return e[z + 4, y + 4, x + 4]
    # inner box [W-1, n-W] on every axis: zero
    assert at(W - 1, W - 1, W - 1) == 0.0 and at(nx - W, ny - W, nz - W) == 0.0
    # one layer axis at a time: depth W-1-a (low side), a-(n-W) (high side)
    assert at(0, 6, 8) == emax * (3 / 4) ** 2
    assert at(nx - 1, 6, 8) == emax * (3 / 4) ** 2
    assert at(-4, 6, 8) == emax * (7 / 4) ** 2              # halo frame: depth W + 3
    assert at(9, ny + 3, 8) == emax * (7 / 4) ** 2
    assert at(9, 6, 1) == emax * (2 / 4) ** 2
    assert at(9, 6, nz - 2) == emax * (2 / 4) ** 2
    # an edge and a corner sum the axes
    assert at(1, 0, 8) == emax * ((2 / 4) ** 2 + (3 / 4) ** 2)
    assert at(-4, -4, -4) == pytest.approx(3 * emax * (7 / 4) ** 2, rel=1e-15)
    # mirror symmetry on each axis, and a transposed grid gives the transpose
    assert np.array_equal(e, e[::-1, :, :]) and np.array_equal(e, e[:, ::-1, :])
    assert np.array_equal(e, e[:, :, ::-1])
    et = oracle.pml_profile(nz, ny, nx, W, emax)
    assert np.array_equal(et, np.transpose(e, (2, 1, 0)))
