"""Pins for the oracle's leapfrog (paper Eq. 2, Algorithm 1) and its adjoint.

Checks: zero stays zero; closed form of the first two steps after a point
injection; the plane-wave (Fourier mode) recursion in the interior; discrete
energy conservation; the CFL stability limit of this stencil; and the
adjoint gradient against central finite differences in FP64.
"""

import math

import numpy as np
import pytest

import oracle
import synth


def test_zero_stays_zero():
    co = synth.star25_coeffs()
    v = synth.layered_velocity(8, 9, 10, 0)
    r = oracle.wave_run(co, v, 1e-3, 10.0, 20)
    assert np.all(r["cur"] == 0) and np.all(r["prev"] == 0)


def test_first_steps_after_point_injection():
    # u^1 = dt^2 v^2 a0 e_src; u^2 = 2 u^1 + m L u^1 + dt^2 v^2 a1 e_src.
    co = synth.star25_coeffs()
    nx, ny, nz = 13, 12, 11
    v = synth.layered_velocity(nx, ny, nz, 5)
    dt, dx = synth.cfl_dt(v, 10.0), 10.0
    src = np.array([[6, 5, 4]], np.int32)
    rec = np.array([[6, 5, 4], [7, 5, 4], [6, 5, 8]], np.int32)
    amp = np.array([[0.7], [-0.3]])
    r = oracle.wave_run(co, v, dt, dx, 2, src=src, amp=amp, rec=rec)
    vs = float(v[4, 5, 6])
    a0 = dt * dt * vs * vs * 0.7
    u1 = np.zeros((nz, ny, nx))
    u1[4, 5, 6] = a0
    assert np.array_equal(oracle.interior(r["prev"]), u1)
    m = (v.astype(np.float64) * dt / dx) ** 2
    # L u1 is a0 times the impulse response
    lap = np.zeros_like(u1)
    lap[4, 5, 6] = co["center"] * a0
    for k in range(1, 5):
        for s in (-1, 1):
            if 0 <= 6 + s * k < nx:
                lap[4, 5, 6 + s * k] = co["ax"][k - 1] * a0
            if 0 <= 5 + s * k < ny:
                lap[4, 5 + s * k, 6] = co["ay"][k - 1] * a0
            if 0 <= 4 + s * k < nz:
                lap[4 + s * k, 5, 6] = co["az"][k - 1] * a0
    u2 = 2 * u1 + m * lap
    u2[4, 5, 6] += dt * dt * vs * vs * -0.3
    assert np.allclose(oracle.interior(r["cur"]), u2, rtol=1e-15, atol=0)
    # receivers record u^{n+1} after injection
    assert r["traces"][0, 0] == a0 and r["traces"][0, 1] == 0.0
    assert np.isclose(r["traces"][1, 1], u2[4, 5, 7], rtol=1e-15, atol=0)
    assert np.isclose(r["traces"][1, 2], u2[8, 5, 6], rtol=1e-15, atol=0)


def test_plane_wave_recursion_in_the_interior():
    # For u = cos(k.x) and constant m, L u = sigma u with
    # sigma = c_xyz + sum_axes sum_r 2 c_r cos(r k_a); the leapfrog gives
    # a_{n+1} = (2 + m sigma) a_n - a_{n-1} wherever the zero halo has not yet
    # been felt (4n cells from every face after n steps).
    co = synth.star25_coeffs()
    n = 40
    kx, ky, kz = 0.7, 0.45, 1.1
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    mode = np.cos(kx * x + ky * y + kz * z)
    sigma = co["center"] + sum(2 * co["ax"][r - 1] * math.cos(r * kx) +
                               2 * co["ay"][r - 1] * math.cos(r * ky) +
                               2 * co["az"][r - 1] * math.cos(r * kz) for r in range(1, 5))
    vel, dx, dt = 2000.0, 10.0, 0.0018
    m = (vel * dt / dx) ** 2
    v = np.full((n, n, n), vel)
    steps = 3
    r = oracle.wave_run(co, v, dt, dx, steps, prev=oracle.padded(mode), cur=oracle.padded(mode))
    a = [1.0, 1.0]
    for _ in range(steps):
        a.append((2 + m * sigma) * a[-1] - a[-2])
    core = slice(4 * steps, n - 4 * steps)
    got = oracle.interior(r["cur"])[core, core, core]
    assert np.allclose(got, a[-1] * mode[core, core, core], rtol=0, atol=1e-12)
    got_prev = oracle.interior(r["prev"])[core, core, core]
    assert np.allclose(got_prev, a[-2] * mode[core, core, core], rtol=0, atol=1e-12)


def test_energy_is_conserved_without_source():
    co = synth.star25_coeffs()
    nx, ny, nz = 14, 13, 12
    v = synth.layered_velocity(nx, ny, nz, 2).astype(np.float64)
    dx = 10.0
    dt = synth.cfl_dt(v, dx, 0.4)
    rng = np.random.default_rng(4)
    prev = oracle.padded(rng.uniform(-1, 1, (nz, ny, nx)))
    cur = oracle.padded(rng.uniform(-1, 1, (nz, ny, nx)))
    e0 = oracle.energy(co, v, dt, dx, prev, cur)
    es = []
    for _ in range(6):
        r = oracle.wave_run(co, v, dt, dx, 50, prev=prev, cur=cur)
        prev, cur = r["prev"], r["cur"]
        es.append(oracle.energy(co, v, dt, dx, prev, cur))
    assert e0 > 0
    drift = max(abs(e - e0) for e in es) / e0
    assert drift < 1e-11


def test_energy_detects_a_wrong_update():
    # Planted mistake on the CPU: a damped update (0.999 * p_prev) is not
    # conservative, and the energy check sees it.
    co = synth.star25_coeffs()
    nx, ny, nz = 10, 10, 10
    v = np.full((nz, ny, nx), 2500.0)
    dx, dt = 10.0, 0.0016
    rng = np.random.default_rng(8)
    prev = oracle.padded(rng.uniform(-1, 1, (nz, ny, nx)))
    cur = oracle.padded(rng.uniform(-1, 1, (nz, ny, nx)))
    e0 = oracle.energy(co, v, dt, dx, prev, cur)
    m = (v * dt / dx) ** 2
    nxt = oracle.padded(2 * oracle.interior(cur) - 0.999 * oracle.interior(prev)
                        + m * oracle.laplacian(cur, co))
    e1 = oracle.energy(co, v, dt, dx, cur, nxt)
    assert abs(e1 - e0) / e0 > 1e-6


@pytest.mark.parametrize("cfl,stable", [(0.44, True), (0.47, False)])
def test_cfl_limit_of_this_stencil(cfl, stable):
    # Nyquist eigenvalue per axis is -2048/315, so the leapfrog is stable for
    # CFL <= sqrt(4 / (3 * 2048/315)) = sqrt(105/512) ~ 0.4529.
    assert abs(math.sqrt(4 / (3 * 2048 / 315)) - math.sqrt(105 / 512)) < 1e-15
    co = synth.star25_coeffs()
    n = 16
    v = np.full((n, n, n), 3000.0)
    dx = 10.0
    dt = cfl * dx / 3000.0
    rng = np.random.default_rng(1)
    u0 = rng.uniform(-1, 1, (n, n, n))
    r = oracle.wave_run(co, v, dt, dx, 400, prev=oracle.padded(u0), cur=oracle.padded(u0))
    amax = float(np.max(np.abs(r["cur"])))
    if stable:
        assert amax < 1e3
    else:
        assert amax > 1e6


def _adjoint_case(n=12, steps=40, seed=0):
    co = synth.star25_coeffs()
    v = synth.layered_velocity(n, n, n, seed).astype(np.float64)
    v_obs = synth.gaussian_bump(v.astype(np.float32), (n // 2, n // 2, n // 2), 2.0, 0.05)
    dx = 10.0
    dt = synth.cfl_dt(v, dx, 0.4)
    src = np.array([[n // 2, n // 2, 2]], np.int32)
    rec = synth.receiver_plane(n, n, 2, 2)
    amp = synth.ricker(steps, dt, 15.0)[:, None] * 1e3
    obs = oracle.wave_run(co, v_obs, dt, dx, steps, src=src, amp=amp, rec=rec)["traces"]
    return co, v, dt, dx, steps, src, amp, rec, obs


def test_adjoint_gradient_matches_finite_differences():
    co, v, dt, dx, steps, src, amp, rec, obs = _adjoint_case()
    J, g = oracle.adjoint_grad(co, v, dt, dx, steps, src, amp, rec, obs)
    assert J > 0
    rng = np.random.default_rng(3)
    for _ in range(3):
        d = rng.uniform(-1, 1, v.shape)
        eps = 1e-2
        jp, _ = oracle.adjoint_grad(co, v + eps * d, dt, dx, steps, src, amp, rec, obs)
        jm, _ = oracle.adjoint_grad(co, v - eps * d, dt, dx, steps, src, amp, rec, obs)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_adjoint_misfit_matches_forward_traces():
    co, v, dt, dx, steps, src, amp, rec, obs = _adjoint_case(n=10, steps=25, seed=3)
    fwd = oracle.wave_run(co, v, dt, dx, steps, src=src, amp=amp, rec=rec)["traces"]
    J, _ = oracle.adjoint_grad(co, v, dt, dx, steps, src, amp, rec, obs)
    assert np.isclose(J, 0.5 * np.sum((fwd - obs) ** 2), rtol=1e-13, atol=0)
    J0, g0 = oracle.adjoint_grad(co, v, dt, dx, steps, src, amp, rec, fwd)
    # the two forward formulations differ only by rounding
    assert J0 <= 1e-20 * J
    J1, g1 = oracle.adjoint_grad(co, v, dt, dx, steps, src, amp, rec, obs)
    assert np.max(np.abs(g0)) <= 1e-9 * np.max(np.abs(g1))


@pytest.mark.parametrize("ckpt", [1, 7, 60])
def test_checkpointed_adjoint_is_bit_identical(ckpt):
    # The checkpointed gradient keeps only segment-start pairs and recomputes
    # each segment; with C = 7 the last segment is ragged (60 = 8 * 7 + 4).
    # Same operations in the same order as the full-storage adjoint, which
    # the finite-difference pin above checks: the results must be identical.
    co, v, dt, dx, steps, src, amp, rec, obs = _adjoint_case(n=24, steps=60, seed=5)
    J, g = oracle.adjoint_grad(co, v, dt, dx, steps, src, amp, rec, obs)
    Jc, gc, tr = oracle.adjoint_grad_ckpt(co, v, dt, dx, steps, src, amp, rec, obs, ckpt,
                                          traces=True)
    assert Jc == J and np.array_equal(gc, g) and np.any(g != 0)
    # its traces are the forward run's (up to the rounding of the injection)
    fwd = oracle.wave_run(co, v, dt, dx, steps, src=src, amp=amp, rec=rec)["traces"]
    assert np.max(np.abs(tr - fwd)) <= 1e-12 * np.max(np.abs(fwd))
    assert np.isclose(Jc, 0.5 * np.sum((tr - obs) ** 2), rtol=1e-13, atol=0)
