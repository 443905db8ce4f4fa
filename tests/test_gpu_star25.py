"""GPU parity of sp_stencil_apply and sp_wave_step against the FP64 oracle.

All calls go through the C ABI (ctypes binding).  Bars:
 * integer weights and integer fields: bit-exact (every partial sum < 2^24);
 * FP32 stencil and per-step leapfrog: relative L2 <= 1e-5 against the
   oracle run on the GPU's own FP32 input widened to FP64;
 * multi-step leapfrog (error compounds over steps): relative L2 <= 1e-4.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import errors, oracle_star_at, oracle_wave_at, sample_points

pytestmark = pytest.mark.gpu

TOL_SWEEP = 1e-5


def _lib():
    from paper_2309_04671_amd import lib
    return lib


def _apply(u_np, coeffs, sweeps, halo_u=None, halo_v=None):
    from paper_2309_04671_amd import fields
    lib = _lib()
    nz, ny, nx = u_np.shape
    g = lib.grid_init(nx, ny, nz)
    u = fields.Field(g)
    v = fields.Field(g)
    if halo_u is not None:
        u.set_padded(halo_u)
    if halo_v is not None:
        v.set_padded(halo_v)
    u.set_interior(u_np)
    where = lib.sp_stencil_apply(g, lib.coeffs(coeffs), sweeps, u.ptr, v.ptr)
    torch.cuda.synchronize()
    return u, v, where


def test_c0_single_sweep_parity(gpu_lib):
    # 64^3 interior, 4-cell zero halo, u ~ U[-1,1] (seed 0), FD8 weights, 1 sweep.
    u = synth.uniform_field((64, 64, 64), 0)
    co = synth.star25_coeffs()
    _, v, where = _apply(u, co, 1)
    assert where == 1
    got = v.get_interior()
    ref = oracle.laplacian(oracle.padded(u), co)
    e = errors(got, ref)
    print("64^3 sweep vs FP64 oracle:", e)
    assert e["rel_l2"] <= TOL_SWEEP


def test_integer_weights_bit_exact(gpu_lib):
    for shape in [(64, 64, 64), (23, 37, 70), (9, 130, 65)]:
        u = synth.integer_field(shape, 1, bound=170)
        co = synth.integer_coeffs()
        _, v, _ = _apply(u, co, 1)
        ref = oracle.laplacian(oracle.padded(u), co)
        assert np.array_equal(v.get_interior().astype(np.float64), ref), shape


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (23, 37, 70), (40, 17, 130),
                                   (33, 64, 129), (70, 20, 3)])
def test_ragged_shapes_with_nonzero_halo(gpu_lib, shape):
    # (nz, ny, nx): tails in every axis, tiles of one point, halos read from memory.
    nz, ny, nx = shape
    co = synth.random_coeffs(sum(shape))
    u = synth.uniform_field(shape, 5)
    halo = synth.uniform_field((nz + 8, ny + 8, nx + 8), 6)
    _, v, _ = _apply(u, co, 1, halo_u=halo)
    up = halo.astype(np.float64)
    up[4:-4, 4:-4, 4:-4] = u
    ref = oracle.laplacian(up, co)
    e = errors(v.get_interior(), ref)
    assert e["rel_l2"] <= TOL_SWEEP, e
    # the library never writes halo cells
    vp = v.get_padded()
    mask = np.ones(vp.shape, bool)
    mask[4:-4, 4:-4, 4:-4] = False
    assert np.all(vp[mask] == 0.0)


@pytest.mark.parametrize("sweeps", [0, 2, 3])
def test_pingpong_sweeps(gpu_lib, sweeps):
    shape = (20, 24, 36)
    co = synth.random_coeffs(2)
    u = synth.integer_field(shape, 3, bound=3)
    ci = synth.integer_coeffs()
    hu = np.zeros((28, 32, 44), np.float32)
    hv = np.zeros((28, 32, 44), np.float32)
    uf, vf, where = _apply(u, {"center": co["center"], "ax": co["ax"], "ay": co["ay"],
                               "az": co["az"]}, sweeps, hu, hv)
    ru, rv, in_v = oracle.stencil_apply(oracle.padded(u), oracle.padded(np.zeros(shape)), co, sweeps)
    assert where == in_v
    got = (vf if where else uf).get_interior()
    ref = oracle.interior(rv if in_v else ru)
    scale = max(float(np.max(np.abs(ref))), 1.0)
    assert np.max(np.abs(got - ref)) / scale <= 1e-5 * max(sweeps, 1)
    del ci


def _wave_setup(nx, ny, nz, seed, nrec=0):
    from paper_2309_04671_amd import fields
    lib = _lib()
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, seed)
    vf = fields.Field(g).set_interior(v)
    return g, v, vf


def test_wave_single_step_parity_random_state(gpu_lib):
    # One step from the same random FP32 state (prev, cur), with a source.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 130, 70, 41
    g, v, vf = _wave_setup(nx, ny, nz, 4)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    prev = synth.uniform_field((nz, ny, nx), 7)
    cur = synth.uniform_field((nz, ny, nx), 8)
    P = fields.Field(g).set_interior(prev)
    C = fields.Field(g).set_interior(cur)
    src_xyz = np.array([[65, 35, 20], [0, 0, 0], [129, 69, 40]], np.int32)
    amp = torch.tensor([[3.0e4, -2.0e4, 1.5e4]], dtype=torch.float32, device="cuda")
    src = lib.make_sources(src_xyz, amp.data_ptr(), 3)
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 1, src=src)
    torch.cuda.synchronize()
    assert st.cur == P.ptr and st.prev == C.ptr and st.step == 1
    got = P.get_interior()
    r = oracle.wave_run(co, v, dt, dx, 1, src=src_xyz, amp=amp.cpu().double().numpy(),
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    e = errors(got, oracle.interior(r["cur"]))
    print("wave step 130x70x41 vs oracle:", e)
    assert e["rel_l2"] <= TOL_SWEEP
    # the source points themselves
    for k, (x, y, z) in enumerate(src_xyz):
        assert abs(got[z, y, x] - oracle.interior(r["cur"])[z, y, x]) <= 1e-5 * abs(float(amp[0, k]))


def test_wave_multi_step_with_receivers(gpu_lib):
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 72, 40, 36
    steps = 60
    g, v, vf = _wave_setup(nx, ny, nz, 1)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src_xyz = np.array([[36, 20, 18]], np.int32)
    w = synth.ricker(steps, dt, 15.0)[:, None]
    rec_xyz = np.concatenate([synth.receiver_plane(nx, ny, 4, 3),
                              np.array([[36, 20, 18], [71, 39, 35], [80, 0, 0]], np.int32)])
    nrec = len(rec_xyz)
    amp = torch.tensor(w, dtype=torch.float32, device="cuda")
    rec_d = torch.tensor(rec_xyz, dtype=torch.int32, device="cuda")
    traces = torch.zeros((steps, nrec), dtype=torch.float32, device="cuda")
    P, C = fields.Field(g), fields.Field(g)
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    src = lib.make_sources(src_xyz, amp.data_ptr(), 1)
    rec = lib.make_receivers(nrec, rec_d.data_ptr(), traces.data_ptr(), nrec)
    # two calls (30 + 30) must equal one run of 60
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 30, src=src, rec=rec)
    rec2 = lib.make_receivers(nrec, rec_d.data_ptr(), traces[30:].data_ptr(), nrec)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 30, src=src, rec=rec2)
    torch.cuda.synchronize()
    assert st.step == steps
    cur = fields.Field(g, buf=P.buf if st.cur == P.ptr else C.buf).get_interior()
    ok_rec = rec_xyz[:-1]
    r = oracle.wave_run(co, v, dt, dx, steps, src=src_xyz, amp=amp.cpu().double().numpy(), rec=ok_rec)
    e = errors(cur, oracle.interior(r["cur"]))
    print("60 steps 72x40x36 vs oracle:", e)
    assert e["rel_l2"] <= 1e-4
    tr = traces.cpu().numpy()
    et = errors(tr[:, :-1], r["traces"])
    assert et["rel_l2"] <= 1e-4
    assert np.all(tr[:, -1] == 0.0)          # out-of-range receiver records 0


def test_wave_full_size_sampled_parity(gpu_lib):
    # 1024x1024x512 (the benchmark workload), bench launch configuration:
    # one step from a random state, checked at sampled points (including the
    # corners and faces) against the oracle evaluated point by point.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 1024, 1024, 512
    g = lib.grid_init(nx, ny, nz)
    gen = torch.Generator(device="cuda").manual_seed(11)
    P, C, V = fields.Field(g), fields.Field(g), fields.Field(g)
    v = synth.layered_velocity(nx, ny, nz, 0)
    V.set_interior(v)
    P.interior().uniform_(-1, 1, generator=gen)
    C.interior().uniform_(-1, 1, generator=gen)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src_xyz = np.array([[512, 512, 256]], np.int32)
    amp = torch.tensor([[5.0e4]], dtype=torch.float32, device="cuda")
    pts = np.concatenate([sample_points(nx, ny, nz, 400, 3), src_xyz])
    prev_pad = P.padded().cpu().numpy()
    cur_pad = C.padded().cpu().numpy()
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, V.ptr, st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    torch.cuda.synchronize()
    out = P.interior()
    got = np.array([float(out[z, y, x]) for (x, y, z) in pts])
    ref = oracle_wave_at(prev_pad, cur_pad, v, co, dt, dx, pts, src=src_xyz, amp_row=[5.0e4])
    e = errors(got, ref)
    print("1024x1024x512 sampled step vs oracle:", e)
    assert e["rel_l2"] <= TOL_SWEEP


def test_apply_full_size_sampled_parity(gpu_lib):
    # sp_stencil_apply at 1024x1024x512 in its own launch configuration,
    # sampled points against the oracle evaluated point by point.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 1024, 1024, 512
    g = lib.grid_init(nx, ny, nz)
    gen = torch.Generator(device="cuda").manual_seed(5)
    U, W = fields.Field(g), fields.Field(g)
    U.interior().uniform_(-1, 1, generator=gen)
    co = synth.star25_coeffs()
    pts = sample_points(nx, ny, nz, 400, 9)
    where = lib.sp_stencil_apply(g, lib.coeffs(co), 1, U.ptr, W.ptr)
    torch.cuda.synchronize()
    assert where == 1
    out = W.interior()
    got = np.array([float(out[z, y, x]) for (x, y, z) in pts])
    ref = oracle_star_at(U.padded().cpu().numpy(), co, pts)
    e = errors(got, ref)
    print("1024x1024x512 sampled apply vs oracle:", e)
    assert e["rel_l2"] <= TOL_SWEEP


TILE_CONFIGS = ["64x16x1", "128x16x2", "128x32x2", "256x16x2", "256x8x2", "256x16x1", "256x8x1",
                "64x16x1x7", "128x16x2x33", "256x16x2x40", "256x8x1x9"]


@pytest.mark.parametrize("tile", TILE_CONFIGS)
def test_every_tile_config_single_step(gpu_lib, tile, monkeypatch):
    # Each compiled launch configuration (SP_TILE=TXxTYxRY[xZCHUNK]) against
    # the oracle: one leapfrog step from a random state with a source, on a
    # ragged grid that spans several tiles in x and y and several z-chunks.
    from paper_2309_04671_amd import fields
    lib = _lib()
    monkeypatch.setenv("SP_TILE", tile)
    nx, ny, nz = 301, 45, 70
    g, v, vf = _wave_setup(nx, ny, nz, 2)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.random_coeffs(4)
    prev = synth.uniform_field((nz, ny, nx), 17)
    cur = synth.uniform_field((nz, ny, nx), 18)
    P = fields.Field(g).set_interior(prev)
    C = fields.Field(g).set_interior(cur)
    src_xyz = np.array([[150, 22, 35], [300, 44, 69]], np.int32)
    amp = torch.tensor([[2.0e4, -1.0e4]], dtype=torch.float32, device="cuda")
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 2))
    torch.cuda.synchronize()
    r = oracle.wave_run(co, v, dt, dx, 1, src=src_xyz, amp=amp.cpu().double().numpy(),
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    e = errors(P.get_interior(), oracle.interior(r["cur"]))
    assert e["rel_l2"] <= TOL_SWEEP, (tile, e)
    # apply in the same configuration
    U, W = fields.Field(g).set_interior(cur), fields.Field(g)
    assert lib.sp_stencil_apply(g, lib.coeffs(co), 1, U.ptr, W.ptr) == 1
    torch.cuda.synchronize()
    e = errors(W.get_interior(), oracle.laplacian(oracle.padded(cur), co))
    assert e["rel_l2"] <= TOL_SWEEP, (tile, e)


SHAPES_DEFAULT = [(1, 1, 1), (5, 1, 3), (300, 300, 1), (17, 260, 9), (700, 33, 18), (129, 129, 129),
                  (520, 260, 50), (96, 384, 31), (1000, 8, 40), (257, 255, 67)]


@pytest.mark.parametrize("shape", SHAPES_DEFAULT)
def test_default_launch_on_many_shapes(gpu_lib, shape):
    # The default tile and z-split choice (which depends on the shape) on
    # shapes from one point to several rounds of blocks: two leapfrog steps
    # from a random state with a source, and one apply sweep, against the
    # oracle.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = shape
    g, v, vf = _wave_setup(nx, ny, nz, 9)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.random_coeffs(nx + 2 * ny + 3 * nz)
    prev = synth.uniform_field((nz, ny, nx), 51)
    cur = synth.uniform_field((nz, ny, nx), 52)
    P = fields.Field(g).set_interior(prev)
    C = fields.Field(g).set_interior(cur)
    src_xyz = np.array([[nx // 3, ny // 2, nz - 1]], np.int32)
    amp = torch.tensor([[2.0e3], [-1.0e3]], dtype=torch.float32, device="cuda")
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 2,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    torch.cuda.synchronize()
    r = oracle.wave_run(co, v, dt, dx, 2, src=src_xyz, amp=amp.cpu().double().numpy(),
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    got = fields.Field(g, buf=C.buf if st.cur == C.ptr else P.buf).get_interior()
    e = errors(got, oracle.interior(r["cur"]))
    assert e["rel_l2"] <= TOL_SWEEP, (shape, e)
    u, out, where = _apply(prev, co, 1)
    assert where == 1
    e = errors(out.get_interior(), oracle.laplacian(oracle.padded(prev), co))
    assert e["rel_l2"] <= TOL_SWEEP, (shape, e)
