"""GPU parity of FP16/BF16 wavefield storage against the storage emulation
(oracle/lowp.py) and the FP64 oracle.

Bars:
 * one step from the same stored state: the new slab scales are equal
   exactly (the exponent decision is taken in FP32 on both sides); every
   stored value is within 1 ulp of the storage format of the emulation's,
   plus the FP32 arithmetic bound of the kernel (2^-4 in stored units, from
   |terms| <= 8 max|inputs| <= 2^15 scaled units and ~32 roundings);
 * the recorded slab maxima equal max|stored| * scale of the GPU's own output;
 * at the full 512^3 size, the same bars at sampled points, against the
   oracle's FP64 step evaluated point by point;
 * multi-step runs: error against the FP64 oracle is reported and must stay
   within twice the emulation's own storage error.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import lowp
import synth
from tests.gpu_util import errors, oracle_wave_at, sample_points

pytestmark = pytest.mark.gpu

FMT = {"f16": 1, "bf16": 2}
TDT = {"f16": torch.float16, "bf16": torch.bfloat16}


def _state_from(fields, g, q_prev, s_prev, q_cur, s_cur, fmt):
    ws = fields.WaveState(g)
    ws.prev().set_interior(q_prev.astype(np.float32))
    ws.cur().set_interior(q_cur.astype(np.float32))
    sc, ac = ws.slot(0)
    sp, ap = ws.slot(-1)
    sc.copy_(torch.tensor(s_cur))
    sp.copy_(torch.tensor(s_prev))
    ac.copy_(torch.tensor(lowp.slab_amax(q_cur, s_cur)))
    ap.copy_(torch.tensor(lowp.slab_amax(q_prev, s_prev)))
    return ws


LOWP_TILES = ["", "128x16x2", "256x8x2", "256x16x1", "256x8x1", "64x16x1x7", "256x16x2x20"]


@pytest.mark.parametrize("tile", LOWP_TILES)
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_single_step_parity(gpu_lib, fmt, tile, monkeypatch):
    # every compiled launch configuration ("" = the default choice)
    from paper_2309_04671_amd import fields, lib
    if tile:
        monkeypatch.setenv("SP_TILE", tile)
    nx, ny, nz = 301, 45, 70                    # ragged in x, y and in the last slab
    g = lib.grid_init(nx, ny, nz, FMT[fmt])
    gv = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 3)
    V = fields.Field(gv).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    rng = np.random.default_rng(12)
    n = lowp.nslab(nz)
    # per-slab magnitudes spanning several binades
    mag = 2.0 ** rng.integers(-20, 4, n)
    plane_mag = mag[np.arange(nz) // 16][:, None, None]
    s_cur = (2.0 ** (np.ceil(np.log2(mag)) - 14)).astype(np.float32)
    s_prev = (s_cur * 2).astype(np.float32)
    q_cur = lowp.round_to(rng.uniform(-1, 1, (nz, ny, nx)) * plane_mag / lowp.plane_scales(s_cur, nz)[:, None, None], fmt)
    q_prev = lowp.round_to(rng.uniform(-1, 1, (nz, ny, nx)) * plane_mag / lowp.plane_scales(s_prev, nz)[:, None, None], fmt)
    ws = _state_from(fields, g, q_prev, s_prev, q_cur, s_cur, fmt)
    src_xyz = np.array([[150, 22, 35], [300, 44, 69]], np.int32)
    amp = torch.tensor([[3.0e-3, -2.0e2]], dtype=torch.float32, device="cuda")
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, gv, V.ptr, ws.st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 2))
    torch.cuda.synchronize()
    assert ws.st.step == 1
    q_gpu = ws.cur().get_interior().astype(np.float64)
    s_gpu = ws.slot(1)[0].cpu().numpy()
    a_gpu = ws.slot(1)[1].cpu().numpy()
    q_ref, s_ref, a_ref, u_ref = lowp.step(co, v, dt, dx, fmt, q_prev, s_prev,
                                           lowp.slab_amax(q_prev, s_prev), q_cur, s_cur,
                                           lowp.slab_amax(q_cur, s_cur), src=src_xyz,
                                           amp_row=amp[0].cpu().numpy())
    assert np.array_equal(s_gpu, s_ref)
    tol = lowp.ulp(q_ref, fmt) + 2.0 ** -4
    d = np.abs(q_gpu - q_ref)
    exact = float(np.mean(d == 0))
    print(fmt, "one step: max |dq| / ulp = %.3f, exact fraction %.5f" % (
        float(np.max(d / lowp.ulp(q_ref, fmt))), exact))
    assert np.all(d <= tol)
    assert exact > 0.95
    assert np.array_equal(a_gpu, lowp.slab_amax(q_gpu, s_gpu))
    assert np.max(np.abs(q_gpu)) <= 2 ** 15
    # the slot of u^{n+2} was cleared for the next step
    assert np.all(ws.slot(2)[0].cpu().numpy() == 0) and np.all(ws.slot(2)[1].cpu().numpy() == 0)
    # decoded error against the exact FP64 step is the storage rounding
    e = errors(ws.decoded(), u_ref)
    assert e["rel_l2"] <= (2.0 ** -11 if fmt == "f16" else 2.0 ** -8)




@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_scale_exponent_clamp(gpu_lib, fmt):
    # A field of magnitude ~2^-100: the next scales' exponent ceil(log2 B) - 15
    # falls below -110 and is clamped there on both sides; the stored values
    # still follow the emulation.
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = 40, 24, 40
    g = lib.grid_init(nx, ny, nz, FMT[fmt])
    gv = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 2)
    V = fields.Field(gv).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    rng = np.random.default_rng(110)
    n = lowp.nslab(nz)
    s_cur = np.full(n, 2.0 ** -110, np.float32)
    s_prev = s_cur.copy()
    q_cur = lowp.round_to(rng.uniform(-2.0 ** 10, 2.0 ** 10, (nz, ny, nx)), fmt)
    q_prev = lowp.round_to(rng.uniform(-2.0 ** 10, 2.0 ** 10, (nz, ny, nx)), fmt)
    ws = _state_from(fields, g, q_prev, s_prev, q_cur, s_cur, fmt)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, gv, V.ptr, ws.st, 1)
    torch.cuda.synchronize()
    q_gpu = ws.cur().get_interior().astype(np.float64)
    s_gpu = ws.slot(1)[0].cpu().numpy()
    q_ref, s_ref, _, _ = lowp.step(co, v, dt, dx, fmt, q_prev, s_prev, lowp.slab_amax(q_prev, s_prev),
                                   q_cur, s_cur, lowp.slab_amax(q_cur, s_cur))
    assert np.all(s_ref == np.float32(2.0 ** -110))
    assert np.array_equal(s_gpu, s_ref)
    assert np.all(np.isfinite(q_gpu))
    d = np.abs(q_gpu - q_ref)
    assert np.all(d <= lowp.ulp(q_ref, fmt) + 2.0 ** -4), float(np.max(d))

@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (5, 1, 17), (2, 19, 3), (7, 3, 33), (66, 2, 16)])
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_single_step_degenerate_shapes(gpu_lib, fmt, shape):
    # Grids thinner than a tile or a load vector in some direction, where
    # most lanes load from clamped positions: one step from a random stored
    # state against the storage emulation, with a source at the centre.
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = shape
    g = lib.grid_init(nx, ny, nz, FMT[fmt])
    gv = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 5)
    V = fields.Field(gv).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    rng = np.random.default_rng(nx * 10007 + ny * 101 + nz)
    n = lowp.nslab(nz)
    s_cur = (2.0 ** rng.integers(-30, -10, n)).astype(np.float32)
    s_prev = (s_cur * 2).astype(np.float32)
    q_cur = lowp.round_to(rng.uniform(-2.0 ** 12, 2.0 ** 12, (nz, ny, nx)), fmt)
    q_prev = lowp.round_to(rng.uniform(-2.0 ** 12, 2.0 ** 12, (nz, ny, nx)), fmt)
    ws = _state_from(fields, g, q_prev, s_prev, q_cur, s_cur, fmt)
    src_xyz = np.array([[nx // 2, ny // 2, nz // 2]], np.int32)
    amp = torch.tensor([[1.0e-2]], dtype=torch.float32, device="cuda")
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, gv, V.ptr, ws.st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    torch.cuda.synchronize()
    q_gpu = ws.cur().get_interior().astype(np.float64)
    s_gpu = ws.slot(1)[0].cpu().numpy()
    a_gpu = ws.slot(1)[1].cpu().numpy()
    q_ref, s_ref, _, _ = lowp.step(co, v, dt, dx, fmt, q_prev, s_prev, lowp.slab_amax(q_prev, s_prev),
                                   q_cur, s_cur, lowp.slab_amax(q_cur, s_cur), src=src_xyz,
                                   amp_row=amp[0].cpu().numpy())
    assert np.array_equal(s_gpu, s_ref), shape
    d = np.abs(q_gpu - q_ref)
    assert np.all(d <= lowp.ulp(q_ref, fmt) + 2.0 ** -4), (shape, float(np.max(d)))
    assert np.array_equal(a_gpu, lowp.slab_amax(q_gpu, s_gpu)), shape

@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_multi_step_with_receivers(gpu_lib, fmt):
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = 72, 40, 52
    steps = 60
    p = synth.wave_problem(nx, ny, nz, steps, seed=4)
    g = lib.grid_init(nx, ny, nz, FMT[fmt])
    gv = lib.grid_init(nx, ny, nz)
    V = fields.Field(gv).set_interior(p["v"])
    co = synth.star25_coeffs()
    amp = torch.tensor(p["amp"] * 1e3, dtype=torch.float32, device="cuda")
    rec_xyz = np.concatenate([synth.receiver_plane(nx, ny, 8, 4), np.array([[36, 20, 26]], np.int32)])
    rec_d = torch.tensor(rec_xyz, dtype=torch.int32, device="cuda")
    traces = torch.zeros((steps, len(rec_xyz)), dtype=torch.float32, device="cuda")
    ws = fields.WaveState(g)
    lib.sp_wave_step(g, lib.coeffs(co), p["dt"], p["dx"], gv, V.ptr, ws.st, steps,
                     src=lib.make_sources(p["src"], amp.data_ptr(), 1),
                     rec=lib.make_receivers(len(rec_xyz), rec_d.data_ptr(), traces.data_ptr(),
                                            len(rec_xyz)))
    torch.cuda.synchronize()
    got = ws.decoded()
    a64 = amp.cpu().double().numpy()
    ref = oracle.wave_run(co, p["v"], p["dt"], p["dx"], steps, src=p["src"], amp=a64, rec=rec_xyz)
    emu, emu_tr = lowp.run(co, p["v"], p["dt"], p["dx"], fmt, steps, p["src"], a64, rec=rec_xyz)
    e_gpu = errors(got, oracle.interior(ref["cur"]))
    e_emu = errors(emu, oracle.interior(ref["cur"]))
    print(fmt, "60 steps vs FP64 oracle: GPU", e_gpu, "emulation", e_emu)
    assert e_gpu["rel_l2"] <= 2 * e_emu["rel_l2"] + 1e-6
    et = errors(traces.cpu().numpy(), ref["traces"])
    assert et["rel_l2"] <= 4 * errors(emu_tr, ref["traces"])["rel_l2"] + 1e-6


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_c2_full_size_single_step_sampled(gpu_lib, fmt):
    # 512^3 (the storage-form workload) in the bench's launch configuration:
    # one step from a stored state with per-slab scales over several
    # binades.  The new slab scales equal the emulation's exactly (they
    # depend only on slab maxima); at sampled points (corners and faces
    # included) the stored value is the oracle's FP64 step, rounded with
    # that scale, within 1 ulp plus the kernel's FP32 bound.
    from paper_2309_04671_amd import fields, lib
    n = 512
    g = lib.grid_init(n, n, n, FMT[fmt])
    gv = lib.grid_init(n, n, n)
    v = synth.layered_velocity(n, n, n, 0)
    V = fields.Field(gv).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    rng = np.random.default_rng(21)
    ns = lowp.nslab(n)
    mag = 2.0 ** rng.integers(-12, 4, ns)
    s_cur = (2.0 ** (np.ceil(np.log2(mag)) - 14)).astype(np.float32)
    s_prev = (s_cur * 2).astype(np.float32)
    pm = (mag[np.arange(n) // 16] / lowp.plane_scales(s_cur, n))[:, None, None]
    q_cur = lowp.round_to(rng.uniform(-1, 1, (n, n, n)).astype(np.float32) * pm, fmt).astype(np.float32)
    pm = (mag[np.arange(n) // 16] / lowp.plane_scales(s_prev, n))[:, None, None]
    q_prev = lowp.round_to(rng.uniform(-1, 1, (n, n, n)).astype(np.float32) * pm, fmt).astype(np.float32)
    del pm
    ws = _state_from(fields, g, q_prev, s_prev, q_cur, s_cur, fmt)
    a_cur, a_prev = lowp.slab_amax(q_cur, s_cur), lowp.slab_amax(q_prev, s_prev)
    src_xyz = np.array([[256, 256, 256], [511, 0, 300]], np.int32)
    amp_row = np.array([4.0e-3, -1.5e2], np.float32)
    amp = torch.tensor(amp_row[None, :], dtype=torch.float32, device="cuda")
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, gv, V.ptr, ws.st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 2))
    torch.cuda.synchronize()
    s_gpu = ws.slot(1)[0].cpu().numpy()
    s_ref = lowp.next_scales(a_cur, a_prev, n, dt, src_xyz, amp_row, v)
    assert np.array_equal(s_gpu, s_ref)
    # decoded inputs, padded with the zero halo, for the point-wise oracle
    pc = np.zeros((n + 8,) * 3, np.float32)
    pc[4:-4, 4:-4, 4:-4] = q_cur * lowp.plane_scales(s_cur, n)[:, None, None]
    pp = np.zeros((n + 8,) * 3, np.float32)
    pp[4:-4, 4:-4, 4:-4] = q_prev * lowp.plane_scales(s_prev, n)[:, None, None]
    del q_cur, q_prev
    pts = np.concatenate([sample_points(n, n, n, 300, 5), src_xyz])
    u_ref = oracle_wave_at(pp, pc, v, co, dt, dx, pts, src=src_xyz, amp_row=amp_row)
    q_out = ws.cur().interior()
    q_gpu = np.array([float(q_out[z, y, x]) for (x, y, z) in pts])
    q_ref = lowp.round_to(u_ref / s_ref[pts[:, 2] // 16], fmt)
    tol = lowp.ulp(q_ref, fmt) + 2.0 ** -4
    d = np.abs(q_gpu - q_ref)
    print(fmt, "512^3 sampled: max |dq| / ulp = %.3f, exact fraction %.4f" % (
        float(np.max(d / lowp.ulp(q_ref, fmt))), float(np.mean(d == 0))))
    assert np.all(d <= tol)
    assert float(np.mean(d == 0)) > 0.9
    # the recorded maxima are those of the GPU's own stored output
    q_all = ws.cur().get_interior().astype(np.float64)
    assert np.array_equal(ws.slot(1)[1].cpu().numpy(), lowp.slab_amax(q_all, s_gpu))
