"""Parity over seeded random grid shapes, each taking its own default launch
choice (tile, z-split, the small-grid rule): the 25-point sweep and one
leapfrog step against the FP64 oracle, one FP16/BF16 step against the
storage emulation, and the two-steps-per-sweep path bitwise against single
steps.  The shapes are drawn once from a fixed seed and include thin and
ragged extents in every direction.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import lowp
import synth
from tests.gpu_util import errors

pytestmark = pytest.mark.gpu


def _shapes(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.choice([int(rng.integers(1, 40)), int(rng.integers(40, 300))]))
        ny = int(rng.choice([int(rng.integers(1, 20)), int(rng.integers(20, 140))]))
        nz = int(rng.choice([int(rng.integers(1, 20)), int(rng.integers(20, 90))]))
        out.append((nx, ny, nz))
    return out


SHAPES = _shapes(16, 2309)


@pytest.mark.parametrize("shape", SHAPES, ids=["%dx%dx%d" % s for s in SHAPES])
def test_apply_and_step_random_shape(gpu_lib, shape):
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = shape
    co = synth.star25_coeffs()
    g = lib.grid_init(nx, ny, nz)
    seed = nx * 7919 + ny * 104729 + nz
    # one sweep of the star
    u = synth.uniform_field((nz, ny, nx), seed)
    U, W = fields.Field(g).set_interior(u), fields.Field(g)
    assert lib.sp_stencil_apply(g, lib.coeffs(co), 1, U.ptr, W.ptr) == 1
    # one leapfrog step from a random state with a source at the centre
    v = synth.layered_velocity(nx, ny, nz, seed % 97)
    V = fields.Field(g).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    prev = synth.uniform_field((nz, ny, nx), seed + 1)
    cur = synth.uniform_field((nz, ny, nx), seed + 2)
    ws = fields.WaveState(g)
    ws.a.set_interior(prev)
    ws.b.set_interior(cur)
    src_xyz = np.array([[nx // 2, ny // 2, nz // 2]], np.int32)
    amp = torch.tensor([[0.5]], dtype=torch.float32, device="cuda")
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, V.ptr, ws.st, 1,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    torch.cuda.synchronize()
    e_apply = errors(W.get_interior(), oracle.laplacian(oracle.padded(u), co))
    r = oracle.wave_run(co, v, dt, dx, 1, src=src_xyz, amp=np.array([[0.5]]),
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    e_step = errors(ws.cur().get_interior(), oracle.interior(r["cur"]))
    assert e_apply["rel_l2"] <= 1e-5, (shape, e_apply)
    assert e_step["rel_l2"] <= 1e-5, (shape, e_step)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES[::2], ids=["%dx%dx%d" % s for s in SHAPES[::2]])
def test_lowp_step_random_shape(gpu_lib, shape, fmt):
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = shape
    g = lib.grid_init(nx, ny, nz, {"f16": lib.SP_F16, "bf16": lib.SP_BF16}[fmt])
    gv = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 3)
    V = fields.Field(gv).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    rng = np.random.default_rng(nx + 1000 * ny + 100000 * nz)
    n = lowp.nslab(nz)
    s_cur = (2.0 ** rng.integers(-24, -8, n)).astype(np.float32)
    s_prev = (s_cur * 2).astype(np.float32)
    q_cur = lowp.round_to(rng.uniform(-2.0 ** 12, 2.0 ** 12, (nz, ny, nx)), fmt)
    q_prev = lowp.round_to(rng.uniform(-2.0 ** 12, 2.0 ** 12, (nz, ny, nx)), fmt)
    ws = fields.WaveState(g)
    ws.prev().set_interior(q_prev.astype(np.float32))
    ws.cur().set_interior(q_cur.astype(np.float32))
    sc, ac = ws.slot(0)
    sp, ap = ws.slot(-1)
    sc.copy_(torch.tensor(s_cur))
    sp.copy_(torch.tensor(s_prev))
    ac.copy_(torch.tensor(lowp.slab_amax(q_cur, s_cur)))
    ap.copy_(torch.tensor(lowp.slab_amax(q_prev, s_prev)))
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, gv, V.ptr, ws.st, 1)
    torch.cuda.synchronize()
    q_gpu = ws.cur().get_interior().astype(np.float64)
    s_gpu = ws.slot(1)[0].cpu().numpy()
    q_ref, s_ref, _, _ = lowp.step(co, v, dt, dx, fmt, q_prev, s_prev, lowp.slab_amax(q_prev, s_prev),
                                   q_cur, s_cur, lowp.slab_amax(q_cur, s_cur))
    assert np.array_equal(s_gpu, s_ref), shape
    d = np.abs(q_gpu - q_ref)
    assert np.all(d <= lowp.ulp(q_ref, fmt) + 2.0 ** -4), (shape, float(np.max(d)))


@pytest.mark.parametrize("shape", SHAPES[1::2], ids=["%dx%dx%d" % s for s in SHAPES[1::2]])
def test_fused_random_shape_bitwise(gpu_lib, shape):
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz = shape
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 11)
    V = fields.Field(g).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = lib.coeffs(synth.star25_coeffs())
    prev = synth.uniform_field((nz, ny, nx), 41)
    cur = synth.uniform_field((nz, ny, nx), 42)
    src_xyz = np.array([[nx // 2, ny // 2, nz // 2]], np.int32)
    amp = torch.tensor(synth.ricker(5, dt, 15.0)[:, None], dtype=torch.float32, device="cuda")
    ws = fields.WaveState(g)
    ws.a.set_interior(prev)
    ws.b.set_interior(cur)
    lib.sp_wave_step(g, co, dt, dx, g, V.ptr, ws.st, 5, src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    wf = fields.WaveState(g, spares=True)
    wf.a.set_interior(prev)
    wf.b.set_interior(cur)
    lib.sp_wave_step_fused(g, co, dt, dx, g, V.ptr, wf.st, 5, wf.spare,
                           src=lib.make_sources(src_xyz, amp.data_ptr(), 1))
    torch.cuda.synchronize()
    assert np.array_equal(ws.cur().get_interior(), wf.cur().get_interior()), shape
    assert np.array_equal(ws.prev().get_interior(), wf.prev().get_interior()), shape
