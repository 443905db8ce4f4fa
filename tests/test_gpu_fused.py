"""GPU parity of sp_wave_step_fused (two leapfrog steps per sweep).

Temporal blocking changes the schedule, not the arithmetic: the fused sweep
must reproduce the FP64 oracle's leapfrog (Eq. 2, Algorithm 1) to the same
bars as the single-step sweep, and it evaluates every point with the same
FP32 operations in the same order as the single-step kernel, so the two GPU
paths are also compared bit for bit.  Inputs span several inner tiles (56 x
24 or 56 x 40 points) with ragged tails, several z-chunks, sources on tile
edges (where a neighbour's ring recomputes them) and receivers.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import errors, oracle_wave_at, sample_points

pytestmark = pytest.mark.gpu

REGIONS = ["64x32", "64x48", "64x32x16", "64x48x7", "64x48x40"]


def _lib():
    from paper_2309_04671_amd import lib
    return lib


def _setup(nx, ny, nz, seed):
    from paper_2309_04671_amd import fields
    lib = _lib()
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, seed)
    vf = fields.Field(g).set_interior(v)
    return g, v, vf


def _fields(g, n):
    from paper_2309_04671_amd import fields
    return [fields.Field(g) for _ in range(n)]


def _edge_sources(nx, ny, nz):
    # inner-tile edges (x = 55/56, y = 23/24 and 39/40), a z-chunk edge, the
    # grid corners and the centre
    pts = [[55, 23, 15], [56, 24, 16], [57, 40, 7], [111, 39, nz - 1], [0, 0, 0],
           [nx - 1, ny - 1, nz - 1], [nx // 2, ny // 2, nz // 2]]
    return np.array([p for p in pts if p[0] < nx and p[1] < ny and p[2] < nz], np.int32)


@pytest.mark.parametrize("region", REGIONS)
def test_fused_random_state_two_steps(gpu_lib, region, monkeypatch):
    # One fused sweep from a random state with sources on tile edges, against
    # two oracle steps.
    lib = _lib()
    monkeypatch.setenv("SP_TILE_FUSED", region)
    nx, ny, nz = 130, 70, 41
    g, v, vf = _setup(nx, ny, nz, 3)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.random_coeffs(6)
    prev = synth.uniform_field((nz, ny, nx), 21)
    cur = synth.uniform_field((nz, ny, nx), 22)
    P, C, S0, S1 = _fields(g, 4)
    P.set_interior(prev)
    C.set_interior(cur)
    src_xyz = _edge_sources(nx, ny, nz)
    ns = len(src_xyz)
    amp = torch.tensor(np.stack([np.linspace(1e4, 3e4, ns), np.linspace(-2e4, 1e4, ns)]),
                       dtype=torch.float32, device="cuda")
    src = lib.make_sources(src_xyz, amp.data_ptr(), ns)
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    spare = [S0.ptr, S1.ptr]
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, vf.ptr, st, 2, spare, src=src)
    torch.cuda.synchronize()
    assert (st.prev, st.cur, st.step) == (S0.ptr, S1.ptr, 2)
    assert spare == [P.ptr, C.ptr]
    r = oracle.wave_run(co, v, dt, dx, 2, src=src_xyz, amp=amp.cpu().double().numpy(),
                        prev=oracle.padded(prev), cur=oracle.padded(cur))
    e1 = errors(S0.get_interior(), oracle.interior(r["prev"]))
    e2 = errors(S1.get_interior(), oracle.interior(r["cur"]))
    print(region, "u^1", e1, "u^2", e2)
    assert e1["rel_l2"] <= 1e-5 and e2["rel_l2"] <= 1e-5
    ref2 = oracle.interior(r["cur"])
    got2 = S1.get_interior()
    for (x, y, z) in src_xyz:
        assert abs(got2[z, y, x] - ref2[z, y, x]) <= 1e-5 * 3e4 + 1e-4 * abs(ref2[z, y, x])


@pytest.mark.parametrize("region", REGIONS[:2])
@pytest.mark.parametrize("nsteps", [0, 1, 2, 7, 40])
def test_fused_bitwise_equal_to_single_step(gpu_lib, region, nsteps, monkeypatch):
    # Same state, sources and receivers through both paths: identical fields
    # and traces (odd counts end with one single-step sweep).
    from paper_2309_04671_amd import fields
    lib = _lib()
    monkeypatch.setenv("SP_TILE_FUSED", region)
    nx, ny, nz = 117, 53, 38
    g, v, vf = _setup(nx, ny, nz, 5)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src_xyz = np.array([[58, 26, 19], [56, 24, 5]], np.int32)
    w = synth.ricker(max(nsteps, 1), dt, 15.0)
    amp = torch.tensor(np.stack([w, -0.5 * w], axis=1), dtype=torch.float32, device="cuda")
    rec_xyz = np.concatenate([synth.receiver_plane(nx, ny, 3, 4),
                              np.array([[56, 24, 19], [116, 52, 37]], np.int32)])
    nrec = len(rec_xyz)
    rec_d = torch.tensor(rec_xyz, dtype=torch.int32, device="cuda")
    prev = synth.uniform_field((nz, ny, nx), 31)
    cur = synth.uniform_field((nz, ny, nx), 32)

    ws = fields.WaveState(g)
    ws.a.set_interior(prev)
    ws.b.set_interior(cur)
    tr1 = torch.zeros((max(nsteps, 1), nrec), dtype=torch.float32, device="cuda")
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, ws.st, nsteps,
                     src=lib.make_sources(src_xyz, amp.data_ptr(), 2),
                     rec=lib.make_receivers(nrec, rec_d.data_ptr(), tr1.data_ptr(), nrec))

    wf = fields.WaveState(g, spares=True)
    wf.a.set_interior(prev)
    wf.b.set_interior(cur)
    tr2 = torch.zeros_like(tr1)
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, vf.ptr, wf.st, nsteps, wf.spare,
                           src=lib.make_sources(src_xyz, amp.data_ptr(), 2),
                           rec=lib.make_receivers(nrec, rec_d.data_ptr(), tr2.data_ptr(), nrec))
    torch.cuda.synchronize()
    assert ws.st.step == wf.st.step == nsteps
    a1, a2 = ws.cur().get_interior(), wf.cur().get_interior()
    b1, b2 = ws.prev().get_interior(), wf.prev().get_interior()
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    assert torch.equal(tr1, tr2)
    # the spares are the two fields the state does not hold
    held = {wf.st.cur, wf.st.prev}
    assert set(wf.spare) == {f.ptr for f in [wf.a, wf.b] + wf.extra} - held


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 1), (5, 3, 2), (9, 70, 3), (57, 25, 9),
                                   (200, 5, 70), (56, 40, 16), (112, 80, 33)])
def test_fused_degenerate_and_exact_shapes_bitwise(gpu_lib, shape):
    # Grids of one point, single planes and rows, fewer planes than the
    # 4-plane start-up, and exact multiples of the 56 x 40 tile: six steps
    # (three fused sweeps) equal six single steps bit for bit.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = shape
    g, v, vf = _setup(nx, ny, nz, 7)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.random_coeffs(nx + ny + nz)
    src_xyz = np.array([[nx // 2, ny // 2, nz // 2], [nx - 1, 0, nz - 1]], np.int32)
    amp = torch.tensor(np.linspace(-1e4, 2e4, 12).reshape(6, 2), dtype=torch.float32, device="cuda")
    prev = synth.uniform_field((nz, ny, nx), 41)
    cur = synth.uniform_field((nz, ny, nx), 42)
    ws, wf = fields.WaveState(g), fields.WaveState(g, spares=True)
    for w in (ws, wf):
        w.a.set_interior(prev)
        w.b.set_interior(cur)
    src = lib.make_sources(src_xyz, amp.data_ptr(), 2)
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, vf.ptr, ws.st, 6, src=src)
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, vf.ptr, wf.st, 6, wf.spare, src=src)
    torch.cuda.synchronize()
    assert np.array_equal(ws.cur().get_interior(), wf.cur().get_interior())
    assert np.array_equal(ws.prev().get_interior(), wf.prev().get_interior())
    # the halos of all four fields are still zero
    for f in [wf.a, wf.b] + wf.extra:
        pad = f.padded().cpu().numpy()
        pad[4:-4, 4:-4, 4:-4] = 0
        assert not pad.any()


def test_fused_multi_step_with_receivers_vs_oracle(gpu_lib):
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 72, 50, 36
    steps = 60
    g, v, vf = _setup(nx, ny, nz, 1)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src_xyz = np.array([[36, 25, 18]], np.int32)
    w = synth.ricker(steps, dt, 15.0)[:, None]
    rec_xyz = np.concatenate([synth.receiver_plane(nx, ny, 4, 3),
                              np.array([[36, 25, 18], [71, 49, 35]], np.int32)])
    nrec = len(rec_xyz)
    amp = torch.tensor(w, dtype=torch.float32, device="cuda")
    rec_d = torch.tensor(rec_xyz, dtype=torch.int32, device="cuda")
    traces = torch.zeros((steps, nrec), dtype=torch.float32, device="cuda")
    ws = fields.WaveState(g, spares=True)
    src = lib.make_sources(src_xyz, amp.data_ptr(), 1)
    # 31 + 29 steps: the first call ends on a single step, the second starts on it
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, vf.ptr, ws.st, 31, ws.spare, src=src,
                           rec=lib.make_receivers(nrec, rec_d.data_ptr(), traces.data_ptr(), nrec))
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, vf.ptr, ws.st, 29, ws.spare, src=src,
                           rec=lib.make_receivers(nrec, rec_d.data_ptr(), traces[31:].data_ptr(), nrec))
    torch.cuda.synchronize()
    assert ws.st.step == steps
    r = oracle.wave_run(co, v, dt, dx, steps, src=src_xyz, amp=amp.cpu().double().numpy(), rec=rec_xyz)
    e = errors(ws.cur().get_interior(), oracle.interior(r["cur"]))
    et = errors(traces.cpu().numpy(), r["traces"])
    print("60 fused steps 72x50x36 vs oracle:", e, "traces", et)
    assert e["rel_l2"] <= 1e-4 and et["rel_l2"] <= 1e-4


def _oracle_two_steps_at(prev_pad, cur_pad, v, co, dt, dx, pts, src, amp):
    """u^{n+2} at each point: two oracle steps on the radius-4 box around it,
    clipped to the grid, with the real 4-cell frame.  u^{n+1} is exact on the
    box and the second step at the centre reads only the box or the zero halo."""
    nz, ny, nx = v.shape
    out = np.empty(len(pts))
    for k, (x, y, z) in enumerate(pts):
        x0, x1 = max(0, x - 4), min(nx, x + 5)
        y0, y1 = max(0, y - 4), min(ny, y + 5)
        z0, z1 = max(0, z - 4), min(nz, z + 5)
        sl = (slice(z0, z1 + 8), slice(y0, y1 + 8), slice(x0, x1 + 8))
        inside = [j for j, (sx, sy, sz) in enumerate(src)
                  if x0 <= sx < x1 and y0 <= sy < y1 and z0 <= sz < z1]
        s = np.array([[src[j][0] - x0, src[j][1] - y0, src[j][2] - z0] for j in inside], np.int32)
        a = amp[:, inside] if inside else None
        r = oracle.wave_run(co, v[z0:z1, y0:y1, x0:x1], dt, dx, 2,
                            src=s if inside else None, amp=a,
                            prev=prev_pad[sl], cur=cur_pad[sl])
        out[k] = r["cur"][z - z0 + 4, y - y0 + 4, x - x0 + 4]
    return out


def test_fused_full_size_sampled_parity(gpu_lib):
    # 1024x1024x512 (the benchmark workload) in the fused path's own launch
    # configuration: one fused sweep from a random state, u^{n+1} and u^{n+2}
    # at sampled points (corners and faces included) against the oracle.
    from paper_2309_04671_amd import fields
    lib = _lib()
    nx, ny, nz = 1024, 1024, 512
    g = lib.grid_init(nx, ny, nz)
    gen = torch.Generator(device="cuda").manual_seed(12)
    P, C, V, S0, S1 = (fields.Field(g) for _ in range(5))
    v = synth.layered_velocity(nx, ny, nz, 0)
    V.set_interior(v)
    P.interior().uniform_(-1, 1, generator=gen)
    C.interior().uniform_(-1, 1, generator=gen)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src_xyz = np.array([[512, 512, 256], [560, 520, 257]], np.int32)
    amp_np = np.array([[5.0e4, -3.0e4], [4.0e4, 2.0e4]])
    amp = torch.tensor(amp_np, dtype=torch.float32, device="cuda")
    pts = np.concatenate([sample_points(nx, ny, nz, 300, 4), src_xyz,
                          np.array([[558, 519, 256], [511, 515, 253]], np.int32)])
    prev_pad = P.padded().cpu().numpy()
    cur_pad = C.padded().cpu().numpy()
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    lib.sp_wave_step_fused(g, lib.coeffs(co), dt, dx, g, V.ptr, st, 2, [S0.ptr, S1.ptr],
                           src=lib.make_sources(src_xyz, amp.data_ptr(), 2))
    torch.cuda.synchronize()
    o1, o2 = S0.interior(), S1.interior()
    got1 = np.array([float(o1[z, y, x]) for (x, y, z) in pts])
    got2 = np.array([float(o2[z, y, x]) for (x, y, z) in pts])
    ref1 = oracle_wave_at(prev_pad, cur_pad, v, co, dt, dx, pts, src=src_xyz, amp_row=amp_np[0])
    ref2 = _oracle_two_steps_at(prev_pad, cur_pad, v, co, dt, dx, pts, src_xyz, amp_np)
    e1, e2 = errors(got1, ref1), errors(got2, ref2)
    print("1024x1024x512 sampled fused sweep vs oracle:", e1, e2)
    assert e1["rel_l2"] <= 1e-5 and e2["rel_l2"] <= 1e-5
