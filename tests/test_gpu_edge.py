"""Degenerate calls on the GPU: zero sweeps and zero steps change nothing.

Every compute entry point accepts a zero count and must then leave every
buffer, the state's field pointers and its step counter exactly as they
were (bitwise), and report the input as the result buffer of a sweep.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _snap(*fields):
    return [f.buf.clone() for f in fields]


def _same(before, *fields):
    return all(torch.equal(b, f.buf) for b, f in zip(before, fields))


def test_zero_sweeps(gpu_lib):
    from paper_2309_04671_amd import fields, lib
    g = lib.grid_init(37, 21, 19)
    U, W = fields.Field(g), fields.Field(g)
    for f in (U, W):    # random bytes everywhere, halos included
        f.buf.copy_(torch.randint(0, 256, f.buf.shape, dtype=torch.uint8, device=f.buf.device))
    before = _snap(U, W)
    assert lib.sp_stencil_apply(g, lib.coeffs(synth.star25_coeffs()), 0, U.ptr, W.ptr) == 0
    w = synth.suite_weights("box3d2r", 0)
    assert lib.sp_apply(g, "box", w, U.ptr, W.ptr, 0) == 0
    torch.cuda.synchronize()
    assert _same(before, U, W)


@pytest.mark.parametrize("entry", ["step", "fused", "seven", "two", "unified"])
def test_zero_steps(gpu_lib, entry):
    from paper_2309_04671_amd import fields, lib
    nx, ny, nz, W = 40, 36, 44, 8
    p = synth.wave_problem(nx, ny, nz, 4, seed=2)
    g = lib.grid_init(nx, ny, nz)
    V = fields.Field(g).set_interior(p["v"])
    ws = fields.WaveState(g, spares=(entry == "fused"))
    ws.cur().set_interior(synth.uniform_field((nz, ny, nx), 3))
    ws.prev().set_interior(synth.uniform_field((nz, ny, nx), 4))
    ws.st.step = 2
    E, PSI = fields.Field(g), fields.Field(g)
    PSI.set_interior(synth.uniform_field((nz, ny, nx), 5))
    amp = torch.ones((4, 1), dtype=torch.float32, device="cuda")
    src = lib.make_sources(p["src"], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    if entry in ("seven", "two", "unified"):
        lib.sp_pml_profile(g, W, synth.pml_eta_max(float(p["v"].max()), W, p["dx"]), E.ptr)
    torch.cuda.synchronize()
    everything = [ws.a, ws.b, V, E, PSI] + ws.extra
    before = _snap(*everything)
    ptrs = (ws.st.cur, ws.st.prev, list(ws.spare))
    if entry == "step":
        lib.sp_wave_step(g, co, p["dt"], p["dx"], g, V.ptr, ws.st, 0, src=src)
    elif entry == "fused":
        lib.sp_wave_step_fused(g, co, p["dt"], p["dx"], g, V.ptr, ws.st, 0, ws.spare, src=src)
    else:
        dec = {"unified": lib.SP_PML_UNIFIED, "seven": lib.SP_PML_SEVEN, "two": lib.SP_PML_TWO}[entry]
        lib.sp_wave_step_pml(g, co, p["dt"], p["dx"], g, V.ptr, ws.st, 0,
                             lib.make_pml(W, E.ptr, PSI.ptr, np.pi * 15, dec), src=src)
    torch.cuda.synchronize()
    assert _same(before, *everything)
    assert (ws.st.cur, ws.st.prev, list(ws.spare)) == ptrs
    assert ws.st.step == 2


@pytest.mark.timeout(600)
def test_leapfrog_beyond_2_32_elements_sampled(gpu_lib):
    # The largest size class: a 2048 x 2048 x 1040 FP32 grid has more than
    # 2^32 elements per field (17.9 GB each), so element offsets of its last
    # planes need 64 bits.  One leapfrog step from a random state (inputs
    # built on the device from a seeded generator), checked against the
    # oracle at sampled points, many of them in the planes beyond 2^32.
    from paper_2309_04671_amd import fields, lib
    import oracle
    nx, ny, nz = 2048, 2048, 1040
    g = lib.grid_init(nx, ny, nz)
    assert g.elems > 2 ** 32
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    V, P, C = fields.Field(g), fields.Field(g), fields.Field(g)
    speeds = np.random.default_rng(0).uniform(1500.0, 4500.0, 8)
    for k in range(8):                           # 8 horizontal layers of 130 planes
        V.interior()[k * 130:(k + 1) * 130].fill_(float(speeds[k]))
    for F in (P, C):
        for z0 in range(0, nz, 65):              # in slabs: uniform_ on a strided view
            F.interior()[z0:z0 + 65].uniform_(-1.0, 1.0, generator=gen)
    dx = 10.0
    dt = 0.4 * dx / float(speeds.max())
    co = synth.star25_coeffs()
    st = lib.sp_wave_state(C.ptr, P.ptr, None, 0)
    Pp = P.padded()
    rng = np.random.default_rng(3)
    pts = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))) for _ in range(120)]
    pts += [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(1001, nz))) for _ in range(120)]
    pts += [(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)]
    # the neighbourhoods of u^{n-1} and u^n before the step (u^{n+1} overwrites u^{n-1})
    before = [(Pp[z:z + 9, y:y + 9, x:x + 9].double().cpu().numpy(),
               C.padded()[z:z + 9, y:y + 9, x:x + 9].double().cpu().numpy()) for (x, y, z) in pts]
    lib.sp_wave_step(g, lib.coeffs(co), dt, dx, g, V.ptr, st, 1)
    torch.cuda.synchronize()
    out = (P if st.cur == P.ptr else C).padded()
    got = np.array([float(out[z + 4, y + 4, x + 4]) for (x, y, z) in pts])
    vi = V.interior()
    ref = np.empty(len(pts))
    for k, ((x, y, z), (pv, cu)) in enumerate(zip(pts, before)):
        r = oracle.wave_run(co, np.array([[[float(vi[z, y, x])]]]), dt, dx, 1, prev=pv, cur=cu)
        ref[k] = r["cur"][4, 4, 4]
    e = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0))
    print("2048x2048x1040 (%d elements per field), %d sampled points: max relative error %.2e"
          % (g.elems, len(pts), e))
    assert e <= 1e-5
