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
