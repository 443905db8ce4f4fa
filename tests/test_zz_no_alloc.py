"""The allocation-free energy entry point against sp_energy.

sp_energy_noalloc keeps its per-block partial sums in a static device array
instead of a caller workspace.  Two calls in a row (a ragged grid spanning
several tiles and z-chunks, then a smaller one, so that the second call
reuses the array the first one filled) must give exactly what sp_energy
gives for the same inputs (same kernels, same fixed summation order), and
both must match the FP64 oracle's energy.  A grid whose sweep needs more
partial sums than the array holds is refused before any launch.
"""

import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _energy_pair(lib, fields, nx, ny, nz, seed):
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, seed)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    V = fields.Field(g).set_interior(v)
    u0 = synth.uniform_field((nz, ny, nx), seed + 1)
    u1 = synth.uniform_field((nz, ny, nx), seed + 2)
    F0, F1 = fields.Field(g).set_interior(u0), fields.Field(g).set_interior(u1)
    out_ws = torch.zeros(1, dtype=torch.float64, device="cuda")
    out_na = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    wsb = torch.empty(int(lib.load().sp_energy_ws_bytes(g)) // 8, dtype=torch.float64, device="cuda")
    lib.sp_energy(g, lib.coeffs(co), dt, dx, g, V.ptr, F0.ptr, F1.ptr, out_ws.data_ptr(), wsb.data_ptr())
    lib.sp_energy_noalloc(g, lib.coeffs(co), dt, dx, g, V.ptr, F0.ptr, F1.ptr, out_na.data_ptr())
    torch.cuda.synchronize()
    ref = oracle.energy(co, v, dt, dx, oracle.padded(u0), oracle.padded(u1))
    return float(out_ws.item()), float(out_na.item()), ref


def test_noalloc_energy_matches_workspace_form(gpu_lib):
    from paper_2309_04671_amd import fields, lib
    assert int(gpu_lib.sp_energy_noalloc_max_partials()) == 1 << 16
    # larger call first, then a smaller one that reuses the array
    for (nx, ny, nz, seed) in ((301, 45, 70, 3), (96, 40, 50, 5)):
        e_ws, e_na, ref = _energy_pair(lib, fields, nx, ny, nz, seed)
        print("energy %dx%dx%d: workspace %.17g, no-alloc %.17g, oracle %.17g" % (nx, ny, nz, e_ws, e_na, ref))
        assert e_na == e_ws, (nx, ny, nz, e_na, e_ws)
        assert abs(e_na - ref) <= 1e-6 * abs(ref)


def test_noalloc_energy_refuses_grids_beyond_its_scratch(gpu_lib, monkeypatch):
    from paper_2309_04671_amd import fields, lib
    # 64x16 tiles with one-plane z-chunks: 16 x 32 tiles x 130 chunks = 66560
    # partial sums, above the 65536 the static array holds
    monkeypatch.setenv("SP_TILE", "64x16x1x1")
    nx, ny, nz = 1024, 512, 130
    g = lib.grid_init(nx, ny, nz)
    V, F0, F1 = fields.Field(g), fields.Field(g), fields.Field(g)
    V.interior().fill_(2000.0)               # m > 0: the energy of zero fields is 0
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    co = lib.coeffs(synth.star25_coeffs())
    rc = gpu_lib.sp_energy_noalloc(g, co, 1e-3, 10.0, g, V.ptr, F0.ptr, F1.ptr, out.data_ptr(),
                                   lib.stream_ptr())
    assert rc == lib.SP_ENOMEM, (rc, lib.last_error())
    assert "partial sums" in lib.last_error()
    torch.cuda.synchronize()
    assert float(out.item()) == 7.0          # nothing was launched
    # the same grid with the workspace form still works
    wsb = torch.empty(int(gpu_lib.sp_energy_ws_bytes(g)) // 8, dtype=torch.float64, device="cuda")
    lib.sp_energy(g, co, 1e-3, 10.0, g, V.ptr, F0.ptr, F1.ptr, out.data_ptr(), wsb.data_ptr())
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0          # zero fields, zero energy
