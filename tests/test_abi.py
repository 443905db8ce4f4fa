"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, lays grids out as documented, and rejects bad arguments
before touching the device."""

import ctypes
import os
import re

import pytest

from paper_2309_04671_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.sp_version().decode().startswith("libstencil")


@pytest.mark.parametrize("dtype,eb", [(lib.SP_F32, 4), (lib.SP_F16, 2), (lib.SP_BF16, 2)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (64, 64, 64), (70, 37, 23), (1024, 1024, 512)])
def test_grid_layout(shape, dtype, eb):
    nx, ny, nz = shape
    g = lib.grid_init(nx, ny, nz, dtype)
    assert g.elem_bytes == eb and g.halo == 4
    assert g.pitch_y == ny + 8 and g.planes == nz + 8
    # interior x = 0 of every row is 128-byte aligned
    assert (g.origin * eb) % 128 == 0 and (g.pitch_x * eb) % 128 == 0
    # the left halo and the previous row's right halo fit in the lead pad
    lead = g.origin - (4 * g.pitch_y + 4) * g.pitch_x
    assert lead >= 8 and g.pitch_x >= lead + nx
    # every padded cell is a distinct element inside the allocation
    sz, sy = g.pitch_x * g.pitch_y, g.pitch_x
    first = g.origin - 4 * sz - 4 * sy - 4
    last = g.origin + (nz + 3) * sz + (ny + 3) * sy + (nx + 3)
    assert first >= 0 and last < g.elems and g.elems * eb <= g.bytes
    assert g.bytes % 256 == 0
    # row y's right halo ends before row y+1's left halo starts
    assert (nx + 3) < sy - 4


def test_grid_init_rejects_bad_arguments():
    L = lib.load()
    g = lib.sp_grid()
    assert L.sp_grid_init(8, 8, 8, 3, lib.SP_F32, ctypes.byref(g)) == lib.SP_EINVAL
    assert "halo" in lib.last_error()
    assert L.sp_grid_init(0, 8, 8, 4, lib.SP_F32, ctypes.byref(g)) == lib.SP_EINVAL
    assert L.sp_grid_init(8, 8, 8, 4, 7, ctypes.byref(g)) == lib.SP_EINVAL
    assert L.sp_grid_init(8, 8, 8, 4, lib.SP_F32, None) == lib.SP_EINVAL


def test_apply_validates_before_launch():
    L = lib.load()
    g = lib.grid_init(16, 16, 16)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    out = ctypes.c_int()
    # overlapping u and v
    rc = L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), 1, ctypes.c_void_p(4096),
                            ctypes.c_void_p(4096 + 256), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL and "overlap" in lib.last_error()
    # misaligned pointer
    rc = L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), 1, ctypes.c_void_p(4100),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL and "aligned" in lib.last_error()
    # descriptor not from sp_grid_init
    bad = lib.grid_init(16, 16, 16)
    bad.pitch_x += 1
    rc = L.sp_stencil_apply(ctypes.byref(bad), ctypes.byref(c), 1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL and "sp_grid_init" in lib.last_error()
    # a descriptor whose own dimensions are invalid: the message keeps the reason
    bad = lib.grid_init(16, 16, 16)
    bad.halo = 3
    rc = L.sp_stencil_apply(ctypes.byref(bad), ctypes.byref(c), 1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    msg = lib.last_error()
    assert rc == lib.SP_EINVAL and "invalid grid descriptor" in msg and "halo" in msg, msg
    # FP16 grids are not supported by apply
    h = lib.grid_init(16, 16, 16, lib.SP_F16)
    rc = L.sp_stencil_apply(ctypes.byref(h), ctypes.byref(c), 1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EUNSUPPORTED
    # negative sweeps
    rc = L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), -1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL


def test_wave_step_validates_before_launch():
    L = lib.load()
    g = lib.grid_init(32, 32, 32)
    gv = lib.grid_init(32, 32, 32)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    st = lib.sp_wave_state(1 << 30, 1 << 36, None, 0)
    v = ctypes.c_void_p(1 << 40)

    def call(**kw):
        a = dict(g=g, gv=gv, dt=1e-3, dx=10.0, st=st, n=1, src=None, rec=None)
        a.update(kw)
        return L.sp_wave_step(ctypes.byref(a["g"]), ctypes.byref(c), a["dt"], a["dx"],
                              ctypes.byref(a["gv"]), v, ctypes.byref(a["st"]), a["n"],
                              ctypes.byref(a["src"]) if a["src"] is not None else None,
                              ctypes.byref(a["rec"]) if a["rec"] is not None else None, None)

    assert call(gv=lib.grid_init(32, 32, 31)) == lib.SP_EINVAL
    assert call(dt=0.0) == lib.SP_EINVAL
    assert call(n=-1) == lib.SP_EINVAL
    assert call(st=lib.sp_wave_state(1 << 30, (1 << 30) + 512, None, 0)) == lib.SP_EINVAL
    src = lib.make_sources([[40, 1, 1]], 1 << 20, 1)
    assert call(src=src) == lib.SP_EINVAL and "outside" in lib.last_error()
    src = lib.make_sources([[4, 1, 1]], None, 1)
    assert call(src=src) == lib.SP_EINVAL
    rec = lib.make_receivers(5, None, None, 5)
    assert call(rec=rec) == lib.SP_EINVAL
    rec = lib.make_receivers(5, 1 << 20, 1 << 21, 4)
    assert call(rec=rec) == lib.SP_EINVAL
    # the state must be untouched by a rejected call
    assert st.cur == 1 << 30 and st.step == 0
    # a 16-bit wavefield placed in the upper part of the (larger) FP32 v
    h, hv = lib.grid_init(256, 8, 8, lib.SP_F16), lib.grid_init(256, 8, 8)
    inside = (1 << 40) + h.bytes                  # past v's first h.bytes, inside v
    hs = lib.sp_wave_state(inside, 1 << 36, 1 << 20, 0)
    assert h.bytes < hv.bytes
    assert call(g=h, gv=hv, st=hs) == lib.SP_EINVAL and "v overlaps" in lib.last_error()


def test_fused_step_validates_before_launch(monkeypatch):
    L = lib.load()
    g = lib.grid_init(32, 32, 32)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    big = g.bytes + 4096
    cur, prev, s0, s1 = (1 << 30), (1 << 30) + big, (1 << 30) + 2 * big, (1 << 30) + 3 * big
    st = lib.sp_wave_state(cur, prev, None, 0)
    v = ctypes.c_void_p(1 << 40)

    def call(spare, gg=g, n=2, state=st):
        arr = (ctypes.c_void_p * 2)(*spare) if spare is not None else None
        return L.sp_wave_step_fused(ctypes.byref(gg), ctypes.byref(c), 1e-3, 10.0, ctypes.byref(g),
                                    v, ctypes.byref(state), n, arr, None, None, None)

    assert call(None) == lib.SP_EINVAL
    assert call([s0, None]) == lib.SP_EINVAL
    assert call([s0, s0]) == lib.SP_EINVAL and "overlap" in lib.last_error()
    assert call([s0, prev + 256]) == lib.SP_EINVAL and "overlap" in lib.last_error()
    assert call([s0, s1 + 4]) == lib.SP_EINVAL and "aligned" in lib.last_error()
    assert call([s0, (1 << 40) + 64]) == lib.SP_EINVAL        # overlaps v
    assert call([s0, s1], n=-1) == lib.SP_EINVAL
    g16 = lib.grid_init(32, 32, 32, dtype=lib.SP_F16)
    assert call([s0, s1], gg=g16) in (lib.SP_EINVAL, lib.SP_EUNSUPPORTED)
    monkeypatch.setenv("SP_TILE_FUSED", "64x40")
    assert call([s0, s1]) == lib.SP_EINVAL and "not compiled" in lib.last_error()
    assert st.cur == cur and st.prev == prev and st.step == 0


def test_unknown_tile_override_is_rejected(monkeypatch):
    monkeypatch.setenv("SP_TILE", "96x7x1")
    L = lib.load()
    g = lib.grid_init(16, 16, 16)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    out = ctypes.c_int()
    rc = L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), 1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL and "not compiled" in lib.last_error()


@pytest.mark.parametrize("shape", [(1, 1), (70, 37), (8192, 8192), (1000, 1000)])
def test_grid_2d_layout(shape):
    nx, ny = shape
    g = lib.grid_init_2d(nx, ny)
    g3 = lib.grid_init(nx, ny, 1)
    assert g.nz == 1 and g.planes == 1 and g.halo == 4
    assert g.pitch_x == g3.pitch_x and g.pitch_y == ny + 8
    assert (g.origin * 4) % 128 == 0
    sy = g.pitch_x
    first = g.origin - 4 * sy - 4
    last = g.origin + (ny + 3) * sy + (nx + 3)
    assert first >= 0 and last < g.elems and g.elems * 4 <= g.bytes and g.bytes % 256 == 0
    assert g.bytes < g3.bytes


def _stencil(shape, ndim, r, w=None):
    import numpy as np
    w = np.ones((2 * r + 1,) * ndim) if w is None else w
    st = lib.sp_stencil()
    st.shape, st.ndim, st.radius = shape, ndim, r
    st.w = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return st, w


def test_suite_apply_validates_before_launch():
    import numpy as np
    L = lib.load()
    g3, g2 = lib.grid_init(16, 16, 16), lib.grid_init_2d(16, 16)
    out = ctypes.c_int()
    U, V = ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 40)

    def call(g, st, sweeps=1, u=U, v=V):
        return L.sp_apply(ctypes.byref(g), ctypes.byref(st), sweeps, u, v, ctypes.byref(out), None)

    box, wb = _stencil(lib.SP_BOX, 3, 2)
    # a star with an off-axis weight
    ws = np.zeros((5, 5, 5))
    ws[2, 2, :] = 1
    ws[0, 0, 0] = 0.5
    st, _ = _stencil(lib.SP_STAR, 3, 2, ws)
    assert call(g3, st) == lib.SP_EINVAL and "off the axes" in lib.last_error()
    for shape, ndim, r in ((5, 3, 2), (lib.SP_BOX, 4, 2), (lib.SP_BOX, 3, 0), (lib.SP_BOX, 3, 5)):
        bad, _ = _stencil(shape, ndim, r, np.ones(9 ** 3))
        assert call(g3, bad) == lib.SP_EINVAL
    nan = np.ones((5, 5, 5))
    nan[1, 2, 3] = np.nan
    bad, _ = _stencil(lib.SP_BOX, 3, 2, nan)
    assert call(g3, bad) == lib.SP_EINVAL and "finite" in lib.last_error()
    # 3D stencil on a 2D grid; 2D grids elsewhere in the library
    assert call(g2, box) == lib.SP_EINVAL and "3D grid" in lib.last_error()
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    assert L.sp_stencil_apply(ctypes.byref(g2), ctypes.byref(c), 1, U, V, ctypes.byref(out),
                              None) == lib.SP_EINVAL
    # aliasing, alignment, dtype, sweeps, forged descriptor
    assert call(g3, box, u=ctypes.c_void_p(4096), v=ctypes.c_void_p(4096 + 256)) == lib.SP_EINVAL
    assert call(g3, box, u=ctypes.c_void_p(4100)) == lib.SP_EINVAL
    assert call(g3, box, sweeps=-1) == lib.SP_EINVAL
    h = lib.grid_init(16, 16, 16, lib.SP_F16)
    assert call(h, box) == lib.SP_EUNSUPPORTED
    forged = lib.grid_init_2d(16, 16)
    forged.origin += 1
    assert call(forged, box) == lib.SP_EINVAL
    # sweeps = 0 is a no-op that launches nothing
    assert call(g3, box, sweeps=0) == lib.SP_OK and out.value == 0


def test_decode_validates_before_launch():
    L = lib.load()
    g = lib.grid_init(32, 32, 32)
    g16 = lib.grid_init(32, 32, 32, dtype=lib.SP_F16)
    f, out = ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 36)
    assert L.sp_decode(None, f, None, 0, out, None) == lib.SP_EINVAL
    assert L.sp_decode(ctypes.byref(g), None, None, 0, out, None) == lib.SP_EINVAL
    assert L.sp_decode(ctypes.byref(g), f, None, 0, None, None) == lib.SP_EINVAL
    # FP16/BF16 fields need their slab records
    assert L.sp_decode(ctypes.byref(g16), f, None, 0, out, None) == lib.SP_EINVAL
    assert "slab records" in lib.last_error()
    # out may not overlap the field
    assert L.sp_decode(ctypes.byref(g), f, None, 0, ctypes.c_void_p((1 << 30) + 4096), None) == lib.SP_EINVAL
    assert "overlaps" in lib.last_error()
    bad = lib.grid_init(32, 32, 32)
    bad.pitch_x += 1
    assert L.sp_decode(ctypes.byref(bad), f, None, 0, out, None) == lib.SP_EINVAL


def test_energy_noalloc_validates_before_launch():
    L = lib.load()
    assert L.sp_energy_noalloc_max_partials() == 1 << 16
    g = lib.grid_init(32, 32, 32)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    v, u0, u1 = ctypes.c_void_p(1 << 40), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 36)
    out = ctypes.c_void_p(1 << 38)

    def call(**kw):
        a = dict(g=g, dt=1e-3, u0=u0, u1=u1, out=out)
        a.update(kw)
        return L.sp_energy_noalloc(ctypes.byref(a["g"]), ctypes.byref(c), a["dt"], 10.0, ctypes.byref(g),
                                   v, a["u0"], a["u1"], a["out"], None)

    assert call(dt=0.0) == lib.SP_EINVAL
    assert call(u0=None) == lib.SP_EINVAL
    assert call(out=ctypes.c_void_p((1 << 38) + 4)) == lib.SP_EINVAL and "misaligned" in lib.last_error()
    assert call(g=lib.grid_init(32, 32, 32, dtype=lib.SP_F16)) in (lib.SP_EINVAL, lib.SP_EUNSUPPORTED)


def test_adjoint_only_tile_is_rejected_for_other_sweeps(monkeypatch):
    # 128x16x1 is compiled for the fused adjoint sweep only
    monkeypatch.setenv("SP_TILE", "128x16x1")
    L = lib.load()
    g = lib.grid_init(16, 16, 16)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    out = ctypes.c_int()
    rc = L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), 1, ctypes.c_void_p(1 << 30),
                            ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    assert rc == lib.SP_EINVAL and "not compiled" in lib.last_error()


def test_huge_planes_with_16bit_storage_are_refused():
    # 32768 x 32768 planes (2^30 elements with the frame) are beyond the
    # 32-bit plane offsets of the 16-bit leapfrog: refused before launch
    L = lib.load()
    g = lib.grid_init(32768, 32768, 1, dtype=lib.SP_F16)
    gv = lib.grid_init(32768, 32768, 1)
    c = lib.coeffs({"center": -1, "ax": [0] * 4, "ay": [0] * 4, "az": [0] * 4})
    st = lib.sp_wave_state(1 << 40, 1 << 44, 1 << 46, 0)
    rc = L.sp_wave_step(ctypes.byref(g), ctypes.byref(c), 1e-3, 10.0, ctypes.byref(gv), ctypes.c_void_p(1 << 42),
                        ctypes.byref(st), 1, None, None, None)
    assert rc == lib.SP_EUNSUPPORTED and "2^30" in lib.last_error()
    assert st.step == 0
