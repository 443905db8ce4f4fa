"""GPU parity of sp_apply (the stencil suite: star/box, radius 1..4, 2D and
3D) against the FP64 oracle, through the C ABI.

Bars:
 * integer weights and integer fields: bit-exact (every partial sum of every
   kernel stays below 2^24, so FP32 is exact in any order);
 * FP32 weights: at every point |gpu - oracle| <= (n + 2) 2^-24 sum_k |w_k
   u(p+k)| (n taps: FP32 rounding of each weight and of each of the n
   fused multiply-adds of a positive-bound sum), the bound evaluated by the
   oracle on |w| and |u|;
 * the accuracy study's report (max abs error and RMSD) is printed.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import errors

pytestmark = pytest.mark.gpu

NAMES = sorted(synth.SUITE)


def _run(u_np, w, kind, ndim, sweeps=1, flat=False, frame=None):
    """u_np: interior (nz, ny, nx); flat: use a 2D grid (nz must be 1)."""
    from paper_2309_04671_amd import fields, lib
    nz, ny, nx = u_np.shape
    g = lib.grid_init_2d(nx, ny) if flat else lib.grid_init(nx, ny, nz)
    u, v = fields.Field(g), fields.Field(g)
    if frame is not None:
        u.set_padded(frame)
    u.set_interior(u_np)
    where = lib.sp_apply(g, kind, w, u.ptr, v.ptr, sweeps)
    torch.cuda.synchronize()
    return (v if where == 1 else u).get_interior().astype(np.float64), where


def _bound(u, w, ndim, frame=None):
    n = np.count_nonzero(w)
    fa = None if frame is None else np.abs(frame)
    return (n + 2) * 2.0 ** -24 * oracle.stencil_general(np.abs(u), np.abs(w), ndim, frame=fa)


def _shape(ndim):
    # two x strips with a ragged tail, several y tiles / chunks, several z chunks
    return (29, 37, 300) if ndim == 3 else (3, 70, 263)


@pytest.mark.parametrize("name", NAMES)
def test_integer_weights_bit_exact(gpu_lib, name):
    kind, ndim, r = synth.SUITE[name]
    rng = np.random.default_rng(len(name))
    w = np.where(synth.stencil_support(kind, ndim, r),
                 rng.integers(-3, 4, (2 * r + 1,) * ndim), 0).astype(np.float64)
    u = rng.integers(-100, 101, _shape(ndim)).astype(np.float64)
    got, where = _run(u, w, kind, ndim)
    assert where == 1
    ref = oracle.stencil_general(u, w, ndim)
    assert np.array_equal(got, ref), name


@pytest.mark.parametrize("name", NAMES)
def test_fp32_within_rounding_bound(gpu_lib, name):
    kind, ndim, r = synth.SUITE[name]
    w = synth.suite_weights(name, seed=11, signed=True)
    u = synth.suite_field(_shape(ndim), seed=12)
    got, _ = _run(u, w, kind, ndim)
    ref = oracle.stencil_general(u, w, ndim)
    err = np.abs(got - ref)
    assert np.all(err <= _bound(u, w, ndim)), (name, err.max())
    e = errors(got, ref)
    print("%-10s max abs %.3e  RMSD %.3e  rel-L2 %.3e" % (name, e["max_abs"], e["rmsd"], e["rel_l2"]))


@pytest.mark.parametrize("name", ["star2d1r", "box2d4r", "star3d3r", "box3d2r"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (9, 17, 257), (40, 5, 64), (4, 129, 33)])
def test_ragged_shapes_with_nonzero_frame(gpu_lib, name, shape):
    kind, ndim, r = synth.SUITE[name]
    if ndim == 2:
        shape = shape[1:]
        shape = (1,) + shape
    w = synth.suite_weights(name, seed=3, signed=True)
    u = synth.uniform_field(shape, 5)
    hz = 4 if ndim == 3 else 0
    nz, ny, nx = shape
    frame = synth.uniform_field((nz + 2 * hz, ny + 8, nx + 8), 6)
    frame_full = frame
    if ndim == 2:
        # a 2D kernel on a 3D grid: the grid also has z halo planes the
        # kernel must not read
        frame_full = np.zeros((nz + 8, ny + 8, nx + 8))
        frame_full[4:-4] = frame
    got, _ = _run(u, w, kind, ndim, frame=frame_full)
    ref = oracle.stencil_general(u, w, ndim, frame=frame)
    assert np.all(np.abs(got - ref) <= _bound(u, w, ndim, frame=frame)), (name, shape)


@pytest.mark.parametrize("name", ["star2d4r", "box2d2r", "j2d9pt-gol"])
def test_2d_grid_matches_2d_kernel_on_a_plane(gpu_lib, name):
    kind, ndim, r = synth.SUITE[name]
    w = synth.suite_weights(name, seed=4, signed=True)
    u = synth.uniform_field((1, 301, 517), 8)
    got, _ = _run(u, w, kind, ndim, flat=True)
    ref = oracle.stencil_general(u, w, ndim)
    assert np.all(np.abs(got - ref) <= _bound(u, w, ndim))
    got3, _ = _run(u, w, kind, ndim, flat=False)
    assert np.array_equal(got, got3)


def test_listing_star2d4r_ping_pong(gpu_lib):
    # The paper's example kernel on its 1000 x 1000 grid, several sweeps
    # ping-ponging u and v; result location alternates.
    w = synth.listing_star2d4r_weights()
    u = synth.uniform_field((1, 1000, 1000), 21)
    for sweeps in (0, 1, 2, 5):
        got, where = _run(u, w, "star", 2, sweeps=sweeps, flat=True)
        assert where == sweeps % 2
        ref = oracle.stencil_general(u, w, 2, sweeps=sweeps) if sweeps else u
        e = errors(got, ref)
        assert e["rel_l2"] <= 1e-6, (sweeps, e)


def test_eq3_star_matches_the_25_point_path(gpu_lib):
    # star3d4r with the symmetric eighth-order weights computes the same
    # operator as sp_stencil_apply (different kernels, both within FP32
    # rounding of the oracle)
    from paper_2309_04671_amd import fields, lib
    co = synth.star25_coeffs()
    w = np.zeros((9, 9, 9))
    w[4, 4, 4] = co["center"]
    for m in range(1, 5):
        w[4, 4, 4 - m] = w[4, 4, 4 + m] = co["ax"][m - 1]
        w[4, 4 - m, 4] = w[4, 4 + m, 4] = co["ay"][m - 1]
        w[4 - m, 4, 4] = w[4 + m, 4, 4] = co["az"][m - 1]
    u = synth.uniform_field((48, 40, 260), 2)
    got, _ = _run(u, w, "star", 3)
    g = lib.grid_init(260, 40, 48)
    a, b = fields.Field(g).set_interior(u), fields.Field(g)
    lib.sp_stencil_apply(g, lib.coeffs(co), 1, a.ptr, b.ptr)
    torch.cuda.synchronize()
    ref = oracle.stencil_general(u, w, 3)
    assert errors(got, ref)["rel_l2"] <= 1e-6
    assert errors(b.get_interior(), ref)["rel_l2"] <= 1e-6


@pytest.mark.parametrize("name,shape", [("star3d4r", (512, 512, 512)), ("box3d1r", (256, 512, 512)),
                                        ("star2d4r", (1, 8192, 8192)), ("box2d2r", (1, 4096, 4096))])
def test_full_size_sampled(gpu_lib, name, shape):
    # Bench-size grids: sampled points against oracle windows.
    from paper_2309_04671_amd import fields, lib
    kind, ndim, r = synth.SUITE[name]
    w = synth.suite_weights(name, seed=1)
    nz, ny, nx = shape
    u_t = torch.rand(shape, generator=torch.Generator().manual_seed(3), dtype=torch.float32)
    flat = ndim == 2
    g = lib.grid_init_2d(nx, ny) if flat else lib.grid_init(nx, ny, nz)
    a, b = fields.Field(g), fields.Field(g)
    a.set_interior(u_t)
    lib.sp_apply(g, kind, w, a.ptr, b.ptr, 1)
    torch.cuda.synchronize()
    out = b.interior()
    u = u_t.numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    pts = [(rng.integers(0, nz), rng.integers(0, ny), rng.integers(0, nx)) for _ in range(300)]
    pts += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, 0, nx - 1), (nz - 1, ny // 2, 0)]
    for z, y, x in pts:
        up = np.zeros(((2 * r + 1) if ndim == 3 else 1, 2 * r + 1, 2 * r + 1))
        zs = range(z - r, z + r + 1) if ndim == 3 else [z]
        for iz, zz in enumerate(zs):
            for iy, yy in enumerate(range(y - r, y + r + 1)):
                for ix, xx in enumerate(range(x - r, x + r + 1)):
                    if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                        up[iz, iy, ix] = u[zz, yy, xx]
        win = up if ndim == 3 else up[0]
        ref = oracle.stencil_general(win, w, ndim)
        c = ref[r, r, r] if ndim == 3 else ref[r, r]
        bnd = (np.count_nonzero(w) + 2) * 2.0 ** -24 * np.sum(np.abs(w) * np.abs(win))
        assert abs(float(out[z, y, x]) - c) <= bnd, (z, y, x)
