"""Device fields laid out by sp_grid_init, held in torch allocations.

PyTorch provides the device memory and the strided views used to move data
in and out; all stencil arithmetic runs in libstencil's kernels.
"""

from __future__ import annotations

import numpy as np
import torch

from . import lib

_TORCH_DTYPE = {lib.SP_F32: torch.float32, lib.SP_F16: torch.float16, lib.SP_BF16: torch.bfloat16}


class Field:
    """One halo-padded field on a grid.  ``buf`` owns grid.bytes bytes."""

    def __init__(self, grid: lib.sp_grid, device="cuda", buf: torch.Tensor | None = None):
        self.grid = grid
        self.tdtype = _TORCH_DTYPE[grid.dtype]
        if buf is None:
            buf = torch.zeros(int(grid.bytes), dtype=torch.uint8, device=device)
        assert buf.numel() >= grid.bytes and buf.dtype == torch.uint8
        self.buf = buf

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    @property
    def hz(self) -> int:
        """z frame width: 4, or 0 for a 2D grid (one plane, no z halo)."""
        return 0 if self.grid.planes == 1 else lib.SP_HALO

    def padded(self) -> torch.Tensor:
        """View of shape (nz+8, ny+8, nx+8) over halo and interior
        ((1, ny+8, nx+8) for a 2D grid)."""
        g = self.grid
        h, hz = lib.SP_HALO, self.hz
        flat = self.buf.view(self.tdtype)
        sy, sz = g.pitch_x, g.pitch_x * g.pitch_y
        off = g.origin - hz * sz - h * sy - h
        return torch.as_strided(flat, (g.nz + 2 * hz, g.ny + 2 * h, g.nx + 2 * h), (sz, sy, 1), off)

    def interior(self) -> torch.Tensor:
        h, hz = lib.SP_HALO, self.hz
        return self.padded()[hz:hz + self.grid.nz, h:-h, h:-h]

    def _as_tensor(self, a) -> torch.Tensor:
        if not isinstance(a, torch.Tensor):
            a = torch.as_tensor(np.ascontiguousarray(a))
        return a.to(self.buf.device, self.tdtype)

    def set_interior(self, a) -> "Field":
        self.interior().copy_(self._as_tensor(a))
        return self

    def set_padded(self, a) -> "Field":
        self.padded().copy_(self._as_tensor(a))
        return self

    def get_interior(self) -> np.ndarray:
        return self.interior().float().cpu().numpy() if self.tdtype != torch.float32 \
            else self.interior().cpu().numpy()

    def get_padded(self) -> np.ndarray:
        return self.padded().float().cpu().numpy()


def field(nx, ny, nz, dtype=lib.SP_F32, device="cuda") -> Field:
    return Field(lib.grid_init(nx, ny, nz, dtype), device)


def nslab(nz: int) -> int:
    return (nz + lib.SP_SLAB - 1) // lib.SP_SLAB


class WaveState:
    """Two wavefields (u^{n-1}, u^n), their FP16/BF16 slab records, and the
    sp_wave_state that the library advances.

    The meta block is 4 slots of [scale[nslab] float32, amax[nslab] float32
    bits]; field u^k uses slot k mod 4 (see include/stencil.h).
    """

    def __init__(self, grid: lib.sp_grid, device="cuda", spares: bool = False):
        self.grid = grid
        self.a = Field(grid, device)
        self.b = Field(grid, device)
        # two more fields for sp_wave_step_fused (two steps per sweep)
        self.extra = [Field(grid, device), Field(grid, device)] if spares else []
        self.spare = [f.ptr for f in self.extra]
        nbytes = int(lib.load().sp_wave_meta_bytes(grid))
        self.meta = torch.zeros(max(nbytes // 4, 1), dtype=torch.float32, device=device)
        self.st = lib.sp_wave_state(self.b.ptr, self.a.ptr,
                                    self.meta.data_ptr() if nbytes else None, 0)

    @property
    def nslab(self) -> int:
        return nslab(self.grid.nz)

    def _by_ptr(self, p) -> Field:
        for f in [self.a, self.b] + self.extra:
            if f.ptr == p:
                return f
        raise ValueError("pointer is not one of this state's fields")

    def cur(self) -> Field:
        return self._by_ptr(self.st.cur)

    def prev(self) -> Field:
        return self._by_ptr(self.st.prev)

    def slot(self, k: int):
        """(scale, amax) float32 views of the records of field u^k."""
        n = self.nslab
        base = (k % 4) * 2 * n
        return self.meta[base:base + n], self.meta[base + n:base + 2 * n]

    def reset(self):
        for f in [self.a, self.b] + self.extra:
            f.buf.zero_()
        self.meta.zero_()
        self.st.cur, self.st.prev, self.st.step = self.b.ptr, self.a.ptr, 0
        self.spare = [f.ptr for f in self.extra]

    def decoded_device(self, which="cur") -> torch.Tensor:
        """Interior of u^n (or u^{n-1}) as FP32 values (nz, ny, nx) on the
        device, decoded with its slab scales by the library (sp_decode)."""
        f = self.cur() if which == "cur" else self.prev()
        k = self.st.step if which == "cur" else self.st.step - 1
        g = self.grid
        out = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=f.buf.device)
        meta = self.meta.data_ptr() if g.dtype != lib.SP_F32 else None
        lib.sp_decode(g, f.ptr, meta, k, out.data_ptr())
        return out

    def decoded(self, which="cur") -> np.ndarray:
        """Interior of u^n (or u^{n-1}) decoded with its slab scales, as FP64."""
        return self.decoded_device(which).cpu().numpy().astype(np.float64)
