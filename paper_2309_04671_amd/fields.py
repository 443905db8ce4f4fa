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

    def padded(self) -> torch.Tensor:
        """View of shape (nz+8, ny+8, nx+8) over halo and interior."""
        g = self.grid
        h = lib.SP_HALO
        flat = self.buf.view(self.tdtype)
        sy, sz = g.pitch_x, g.pitch_x * g.pitch_y
        off = g.origin - h * sz - h * sy - h
        return torch.as_strided(flat, (g.nz + 2 * h, g.ny + 2 * h, g.nx + 2 * h), (sz, sy, 1), off)

    def interior(self) -> torch.Tensor:
        h = lib.SP_HALO
        return self.padded()[h:-h, h:-h, h:-h]

    def set_interior(self, a) -> "Field":
        t = torch.as_tensor(np.ascontiguousarray(a)).to(self.buf.device, self.tdtype)
        self.interior().copy_(t)
        return self

    def set_padded(self, a) -> "Field":
        t = torch.as_tensor(np.ascontiguousarray(a)).to(self.buf.device, self.tdtype)
        self.padded().copy_(t)
        return self

    def get_interior(self) -> np.ndarray:
        return self.interior().float().cpu().numpy() if self.tdtype != torch.float32 \
            else self.interior().cpu().numpy()

    def get_padded(self) -> np.ndarray:
        return self.padded().float().cpu().numpy()


def field(nx, ny, nz, dtype=lib.SP_F32, device="cuda") -> Field:
    return Field(lib.grid_init(nx, ny, nz, dtype), device)
