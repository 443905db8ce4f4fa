"""Client side of the continuous-batching shot queue (sp_queue_* in the C ABI).

The queue's worker thread, admission, arena and batched graph launches are
native; this module only marshals shot descriptions and torch-owned buffers.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lib


class Shot:
    """Device buffers of one request (kept alive until it finishes)."""

    def __init__(self, v, dt, dx, nsteps, coeffs, src, amp, rec=None, dtype=lib.SP_F32,
                 final=True, device="cuda"):
        self.v = torch.as_tensor(v, dtype=torch.float32).to(device).contiguous()
        nz, ny, nx = self.v.shape
        self.shape = (nz, ny, nx)
        self.src = np.asarray(src, np.int32).reshape(-1, 3)
        self.amp = torch.as_tensor(np.asarray(amp, np.float32)).reshape(nsteps, len(self.src)).to(device).contiguous()
        self.rec = np.zeros((0, 3), np.int32) if rec is None else np.asarray(rec, np.int32).reshape(-1, 3)
        self.rec_d = torch.as_tensor(self.rec).to(device).contiguous()
        self.traces = torch.zeros((nsteps, max(len(self.rec), 1)), dtype=torch.float32, device=device)
        self.final = torch.zeros(self.shape, dtype=torch.float32, device=device) if final else None
        d = lib.sp_shot_desc()
        d.nx, d.ny, d.nz = nx, ny, nz
        d.dtype = dtype
        d.nsteps = nsteps
        d.dt, d.dx = float(dt), float(dx)
        d.coeffs = lib.coeffs(coeffs)
        d.v = self.v.data_ptr()
        d.nsrc = len(self.src)
        for k, p in enumerate(self.src):
            for j in range(3):
                d.src_xyz[k][j] = int(p[j])
        d.src_amp = self.amp.data_ptr()
        d.nrec = len(self.rec)
        d.rec_xyz = self.rec_d.data_ptr() if len(self.rec) else None
        d.traces = self.traces.data_ptr() if len(self.rec) else None
        d.final_out = self.final.data_ptr() if final else None
        self.desc = d
        self.ticket = None
        self.points = nx * ny * nz * nsteps

    def bytes(self) -> int:
        return int(lib.load().sp_shot_bytes(ctypes.byref(self.desc)))


class ServeClient:
    """Owns a queue over a torch-allocated arena."""

    def __init__(self, arena_bytes, budget_bytes=0, max_slots=64, chunk_steps=16, flags=0,
                 device="cuda", arena_ptr=None):
        L = lib.load()
        self.arena = None
        if arena_ptr is None:
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
            arena_ptr = self.arena.data_ptr()
        cfg = lib.sp_queue_cfg()
        cfg.arena = arena_ptr
        cfg.arena_bytes = int(arena_bytes)
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.chunk_steps = int(chunk_steps)
        cfg.flags = int(flags)
        cfg.stream = None if flags & lib.SP_QUEUE_FAKE else torch.cuda.current_stream().cuda_stream
        self.q = ctypes.c_void_p()
        lib.check(L.sp_queue_create(ctypes.byref(cfg), ctypes.byref(self.q)))
        self.shots = {}

    def submit(self, shot: Shot) -> int:
        t = ctypes.c_uint64()
        lib.check(lib.load().sp_submit(self.q, ctypes.byref(shot.desc), ctypes.byref(t)))
        shot.ticket = t.value
        # the queue holds raw pointers into the shot's buffers until it finishes
        self.shots[t.value] = shot
        return t.value

    def poll(self, ticket):
        st = lib.sp_shot_status()
        rc = lib.load().sp_poll(self.q, ctypes.c_uint64(ticket), ctypes.byref(st))
        if rc not in (lib.SP_OK, lib.SP_EPENDING):
            lib.check(rc)
        done = rc == lib.SP_OK
        if done:
            self.shots.pop(ticket, None)    # finished: the queue no longer uses its buffers
        return done, st

    def drain(self):
        lib.check(lib.load().sp_queue_drain(self.q))

    def close(self):
        if self.q:
            lib.check(lib.load().sp_queue_destroy(self.q))
            self.q = ctypes.c_void_p()
        self.shots.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
