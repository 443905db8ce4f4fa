// Internal declarations shared by the kernel translation unit and the C-ABI
// host code.  Not part of the public interface (include/stencil.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stencil.h"

namespace sp {

enum Mode : int {
    MODE_APPLY = 0,   // out = L u
    MODE_WAVE = 1,    // out = 2u - prev + m L u (+ sources)
};

// Stencil weights rounded once to FP32 (paper Eq. 3).
struct StarCoef {
    float c0;
    float cx[4], cy[4], cz[4];
};

// Point sources for one step: coordinates by value, amplitude row on device.
struct SrcList {
    int n;
    int x[SP_MAX_SOURCES], y[SP_MAX_SOURCES], z[SP_MAX_SOURCES];
    const float *amp;   // amplitudes of this step, amp[s]
    float dt2;          // dt^2 (injection = dt^2 v^2 amp)
};

// Arguments of one sweep of the streaming star kernel (FP32 storage).
struct SweepArgs {
    const float *u;      // input field at interior origin
    const float *prev;   // u^{n-1} at origin (MODE_WAVE; may alias out)
    const float *v;      // velocity at its origin (MODE_WAVE)
    float *out;          // output at origin
    int nx, ny, nz;
    int64_t sy, sz;      // row / plane strides of u, prev, out (elements)
    int64_t vsy, vsz;    // row / plane strides of v
    float m_scale;       // (dt / dx)^2, so m = v^2 m_scale
    StarCoef c;
    SrcList src;
    int tiles_x, tiles_y, zchunk, nzc;
};

// Launch configuration chosen by the host for a grid shape.
struct TileCfg {
    int tx, ty;          // tile extent in x (points) and y (rows)
    int ry;              // adjacent rows per thread
    int zchunk;          // planes per block
};

TileCfg choose_tiles(int nx, int ny, int nz);
hipError_t launch_sweep(int mode, const TileCfg &t, const SweepArgs &a, hipStream_t s);
hipError_t launch_record(const float *u, int64_t sy, int64_t sz, int nx, int ny, int nz,
                         const int32_t *xyz, int n, float *traces, hipStream_t s);

}  // namespace sp
