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
    MODE_GRAD = 2,    // G += w * (L u + dx^2 f e_src)      (FP64 G; w in `prev`)
    MODE_ENERGY = 3,  // partial[block] = sum (w - u)^2 / m - w L u   (FP64; w in `prev`)
    MODE_PML = 4,     // absorbing-layer leapfrog (damping eta, auxiliary psi; FP32)
    MODE_ADJ = 5,     // out = 2u - prev + m L u and G += out * (L u2 + dx^2 f e_src)  (FP64 G)
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

// Per-slab scale records of FP16/BF16 fields (SP_SLAB planes per slab).
// Slot layout in the caller's meta block: 4 slots, each holding
// float scale[nslab] followed by uint32 amax[nslab] (IEEE bits of a
// non-negative float, so integer max is float max).  Field u^k uses slot
// k mod 4.
struct SlabMeta {
    const float *s_u;        // scales of u^n
    const float *s_prev;     // scales of u^{n-1}
    const uint32_t *a_u;     // maxima of |u^n|
    const uint32_t *a_prev;  // maxima of |u^{n-1}|
    float *s_out;            // scales of u^{n+1} (written here)
    uint32_t *a_out;         // maxima of |u^{n+1}| (atomic max; zero on entry)
    float *s_clear;          // slot of u^{n+2}: cleared by block 0
    uint32_t *a_clear;
    int nslab;
};

// Arguments of one sweep of the streaming star kernel.  Field pointers are
// at the interior origin and typed by the storage type of the launch.
struct SweepArgs {
    const void *u;       // input field
    const float *u2;     // MODE_ADJ: the forward field whose Laplacian weights the gradient
    const void *prev;    // u^{n-1} (MODE_WAVE; may alias out)
    const float *v;      // velocity at its origin (MODE_WAVE)
    void *out;           // output field
    int nx, ny, nz;
    int64_t sy, sz;      // row / plane strides of u, prev, out (elements)
    int64_t vsy, vsz;    // row / plane strides of v
    float m_scale;       // (dt / dx)^2, so m = v^2 m_scale
    StarCoef c;
    SrcList src;
    SlabMeta meta;       // FP16/BF16 storage only
    double *gacc;        // MODE_GRAD: FP64 field on the FP32 layout; MODE_ENERGY: partial sums
    float dx2;           // MODE_GRAD: dx^2 (source term)
    const float *eta;    // MODE_PML: damping (1/s) on v's layout, frame included
    float *psi;          // MODE_PML: auxiliary field on u's layout, updated in place
    float dt, alpha_dt;  // MODE_PML: time step and frequency shift times dt
    uint32_t *nonfinite; // batched MODE_WAVE: set non-zero when an output value is not finite
    int tiles_x, tiles_y, zchunk, nzc;
};

// Largest z-chunk of one block for FP16/BF16 storage (its slab scales are
// staged in LDS).
constexpr int MAX_ZCHUNK_SCALED = 1024;

// Launch configuration chosen by the host for a grid shape.
struct TileCfg {
    int tx, ty;          // tile extent in x (points) and y (rows)
    int ry;              // adjacent rows per thread
    int zchunk;          // planes per block
};

// Launch configuration of the k_star25 sweeps for a grid, storage type and mode.
TileCfg choose_tiles(int nx, int ny, int nz, int dtype, int mode);
// Planes per block for `tiles` xy tiles when per_round blocks fill the GPU.
int occupancy_zchunk(int64_t tiles, int nz, int per_round);

// Up to MAX_BOXES boxes of one grid swept by one launch of 512-thread
// blocks: box k takes blocks [first[k], first[k+1]), on 256x8x1 tiles if
// wide[k], else on 32x64x1 tiles (kernel arguments: 6 x 480 B fits the
// 4 KB limit).
constexpr int MAX_BOXES = 6;
struct BoxSet {
    SweepArgs a[MAX_BOXES];
    int first[MAX_BOXES + 1];
    int wide[MAX_BOXES];
    int n;
};
hipError_t launch_sweep_boxes(int mode, const BoxSet &bs, hipStream_t s);
// Configurations the batched (multi-grid) sweep is compiled for.
bool batch_supported(const TileCfg &t);
bool tile_supported(const TileCfg &t, int mode);
hipError_t launch_sweep(int mode, int dtype, const TileCfg &t, const SweepArgs &a, hipStream_t s);
// Record u at receiver points (decoding with per-slab scales if `scale`).
hipError_t launch_record(int dtype, const void *u, const float *scale, int64_t sy, int64_t sz,
                         int nx, int ny, int nz, const int32_t *xyz, int n, float *traces,
                         hipStream_t s);

// field[x_r] += scale * v[x_r]^2 * amp[r] for r < n (atomic: duplicates add).
hipError_t launch_inject(float *field, int64_t sy, int64_t sz, const float *v, int64_t vsy,
                         int64_t vsz, int nx, int ny, int nz, const int32_t *xyz, int n,
                         const float *amp, float scale, hipStream_t s);
// The receiver term of one fused adjoint step (after the MODE_ADJ sweep a):
// for r < n, w = scale * v[x_r]^2 * amp[r]; out[x_r] += w and
// G[x_r] += w * (L u2 + dx^2 f e_src)[x_r]  (atomic: duplicates add).
hipError_t launch_inject_grad(const SweepArgs &a, const int32_t *xyz, int n, const float *amp,
                              float scale, hipStream_t s);
// out = 2 G / v on the interior (FP32 grid layout for out, v; FP64 G).
hipError_t launch_grad_finish(const double *G, const float *v, float *out, int64_t sy, int64_t sz,
                              int nx, int ny, int nz, hipStream_t s);
// *out = sum of n partials, in index order.
hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t s);

// Error reporting shared by the C-ABI translation units (thread-local message).
int fail(int code, const char *fmt, ...);
int ok();
// Validate the arguments common to the leapfrog calls and fill a, t.
int prep_wave(const char *who, const sp_grid *g, const sp_coeffs *c, double dt, double dx,
              const sp_grid *gv, const float *v, const sp_sources *src, const sp_receivers *rec,
              SweepArgs *a, TileCfg *t);
// Per-step pointers (fields given by allocation base), slab records and source row.
void step_args(SweepArgs &a, const sp_grid *g, void *cur, void *prev, void *out, float *meta,
               int64_t n, const float *amp, int64_t amp_stride);

// Receiver recording of one grid in a batched launch (newest field).
struct RecArgs {
    const void *field;       // at interior origin, storage type of the launch
    const float *scale;      // per-slab scales of the field (FP16/BF16) or null
    const int32_t *xyz;      // device [n][3]
    float *traces;           // this step's row
    int64_t sy, sz;
    int nx, ny, nz, n;
};

// Batched sweep: nblk blocks; block b computes tile table[b].y of the grid
// whose arguments are args[table[b].x] (device arrays).
hipError_t launch_sweep_batch(int mode, int dtype, const TileCfg &t, const SweepArgs *args,
                              const int2 *table, int nblk, hipStream_t s);
// Batched receivers: thread r records receiver rmap[r].y of grid rmap[r].x.
hipError_t launch_record_batch(int dtype, const RecArgs *recs, const int2 *rmap, int total,
                               hipStream_t s);
// Interior-dense FP32 [nz][ny][nx] <-> field at interior origin.
hipError_t launch_pack(const float *dense, float *field, int64_t sy, int64_t sz, int nx, int ny,
                       int nz, hipStream_t s);
hipError_t launch_unpack(int dtype, const void *field, const float *scale, float *dense,
                         int64_t sy, int64_t sz, int nx, int ny, int nz, hipStream_t s);

// Two fused leapfrog steps (FP32): u^{n+1} into out1, u^{n+2} into out2.
// Pointers at the interior origin; out1 and out2 distinct from u and prev.
struct Tb2Args {
    const float *u;      // u^n
    const float *prev;   // u^{n-1}
    const float *v;
    float *out1, *out2;
    int nx, ny, nz;
    int64_t sy, sz;      // strides of u, prev, out1, out2
    int64_t vsy, vsz;
    float m_scale;       // (dt / dx)^2
    StarCoef c;
    SrcList src;         // amp: amplitudes of step n
    const float *amp1;   // amplitudes of step n+1
    int tiles_x, tiles_y, zchunk, nzc;
};
// tx x ty = region (inner tile plus a 4-point ring), zchunk planes per block.
TileCfg choose_tiles_tb2(int nx, int ny, int nz);
int tb2_zchunk(const TileCfg &t, int nx, int ny, int nz);
bool tb2_supported(const TileCfg &t);
hipError_t launch_tb2(const TileCfg &t, const Tb2Args &a, hipStream_t s);

// Stencil suite (star/box, radius 1..4, 2D/3D, arbitrary weights; FP32).
// u and out point at interior (0, 0, 0); a 2D kernel on a grid of several
// planes treats each interior plane as its own 2D grid.
struct SuiteArgs {
    const float *u;
    float *out;
    int nx, ny, nz;
    int64_t sy, sz;
};
// w: dense (2r+1)^ndim FP32 weights, x offset fastest, zero off a star's
// axes.  shape 0 = star, 1 = box.
hipError_t launch_suite(int shape, int ndim, int radius, const float *w, const SuiteArgs &a,
                        hipStream_t s);

// eta = eta_max * sum over axes (d_a / width)^2 on every cell of the padded
// extent, d_a = max(0, width - 1 - a, a - (n_a - width)).
hipError_t launch_pml_profile(float *eta, int64_t sy, int64_t sz, int nx, int ny, int nz, int width,
                              float eta_max, hipStream_t s);

}  // namespace sp
