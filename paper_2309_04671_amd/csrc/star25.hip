// Streaming 25-point star stencil for gfx950 (CDNA4, wave64).
//
// One kernel computes one sweep of the star of the paper's Eq. 3 over the
// interior, optionally fused with the leapfrog update of Eq. 2 and the point
// source term of Algorithm 1.
//
// Design (MI355X-first, HBM-bound: ~41 FLOP per 16 B moved):
//  * A workgroup owns an xy tile of TX x TY points and streams along z over a
//    chunk of planes (2.5D blocking).  Each lane owns 4 consecutive x points
//    of one row and moves them with one 16-byte load/store (x-contiguous,
//    128-byte aligned rows, so a wave's row segments fill whole cache lines).
//  * z-neighbours come from a 9-deep register queue per lane (planes z-4 ..
//    z+4); each plane of u is fetched from HBM once per tile.
//  * x/y-neighbours come from an LDS copy of plane z: the tile plus a 4-wide
//    frame of halo chunks (star shape: no corners), double-buffered so one
//    barrier per plane suffices.
//  * All loads for plane z+1 (queue head, halo frame, u^{n-1}, v) are issued
//    before the barrier of plane z, so HBM latency overlaps the compute.
//  * Tiles are mapped to blocks so that consecutive tiles run on the same XCD
//    (workgroups are dealt round-robin over the 8 XCDs, each with its own L2):
//    y-neighbouring tiles then share halo rows through that XCD's L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace sp {

namespace {

__device__ __forceinline__ float4 ld4(const float *p) {
    return *reinterpret_cast<const float4 *>(p);
}

__device__ __forceinline__ void st4(float *p, float4 v) {
    *reinterpret_cast<float4 *>(p) = v;
}

// Barrier that orders LDS traffic only; pending global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ float4 f4(float a) { return make_float4(a, a, a, a); }

__device__ __forceinline__ float4 fma4(float c, float4 a, float4 acc) {
    acc.x = fmaf(c, a.x, acc.x);
    acc.y = fmaf(c, a.y, acc.y);
    acc.z = fmaf(c, a.z, acc.z);
    acc.w = fmaf(c, a.w, acc.w);
    return acc;
}

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// Map a block index to a tile index so that each XCD receives one contiguous
// range of tiles.  Bijective on [0, n) for any n.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    const int xcd = bid & 7, loc = bid >> 3, q = n >> 3, r = n & 7;
    return xcd * q + (xcd < r ? xcd : r) + loc;
}

template <int TX, int TY, int MODE>
__global__ void __launch_bounds__((TX / 4) * TY)
k_star25(SweepArgs a) {
    constexpr int LX = TX / 4;           // lanes per tile row
    constexpr int NT = LX * TY;          // threads per block
    constexpr int LC = LX + 2;           // LDS chunks per row (incl. x halo)
    constexpr int LR = TY + 8;           // LDS rows (incl. y halo)
    constexpr int HY = 8 * LX;           // y-halo chunks per plane
    constexpr int HC = HY + 2 * TY;      // all halo chunks per plane
    __shared__ float4 lds[2][LR][LC];

    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    const int tix = lin % a.tiles_x;
    const int rest = lin / a.tiles_x;
    const int tiy = rest % a.tiles_y;
    const int zc = rest / a.tiles_y;
    const int x0 = tix * TX, y0 = tiy * TY;
    const int zb = zc * a.zchunk;
    const int ze = min(a.nz, zb + a.zchunk);

    const int tid = threadIdx.x;
    const int lx = tid % LX, ly = tid / LX;
    const int x = x0 + 4 * lx, y = y0 + ly;
    const int64_t sz = a.sz;

    // Own column: loaded while inside the padded extent (rows < ny+4,
    // chunks starting before nx+4); stored only for interior points.
    const bool ld_ok = (y < a.ny + 4) && (x < a.nx + 4);
    const bool st_ok = (y < a.ny) && (x < a.nx);
    const int64_t own = (int64_t)y * a.sy + x;

    // Halo chunks owned by this thread (HPT per plane at most).
    constexpr int HPT = (HC + NT - 1) / NT;
    int hrow[HPT], hchk[HPT];
    bool h_ok[HPT];
    int64_t hoff[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int k = tid + j * NT;
        int dy = 0, dx = 0;
        hrow[j] = 0;
        hchk[j] = 0;
        if (k < HY) {
            const int rr = k / LX, cc = k % LX;
            dy = rr < 4 ? rr - 4 : TY + rr - 4;
            dx = 4 * cc;
            hrow[j] = dy + 4;
            hchk[j] = cc + 1;
        } else if (k < HC) {
            const int kk = k - HY, rr = kk >> 1, side = kk & 1;
            dy = rr;
            dx = side ? TX : -4;
            hrow[j] = rr + 4;
            hchk[j] = side ? LX + 1 : 0;
        }
        h_ok[j] = (k < HC) && (y0 + dy < a.ny + 4) && (x0 + dx < a.nx + 4);
        hoff[j] = (int64_t)(y0 + dy) * a.sy + (x0 + dx);
    }

    const float4 zero = f4(0.f);
    const float *u = a.u;

    float4 q[9];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        q[i] = ld_ok ? ld4(u + (int64_t)(zb - 4 + i) * sz + own) : zero;
    float4 nq = ld_ok ? ld4(u + (int64_t)(zb + 4) * sz + own) : zero;
    float4 hv[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) hv[j] = h_ok[j] ? ld4(u + (int64_t)zb * sz + hoff[j]) : zero;

    float4 pp = zero, vv = zero;
    const int64_t vown = (int64_t)y * a.vsy + x;
    if (MODE == MODE_WAVE && st_ok) {
        pp = ld4(a.prev + (int64_t)zb * sz + own);
        vv = ld4(a.v + (int64_t)zb * a.vsz + vown);
    }

    const StarCoef &c = a.c;

    for (int z = zb; z < ze; ++z) {
        q[8] = nq;
        const int b = z & 1;
        lds[b][ly + 4][lx + 1] = q[4];
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (tid + j * NT < HC) lds[b][hrow[j]][hchk[j]] = hv[j];

        float4 pp_n = zero, vv_n = zero;
        if (z + 1 < ze) {
            nq = ld_ok ? ld4(u + (int64_t)(z + 5) * sz + own) : zero;
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                hv[j] = h_ok[j] ? ld4(u + (int64_t)(z + 1) * sz + hoff[j]) : zero;
            if (MODE == MODE_WAVE && st_ok) {
                pp_n = ld4(a.prev + (int64_t)(z + 1) * sz + own);
                vv_n = ld4(a.v + (int64_t)(z + 1) * a.vsz + vown);
            }
        }

        lds_barrier();

        const float4 ctr = q[4];
        float4 acc = make_float4(c.c0 * ctr.x, c.c0 * ctr.y, c.c0 * ctr.z, c.c0 * ctr.w);
#pragma unroll
        for (int r = 1; r <= 4; ++r) acc = fma4(c.cz[r - 1], add4(q[4 + r], q[4 - r]), acc);
#pragma unroll
        for (int r = 1; r <= 4; ++r)
            acc = fma4(c.cy[r - 1], add4(lds[b][ly + 4 + r][lx + 1], lds[b][ly + 4 - r][lx + 1]), acc);
        {
            const float4 L = lds[b][ly + 4][lx], R = lds[b][ly + 4][lx + 2];
            const float w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w,
                                 R.x, R.y, R.z, R.w};
            float o[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 1; r <= 4; ++r)
                    o[i] = fmaf(c.cx[r - 1], w[4 + i + r] + w[4 + i - r], o[i]);
            acc = make_float4(o[0], o[1], o[2], o[3]);
        }

        float4 res;
        if (MODE == MODE_WAVE) {
            const float ms = a.m_scale;
            float4 m = make_float4(vv.x * vv.x * ms, vv.y * vv.y * ms, vv.z * vv.z * ms,
                                   vv.w * vv.w * ms);
            res.x = fmaf(m.x, acc.x, 2.f * ctr.x - pp.x);
            res.y = fmaf(m.y, acc.y, 2.f * ctr.y - pp.y);
            res.z = fmaf(m.z, acc.z, 2.f * ctr.z - pp.z);
            res.w = fmaf(m.w, acc.w, 2.f * ctr.w - pp.w);
            for (int s = 0; s < a.src.n; ++s) {
                if (a.src.z[s] == z && a.src.y[s] == y) {
                    const int d = a.src.x[s] - x;
                    if (d >= 0 && d < 4) {
                        const float vs = d == 0 ? vv.x : d == 1 ? vv.y : d == 2 ? vv.z : vv.w;
                        const float inj = a.src.dt2 * (vs * vs) * a.src.amp[s];
                        if (d == 0) res.x += inj;
                        else if (d == 1) res.y += inj;
                        else if (d == 2) res.z += inj;
                        else res.w += inj;
                    }
                }
            }
        } else {
            res = acc;
        }

        if (st_ok) {
            float *o = a.out + (int64_t)z * sz + own;
            if (x + 4 <= a.nx) {
                st4(o, res);
            } else {
                o[0] = res.x;
                if (x + 1 < a.nx) o[1] = res.y;
                if (x + 2 < a.nx) o[2] = res.z;
            }
        }

#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
        pp = pp_n;
        vv = vv_n;
    }
}

__global__ void k_record(const float *u, int64_t sy, int64_t sz, int nx, int ny, int nz,
                         const int32_t *xyz, int n, float *traces) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
    float val = 0.f;
    if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
        val = u[(int64_t)z * sz + (int64_t)y * sy + x];
    traces[r] = val;
}

template <int TX, int TY>
hipError_t launch_t(int mode, const SweepArgs &a, hipStream_t s) {
    const int nblk = a.tiles_x * a.tiles_y * a.nzc;
    const dim3 grid(nblk), block((TX / 4) * TY);
    if (mode == MODE_WAVE)
        hipLaunchKernelGGL((k_star25<TX, TY, MODE_WAVE>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_star25<TX, TY, MODE_APPLY>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

TileCfg choose_tiles(int nx, int ny, int nz) {
    TileCfg t;
    t.tx = 64;
    t.ty = 16;
    const int tiles = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    // Enough blocks to give every CU work; split z only when the xy tiling
    // alone leaves the GPU underfilled (each split re-reads 8 planes of u).
    const int want = 1024;
    int chunks = (want + tiles - 1) / tiles;
    int zc = (nz + chunks - 1) / chunks;
    if (zc < 32) zc = 32;
    if (zc > nz) zc = nz;
    t.zchunk = zc < 1 ? 1 : zc;
    return t;
}

hipError_t launch_sweep(int mode, const TileCfg &t, const SweepArgs &a, hipStream_t s) {
    if (t.tx == 64 && t.ty == 16) return launch_t<64, 16>(mode, a, s);
    if (t.tx == 64 && t.ty == 8) return launch_t<64, 8>(mode, a, s);
    if (t.tx == 128 && t.ty == 8) return launch_t<128, 8>(mode, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_record(const float *u, int64_t sy, int64_t sz, int nx, int ny, int nz,
                         const int32_t *xyz, int n, float *traces, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_record, dim3((n + bs - 1) / bs), dim3(bs), 0, s, u, sy, sz, nx, ny, nz,
                       xyz, n, traces);
    return hipGetLastError();
}

}  // namespace sp
