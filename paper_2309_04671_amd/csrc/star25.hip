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

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v ld4(const float *p) {
    return *reinterpret_cast<const f4v *>(p);
}

// Streamed-once data: non-temporal hint keeps it from displacing reused lines.
__device__ __forceinline__ f4v ld4_nt(const float *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
}

__device__ __forceinline__ void st4_nt(float *p, f4v v) {
    __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(p));
}

// Barrier that orders LDS traffic only; pending global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Map a block index to a tile index so that each XCD receives one contiguous
// range of tiles.  Bijective on [0, n) for any n.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    const int xcd = bid & 7, loc = bid >> 3, q = n >> 3, r = n & 7;
    return xcd * q + (xcd < r ? xcd : r) + loc;
}

// One sweep over the block's tile and z-chunk.
//   TX: tile width in points (4 per lane), TY: tile height in rows,
//   RY: adjacent rows per thread (register blocking in y).
template <int TX, int TY, int RY, int MODE>
__global__ void __launch_bounds__((TX / 4) * (TY / RY))
k_star25(SweepArgs a) {
    constexpr int LX = TX / 4;           // lanes per tile row
    constexpr int NT = LX * (TY / RY);   // threads per block
    constexpr int LC = LX + 2;           // LDS chunks per row (incl. x halo)
    constexpr int LR = TY + 8;           // LDS rows (incl. y halo)
    constexpr int HY = 8 * LX;           // y-halo chunks per plane
    constexpr int HC = HY + 2 * TY;      // all halo chunks per plane
    constexpr int HPT = (HC + NT - 1) / NT;
    static_assert(TY % RY == 0, "RY must divide TY");
    __shared__ f4v lds[2][LR][LC];

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
    const int x = x0 + 4 * lx;
    const int ybase = y0 + ly * RY;       // first of this thread's RY rows
    const int64_t sz = a.sz;

    // Own columns: loaded while inside the padded extent (rows < ny+4,
    // chunks starting before nx+4); stored only for interior points.
    bool ld_ok[RY], st_ok[RY];
    int64_t own[RY], vown[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int y = ybase + j;
        ld_ok[j] = (y < a.ny + 4) && (x < a.nx + 4);
        st_ok[j] = (y < a.ny) && (x < a.nx);
        own[j] = (int64_t)y * a.sy + x;
        vown[j] = (int64_t)y * a.vsy + x;
    }

    // Halo chunks owned by this thread (HPT per plane at most).
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

    const f4v zero = {0.f, 0.f, 0.f, 0.f};
    const float *u = a.u;

    f4v q[RY][9];
    f4v nq[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            q[j][i] = ld_ok[j] ? ld4(u + (int64_t)(zb - 4 + i) * sz + own[j]) : zero;
        nq[j] = ld_ok[j] ? ld4(u + (int64_t)(zb + 4) * sz + own[j]) : zero;
    }
    f4v hv[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) hv[j] = h_ok[j] ? ld4(u + (int64_t)zb * sz + hoff[j]) : zero;

    f4v pp[RY], vv[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        pp[j] = zero;
        vv[j] = zero;
        if (MODE == MODE_WAVE && st_ok[j]) {
            pp[j] = ld4_nt(a.prev + (int64_t)zb * sz + own[j]);
            vv[j] = ld4_nt(a.v + (int64_t)zb * a.vsz + vown[j]);
        }
    }

    const StarCoef &c = a.c;

    for (int z = zb; z < ze; ++z) {
        const int b = z & 1;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][8] = nq[j];
            lds[b][ly * RY + j + 4][lx + 1] = q[j][4];
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (tid + j * NT < HC) lds[b][hrow[j]][hchk[j]] = hv[j];

        f4v pp_n[RY], vv_n[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            pp_n[j] = zero;
            vv_n[j] = zero;
        }
        if (z + 1 < ze) {
#pragma unroll
            for (int j = 0; j < RY; ++j)
                nq[j] = ld_ok[j] ? ld4(u + (int64_t)(z + 5) * sz + own[j]) : zero;
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                hv[j] = h_ok[j] ? ld4(u + (int64_t)(z + 1) * sz + hoff[j]) : zero;
            if (MODE == MODE_WAVE) {
#pragma unroll
                for (int j = 0; j < RY; ++j)
                    if (st_ok[j]) {
                        pp_n[j] = ld4_nt(a.prev + (int64_t)(z + 1) * sz + own[j]);
                        vv_n[j] = ld4_nt(a.v + (int64_t)(z + 1) * a.vsz + vown[j]);
                    }
            }
        }

        lds_barrier();

        // y-neighbour rows d = -4 .. RY+3 relative to this thread's first row:
        // own rows from registers, the rest from LDS.
        f4v yrow[RY + 8];
#pragma unroll
        for (int d = -4; d < RY + 4; ++d)
            yrow[d + 4] = (d >= 0 && d < RY) ? q[d][4] : lds[b][ly * RY + d + 4][lx + 1];

#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const f4v ctr = q[j][4];
            f4v acc = c.c0 * ctr;
#pragma unroll
            for (int r = 1; r <= 4; ++r) acc += c.cz[r - 1] * (q[j][4 + r] + q[j][4 - r]);
#pragma unroll
            for (int r = 1; r <= 4; ++r) acc += c.cy[r - 1] * (yrow[j + 4 + r] + yrow[j + 4 - r]);
            {
                const f4v L = lds[b][ly * RY + j + 4][lx], R = lds[b][ly * RY + j + 4][lx + 2];
                const float w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w,
                                     R.x, R.y, R.z, R.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float o = acc[i];
#pragma unroll
                    for (int r = 1; r <= 4; ++r) o = fmaf(c.cx[r - 1], w[4 + i + r] + w[4 + i - r], o);
                    acc[i] = o;
                }
            }

            f4v res;
            if (MODE == MODE_WAVE) {
                const f4v m = vv[j] * vv[j] * a.m_scale;
                res = m * acc + (2.f * ctr - pp[j]);
                const int y = ybase + j;
                for (int s = 0; s < a.src.n; ++s) {
                    if (a.src.z[s] == z && a.src.y[s] == y) {
                        const int d = a.src.x[s] - x;
                        if (d >= 0 && d < 4) {
                            const float vs = vv[j][d];
                            res[d] += a.src.dt2 * (vs * vs) * a.src.amp[s];
                        }
                    }
                }
            } else {
                res = acc;
            }

            if (st_ok[j]) {
                float *o = a.out + (int64_t)z * sz + own[j];
                if (x + 4 <= a.nx) {
                    st4_nt(o, res);
                } else {
                    o[0] = res.x;
                    if (x + 1 < a.nx) o[1] = res.y;
                    if (x + 2 < a.nx) o[2] = res.z;
                }
            }
        }

#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int i = 0; i < 8; ++i) q[j][i] = q[j][i + 1];
            pp[j] = pp_n[j];
            vv[j] = vv_n[j];
        }
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

template <int TX, int TY, int RY>
hipError_t launch_t(int mode, const SweepArgs &a, hipStream_t s) {
    const int nblk = a.tiles_x * a.tiles_y * a.nzc;
    const dim3 grid(nblk), block((TX / 4) * (TY / RY));
    if (mode == MODE_WAVE)
        hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_WAVE>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_APPLY>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

TileCfg choose_tiles(int nx, int ny, int nz) {
    // Wide tiles keep the x-halo (one 128-byte line per side per row) and
    // the y-halo rows small relative to the tile; two rows per thread share
    // their y-neighbour reads.
    TileCfg t;
    if (nx >= 192) {
        t.tx = 256; t.ty = 16; t.ry = 2;
    } else if (nx >= 96) {
        t.tx = 128; t.ty = 16; t.ry = 2;
    } else {
        t.tx = 64; t.ty = 16; t.ry = 1;
    }
    const int tiles = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    // At least one block per CU; split z only when the xy tiling alone
    // leaves the GPU underfilled (each split re-reads 8 planes of u).
    const int want = 256;
    const int chunks = (want + tiles - 1) / tiles;
    int zc = (nz + chunks - 1) / chunks;
    if (zc < 32) zc = 32;
    if (zc > nz) zc = nz;
    t.zchunk = zc < 1 ? 1 : zc;
    return t;
}

hipError_t launch_sweep(int mode, const TileCfg &t, const SweepArgs &a, hipStream_t s) {
    if (t.tx == 64 && t.ty == 16 && t.ry == 1) return launch_t<64, 16, 1>(mode, a, s);
    if (t.tx == 128 && t.ty == 16 && t.ry == 2) return launch_t<128, 16, 2>(mode, a, s);
    if (t.tx == 128 && t.ty == 32 && t.ry == 2) return launch_t<128, 32, 2>(mode, a, s);
    if (t.tx == 256 && t.ty == 16 && t.ry == 2) return launch_t<256, 16, 2>(mode, a, s);
    if (t.tx == 256 && t.ty == 16 && t.ry == 4) return launch_t<256, 16, 4>(mode, a, s);
    if (t.tx == 64 && t.ty == 32 && t.ry == 2) return launch_t<64, 32, 2>(mode, a, s);
    if (t.tx == 256 && t.ty == 8 && t.ry == 2) return launch_t<256, 8, 2>(mode, a, s);
    if (t.tx == 256 && t.ty == 8 && t.ry == 1) return launch_t<256, 8, 1>(mode, a, s);
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
