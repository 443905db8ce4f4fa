// Stencil-suite kernels for gfx950: star- and box-shaped stencils of radius
// 1..4 in 2D and 3D with an arbitrary weight per offset (the kernel family of
// the paper's accuracy study, Sec. 6; the 25-point star of Eq. 3 is star3d4r
// with symmetric weights).  FP32 storage and arithmetic:
//     out(p) = sum over offsets k in [-r, r]^ndim of w[k] * u(p + k).
//
// 2D (one wave = one 256-point-wide strip of a plane, streaming along y):
//  * a lane owns 4 consecutive x points; rows y-r .. y+r of its 4 columns
//    sit in a register queue, each row fetched from HBM once per strip;
//  * x-neighbours come from the two adjacent 16-byte chunks of the row (L1/L2
//    hits: the neighbouring lanes fetched them), for every queued row of a
//    box and for the centre row of a star;
//  * no LDS and no barriers: the four waves of a block are independent, and
//    loads of row y+r+1 are in flight while row y is computed.
// 3D (a workgroup = a 256 x TY tile streaming along z; the accumulating, or
// semi-stencil, arrangement):
//  * each plane of the tile plus an r-row, 4-column frame (corners included)
//    is fetched once into a double-buffered LDS slot, one barrier per plane;
//  * the plane's contribution to the 2r+1 output planes it touches is added
//    to 2r+1 register accumulators per point (forward and backward partial
//    sums); the oldest accumulator is complete and is stored when the plane
//    r ahead of it has been added.  No queue of input planes is kept.
//  * the fetch of plane z+1 is issued before the barrier of plane z.
// Block indices are mapped so that consecutive tiles run on the same XCD
// (blocks are dealt round-robin over the 8 XCDs, each with its own L2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "kcommon.h"

namespace sp {

namespace {

// Element k (-4 <= k < 8) of the 12 values l | c | r around a lane's chunk.
__device__ __forceinline__ float pick(const f4v &l, const f4v &c, const f4v &r, int k) {
    return k < 0 ? l[k + 4] : (k < 4 ? c[k] : r[k - 4]);
}

// Weight storage passed by value (kernel arguments, read through the scalar
// cache).  Star: per-axis arrays of 2r+1 (x first; the centre weight is in
// the x array, the y and z centre entries are zero).  Box: the dense array.
template <int N> struct Wts {
    float w[N];
};

template <int R, bool BOX, int NDIM> struct WCount {
    static constexpr int D = 2 * R + 1;
    static constexpr int value = BOX ? (NDIM == 3 ? D * D * D : D * D) : NDIM * D;
};

constexpr int WAVES2 = 4;      // waves per 2D block

struct Tile2 {
    int tiles_x, ychunk, groups;   // groups: blocks per strip and plane
};

template <int R, bool BOX>
__global__ __launch_bounds__(64 * WAVES2) void k_suite2(SuiteArgs a, Tile2 t,
                                                        Wts<WCount<R, BOX, 2>::value> W) {
    constexpr int D = 2 * R + 1;
    constexpr int QS = BOX ? D : 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int lin = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = lin % t.tiles_x;
    lin /= t.tiles_x;
    const int grp = lin % t.groups;
    const int z = lin / t.groups;
    const int yb = (grp * WAVES2 + wv) * t.ychunk;
    if (yb >= a.ny) return;                              // whole wave
    const int ye = min(yb + t.ychunk, a.ny);
    const int x = tx * 256 + lane * 4;
    // lanes past the row end load a valid chunk and store nothing
    const int xl = min(x, (a.nx - 1) & ~3);
    const float *src = a.u + (int64_t)z * a.sz + xl;
    float *dst = a.out + (int64_t)z * a.sz + x;
    const int nst = a.nx - x;                           // values this lane stores per row

    f4v qc[D], ql[QS], qr[QS];
    for (int k = 0; k < D; ++k) {
        const float *p = src + (int64_t)(yb - R + k) * a.sy;
        qc[k] = ld4(p);
        if constexpr (BOX) {
            ql[k] = ld4(p - 4);
            qr[k] = ld4(p + 4);
        }
    }
    if constexpr (!BOX) {
        const float *p = src + (int64_t)yb * a.sy;
        ql[0] = ld4(p - 4);
        qr[0] = ld4(p + 4);
    }

    for (int y = yb; y < ye; ++y) {
        // fetch ahead: row y+r+1 (clamped: the last pass re-reads a row)
        const int yn = min(y + R + 1, ye + R - 1);
        const float *pn = src + (int64_t)yn * a.sy;
        const f4v nc = ld4(pn);
        f4v nl, nr;
        if constexpr (BOX) {
            nl = ld4(pn - 4);
            nr = ld4(pn + 4);
        } else {
            const float *pc = src + (int64_t)min(y + 1, ye - 1) * a.sy;
            nl = ld4(pc - 4);
            nr = ld4(pc + 4);
        }

        f4v res;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = 0.f;
            if constexpr (BOX) {
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx)
                        s = fmaf(W.w[(dy + R) * D + dx + R], pick(ql[dy + R], qc[dy + R], qr[dy + R], i + dx), s);
            } else {
#pragma unroll
                for (int dx = -R; dx <= R; ++dx) s = fmaf(W.w[dx + R], pick(ql[0], qc[R], qr[0], i + dx), s);
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
                    if (dy != 0) s = fmaf(W.w[D + dy + R], qc[dy + R][i], s);
            }
            res[i] = s;
        }
        if (nst > 0) st_part(dst + (int64_t)y * a.sy, res, nst);

#pragma unroll
        for (int k = 0; k + 1 < D; ++k) {
            qc[k] = qc[k + 1];
            if constexpr (BOX) {
                ql[k] = ql[k + 1];
                qr[k] = qr[k + 1];
            }
        }
        qc[D - 1] = nc;
        if constexpr (BOX) {
            ql[D - 1] = nl;
            qr[D - 1] = nr;
        } else {
            ql[0] = nl;
            qr[0] = nr;
        }
    }
}

struct Tile3 {
    int tiles_x, tiles_y, zchunk;
};

constexpr int LC = 66;         // 16-byte chunks per LDS row: x0-4 .. x0+259

template <int R, bool BOX, int TY, int RY>
__global__ __launch_bounds__(64 * TY / RY) void k_suite3(SuiteArgs a, Tile3 t,
                                                        Wts<WCount<R, BOX, 3>::value> W) {
    constexpr int NT = 64 * TY / RY, D = 2 * R + 1;
    constexpr int LR = TY + 2 * R;               // LDS rows: tile plus r-row frame
    constexpr int NCH = LR * LC;
    constexpr int K = (NCH + NT - 1) / NT;       // chunks fetched per thread and plane
    __shared__ f4v lds[2][NCH];

    const int tid = threadIdx.x, lane = tid & 63, rg = tid >> 6;
    int lin = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = lin % t.tiles_x;
    lin /= t.tiles_x;
    const int ty = lin % t.tiles_y;
    const int zc = lin / t.tiles_y;
    const int x0 = tx * 256, y0 = ty * TY;
    const int zb = zc * t.zchunk, ze = min(zb + t.zchunk, a.nz);

    // This thread's chunks of every plane: in-plane element offsets (0 for a
    // chunk outside the grid's frame, fetched from a valid address and
    // replaced by zero).
    int32_t off[K];
    bool okc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = tid + k * NT;
        const int row = c / LC, col = c - row * LC;
        const int gy = y0 - R + row, gx = x0 - 4 + 4 * col;
        okc[k] = c < NCH && gy < a.ny + R && gx < a.nx + 4;
        off[k] = okc[k] ? (int32_t)(gy * a.sy + gx) : 0;
    }
    auto fetch = [&](int zp, f4v *d) {
        const float *p = a.u + (int64_t)zp * a.sz;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const f4v v = ld4(p + off[k]);
            d[k] = okc[k] ? v : f4v{0.f, 0.f, 0.f, 0.f};
        }
    };

    f4v acc[RY][D];
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int k = 0; k < D; ++k) acc[j][k] = f4v{0.f, 0.f, 0.f, 0.f};

    const int x = x0 + lane * 4;
    const int nst = a.nx - x;
    f4v cur[K];
    fetch(zb - R, cur);
    for (int zp = zb - R; zp < ze + R; ++zp) {
        f4v nxt[K];
        fetch(min(zp + 1, ze + R - 1), nxt);
        f4v *L = lds[(zp - zb + R) & 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = tid + k * NT;
            if (k + 1 < K || c < NCH) L[c] = cur[k];
        }
        lds_barrier();
        // plane zp adds w[dz] * (its xy part) to output plane zp - dz, held
        // in acc[j][R - dz]
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int lr = rg * RY + j + R;          // LDS row of this output row
            if constexpr (BOX) {
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
                    const f4v *row = L + (lr + dy) * LC + lane;
                    const f4v l = row[0], c = row[1], r = row[2];
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float s = acc[j][R - dz][i];
#pragma unroll
                            for (int dx = -R; dx <= R; ++dx)
                                s = fmaf(W.w[((dz + R) * D + dy + R) * D + dx + R], pick(l, c, r, i + dx), s);
                            acc[j][R - dz][i] = s;
                        }
                }
            } else {
                const f4v *row = L + lr * LC + lane;
                const f4v l = row[0], c = row[1], r = row[2];
                f4v col[D];
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
                    if (dy != 0) col[dy + R] = L[(lr + dy) * LC + lane + 1];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float s = acc[j][R][i];
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) s = fmaf(W.w[dx + R], pick(l, c, r, i + dx), s);
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
                        if (dy != 0) s = fmaf(W.w[D + dy + R], col[dy + R][i], s);
                    acc[j][R][i] = s;
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
                        if (dz != 0) acc[j][R - dz][i] = fmaf(W.w[2 * D + dz + R], c[i], acc[j][R - dz][i]);
                }
            }
        }
        // output plane zp - r has all its contributions
        const int zo = zp - R;
        if (zo >= zb && nst > 0) {
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const int y = y0 + rg * RY + j;
                if (y < a.ny) st_part(a.out + (int64_t)zo * a.sz + (int64_t)y * a.sy + x, acc[j][0], nst);
            }
        }
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int k = 0; k + 1 < D; ++k) acc[j][k] = acc[j][k + 1];
            acc[j][D - 1] = f4v{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int k = 0; k < K; ++k) cur[k] = nxt[k];
    }
}

template <int N> Wts<N> pack_w(int shape, int ndim, int R, const float *w) {
    Wts<N> o = {};
    const int D = 2 * R + 1;
    if (shape == 1) {
        for (int i = 0; i < N; ++i) o.w[i] = w[i];
        return o;
    }
    // star: axis lines through the centre of the dense array
    const int c = ndim == 3 ? (R * D + R) * D + R : R * D + R;
    for (int d = -R; d <= R; ++d) {
        o.w[d + R] = w[c + d];                                  // x (and the centre)
        o.w[D + d + R] = d ? w[c + d * D] : 0.f;                // y
        if (ndim == 3) o.w[2 * D + d + R] = d ? w[c + d * D * D] : 0.f;   // z
    }
    return o;
}

template <int R, bool BOX>
hipError_t run2(const float *w, const SuiteArgs &a, hipStream_t s) {
    Tile2 t;
    t.tiles_x = (a.nx + 255) / 256;
    // rows per wave: about 4096 waves (16 per CU; measured best), at least
    // 8r rows so the 2r re-read rows stay a small share
    const int64_t strips = (int64_t)t.tiles_x * a.nz;
    int64_t yc = (strips * a.ny + 4095) / 4096;
    yc = std::max<int64_t>(yc, 8 * R);
    t.ychunk = (int)std::min<int64_t>(yc, a.ny);
    const int nchunks = (a.ny + t.ychunk - 1) / t.ychunk;
    t.groups = (nchunks + WAVES2 - 1) / WAVES2;
    const int64_t nblk = strips * t.groups;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    constexpr int N = WCount<R, BOX, 2>::value;
    const Wts<N> W = pack_w<N>(BOX ? 1 : 0, 2, R, w);
    hipLaunchKernelGGL((k_suite2<R, BOX>), dim3((unsigned)nblk), dim3(64 * WAVES2), 0, s, a, t, W);
    return hipGetLastError();
}

template <int R, bool BOX>
hipError_t run3(const float *w, const SuiteArgs &a, hipStream_t s) {
    // box kernels of radius >= 3 are long unrolled bodies: one row per thread
    constexpr bool small = BOX && R >= 3;
    constexpr int TY = small ? 8 : 16, RY = small ? 1 : 2;
    Tile3 t;
    t.tiles_x = (a.nx + 255) / 256;
    t.tiles_y = (a.ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)t.tiles_x * t.tiles_y;
    // split z only as far as needed for about one block per CU: longer
    // chunks re-read fewer frame planes (measured best)
    const int64_t want = 256;
    int64_t chunks = (want + tiles - 1) / tiles;
    int64_t zc = (a.nz + chunks - 1) / chunks;
    zc = std::max<int64_t>(zc, std::min<int64_t>(4 * R, a.nz));
    t.zchunk = (int)std::min<int64_t>(zc, a.nz);
    const int64_t nblk = tiles * ((a.nz + t.zchunk - 1) / t.zchunk);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    constexpr int N = WCount<R, BOX, 3>::value;
    const Wts<N> W = pack_w<N>(BOX ? 1 : 0, 3, R, w);
    hipLaunchKernelGGL((k_suite3<R, BOX, TY, RY>), dim3((unsigned)nblk), dim3(64 * TY / RY), 0, s, a, t,
                       W);
    return hipGetLastError();
}

template <bool BOX>
hipError_t dispatch(int ndim, int radius, const float *w, const SuiteArgs &a, hipStream_t s) {
    if (ndim == 2) {
        switch (radius) {
            case 1: return run2<1, BOX>(w, a, s);
            case 2: return run2<2, BOX>(w, a, s);
            case 3: return run2<3, BOX>(w, a, s);
            case 4: return run2<4, BOX>(w, a, s);
        }
    } else {
        switch (radius) {
            case 1: return run3<1, BOX>(w, a, s);
            case 2: return run3<2, BOX>(w, a, s);
            case 3: return run3<3, BOX>(w, a, s);
            case 4: return run3<4, BOX>(w, a, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_suite(int shape, int ndim, int radius, const float *w, const SuiteArgs &a,
                        hipStream_t s) {
    return shape == 1 ? dispatch<true>(ndim, radius, w, a, s) : dispatch<false>(ndim, radius, w, a, s);
}

}  // namespace sp
