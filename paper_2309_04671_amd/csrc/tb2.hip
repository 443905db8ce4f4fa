// Two leapfrog steps per sweep (temporal blocking), FP32 storage.
//
// The same update as the single-step sweep (the 25-point star of the
// paper's Eq. 3 inside the leapfrog of Eq. 2, point sources as in
// Algorithm 1), applied twice in one pass over the grid: the sweep reads
// u^n, u^{n-1} and v once and writes u^{n+1} and u^{n+2}, 20 B per point
// for two steps instead of 32.  The paper lists the number of fused time
// steps as a tuning dimension of its GPU tilings; this is the two-step
// member of that space, designed for gfx950.
//
// Design:
//  * A workgroup owns an inner xy tile of (RX-8) x (RR-8) points and a
//    region of RX x RR points around it (the inner tile plus a 4-point
//    ring).  One thread holds one 4-point chunk of one region row and
//    streams along z over a chunk of planes.
//  * First step: u^{n+1} is computed on the whole region, so that the
//    second step finds every x/y neighbour it needs inside the block.  The
//    ring values duplicate work of the neighbouring tiles; they are never
//    stored.  z-neighbours of u^n come from a 9-plane register queue, x/y
//    neighbours from an LDS copy of plane z (region plus a 4-wide frame).
//  * Second step, 4 planes behind the first: u^{n+2} on the inner tile.
//    z-neighbours of u^{n+1} come from a second 9-plane register queue that
//    the first step fills; x/y neighbours from an LDS copy of u^{n+1} at
//    that plane, written from the same queues; u^n at that plane is the
//    oldest entry of the first queue; v at that plane comes from a 5-plane
//    ring in LDS that each thread writes and reads for its own chunk only.
//  * u^{n+1} is zero outside the interior (the Dirichlet halo), which the
//    first step enforces on the ring; planes outside the grid are zero too.
//    Each block starts 4 planes before its z-chunk (8 for u^n) and ends 4
//    planes after, so chunks are independent.
//  * One LDS barrier per plane: both LDS planes are double-buffered.
//
// Both outputs must be distinct from both inputs: a neighbour's ring reads
// u^n and u^{n-1} at this tile's points while this tile streams.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "kcommon.h"

namespace sp {

namespace {

// Depth of the frame-chunk register queue (planes fetched ahead); measured
// best of 1..5 on MI355X.
constexpr int TB_HD = 3;

template <int RX, int RR>
__global__ void __launch_bounds__((RX / 4) * RR) k_tb2(const Tb2Args a) {
    constexpr int LX = RX / 4;           // lanes per region row
    constexpr int NT = LX * RR;          // one region chunk per thread
    constexpr int TXI = RX - 8, TYI = RR - 8;   // inner (output) tile
    constexpr int HY = 8 * LX;           // frame chunks above and below the region
    constexpr int HC = HY + 2 * RR;      // plus one chunk left and right of each row
    constexpr int HPT = (HC + NT - 1) / NT;
    constexpr int HD = TB_HD;
    __shared__ f4v la[2][RR + 8][LX + 2];   // u^n of plane z: region and frame
    __shared__ f4v lb[2][RR][LX];           // u^{n+1} of plane z-4: region
    __shared__ f4v lv[5][NT];               // v of planes z-4 .. z, own chunk
    __shared__ float s_amp[2][SP_MAX_SOURCES];

    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    const int tix = lin % a.tiles_x;
    const int rest = lin / a.tiles_x;
    const int tiy = rest % a.tiles_y;
    const int zc = rest / a.tiles_y;
    const int x0 = tix * TXI, y0 = tiy * TYI;
    const int zb = zc * a.zchunk;
    const int ze = min(a.nz, zb + a.zchunk);

    const int tid = threadIdx.x;
    const int lx = tid % LX, rr = tid / LX;
    const int gx = x0 - 4 + 4 * lx, gy = y0 - 4 + rr;
    const bool inner = lx >= 1 && lx <= LX - 2 && rr >= 4 && rr < RR - 4;
    const bool in_ok = gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny;   // chunk holds interior points
    bool em[4];                                                          // ... and which of its 4
#pragma unroll
    for (int i = 0; i < 4; ++i) em[i] = in_ok && gx + i < a.nx;

    // Loads are not predicated: each reads a clamped address inside the
    // allocation.  An interior point reads u^n only within the padded extent
    // and u^{n-1}, v only at itself, where clamping changes nothing; a value
    // read at a clamped position reaches only points outside the interior,
    // which the first step sets to zero.  So the plane loop carries no
    // per-lane predicate work (the plane clamps are uniform).
    const int xu = 4 * ((a.nx + 3) / 4), xp = 4 * ((a.nx - 1) / 4);
    const int64_t own = (int64_t)clampi(gy, -4, a.ny + 3) * a.sy + clampi(gx, -4, xu);
    const int64_t pown = (int64_t)clampi(gy, 0, a.ny - 1) * a.sy + clampi(gx, 0, xp);
    const int64_t vown = (int64_t)clampi(gy, 0, a.ny - 1) * a.vsy + clampi(gx, 0, xp);
    const float *u = a.u;
    const int64_t sz = a.sz;

    int hrow[HPT], hcol[HPT];
    bool has_h[HPT];
    int64_t hoff[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int k = tid + j * NT;
        int ar = 0, hx = 0, hc = 0;
        if (k < HY) {
            const int rf = k / LX, cc = k % LX;
            ar = rf < 4 ? rf : RR + rf;
            hx = x0 - 4 + 4 * cc;
            hc = cc + 1;
        } else if (k < HC) {
            const int kk = k - HY, side = kk & 1;
            ar = (kk >> 1) + 4;
            hx = side ? x0 - 4 + RX : x0 - 8;
            hc = side ? LX + 1 : 0;
        }
        hrow[j] = ar;
        hcol[j] = hc;
        has_h[j] = k < HC;
        hoff[j] = (int64_t)clampi(y0 - 8 + ar, -4, a.ny + 3) * a.sy + clampi(hx, -4, xu);
    }

    // sources in this thread's chunk column, as a bit set
    unsigned smask = 0;
    for (int s = 0; s < a.src.n; ++s) {
        const int d = a.src.x[s] - gx;
        if (a.src.y[s] == gy && d >= 0 && d < 4) smask |= 1u << s;
    }

    const f4v zero = {0.f, 0.f, 0.f, 0.f};
    auto ldu = [&](int z, int64_t off) { return ld4(u + (int64_t)clampi(z, -4, a.nz + 3) * sz + off); };
    auto ldp = [&](int z) { return ld4(a.prev + (int64_t)clampi(z, 0, a.nz - 1) * sz + pown); };
    auto ldv = [&](int z) { return ld4(a.v + (int64_t)clampi(z, 0, a.nz - 1) * a.vsz + vown); };

    const int zs = zb - 4, zl = ze + 4;    // planes of the first step
    f4v q1[9], q2[9];
#pragma unroll
    for (int i = 0; i < 8; ++i) q1[i] = ldu(zs - 4 + i, own);
    q1[8] = zero;
    f4v nq = ldu(zs + 4, own);
#pragma unroll
    for (int i = 0; i < 9; ++i) q2[i] = zero;
    f4v hq[HPT][HD];
#pragma unroll
    for (int j = 0; j < HPT; ++j)
#pragma unroll
        for (int k = 0; k < HD; ++k) hq[j][k] = has_h[j] ? ldu(zs + k, hoff[j]) : zero;
    f4v pp = ldp(zs), vv = ldv(zs);

    // both steps' source amplitudes, read once per block
    if (tid < a.src.n) {
        s_amp[0][tid] = a.src.amp[tid];
        s_amp[1][tid] = a.amp1[tid];
    }
    __syncthreads();

    const StarCoef &c = a.c;
    int slot = 0;                         // lv slot of plane z; plane z-4 is slot+1 (mod 5)
    for (int z = zs; z < zl; ++z) {
        const int b = z & 1;
        q1[8] = nq;
        la[b][rr + 4][lx + 1] = q1[4];
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (has_h[j]) la[b][hrow[j]][hcol[j]] = hq[j][0];
        lb[b][rr][lx] = q2[5];            // u^{n+1} of plane z-4
        lv[slot][tid] = vv;

        // next plane's loads (clamped past the last plane, never used there)
        nq = ldu(z + 5, own);
        f4v hn[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) hn[j] = has_h[j] ? ldu(z + HD, hoff[j]) : zero;
        const f4v pp_n = ldp(z + 1), vv_n = ldv(z + 1);

        lds_barrier();

        // first step, plane z, whole region
        f4v r1;
        {
            const f4v ctr = q1[4];
            f4v acc = c.c0 * ctr;
#pragma unroll
            for (int r = 1; r <= 4; ++r) acc += c.cz[r - 1] * (q1[4 + r] + q1[4 - r]);
#pragma unroll
            for (int r = 1; r <= 4; ++r)
                acc += c.cy[r - 1] * (la[b][rr + 4 + r][lx + 1] + la[b][rr + 4 - r][lx + 1]);
            const f4v L = la[b][rr + 4][lx], R = la[b][rr + 4][lx + 2];
            const float w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w, R.x, R.y, R.z, R.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float o = acc[i];
#pragma unroll
                for (int r = 1; r <= 4; ++r) o = fmaf(c.cx[r - 1], w[4 + i + r] + w[4 + i - r], o);
                acc[i] = o;
            }
            const f4v m = vv * vv * a.m_scale;
            r1 = m * acc + (2.f * ctr - pp);
            if (smask) {
                for (int s = 0; s < a.src.n; ++s) {
                    if (((smask >> s) & 1u) && a.src.z[s] == z) {
                        const int d = a.src.x[s] - gx;
                        r1[d] += a.src.dt2 * (vv[d] * vv[d]) * s_amp[0][s];
                    }
                }
            }
            const bool zin = z >= 0 && z < a.nz;
#pragma unroll
            for (int i = 0; i < 4; ++i) r1[i] = (zin && em[i]) ? r1[i] : 0.f;
            if (inner && in_ok && z >= zb && z < ze) st_part(a.out1 + (int64_t)z * sz + pown, r1, a.nx - gx);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) q2[i] = q2[i + 1];
        q2[8] = r1;

        // second step, plane z-4, inner tile
        const int zz = z - 4;
        const int slot4 = slot == 4 ? 0 : slot + 1;
        if (inner && zz >= zb) {
            const f4v ctr = q2[4];
            f4v acc = c.c0 * ctr;
#pragma unroll
            for (int r = 1; r <= 4; ++r) acc += c.cz[r - 1] * (q2[4 + r] + q2[4 - r]);
#pragma unroll
            for (int r = 1; r <= 4; ++r) acc += c.cy[r - 1] * (lb[b][rr + r][lx] + lb[b][rr - r][lx]);
            const f4v L = lb[b][rr][lx - 1], R = lb[b][rr][lx + 1];
            const float w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w, R.x, R.y, R.z, R.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float o = acc[i];
#pragma unroll
                for (int r = 1; r <= 4; ++r) o = fmaf(c.cx[r - 1], w[4 + i + r] + w[4 + i - r], o);
                acc[i] = o;
            }
            const f4v v2 = lv[slot4][tid];
            const f4v m = v2 * v2 * a.m_scale;
            f4v r2 = m * acc + (2.f * ctr - q1[0]);
            if (smask) {
                for (int s = 0; s < a.src.n; ++s) {
                    if (((smask >> s) & 1u) && a.src.z[s] == zz) {
                        const int d = a.src.x[s] - gx;
                        r2[d] += a.src.dt2 * (v2[d] * v2[d]) * s_amp[1][s];
                    }
                }
            }
            if (in_ok) st_part(a.out2 + (int64_t)zz * sz + pown, r2, a.nx - gx);
        }

#pragma unroll
        for (int i = 0; i < 8; ++i) q1[i] = q1[i + 1];
        pp = pp_n;
        vv = vv_n;
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
#pragma unroll
            for (int k = 0; k + 1 < HD; ++k) hq[j][k] = hq[j][k + 1];
            hq[j][HD - 1] = hn[j];
        }
        slot = slot4;
    }
}

}  // namespace

TileCfg choose_tiles_tb2(int nx, int ny, int nz) {
    // 64 x 48 regions (56 x 40 inner tiles), 768 threads at up to 168
    // VGPRs: three waves per SIMD, one block per CU.  The z-split minimises
    // (rounds of 256 blocks) x (planes per block, including the 8 planes of
    // start-up and drain).
    TileCfg t;
    t.tx = 64;
    t.ty = 48;
    t.ry = 1;
    t.zchunk = tb2_zchunk(t, nx, ny, nz);
    return t;
}

int tb2_zchunk(const TileCfg &t, int nx, int ny, int nz) {
    const int64_t tiles = (int64_t)((nx + t.tx - 9) / (t.tx - 8)) * ((ny + t.ty - 9) / (t.ty - 8));
    int best_k = 1;
    int64_t best = -1;
    for (int k = 1; k <= 64; ++k) {
        const int zc = (nz + k - 1) / k;
        if (k > 1 && zc < 16) break;
        const int64_t rounds = (tiles * k + 255) / 256;
        const int64_t cost = rounds * (zc + 8);
        if (best < 0 || cost < best) {
            best = cost;
            best_k = k;
        }
    }
    return (nz + best_k - 1) / best_k;
}

bool tb2_supported(const TileCfg &t) { return t.tx == 64 && (t.ty == 32 || t.ty == 48) && t.ry == 1; }

hipError_t launch_tb2(const TileCfg &t, const Tb2Args &a, hipStream_t s) {
    const dim3 grid(a.tiles_x * a.tiles_y * a.nzc);
    if (t.tx == 64 && t.ty == 32 && t.ry == 1)
        hipLaunchKernelGGL((k_tb2<64, 32>), grid, dim3(512), 0, s, a);
    else if (t.tx == 64 && t.ty == 48 && t.ry == 1)
        hipLaunchKernelGGL((k_tb2<64, 48>), grid, dim3(768), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace sp
