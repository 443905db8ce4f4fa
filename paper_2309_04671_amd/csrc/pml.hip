// Absorbing layer ("PML" region of the paper's Sec. 2.2) for gfx950.
//
// Reading of the layer (the paper cites its PML without equations): all
// coordinates are stretched by one position-dependent factor, with a
// frequency shift alpha in the auxiliary equation,
//     (d/dt + eta)^2 u = V^2 (lap u + phi),
//     (d/dt + eta + alpha) phi = -grad eta . grad u,
// centred in time with psi = dx^2 phi held at half steps (a = eta dt,
// b = a + alpha dt, m = (v dt / dx)^2):
//     psi^{n+1/2} = [ (1 - b/2) psi^{n-1/2} - dt G ] / (1 + b/2),
//     G = 1/4 sum over axes (eta(+1) - eta(-1)) (u^n(+1) - u^n(-1)),
//     u^{n+1} = [ (2 - a^2) u^n - (1 - a) u^{n-1}
//                 + m (L u^n + (psi^{n-1/2} + psi^{n+1/2}) / 2) ] / (1 + a).
// The layer kernel thus applies the 25-point star to u and a 7-point star
// (eta and u at +-1 on each axis) for the auxiliary array, as the paper
// describes its PML kernel.  Where eta vanishes with its neighbours the
// update is the plain leapfrog, so the inner box runs the streaming
// leapfrog kernel and only the layer runs this one.
//
// Design: the layer is a thin shell (23 % of a 1024x1024x512 grid at width
// 32), so the kernel is a direct gather.  A lane owns one 16-byte chunk (4
// x points) of one row: its x-neighbours are the adjacent chunks and its
// y/z-neighbours are chunk loads at row/plane strides, mostly L2 hits.  A
// launch covers a list of boxes; lanes outside their box are masked at the
// store, so each point is written by exactly one launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace sp {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v ld4(const float *p) { return *reinterpret_cast<const f4v *>(p); }

// Element k (-4 <= k < 8) of the 12 values l | c | r around a chunk.
__device__ __forceinline__ float pick(const f4v &l, const f4v &c, const f4v &r, int k) {
    return k < 0 ? l[k + 4] : (k < 4 ? c[k] : r[k - 4]);
}

constexpr int PML_THREADS = 256;

struct PmlPlan {
    int ncx[7], rows[7], first[8];   // chunk columns, rows*planes and first block of each box
    int cx0[7];
};

__global__ __launch_bounds__(PML_THREADS) void k_pml(PmlArgs a, PmlPlan p) {
    const int bid = blockIdx.x;
    int k = 0;
    while (k + 1 < a.nbox && bid >= p.first[k + 1]) ++k;
    const PmlBox &bx = a.box[k];
    const int64_t item = (int64_t)(bid - p.first[k]) * PML_THREADS + threadIdx.x;
    const int64_t total = (int64_t)p.ncx[k] * p.rows[k];
    if (item >= total) return;
    const int cx = p.cx0[k] + (int)(item % p.ncx[k]);
    const int r = (int)(item / p.ncx[k]);
    const int nyb = bx.y1 - bx.y0;
    const int y = bx.y0 + r % nyb;
    const int z = bx.z0 + r / nyb;
    const int x = 4 * cx;
    const int64_t off = (int64_t)z * a.sz + (int64_t)y * a.sy + x;
    const float *pu = a.u + off;
    const float *pe = a.eta + off;

    const f4v C = ld4(pu), L = ld4(pu - 4), R = ld4(pu + 4);
    f4v yp[4], ym[4], zp[4], zm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        yp[q] = ld4(pu + (q + 1) * a.sy);
        ym[q] = ld4(pu - (q + 1) * a.sy);
        zp[q] = ld4(pu + (q + 1) * a.sz);
        zm[q] = ld4(pu - (q + 1) * a.sz);
    }
    const f4v EC = ld4(pe), EL = ld4(pe - 4), ER = ld4(pe + 4);
    const f4v Eyp = ld4(pe + a.sy), Eym = ld4(pe - a.sy), Ezp = ld4(pe + a.sz), Ezm = ld4(pe - a.sz);
    const f4v P = ld4(a.prev + off), V = ld4(a.v + off), S = ld4(a.psi + off);

    const StarCoef &c = a.c;
    f4v un, pn;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float lap = c.c0 * C[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lap = fmaf(c.cx[q], pick(L, C, R, i + q + 1) + pick(L, C, R, i - q - 1), lap);
            lap = fmaf(c.cy[q], yp[q][i] + ym[q][i], lap);
            lap = fmaf(c.cz[q], zp[q][i] + zm[q][i], lap);
        }
        const float G = 0.25f * ((pick(EL, EC, ER, i + 1) - pick(EL, EC, ER, i - 1)) *
                                     (pick(L, C, R, i + 1) - pick(L, C, R, i - 1)) +
                                 (Eyp[i] - Eym[i]) * (yp[0][i] - ym[0][i]) +
                                 (Ezp[i] - Ezm[i]) * (zp[0][i] - zm[0][i]));
        const float ae = EC[i] * a.dt;
        const float b = ae + a.alpha_dt;
        const float psn = ((1.f - 0.5f * b) * S[i] - a.dt * G) / (1.f + 0.5f * b);
        const float m = V[i] * V[i] * a.m_scale;
        un[i] = ((2.f - ae * ae) * C[i] - (1.f - ae) * P[i] + m * (lap + 0.5f * (S[i] + psn))) /
                (1.f + ae);
        pn[i] = psn;
    }
    for (int s = 0; s < a.src.n; ++s) {
        if (a.src.z[s] == z && a.src.y[s] == y) {
            const int d = a.src.x[s] - x;
            if (d >= 0 && d < 4) un[d] += a.src.dt2 * (V[d] * V[d]) * a.src.amp[s];
        }
    }
    // points of this chunk inside the box
    const int lo = max(bx.x0 - x, 0), hi = min(bx.x1 - x, 4);
    float *po = a.prev + off, *ps = a.psi + off;
    if (lo == 0 && hi == 4) {
        *reinterpret_cast<f4v *>(po) = un;
        *reinterpret_cast<f4v *>(ps) = pn;
    } else {
        for (int i = lo; i < hi; ++i) {
            po[i] = un[i];
            ps[i] = pn[i];
        }
    }
}

__global__ void k_pml_profile(float *eta, int64_t sy, int64_t sz, int nx, int ny, int nz, int w,
                              float eta_max) {
    const int px = nx + 8, py = ny + 8, pz = nz + 8;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)px * py * pz) return;
    const int x = (int)(t % px) - 4;
    const int y = (int)((t / px) % py) - 4;
    const int z = (int)(t / ((int64_t)px * py)) - 4;
    auto depth = [&](int q, int n) { return (float)max(0, max(w - 1 - q, q - (n - w))) / (float)w; };
    const float dx = depth(x, nx), dy = depth(y, ny), dz = depth(z, nz);
    eta[(int64_t)z * sz + (int64_t)y * sy + x] = eta_max * (dz * dz + dy * dy + dx * dx);
}

}  // namespace

hipError_t launch_pml(const PmlArgs &a, hipStream_t s) {
    PmlPlan p = {};
    int nblk = 0;
    for (int k = 0; k < a.nbox; ++k) {
        const PmlBox &b = a.box[k];
        p.cx0[k] = b.x0 >> 2;
        p.ncx[k] = ((b.x1 + 3) >> 2) - p.cx0[k];
        p.rows[k] = (b.y1 - b.y0) * (b.z1 - b.z0);
        p.first[k] = nblk;
        const int64_t items = (int64_t)p.ncx[k] * p.rows[k];
        const int64_t blocks = (items + PML_THREADS - 1) / PML_THREADS;
        if (nblk + blocks > 0x7fffffff) return hipErrorInvalidValue;
        nblk += (int)blocks;
    }
    p.first[a.nbox] = nblk;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pml, dim3(nblk), dim3(PML_THREADS), 0, s, a, p);
    return hipGetLastError();
}

hipError_t launch_pml_profile(float *eta, int64_t sy, int64_t sz, int nx, int ny, int nz, int width,
                              float eta_max, hipStream_t s) {
    const int64_t n = (int64_t)(nx + 8) * (ny + 8) * (nz + 8);
    const int bs = 256;
    hipLaunchKernelGGL(k_pml_profile, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, eta, sy, sz,
                       nx, ny, nz, width, eta_max);
    return hipGetLastError();
}

}  // namespace sp
