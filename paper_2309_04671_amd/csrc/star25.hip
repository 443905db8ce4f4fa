// Streaming 25-point star stencil for gfx950 (CDNA4, wave64).
//
// One kernel computes one sweep of the star of the paper's Eq. 3 over the
// interior, optionally fused with the leapfrog update of Eq. 2 and the point
// source term of Algorithm 1.  Wavefields may be stored in FP32, FP16 or
// BF16; all arithmetic is FP32.
//
// Design (MI355X-first, HBM-bound: ~41 FLOP per 16 B moved in FP32):
//  * A workgroup owns an xy tile of TX x TY points and streams along z over a
//    chunk of planes (2.5D blocking).  Each lane owns 4 consecutive x points
//    of RY adjacent rows and moves each row's 4 values with one vector
//    load/store (x-contiguous, 128-byte aligned rows).
//  * z-neighbours come from a 9-deep register queue per row (planes z-4 ..
//    z+4); each plane of u is fetched from HBM once per tile.
//  * x/y-neighbours come from an LDS copy of plane z: the tile plus a 4-wide
//    frame of halo chunks (star shape: no corners), double-buffered so one
//    barrier per plane suffices; rows owned by the thread itself are taken
//    from registers.
//  * Loads for plane z+1 (queue head, halo frame, u^{n-1}, v) are issued
//    before the barrier of plane z, so HBM latency overlaps the compute.
//    u^{n-1}, v and the output are touched once: non-temporal accesses keep
//    them from displacing u lines that neighbouring tiles re-read from L2.
//  * Tiles are mapped to blocks so that consecutive tiles run on the same XCD
//    (workgroups are dealt round-robin over the 8 XCDs, each with its own L2):
//    neighbouring tiles then share halo lines through that XCD's L2.
//  * FP16/BF16 storage: value = stored * 2^e per 16-plane slab.  Each step
//    chooses the output slab exponent a priori from the maxima of its inputs
//    (so the stored magnitude stays <= 2^15), and reduces the output maxima
//    for the next step with one atomic max per wave and slab.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "internal.h"
#include "kcommon.h"

namespace sp {

namespace {

typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef uint16_t u4v __attribute__((ext_vector_type(4)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));

// Storage type <-> FP32.  dec(raw, s) = stored * s; enc(v, inv) stores
// round-to-nearest-even(v * inv), inv = 1/s (a power of two, so exact).
template <typename T> struct Io;

template <> struct Io<float> {
    typedef f4v raw;
    static constexpr bool scaled = false;
    __device__ static raw ld(const float *p) { return *reinterpret_cast<const f4v *>(p); }
    __device__ static raw ld_nt(const float *p) {
        return __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    }
    __device__ static f4v dec(raw r, float) { return r; }
    __device__ static raw enc(f4v v, float) { return v; }
    __device__ static void st_nt(float *p, raw r) {
        __builtin_nontemporal_store(r, reinterpret_cast<f4v *>(p));
    }
    __device__ static float dec1(float r, float) { return r; }
    __device__ static f4v mag(raw r) { return __builtin_elementwise_abs(r); }
};

template <> struct Io<_Float16> {
    typedef h4v raw;
    static constexpr bool scaled = true;
    __device__ static raw ld(const _Float16 *p) { return *reinterpret_cast<const h4v *>(p); }
    __device__ static raw ld_nt(const _Float16 *p) {
        return __builtin_nontemporal_load(reinterpret_cast<const h4v *>(p));
    }
    __device__ static f4v dec(raw r, float s) { return __builtin_convertvector(r, f4v) * s; }
    __device__ static raw enc(f4v v, float inv) { return __builtin_convertvector(v * inv, h4v); }
    __device__ static void st_nt(_Float16 *p, raw r) {
        __builtin_nontemporal_store(r, reinterpret_cast<h4v *>(p));
    }
    __device__ static float dec1(_Float16 r, float s) { return (float)r * s; }
    __device__ static f4v mag(raw r) {
        return __builtin_elementwise_abs(__builtin_convertvector(r, f4v));
    }
};

template <> struct Io<__bf16> {
    typedef b4v raw;
    static constexpr bool scaled = true;
    __device__ static raw ld(const __bf16 *p) { return *reinterpret_cast<const b4v *>(p); }
    __device__ static raw ld_nt(const __bf16 *p) {
        return __builtin_bit_cast(
            b4v, __builtin_nontemporal_load(reinterpret_cast<const u4v *>(p)));
    }
    __device__ static f4v dec(raw r, float s) { return __builtin_convertvector(r, f4v) * s; }
    __device__ static raw enc(f4v v, float inv) { return __builtin_convertvector(v * inv, b4v); }
    __device__ static void st_nt(__bf16 *p, raw r) {
        __builtin_nontemporal_store(__builtin_bit_cast(u4v, r), reinterpret_cast<u4v *>(p));
    }
    __device__ static float dec1(__bf16 r, float s) { return (float)r * s; }
    __device__ static f4v mag(raw r) {
        return __builtin_elementwise_abs(__builtin_convertvector(r, f4v));
    }
};

// True if any of the first n (1..4) values is an infinity or a NaN.
__device__ __forceinline__ bool nonfinite4(const f4v r, int n) {
    bool bad = !__builtin_isfinite(r.x);
    if (n > 1) bad |= !__builtin_isfinite(r.y);
    if (n > 2) bad |= !__builtin_isfinite(r.z);
    if (n > 3) bad |= !__builtin_isfinite(r.w);
    return bad;
}

// One atomic OR per wave whose lanes saw a non-finite output.
__device__ __forceinline__ void report_nonfinite(uint32_t *flag, bool bad) {
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// Depth of the halo-chunk register queue: the LDS frame of plane z is
// fetched at iteration z-5, the iteration at which the tiles that own those
// rows fetch them as their z-queue head, so the shared lines are read from
// HBM once and found in L2 by the neighbour (fetched one plane ahead, they
// had left a 4 MB XCD L2 again after the owner's four further planes).
constexpr int HQ = 5;

// Slabs one block may touch (z-chunk of at most MAX_ZCHUNK_SCALED planes plus
// the 4-plane margins), for the FP16/BF16 scale tables in LDS.
constexpr int MAX_BLOCK_SLABS = MAX_ZCHUNK_SCALED / SP_SLAB + 2;

// Slab exponent rule: B = 8 max(|u^n| on slabs k-1..k+1, |u^{n-1}| on slab k)
// + sum of |injections| in slab k; scale = 2^(ceil(log2 B) - 15), or 1 when
// B = 0.  Since |u^{n+1}| <= (3 + m sum|c|) max|inputs| < 8 max|inputs| for
// any Courant number inside the stability limit, |stored| <= 2^15.
__device__ float slab_scale(const SweepArgs &a, int k) {
    const SlabMeta &m = a.meta;
    float M = __uint_as_float(m.a_u[k]);
    if (k > 0) M = fmaxf(M, __uint_as_float(m.a_u[k - 1]));
    if (k + 1 < m.nslab) M = fmaxf(M, __uint_as_float(m.a_u[k + 1]));
    M = fmaxf(M, __uint_as_float(m.a_prev[k]));
    float B = 8.f * M;
    for (int s = 0; s < a.src.n; ++s) {
        if ((a.src.z[s] >> 4) == k) {
            const float vs = a.v[(int64_t)a.src.z[s] * a.vsz + (int64_t)a.src.y[s] * a.vsy + a.src.x[s]];
            B += fabsf(a.src.dt2 * (vs * vs) * a.src.amp[s]);
        }
    }
    if (!(B > 0.f)) return 1.f;
    int E;
    const float mant = frexpf(B, &E);          // B = mant * 2^E, mant in [0.5, 1)
    int e = (mant == 0.5f ? E - 1 : E) - 15;   // ceil(log2 B) - 15
    e = clampi(e, -110, 110);
    return ldexpf(1.f, e);
}

// Leapfrog step with FP16 or BF16 storage.  The register queue and the LDS
// plane keep the stored 16-bit values (two per VGPR) instead of decoded FP32
// values, and every tap multiplies a stored value by an FP32 coefficient
// that already carries the slab scale of the tap's plane: scales are powers
// of two, so coefficient x scale is exact and no separate decode multiply is
// needed.  For FP16 a tap is one mixed-precision FMA (half operand, FP32
// coefficient and accumulator); a BF16 value widens to FP32 exactly by a
// 16-bit shift or mask, then one FMA.  Same tiles, halo mapping, slab
// records and rounding as the generic body; about half the queue and LDS
// footprint.
template <int TX, int TY, int RY, typename T, bool NF>
__device__ __forceinline__ void star25_wave_raw16(const SweepArgs &a, const int lin) {
    typedef Io<T> IO;
    typedef typename IO::raw raw;
    constexpr int LX = TX / 4;
    constexpr int NT = LX * (TY / RY);
    constexpr int LC = LX + 2;
    constexpr int LR = TY + 8;
    constexpr int HY = 8 * LX;
    constexpr int HC = HY + 2 * TY;
    constexpr int HPT = (HC + NT - 1) / NT;
    static_assert(TY % RY == 0, "RY must divide TY");
    __shared__ raw lds[2][LR][LC];

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
    const int ybase = y0 + ly * RY;
    const int64_t sz = a.sz;
    const T *u = static_cast<const T *>(a.u);
    const T *uprev = static_cast<const T *>(a.prev);
    T *out = static_cast<T *>(a.out);
    const int nslab = a.meta.nslab;

    if (lin == 0)
        for (int i = tid; i < nslab; i += NT) {
            a.meta.s_clear[i] = 0.f;
            a.meta.a_clear[i] = 0u;
        }

    // Addresses are a uniform plane base (the frame corner (-4, -4) of the
    // plane) plus a 32-bit per-lane byte offset: the loads take the
    // scalar-base form and each offset costs the lane one VGPR.
    const int64_t corner = -4 * a.sy - 4, vcorner = -4 * a.vsy - 4;
    auto plane = [&](const T *f, int zz) {
        return reinterpret_cast<const char *>(f + (int64_t)zz * sz + corner);
    };
    auto vplane = [&](int zz) { return reinterpret_cast<const char *>(a.v + (int64_t)zz * a.vsz + vcorner); };
    auto at = [](const char *base, uint32_t off) { return reinterpret_cast<const T *>(base + off); };
    auto vat = [](const char *base, uint32_t off) { return reinterpret_cast<const float *>(base + off); };

    // Every load takes a position clamped into the range that some lane
    // really needs: the frame for u^n (queue and halo chunks), the interior
    // for u^{n-1} and v.  A lane outside that range loads what an in-range
    // lane loads; its values reach no stored output, so the loads need no
    // per-lane predicate and no zero fill.
    const int xl = min(x, ((a.nx + 3) >> 2) << 2);   // last vector inside the frame
    const int xs = min(x, ((a.nx - 1) >> 2) << 2);   // last vector inside the interior
    bool st_ok[RY];
    uint32_t lown[RY], own[RY], vown[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int y = ybase + j;
        const int yl = min(y, a.ny + 3), ys = min(y, a.ny - 1);
        st_ok[j] = (y < a.ny) && (x < a.nx);
        lown[j] = (uint32_t)(((int64_t)(yl + 4) * a.sy + xl + 4) * (int64_t)sizeof(T));
        own[j] = (uint32_t)(((int64_t)(ys + 4) * a.sy + xs + 4) * (int64_t)sizeof(T));
        vown[j] = (uint32_t)(((int64_t)(ys + 4) * a.vsy + xs + 4) * 4);
    }

    int hrow[HPT], hchk[HPT];
    uint32_t hoff[HPT];
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
        const int yh = min(y0 + dy, a.ny + 3), xh = min(x0 + dx, ((a.nx + 3) >> 2) << 2);
        hoff[j] = (uint32_t)(((int64_t)(yh + 4) * a.sy + xh + 4) * (int64_t)sizeof(T));
    }

    __shared__ float s_in[MAX_BLOCK_SLABS], s_pv[MAX_BLOCK_SLABS], s_o[MAX_BLOCK_SLABS];
    const int ks = clampi((zb - 4) >> 4, 0, nslab - 1);
    {
        const int ke = clampi((ze + 3) >> 4, 0, nslab - 1);
        for (int t = tid; t <= ke - ks; t += NT) {
            const int k = ks + t;
            s_in[t] = a.meta.s_u[k];
            s_pv[t] = a.meta.s_prev[k];
            const float so = slab_scale(a, k);
            s_o[t] = so;
            if (lin % (a.tiles_x * a.tiles_y) == 0 && k >= (zb >> 4) && k <= ((ze - 1) >> 4))
                a.meta.s_out[k] = so;
        }
        __syncthreads();
    }
    auto slab_of = [&](int zz) { return clampi(zz >> 4, 0, nslab - 1) - ks; };
    auto su = [&](int zz) { return s_in[slab_of(zz)]; };

    raw q[RY][9];
    raw nq[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int zz = zb - 4 + i;
            q[j][i] = IO::ld(at(plane(u, zz), lown[j]));
        }
        nq[j] = IO::ld(at(plane(u, zb + 4), lown[j]));
    }
    // Halo chunks of planes z .. z+HQR-1.  The FP32 sweeps fetch them 5
    // planes ahead, when their owners fetch the same rows (L2 reuse); the
    // raw 16-bit body keeps a shallower queue for occupancy: at depth 5
    // the BF16 body needs 178 VGPRs (two waves per SIMD), at depth 1 it
    // fits three, and FP16 keeps three at depth 2.  Measured side by side
    // on MI355X, 128x16x2 tiles: BF16 485 against 429 GPts/s at 512^3 and
    // 491 against 470 at 1024x1024x512; FP16 498 against 493 and 499
    // against 499.
    constexpr int HQR = std::is_same<T, __bf16>::value ? 1 : 2;
    raw hq[HPT][HQR];
#pragma unroll
    for (int j = 0; j < HPT; ++j)
#pragma unroll
        for (int k = 0; k < HQR; ++k)
            hq[j][k] = IO::ld(at(plane(u, zb + k), hoff[j]));

    // u^{n-1} and v one plane ahead (two planes ahead measured 2-3 % slower:
    // the extra registers cost BF16 its third wave per SIMD)
    raw pp[RY];
    f4v vv[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        pp[j] = IO::ld_nt(at(plane(uprev, zb), own[j]));
        vv[j] = ld4_nt(vat(vplane(zb), vown[j]));
    }

    // this step's source amplitudes, read once per block
    __shared__ float s_amp[SP_MAX_SOURCES];
    if (tid < a.src.n) s_amp[tid] = a.src.amp[tid];
    __syncthreads();

    const StarCoef &c = a.c;
    float s_out = 1.f, inv_out = 1.f;
    float tmax = 0.f;
    bool bad = false;                     // a non-finite output seen by this lane

    // One plane of the chunk; MORE: issue the next plane's loads and advance
    // the queues (every plane but the chunk's last, which is peeled off the
    // loop so that no load needs a predicate).
    auto sweep_plane = [&](const int z, auto more) {
        constexpr bool MORE = decltype(more)::value;
        const int b = z & 1;
        if (z == zb || (z & (SP_SLAB - 1)) == 0) {
            s_out = s_o[slab_of(z)];
            inv_out = 1.f / s_out;
        }
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][8] = nq[j];
            lds[b][ly * RY + j + 4][lx + 1] = q[j][4];
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (tid + j * NT < HC) lds[b][hrow[j]][hchk[j]] = hq[j][0];

        raw hn[HPT];
        raw pp_n[RY];
        f4v vv_n[RY];
        if constexpr (MORE) {
#pragma unroll
            for (int j = 0; j < RY; ++j) nq[j] = IO::ld(at(plane(u, z + 5), lown[j]));
#pragma unroll
            for (int j = 0; j < HPT; ++j) hn[j] = IO::ld(at(plane(u, z + HQR), hoff[j]));
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                pp_n[j] = IO::ld_nt(at(plane(uprev, z + 1), own[j]));
                vv_n[j] = ld4_nt(vat(vplane(z + 1), vown[j]));
            }
        }

        lds_barrier();

        raw yrow[RY + 8];
#pragma unroll
        for (int d = -4; d < RY + 4; ++d)
            yrow[d + 4] = (d >= 0 && d < RY) ? q[d][4] : lds[b][ly * RY + d + 4][lx + 1];

        // FP32 coefficients of this plane's taps, each times the slab scale
        // of the plane the tap reads (exact: scales are powers of two)
        const float s0 = su(z);
        const float c0s = c.c0 * s0, two_s = 2.f * s0, nsp = -s_pv[slab_of(z)];
        float czp[4], czm[4], cys[4], cxs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            czp[r] = c.cz[r] * su(z + r + 1);
            czm[r] = c.cz[r] * su(z - r - 1);
            cys[r] = c.cy[r] * s0;
            cxs[r] = c.cx[r] * s0;
        }
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const raw ctr = q[j][4];
            const raw L = lds[b][ly * RY + j + 4][lx], R = lds[b][ly * RY + j + 4][lx + 2];
            const T w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w, R.x, R.y, R.z, R.w};
            f4v acc;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float o = c0s * (float)ctr[i];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    o = fmaf(czp[r], (float)q[j][5 + r][i], o);
                    o = fmaf(czm[r], (float)q[j][3 - r][i], o);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    o = fmaf(cys[r], (float)yrow[j + 5 + r][i], o);
                    o = fmaf(cys[r], (float)yrow[j + 3 - r][i], o);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    o = fmaf(cxs[r], (float)w[5 + i + r], o);
                    o = fmaf(cxs[r], (float)w[3 + i - r], o);
                }
                acc[i] = o;
            }
            const f4v m = vv[j] * vv[j] * a.m_scale;
            f4v res;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float t = fmaf(two_s, (float)ctr[i], nsp * (float)pp[j][i]);
                res[i] = fmaf(m[i], acc[i], t);
            }
            const int y = ybase + j;
            for (int s = 0; s < a.src.n; ++s) {
                if (a.src.z[s] == z && a.src.y[s] == y) {
                    const int d = a.src.x[s] - x;
                    if (d >= 0 && d < 4) {
                        const float vs = vv[j][d];
                        res[d] += a.src.dt2 * (vs * vs) * s_amp[s];
                    }
                }
            }
            if (st_ok[j]) {
                if (NF) bad |= nonfinite4(res, a.nx - x);
                T *o = const_cast<T *>(at(plane(out, z), own[j]));
                // the slab maximum is taken on the scaled FP32 values and
                // rounded once per wave below: rounding to nearest even is
                // monotone and odd, so max |round(v)| = round(max |v|)
                const f4v sc = res * inv_out;
                const raw enc = __builtin_convertvector(sc, raw);
                float mm = fabsf(sc.x);
                if (x + 1 < a.nx) mm = fmaxf(mm, fabsf(sc.y));
                if (x + 2 < a.nx) mm = fmaxf(mm, fabsf(sc.z));
                if (x + 3 < a.nx) mm = fmaxf(mm, fabsf(sc.w));
                tmax = fmaxf(tmax, mm);
                if (x + 4 <= a.nx) {
                    IO::st_nt(o, enc);
                } else {
                    o[0] = enc[0];
                    if (x + 1 < a.nx) o[1] = enc[1];
                    if (x + 2 < a.nx) o[2] = enc[2];
                }
            }
        }

        if (z + 1 == ze || ((z + 1) & (SP_SLAB - 1)) == 0) {
            float w = tmax;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) w = fmaxf(w, __shfl_xor(w, off, 64));
            w = (float)(T)w;                        // the stored magnitude
            if ((tid & 63) == 0) atomicMax(&a.meta.a_out[z >> 4], __float_as_uint(w * s_out));
            tmax = 0.f;
        }

        if constexpr (MORE) {
#pragma unroll
            for (int j = 0; j < RY; ++j) {
#pragma unroll
                for (int i = 0; i < 8; ++i) q[j][i] = q[j][i + 1];
                pp[j] = pp_n[j];
                vv[j] = vv_n[j];
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
#pragma unroll
                for (int k = 0; k + 1 < HQR; ++k) hq[j][k] = hq[j][k + 1];
                hq[j][HQR - 1] = hn[j];
            }
        }
    };
    for (int z = zb; z + 1 < ze; ++z) sweep_plane(z, std::true_type());
    sweep_plane(ze - 1, std::false_type());
    if (NF) report_nonfinite(a.nonfinite, bad);
}

// One sweep over the block's tile and z-chunk.
//   TX: tile width in points (4 per lane), TY: tile height in rows,
//   RY: adjacent rows per thread (register blocking in y), T: storage type,
//   NF: the leapfrog reports non-finite outputs through a.nonfinite (the
//   served batches; the single-grid sweeps compile without the check).
template <int TX, int TY, int RY, int MODE, typename T, bool NF = false>
__device__ __forceinline__ void star25_body(const SweepArgs &a, const int lin) {
    if constexpr (MODE == MODE_WAVE && Io<T>::scaled) {
        star25_wave_raw16<TX, TY, RY, T, NF>(a, lin);
        return;
    }
    typedef Io<T> IO;
    typedef typename IO::raw raw;
    constexpr int LX = TX / 4;           // lanes per tile row
    constexpr int NT = LX * (TY / RY);   // threads per block
    constexpr int LC = LX + 2;           // LDS chunks per row (incl. x halo)
    constexpr int LR = TY + 8;           // LDS rows (incl. y halo)
    constexpr int HY = 8 * LX;           // y-halo chunks per plane
    constexpr int HC = HY + 2 * TY;      // all halo chunks per plane
    constexpr int HPT = (HC + NT - 1) / NT;
    static_assert(TY % RY == 0, "RY must divide TY");
    static_assert(MODE == MODE_WAVE || !IO::scaled, "only the leapfrog step has FP16/BF16 storage");
    static_assert(MODE != MODE_PML || RY == 1, "the absorbing-layer mode runs one row per thread");
    static_assert(MODE != MODE_ADJ || RY == 1, "the fused adjoint mode runs one row per thread");
    constexpr bool VW = (MODE == MODE_WAVE || MODE == MODE_ENERGY || MODE == MODE_PML ||
                         MODE == MODE_ADJ);  // reads v
    typedef double d4v __attribute__((ext_vector_type(4)));
    constexpr bool PW = (MODE == MODE_WAVE || MODE == MODE_GRAD || MODE == MODE_ENERGY ||
                         MODE == MODE_PML || MODE == MODE_ADJ);  // reads `prev`
    constexpr bool GW = (MODE == MODE_GRAD || MODE == MODE_ADJ);   // accumulates FP64 G
    // MODE_ADJ streams a second stencil field u2 (its own register queue,
    // LDS plane and halo chunks); the other modes compile these to size 1
    constexpr bool TWO = (MODE == MODE_ADJ);
    constexpr int R2 = TWO ? RY : 1;
    __shared__ f4v lds[2][LR][LC];
    __shared__ f4v lds2[TWO ? 2 : 1][TWO ? LR : 1][TWO ? LC : 1];

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
    const T *u = static_cast<const T *>(a.u);
    const T *uprev = static_cast<const T *>(a.prev);
    T *out = static_cast<T *>(a.out);
    const int nslab = a.meta.nslab;

    if constexpr (IO::scaled) {
        // retire the records of u^{n-2}: that slot receives u^{n+2} next step
        if (lin == 0)
            for (int i = tid; i < nslab; i += NT) {
                a.meta.s_clear[i] = 0.f;
                a.meta.a_clear[i] = 0u;
            }
    }

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
    const raw rzero = IO::enc(zero, 1.f);

    // FP16/BF16: the block's slab scales (inputs, and the outputs chosen by
    // the rule) are computed once into LDS; the plane loop reads them there
    // instead of issuing dependent global loads that would drain the
    // outstanding prefetches.
    constexpr int MAXS = IO::scaled ? MAX_BLOCK_SLABS : 1;
    __shared__ float s_in[MAXS], s_pv[MAXS], s_o[MAXS];
    int ks = 0;
    if constexpr (IO::scaled) {
        ks = clampi((zb - 4) >> 4, 0, nslab - 1);
        const int ke = clampi((ze + 3) >> 4, 0, nslab - 1);
        for (int t = tid; t <= ke - ks; t += NT) {
            const int k = ks + t;
            s_in[t] = a.meta.s_u[k];
            s_pv[t] = a.meta.s_prev[k];
            const float so = slab_scale(a, k);
            s_o[t] = so;
            if (lin % (a.tiles_x * a.tiles_y) == 0 && k >= (zb >> 4) && k <= ((ze - 1) >> 4))
                a.meta.s_out[k] = so;
        }
        __syncthreads();
    }
    auto slab_of = [&](int zz) { return clampi(zz >> 4, 0, nslab - 1) - ks; };
    auto su = [&](int zz) {
        if constexpr (IO::scaled) return s_in[slab_of(zz)];
        else return 1.f;
    };
    auto sprev = [&](int zz) {
        if constexpr (IO::scaled) return s_pv[slab_of(zz)];
        else return 1.f;
    };

    f4v q[RY][9];
    raw nq[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int zz = zb - 4 + i;
            q[j][i] = ld_ok[j] ? IO::dec(IO::ld(u + (int64_t)zz * sz + own[j]), su(zz)) : zero;
        }
        nq[j] = ld_ok[j] ? IO::ld(u + (int64_t)(zb + 4) * sz + own[j]) : rzero;
    }
    // halo chunks of planes z .. z+HD-1; the FP32 leapfrog, gradient and
    // energy sweeps on 1024-thread blocks (a 128-VGPR budget) and the fused
    // adjoint (two fields) keep depth 1
    constexpr int HD = ((NT > 512 && MODE != MODE_APPLY && std::is_same<T, float>::value) || TWO) ? 1 : HQ;
    raw hq[HPT][HD];
#pragma unroll
    for (int j = 0; j < HPT; ++j)
#pragma unroll
        for (int k = 0; k < HD; ++k)
            hq[j][k] = h_ok[j] ? IO::ld(u + (int64_t)(zb + k) * sz + hoff[j]) : rzero;
    // MODE_ADJ: the same queue, halo chunks and next plane for u2 (FP32)
    f4v q2[R2][9], nq2[R2], hq2[TWO ? HPT : 1];
    if constexpr (TWO) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                q2[j][i] = ld_ok[j] ? ld4(a.u2 + (int64_t)(zb - 4 + i) * sz + own[j]) : zero;
            nq2[j] = ld_ok[j] ? ld4(a.u2 + (int64_t)(zb + 4) * sz + own[j]) : zero;
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) hq2[j] = h_ok[j] ? ld4(a.u2 + (int64_t)zb * sz + hoff[j]) : zero;
    }

    // Single-use streams (u^{n-1}, v) are fetched PF planes ahead: pp/vv hold
    // plane z, pp1/vv1 plane z+1 when PF = 2 (plane zb+1 <= nz lies in the
    // frame).  1024-thread blocks (a 128-VGPR budget) and the FP64 gradient
    // sweep keep PF = 1.
    constexpr int PF = (NT > 512 || GW || MODE == MODE_PML) ? 1 : 2;
    raw pp[RY], pp1[RY];
    f4v vv[RY], vv1[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        pp[j] = rzero;
        vv[j] = zero;
        pp1[j] = rzero;
        vv1[j] = zero;
        if (PW && st_ok[j]) {
            pp[j] = IO::ld_nt(uprev + (int64_t)zb * sz + own[j]);
            if constexpr (PF == 2) pp1[j] = IO::ld_nt(uprev + (int64_t)(zb + 1) * sz + own[j]);
        }
        if (VW && st_ok[j]) {
            vv[j] = ld4_nt(a.v + (int64_t)zb * a.vsz + vown[j]);
            if constexpr (PF == 2) vv1[j] = ld4_nt(a.v + (int64_t)(zb + 1) * a.vsz + vown[j]);
        }
    }
    d4v gg[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        gg[j] = d4v{0.0, 0.0, 0.0, 0.0};
        if (GW && st_ok[j])
            gg[j] = *reinterpret_cast<const d4v *>(a.gacc + (int64_t)zb * sz + own[j]);
    }
    double esum = 0.0;                    // MODE_ENERGY: this thread's partial sum

    // MODE_PML (one row per thread): damping eta as a 3-plane queue of the
    // own chunk (planes z-1, z, z+1) plus the x/y-neighbour chunks of plane
    // z (x-4, x+4, y-1, y+1); psi of plane z.  All fetched one plane ahead
    // from offsets that are valid for every lane.
    f4v eq[3], ex[4], ps;
    const int64_t ve = st_ok[0] ? vown[0] : 0, pe = st_ok[0] ? own[0] : 0;
    auto eta_xy = [&](int zz, f4v *d) {
        const float *e = a.eta + (int64_t)zz * a.vsz + ve;
        d[0] = ld4(e - 4);
        d[1] = ld4(e + 4);
        d[2] = ld4(e - a.vsy);
        d[3] = ld4(e + a.vsy);
    };
    if constexpr (MODE == MODE_PML) {
#pragma unroll
        for (int k = 0; k < 3; ++k) eq[k] = ld4(a.eta + (int64_t)(zb - 1 + k) * a.vsz + ve);
        eta_xy(zb, ex);
        ps = ld4(a.psi + (int64_t)zb * sz + pe);
    }

    // this step's source amplitudes, read once per block: a global load in
    // the plane loop would wait for every outstanding prefetch
    __shared__ float s_amp[SP_MAX_SOURCES];
    if (tid < a.src.n) s_amp[tid] = a.src.amp[tid];
    __syncthreads();

    const StarCoef &c = a.c;
    float s_out = 1.f, inv_out = 1.f;     // output scale of the current slab
    float tmax = 0.f;                     // running max |stored output| in the slab
    bool bad = false;                     // MODE_WAVE: a non-finite output seen by this lane

    for (int z = zb; z < ze; ++z) {
        const int b = z & 1;
        if constexpr (IO::scaled) {
            if (z == zb || (z & (SP_SLAB - 1)) == 0) {
                s_out = s_o[slab_of(z)];
                inv_out = 1.f / s_out;
            }
        }
        const float s4 = su(z + 4), s0 = su(z);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][8] = IO::dec(nq[j], s4);
            lds[b][ly * RY + j + 4][lx + 1] = q[j][4];
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (tid + j * NT < HC) lds[b][hrow[j]][hchk[j]] = IO::dec(hq[j][0], s0);
        if constexpr (TWO) {
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                q2[j][8] = nq2[j];
                lds2[b][ly * RY + j + 4][lx + 1] = q2[j][4];
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                if (tid + j * NT < HC) lds2[b][hrow[j]][hchk[j]] = hq2[j];
        }

        raw hn[HPT];
        f4v hn2[TWO ? HPT : 1];
#pragma unroll
        for (int j = 0; j < HPT; ++j) hn[j] = rzero;
#pragma unroll
        for (int j = 0; j < (TWO ? HPT : 1); ++j) hn2[j] = zero;
        raw pp_n[RY];
        f4v vv_n[RY];
        d4v gg_n[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            pp_n[j] = rzero;
            vv_n[j] = zero;
            gg_n[j] = d4v{0.0, 0.0, 0.0, 0.0};
        }
        if (z + 1 < ze) {
#pragma unroll
            for (int j = 0; j < RY; ++j)
                nq[j] = ld_ok[j] ? IO::ld(u + (int64_t)(z + 5) * sz + own[j]) : rzero;
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                hn[j] = h_ok[j] ? IO::ld(u + (int64_t)(z + HD) * sz + hoff[j]) : rzero;
#pragma unroll
            for (int j = 0; j < RY; ++j)
                if (st_ok[j]) {
                    if (PW) pp_n[j] = IO::ld_nt(uprev + (int64_t)(z + PF) * sz + own[j]);
                    if (VW) vv_n[j] = ld4_nt(a.v + (int64_t)(z + PF) * a.vsz + vown[j]);
                    if (GW)
                        gg_n[j] = __builtin_nontemporal_load(
                            reinterpret_cast<const d4v *>(a.gacc + (int64_t)(z + 1) * sz + own[j]));
                }
            if constexpr (TWO) {
#pragma unroll
                for (int j = 0; j < RY; ++j)
                    nq2[j] = ld_ok[j] ? ld4(a.u2 + (int64_t)(z + 5) * sz + own[j]) : zero;
#pragma unroll
                for (int j = 0; j < HPT; ++j)
                    hn2[j] = h_ok[j] ? ld4(a.u2 + (int64_t)(z + 1) * sz + hoff[j]) : zero;
            }
        }
        f4v eq_n, ex_n[4], ps_n;
        if constexpr (MODE == MODE_PML) {
            // planes z+2 (<= nz+1) and z+1 always lie in the frame
            eq_n = ld4(a.eta + (int64_t)(z + 2) * a.vsz + ve);
            eta_xy(z + 1, ex_n);
            ps_n = ld4(a.psi + (int64_t)(z + 1) * sz + pe);
        }

        lds_barrier();

        // y-neighbour rows d = -4 .. RY+3 relative to this thread's first row:
        // own rows from registers, the rest from LDS.
        f4v yrow[RY + 8];
#pragma unroll
        for (int d = -4; d < RY + 4; ++d)
            yrow[d + 4] = (d >= 0 && d < RY) ? q[d][4] : lds[b][ly * RY + d + 4][lx + 1];

        const float sp0 = sprev(z);
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
            if constexpr (MODE == MODE_ADJ) {
                // nu^k = 2 nu^{k+1} - nu^{k+2} + m L nu^{k+1} (the receiver term
                // follows in a separate kernel); G += nu^k (L u2 + dx^2 f e_src)
                const f4v m = vv[j] * vv[j] * a.m_scale;
                res = m * acc + (2.f * ctr - IO::dec(pp[j], 1.f));
                const f4v c2 = q2[j][4];
                f4v term = c.c0 * c2;
#pragma unroll
                for (int r = 1; r <= 4; ++r) term += c.cz[r - 1] * (q2[j][4 + r] + q2[j][4 - r]);
                const int row = ly * RY + j + 4;
#pragma unroll
                for (int r = 1; r <= 4; ++r)
                    term += c.cy[r - 1] * (lds2[b][row + r][lx + 1] + lds2[b][row - r][lx + 1]);
                {
                    const f4v L = lds2[b][row][lx], R = lds2[b][row][lx + 2];
                    const float w[12] = {L.x, L.y, L.z, L.w, c2.x, c2.y, c2.z, c2.w, R.x, R.y, R.z, R.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float o = term[i];
#pragma unroll
                        for (int r = 1; r <= 4; ++r) o = fmaf(c.cx[r - 1], w[4 + i + r] + w[4 + i - r], o);
                        term[i] = o;
                    }
                }
                const int y = ybase + j;
                for (int s = 0; s < a.src.n; ++s) {
                    if (a.src.z[s] == z && a.src.y[s] == y) {
                        const int d = a.src.x[s] - x;
                        if (d >= 0 && d < 4) term[d] += a.dx2 * s_amp[s];
                    }
                }
                if (st_ok[j]) {
                    d4v gnew = gg[j];
#pragma unroll
                    for (int i = 0; i < 4; ++i) gnew[i] = fma((double)res[i], (double)term[i], gnew[i]);
                    double *go = a.gacc + (int64_t)z * sz + own[j];
                    if (x + 4 <= a.nx) {
                        __builtin_nontemporal_store(gnew, reinterpret_cast<d4v *>(go));
                    } else {
                        go[0] = gnew[0];
                        if (x + 1 < a.nx) go[1] = gnew[1];
                        if (x + 2 < a.nx) go[2] = gnew[2];
                    }
                }
            } else if (MODE == MODE_WAVE) {
                const f4v m = vv[j] * vv[j] * a.m_scale;
                res = m * acc + (2.f * ctr - IO::dec(pp[j], sp0));
                const int y = ybase + j;
                for (int s = 0; s < a.src.n; ++s) {
                    if (a.src.z[s] == z && a.src.y[s] == y) {
                        const int d = a.src.x[s] - x;
                        if (d >= 0 && d < 4) {
                            const float vs = vv[j][d];
                            res[d] += a.src.dt2 * (vs * vs) * s_amp[s];
                        }
                    }
                }
            } else if (MODE == MODE_PML) {
                // layer update (see the absorbing-layer equations): acc = L u
                const f4v L = lds[b][ly * RY + j + 4][lx], R = lds[b][ly * RY + j + 4][lx + 2];
                const f4v eC = eq[1];
                f4v pn;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float ux = (i < 3 ? ctr[i + 1] : R[0]) - (i > 0 ? ctr[i - 1] : L[3]);
                    const float ex1 = (i < 3 ? eC[i + 1] : ex[1][0]) - (i > 0 ? eC[i - 1] : ex[0][3]);
                    const float G = 0.25f * (ex1 * ux + (ex[3][i] - ex[2][i]) * (yrow[j + 5][i] - yrow[j + 3][i]) +
                                             (eq[2][i] - eq[0][i]) * (q[j][5][i] - q[j][3][i]));
                    const float ae = eC[i] * a.dt;
                    const float bb = ae + a.alpha_dt;
                    // the two quotients take the hardware reciprocal (1 ulp)
                    // instead of a correctly rounded division: about 70
                    // fewer instructions per plane in this compute-bound mode
                    pn[i] = ((1.f - 0.5f * bb) * ps[i] - a.dt * G) * __builtin_amdgcn_rcpf(1.f + 0.5f * bb);
                    const float m = vv[j][i] * vv[j][i] * a.m_scale;
                    res[i] = ((2.f - ae * ae) * ctr[i] - (1.f - ae) * IO::dec(pp[j], 1.f)[i] +
                              m * (acc[i] + 0.5f * (ps[i] + pn[i]))) * __builtin_amdgcn_rcpf(1.f + ae);
                }
                const int y = ybase + j;
                for (int s = 0; s < a.src.n; ++s) {
                    if (a.src.z[s] == z && a.src.y[s] == y) {
                        const int d = a.src.x[s] - x;
                        if (d >= 0 && d < 4) {
                            const float vs = vv[j][d];
                            res[d] += a.src.dt2 * (vs * vs) * s_amp[s];
                        }
                    }
                }
                if (st_ok[j]) {
                    float *po = a.psi + (int64_t)z * sz + own[j];
                    if (x + 4 <= a.nx) {
                        *reinterpret_cast<f4v *>(po) = pn;
                    } else {
                        po[0] = pn[0];
                        if (x + 1 < a.nx) po[1] = pn[1];
                        if (x + 2 < a.nx) po[2] = pn[2];
                    }
                }
            } else if (MODE == MODE_GRAD) {
                // G += w (L u + dx^2 f at sources), products and sums in FP64
                f4v term = acc;
                const int y = ybase + j;
                for (int s = 0; s < a.src.n; ++s) {
                    if (a.src.z[s] == z && a.src.y[s] == y) {
                        const int d = a.src.x[s] - x;
                        if (d >= 0 && d < 4) term[d] += a.dx2 * s_amp[s];
                    }
                }
                if (st_ok[j]) {
                    const f4v w = IO::dec(pp[j], 1.f);
                    d4v gnew = gg[j];
#pragma unroll
                    for (int i = 0; i < 4; ++i) gnew[i] = fma((double)w[i], (double)term[i], gnew[i]);
                    double *go = a.gacc + (int64_t)z * sz + own[j];
                    if (x + 4 <= a.nx) {
                        __builtin_nontemporal_store(gnew, reinterpret_cast<d4v *>(go));
                    } else {
                        go[0] = gnew[0];
                        if (x + 1 < a.nx) go[1] = gnew[1];
                        if (x + 2 < a.nx) go[2] = gnew[2];
                    }
                }
                continue;
            } else if (MODE == MODE_ENERGY) {
                // (u1 - u0)^2 / m - u1 (L u0), u0 = ctr, u1 = w; FP64 accumulation
                if (st_ok[j]) {
                    const f4v w = IO::dec(pp[j], 1.f);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (x + i < a.nx) {
                            const double vv2 = (double)vv[j][i] * (double)vv[j][i];
                            const double m = vv2 * (double)a.m_scale;
                            const double dd = (double)w[i] - (double)ctr[i];
                            esum += dd * dd / m - (double)w[i] * (double)acc[i];
                        }
                    }
                }
                continue;
            } else {
                res = acc;
            }

            if (st_ok[j]) {
                if (MODE == MODE_WAVE && NF) bad |= nonfinite4(res, a.nx - x);
                T *o = out + (int64_t)z * sz + own[j];
                const raw enc = IO::enc(res, inv_out);
                if constexpr (IO::scaled) {
                    const f4v mg = IO::mag(enc);
                    float mm = mg.x;
                    if (x + 1 < a.nx) mm = fmaxf(mm, mg.y);   // ragged chunk: interior points only
                    if (x + 2 < a.nx) mm = fmaxf(mm, mg.z);
                    if (x + 3 < a.nx) mm = fmaxf(mm, mg.w);
                    tmax = fmaxf(tmax, mm);
                }
                if (x + 4 <= a.nx) {
                    IO::st_nt(o, enc);
                } else {
                    o[0] = enc[0];
                    if (x + 1 < a.nx) o[1] = enc[1];
                    if (x + 2 < a.nx) o[2] = enc[2];
                }
            }
        }

        if constexpr (IO::scaled) {
            if (z + 1 == ze || ((z + 1) & (SP_SLAB - 1)) == 0) {
                float w = tmax;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) w = fmaxf(w, __shfl_xor(w, off, 64));
                if ((tid & 63) == 0) atomicMax(&a.meta.a_out[z >> 4], __float_as_uint(w * s_out));
                tmax = 0.f;
            }
        }

#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int i = 0; i < 8; ++i) q[j][i] = q[j][i + 1];
            if constexpr (PF == 2) {
                pp[j] = pp1[j];
                vv[j] = vv1[j];
                pp1[j] = pp_n[j];
                vv1[j] = vv_n[j];
            } else {
                pp[j] = pp_n[j];
                vv[j] = vv_n[j];
            }
            gg[j] = gg_n[j];
        }
        if constexpr (TWO) {
#pragma unroll
            for (int j = 0; j < RY; ++j)
#pragma unroll
                for (int i = 0; i < 8; ++i) q2[j][i] = q2[j][i + 1];
#pragma unroll
            for (int j = 0; j < HPT; ++j) hq2[j] = hn2[j];
        }
        if constexpr (MODE == MODE_PML) {
            eq[0] = eq[1];
            eq[1] = eq[2];
            eq[2] = eq_n;
#pragma unroll
            for (int k = 0; k < 4; ++k) ex[k] = ex_n[k];
            ps = ps_n;
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
#pragma unroll
            for (int k = 0; k + 1 < HD; ++k) hq[j][k] = hq[j][k + 1];
            hq[j][HD - 1] = hn[j];
        }
    }

    if constexpr (MODE == MODE_WAVE && NF) report_nonfinite(a.nonfinite, bad);

    if constexpr (MODE == MODE_ENERGY) {
        // block sum in a fixed order: waves by shuffles, then wave 0 over LDS
        __shared__ double wsum[NT / 64];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) esum += __shfl_xor(esum, off, 64);
        if ((tid & 63) == 0) wsum[tid >> 6] = esum;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += wsum[w];
            a.gacc[blockIdx.x] = t;
        }
    }
}

// Register cap of a kernel instance: the 16-bit leapfrog on its default
// 128x16x2 tiles is held to 168 VGPRs, three waves per SIMD.  Left alone the
// compiler takes 170-180 and drops to two waves (served batches: 342
// against 372 GPts/s, measured); at the cap the batched form spills a few
// bytes outside its plane loop.  The other instances take what they need.
template <int TX, int TY, int RY, int MODE, typename T>
constexpr int waves_per_simd() {
    return Io<T>::scaled && MODE == MODE_WAVE && TX == 128 && TY == 16 && RY == 2 ? 3 : 1;
}

template <int TX, int TY, int RY, int MODE, typename T>
__global__ void __launch_bounds__((TX / 4) * (TY / RY))
__attribute__((amdgpu_waves_per_eu(waves_per_simd<TX, TY, RY, MODE, T>())))
k_star25(SweepArgs a) {
    star25_body<TX, TY, RY, MODE, T>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Several boxes of one grid in one launch (the absorbing layer's shell as
// one region): block b sweeps tile b - first[k] of box k, the box whose
// block range holds b; each XCD receives one contiguous range of blocks.
// The wide z and y slabs run on 256x8x1 tiles and the 32-wide x slabs on
// 32x64x1 tiles (both 512 threads; the choice is uniform per block), so the
// thin x slabs overlap the wide ones.
template <int MODE, typename T>
__global__ void __launch_bounds__(512) k_star25_shell(const BoxSet bs) {
    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    int k = 0;
#pragma unroll
    for (int i = 1; i < MAX_BOXES; ++i)
        if (i < bs.n && lin >= bs.first[i]) k = i;
    if (bs.wide[k])
        star25_body<256, 8, 1, MODE, T>(bs.a[k], lin - bs.first[k]);
    else
        star25_body<32, 64, 1, MODE, T>(bs.a[k], lin - bs.first[k]);
}

// Batched form: block b computes tile table[b].y of grid table[b].x, whose
// arguments are args[table[b].x].  The host lays the table out so that each
// XCD receives contiguous tiles of the same grid.
template <int TX, int TY, int RY, int MODE, typename T>
__global__ void __launch_bounds__((TX / 4) * (TY / RY))
__attribute__((amdgpu_waves_per_eu(waves_per_simd<TX, TY, RY, MODE, T>())))
k_star25_batch(const SweepArgs *__restrict__ args, const int2 *__restrict__ table) {
    const int2 e = table[blockIdx.x];
    star25_body<TX, TY, RY, MODE, T, true>(args[e.x], e.y);
}

__global__ void k_inject(float *field, int64_t sy, int64_t sz, const float *v, int64_t vsy,
                         int64_t vsz, int nx, int ny, int nz, const int32_t *xyz, int n,
                         const float *amp, float scale) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return;
    const float vs = v[(int64_t)z * vsz + (int64_t)y * vsy + x];
    atomicAdd(field + (int64_t)z * sz + (int64_t)y * sy + x, scale * (vs * vs) * amp[r]);
}

// The receiver term of a fused adjoint step: the MODE_ADJ sweep wrote nu^k
// without it and added nu^k (L u2 + dx^2 f) to G, so each receiver adds
// its injection w to nu^k and w (L u2 + dx^2 f) to G at its point.
__global__ void k_inject_grad(const SweepArgs a, const int32_t *xyz, int n, const float *amp,
                              float scale) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
    if (x < 0 || x >= a.nx || y < 0 || y >= a.ny || z < 0 || z >= a.nz) return;
    const float vs = a.v[(int64_t)z * a.vsz + (int64_t)y * a.vsy + x];
    const float w = scale * (vs * vs) * amp[r];
    const int64_t o = (int64_t)z * a.sz + (int64_t)y * a.sy + x;
    atomicAdd(static_cast<float *>(a.out) + o, w);
    const float *p = a.u2 + o;
    const StarCoef &c = a.c;
    float t = c.c0 * p[0];
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        t += c.cz[k - 1] * (p[k * a.sz] + p[-k * a.sz]);
        t += c.cy[k - 1] * (p[k * a.sy] + p[-k * a.sy]);
        t += c.cx[k - 1] * (p[k] + p[-k]);
    }
    for (int s = 0; s < a.src.n; ++s)
        if (a.src.x[s] == x && a.src.y[s] == y && a.src.z[s] == z) t += a.dx2 * a.src.amp[s];
    atomicAdd(a.gacc + o, (double)w * (double)t);
}

__global__ void k_grad_finish(const double *G, const float *v, float *out, int64_t sy, int64_t sz,
                              int nx, int ny, int nz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)nx * ny * nz;
    if (i >= n) return;
    const int x = (int)(i % nx);
    const int64_t r = i / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const int64_t o = (int64_t)z * sz + (int64_t)y * sy + x;
    out[o] = (float)(2.0 * G[o] / (double)v[o]);
}

__global__ void k_sum(const double *partial, int n, double *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += partial[i];
        *out = t;
    }
}

template <typename T>
__global__ void k_record(const T *u, const float *scale, int64_t sy, int64_t sz, int nx, int ny,
                         int nz, const int32_t *xyz, int n, float *traces) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
    float val = 0.f;
    if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) {
        const float s = scale ? scale[z >> 4] : 1.f;
        val = Io<T>::dec1(u[(int64_t)z * sz + (int64_t)y * sy + x], s);
    }
    traces[r] = val;
}

template <typename T>
__global__ void k_record_batch(const RecArgs *__restrict__ recs, const int2 *__restrict__ rmap,
                               int total) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= total) return;
    const int2 e = rmap[r];
    const RecArgs &a = recs[e.x];
    const int i = e.y;
    const int x = a.xyz[3 * i], y = a.xyz[3 * i + 1], z = a.xyz[3 * i + 2];
    float val = 0.f;
    if (x >= 0 && x < a.nx && y >= 0 && y < a.ny && z >= 0 && z < a.nz) {
        const float sc = a.scale ? a.scale[z >> 4] : 1.f;
        val = Io<T>::dec1(static_cast<const T *>(a.field)[(int64_t)z * a.sz + (int64_t)y * a.sy + x], sc);
    }
    a.traces[i] = val;
}

__global__ void k_pack(const float *dense, float *field, int64_t sy, int64_t sz, int nx, int ny, int nz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny * nz) return;
    const int x = (int)(i % nx);
    const int64_t r = i / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    field[(int64_t)z * sz + (int64_t)y * sy + x] = dense[i];
}

template <typename T>
__global__ void k_unpack(const T *field, const float *scale, float *dense, int64_t sy, int64_t sz,
                         int nx, int ny, int nz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny * nz) return;
    const int x = (int)(i % nx);
    const int64_t r = i / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const float sc = scale ? scale[z >> 4] : 1.f;
    dense[i] = Io<T>::dec1(field[(int64_t)z * sz + (int64_t)y * sy + x], sc);
}

template <int TX, int TY, int RY, typename T>
hipError_t launch_batch_t(int mode, const SweepArgs *args, const int2 *table, int nblk, hipStream_t s) {
    const dim3 grid(nblk), block((TX / 4) * (TY / RY));
    if (mode != MODE_WAVE) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_star25_batch<TX, TY, RY, MODE_WAVE, T>), grid, block, 0, s, args, table);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_cfg(int mode, const TileCfg &t, const SweepArgs *args, const int2 *table,
                            int nblk, hipStream_t s) {
    if (t.tx == 256 && t.ty == 16 && t.ry == 2) return launch_batch_t<256, 16, 2, T>(mode, args, table, nblk, s);
    if (t.tx == 128 && t.ty == 16 && t.ry == 2) return launch_batch_t<128, 16, 2, T>(mode, args, table, nblk, s);
    if (t.tx == 64 && t.ty == 16 && t.ry == 1) return launch_batch_t<64, 16, 1, T>(mode, args, table, nblk, s);
    if (t.tx == 256 && t.ty == 16 && t.ry == 1) return launch_batch_t<256, 16, 1, T>(mode, args, table, nblk, s);
    return hipErrorInvalidValue;
}

template <int TX, int TY, int RY, typename T>
hipError_t launch_t(int mode, const SweepArgs &a, hipStream_t s) {
    const int nblk = a.tiles_x * a.tiles_y * a.nzc;
    const dim3 grid(nblk), block((TX / 4) * (TY / RY));
    if (mode == MODE_WAVE) {
        hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_WAVE, T>), grid, block, 0, s, a);
    } else if (mode == MODE_PML) {
        // the absorbing layer: FP32, one row per thread, 512 or 256 threads
        if constexpr (std::is_same<T, float>::value && RY == 1 && TX * TY / 4 <= 512)
            hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_PML, T>), grid, block, 0, s, a);
        else
            return hipErrorInvalidValue;
    } else {
        if constexpr (Io<T>::scaled) {
            return hipErrorInvalidValue;
        } else {
            if (mode == MODE_APPLY)
                hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_APPLY, T>), grid, block, 0, s, a);
            else if (mode == MODE_GRAD)
                hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_GRAD, T>), grid, block, 0, s, a);
            else if (mode == MODE_ADJ) {
                // one row per thread, at most 512 threads (two queues per thread)
                if constexpr (RY == 1 && TX * TY / 4 <= 512)
                    hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_ADJ, T>), grid, block, 0, s, a);
                else
                    return hipErrorInvalidValue;
            }
            else if (mode == MODE_ENERGY)
                hipLaunchKernelGGL((k_star25<TX, TY, RY, MODE_ENERGY, T>), grid, block, 0, s, a);
            else
                return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cfg(int mode, const TileCfg &t, const SweepArgs &a, hipStream_t s) {
    if (t.tx == 256 && t.ty == 16 && t.ry == 2) return launch_t<256, 16, 2, T>(mode, a, s);
    if (t.tx == 128 && t.ty == 16 && t.ry == 2) return launch_t<128, 16, 2, T>(mode, a, s);
    if (t.tx == 64 && t.ty == 16 && t.ry == 1) return launch_t<64, 16, 1, T>(mode, a, s);
    if (t.tx == 128 && t.ty == 32 && t.ry == 2) return launch_t<128, 32, 2, T>(mode, a, s);
    if (t.tx == 256 && t.ty == 8 && t.ry == 2) return launch_t<256, 8, 2, T>(mode, a, s);
    if (t.tx == 256 && t.ty == 16 && t.ry == 1) return launch_t<256, 16, 1, T>(mode, a, s);
    if (t.tx == 256 && t.ty == 8 && t.ry == 1) return launch_t<256, 8, 1, T>(mode, a, s);
    if (t.tx == 128 && t.ty == 16 && t.ry == 1) {
        if constexpr (std::is_same<T, float>::value) {
            if (mode == MODE_ADJ) {
                const dim3 grid(a.tiles_x * a.tiles_y * a.nzc), block(512);
                hipLaunchKernelGGL((k_star25<128, 16, 1, MODE_ADJ, float>), grid, block, 0, s, a);
                return hipGetLastError();
            }
        }
        return hipErrorInvalidValue;
    }
    if (t.tx == 32 && t.ty == 32 && t.ry == 1) {
        // the absorbing layer's x slabs: one 128-byte line per tile row
        if constexpr (std::is_same<T, float>::value) {
            if (mode == MODE_PML) {
                const dim3 grid(a.tiles_x * a.tiles_y * a.nzc), block(256);
                hipLaunchKernelGGL((k_star25<32, 32, 1, MODE_PML, float>), grid, block, 0, s, a);
                return hipGetLastError();
            }
        }
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool tile_supported(const TileCfg &t, int mode) {
    // 128x16x1 is compiled for the fused adjoint sweep only
    if (t.tx == 128 && t.ty == 16 && t.ry == 1) return mode == MODE_ADJ;
    return (t.tx == 256 && t.ty == 16 && t.ry == 2) || (t.tx == 128 && t.ty == 16 && t.ry == 2) ||
           (t.tx == 64 && t.ty == 16 && t.ry == 1) || (t.tx == 128 && t.ty == 32 && t.ry == 2) ||
           (t.tx == 256 && t.ty == 8 && t.ry == 2) || (t.tx == 256 && t.ty == 16 && t.ry == 1) ||
           (t.tx == 256 && t.ty == 8 && t.ry == 1);
}

int occupancy_zchunk(int64_t tiles, int nz, int per_round) {
    // Pick the z-split that maximises the filled share of the last round of
    // per_round blocks times zc / (zc + 8) (each chunk also streams 8
    // planes of start-up).  This keeps one chunk per tile when the tiles
    // fill whole rounds (1024^2 planes: 256 tiles) and avoids, for example,
    // 288 blocks on a 768^2 plane (1.125 rounds: 64-plane chunks run 30 %
    // faster there, measured).
    //
    // A grid too small to fill one round even with 16-plane chunks is
    // latency-bound: all its blocks run at once, each for its chunk plus the
    // 8 start-up planes, so the shortest chunks that still fit one round
    // win, down to a single plane (64^3 apply: 3.8 us per sweep with
    // 1-plane chunks against 13.3 us with 16-plane chunks, measured).
    const int64_t at16 = tiles * ((nz + 15) / 16);
    if (at16 < per_round) {
        for (int z = 1; z < 16; ++z)
            if (tiles * ((nz + z - 1) / z) <= per_round) return z;
        return nz < 16 ? nz : 16;
    }
    int best_k = 1;
    double best = -1.0;
    for (int k = 1; k <= 64; ++k) {
        const int z = (nz + k - 1) / k;
        if (k > 1 && z < 16) break;
        const double rounds = (double)tiles * ((nz + z - 1) / z) / per_round;
        const double eff = rounds / std::ceil(rounds) * z / (z + 8.0);
        if (eff > best + 1e-9) {
            best = eff;
            best_k = k;
        }
    }
    return (nz + best_k - 1) / best_k;
}

TileCfg choose_tiles(int nx, int ny, int nz, int dtype, int mode) {
    // Widest tile that does not waste more than a quarter of its columns on
    // the ragged x edge: wide tiles keep the x-halo (one 128-byte line per
    // side per row) and the y-halo rows small relative to the tile, and two
    // rows per thread share their y-neighbour reads.  The candidates depend
    // on the storage type, because what limits each kernel differs:
    //  * FP32 (231 VGPRs, 16-byte accesses): 512-thread 256x16x2 tiles, one
    //    block per CU, z split only when there are fewer than 256 tiles
    //    (the leapfrog on grids that need 16-plane chunks: 256x16x1);
    //  * FP16 and BF16 (the raw 16-bit body, held to 168 VGPRs for three
    //    waves per SIMD, 8-byte accesses): 256-thread 128x16x2 tiles and many
    //    short z-chunks (about 4096 blocks) so that the CUs stay evenly
    //    loaded (BF16 at 512^3: 453 GPts/s against 345 on the 1024-thread
    //    256x16x1 tiles the decoding body had used);
    //  * the FP32 APPLY sweep (8 B per point) runs best on 128x32x2 tiles
    //    with about 256 blocks (one long z-chunk per tile at 1024^2),
    //    measured on live data: constant or overflowed fields run the same
    //    kernel faster and had favoured other tiles;
    //  * the absorbing-layer mode runs one row per thread in 512-thread
    //    256x8x1 tiles, 64x16x1 or 32x32x1 for narrow boxes (the x slabs),
    //    with the FP32 rule for the z-split;
    //  * the fused adjoint sweep (two stencil fields per thread) runs one
    //    row per thread in 512-thread 128x16x1 tiles, 64x16x1 for narrow
    //    grids, with the FP32 rule for the z-split (256^3 x 1000 forward
    //    plus backward: 0.220 s against 0.224 on 256x8x1 and 0.233 on
    //    64x16x1 tiles);
    // z-chunks are at least 16 planes (each chunk re-reads 8 planes of u,
    // mostly from L2) unless the grid is too small to fill the GPU (see
    // occupancy_zchunk).  These targets are measured optima on MI355X.
    struct Cand {
        int tx, ty, ry, want, min_tiles_x;
    };
    static const Cand c32[3] = {{256, 16, 2, 256, 1}, {128, 16, 2, 512, 1}, {64, 16, 1, 512, 1}};
    static const Cand c16[3] = {{128, 16, 2, 4096, 1}, {128, 16, 2, 4096, 1}, {64, 16, 1, 4096, 1}};
    static const Cand cap[3] = {{128, 32, 2, 256, 1}, {128, 16, 2, 512, 1}, {64, 16, 1, 512, 1}};
    static const Cand cpm[3] = {{256, 8, 1, 256, 1}, {64, 16, 1, 512, 1}, {32, 32, 1, 512, 1}};
    static const Cand cad[3] = {{128, 16, 1, 256, 1}, {64, 16, 1, 512, 1}, {64, 16, 1, 512, 1}};
    const Cand *cand = dtype != SP_F32       ? c16
                       : mode == MODE_APPLY ? cap
                       : mode == MODE_PML   ? cpm
                       : mode == MODE_ADJ   ? cad
                                            : c32;
    TileCfg t;
    int want = 256;
    for (int c = 0; c < 3; ++c) {
        t.tx = cand[c].tx;
        t.ty = cand[c].ty;
        t.ry = cand[c].ry;
        want = cand[c].want;
        const int tiles_x = (nx + t.tx - 1) / t.tx;
        if ((4 * tiles_x * t.tx <= 5 * nx && tiles_x >= cand[c].min_tiles_x) || c == 2) break;
    }
    const int tiles = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    int zc;
    if (cand == c32 || cand == cpm || cand == cap || cand == cad) {
        // FP32 sweeps (leapfrog, gradient, energy, layer, apply): `want`
        // blocks fill the GPU once (one 512-thread or two 256-thread blocks
        // per CU).
        zc = occupancy_zchunk(tiles, nz, want);
        // A leapfrog grid this small fills the GPU only with the shortest
        // chunks; there four waves per SIMD (1024-thread 256x16x1 tiles,
        // one row per thread, same tile count) hide more latency than the
        // two of 256x16x2 (256^3: 360 against 347 GPts/s, measured).
        if (cand == c32 && mode == MODE_WAVE && t.tx == 256 && t.ry == 2 && zc <= 16 && nz > 16)
            t.ry = 1;
    } else {
        const int chunks = (want + tiles - 1) / tiles;
        zc = (nz + chunks - 1) / chunks;
        if (zc < 16) zc = 16;
    }
    if (zc > nz) zc = nz;
    t.zchunk = zc < 1 ? 1 : zc;
    return t;
}

hipError_t launch_sweep_boxes(int mode, const BoxSet &bs, hipStream_t s) {
    if (mode != MODE_PML || bs.n < 1 || bs.n > MAX_BOXES) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_star25_shell<MODE_PML, float>), dim3(bs.first[bs.n]), dim3(512), 0, s, bs);
    return hipGetLastError();
}

bool batch_supported(const TileCfg &t) {
    return (t.tx == 256 && t.ty == 16 && (t.ry == 2 || t.ry == 1)) ||
           (t.tx == 128 && t.ty == 16 && t.ry == 2) || (t.tx == 64 && t.ty == 16 && t.ry == 1);
}

hipError_t launch_sweep(int mode, int dtype, const TileCfg &t, const SweepArgs &a, hipStream_t s) {
    switch (dtype) {
        case SP_F32: return launch_cfg<float>(mode, t, a, s);
        case SP_F16: return launch_cfg<_Float16>(mode, t, a, s);
        case SP_BF16: return launch_cfg<__bf16>(mode, t, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inject(float *field, int64_t sy, int64_t sz, const float *v, int64_t vsy,
                         int64_t vsz, int nx, int ny, int nz, const int32_t *xyz, int n,
                         const float *amp, float scale, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_inject, dim3((n + bs - 1) / bs), dim3(bs), 0, s, field, sy, sz, v, vsy,
                       vsz, nx, ny, nz, xyz, n, amp, scale);
    return hipGetLastError();
}

hipError_t launch_inject_grad(const SweepArgs &a, const int32_t *xyz, int n, const float *amp,
                              float scale, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_inject_grad, dim3((n + bs - 1) / bs), dim3(bs), 0, s, a, xyz, n, amp, scale);
    return hipGetLastError();
}

hipError_t launch_grad_finish(const double *G, const float *v, float *out, int64_t sy, int64_t sz,
                              int nx, int ny, int nz, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int bs = 256;
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, G, v,
                       out, sy, sz, nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_record(int dtype, const void *u, const float *scale, int64_t sy, int64_t sz,
                         int nx, int ny, int nz, const int32_t *xyz, int n, float *traces,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    const dim3 g((n + bs - 1) / bs), b(bs);
    switch (dtype) {
        case SP_F32:
            hipLaunchKernelGGL(k_record<float>, g, b, 0, s, static_cast<const float *>(u), scale,
                               sy, sz, nx, ny, nz, xyz, n, traces);
            break;
        case SP_F16:
            hipLaunchKernelGGL(k_record<_Float16>, g, b, 0, s, static_cast<const _Float16 *>(u),
                               scale, sy, sz, nx, ny, nz, xyz, n, traces);
            break;
        case SP_BF16:
            hipLaunchKernelGGL(k_record<__bf16>, g, b, 0, s, static_cast<const __bf16 *>(u),
                               scale, sy, sz, nx, ny, nz, xyz, n, traces);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_batch(int mode, int dtype, const TileCfg &t, const SweepArgs *args,
                              const int2 *table, int nblk, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    switch (dtype) {
        case SP_F32: return launch_batch_cfg<float>(mode, t, args, table, nblk, s);
        case SP_F16: return launch_batch_cfg<_Float16>(mode, t, args, table, nblk, s);
        case SP_BF16: return launch_batch_cfg<__bf16>(mode, t, args, table, nblk, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_record_batch(int dtype, const RecArgs *recs, const int2 *rmap, int total,
                               hipStream_t s) {
    if (total <= 0) return hipSuccess;
    const int bs = 256;
    const dim3 g((total + bs - 1) / bs), b(bs);
    switch (dtype) {
        case SP_F32: hipLaunchKernelGGL(k_record_batch<float>, g, b, 0, s, recs, rmap, total); break;
        case SP_F16: hipLaunchKernelGGL(k_record_batch<_Float16>, g, b, 0, s, recs, rmap, total); break;
        case SP_BF16: hipLaunchKernelGGL(k_record_batch<__bf16>, g, b, 0, s, recs, rmap, total); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack(const float *dense, float *field, int64_t sy, int64_t sz, int nx, int ny,
                       int nz, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int bs = 256;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, dense, field,
                       sy, sz, nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_unpack(int dtype, const void *field, const float *scale, float *dense,
                         int64_t sy, int64_t sz, int nx, int ny, int nz, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int bs = 256;
    const dim3 g((unsigned)((n + bs - 1) / bs)), b(bs);
    switch (dtype) {
        case SP_F32:
            hipLaunchKernelGGL(k_unpack<float>, g, b, 0, s, static_cast<const float *>(field), scale,
                               dense, sy, sz, nx, ny, nz);
            break;
        case SP_F16:
            hipLaunchKernelGGL(k_unpack<_Float16>, g, b, 0, s, static_cast<const _Float16 *>(field),
                               scale, dense, sy, sz, nx, ny, nz);
            break;
        case SP_BF16:
            hipLaunchKernelGGL(k_unpack<__bf16>, g, b, 0, s, static_cast<const __bf16 *>(field),
                               scale, dense, sy, sz, nx, ny, nz);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sp
