// C-ABI of libstencil: argument validation, grid layout and launch sequencing.
// Every entry point validates before enqueueing anything and reports errors
// through a status code plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "log.h"

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace sp {

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int ok() {
    g_err[0] = '\0';
    return SP_OK;
}

bool log_on() {
    static const bool on = [] {
        const char *e = std::getenv("SP_LOG");
        return e && e[0] && std::strcmp(e, "0") != 0;
    }();
    return on;
}

void log_line(const char *fmt, ...) {
    if (!log_on()) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[libstencil] %s\n", buf);
}

}  // namespace sp

namespace {
using sp::fail;
using sp::ok;

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// A descriptor is valid if it equals what sp_grid_init (or, where 2D grids
// are accepted, sp_grid_init_2d) makes of its own dimensions.
int check_grid(const sp_grid *g, const char *what, bool allow_2d = false) {
    if (!g) return fail(SP_EINVAL, "%s: grid descriptor is NULL", what);
    sp_grid ref;
    const bool flat = g->planes == 1;
    if (flat && !allow_2d) return fail(SP_EINVAL, "%s: 2D grids are not accepted here", what);
    const int rc = flat ? sp_grid_init_2d(g->nx, g->ny, g->halo, g->dtype, &ref)
                        : sp_grid_init(g->nx, g->ny, g->nz, g->halo, g->dtype, &ref);
    if (rc != SP_OK) {
        // the message lives in the buffer that fail() writes: copy it first
        char why[sizeof g_err];
        std::snprintf(why, sizeof why, "%s", g_err);
        return fail(SP_EINVAL, "%s: invalid grid descriptor (%s)", what, why);
    }
    if (std::memcmp(&ref, g, sizeof ref) != 0)
        return fail(SP_EINVAL, "%s: grid descriptor was not produced by sp_grid_init", what);
    return SP_OK;
}

// Do [a, a + abytes) and [b, b + bbytes) intersect?
bool overlaps(const void *a, int64_t abytes, const void *b, int64_t bbytes) {
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)bbytes && y < x + (uintptr_t)abytes;
}

bool overlaps(const void *a, const void *b, int64_t bytes) { return overlaps(a, bytes, b, bytes); }

sp::StarCoef to_f32(const sp_coeffs *c) {
    sp::StarCoef s;
    s.c0 = (float)c->center;
    for (int i = 0; i < 4; ++i) {
        s.cx[i] = (float)c->ax[i];
        s.cy[i] = (float)c->ay[i];
        s.cz[i] = (float)c->az[i];
    }
    return s;
}

void fill_tiling(sp::SweepArgs &a, const sp::TileCfg &t) {
    a.tiles_x = (a.nx + t.tx - 1) / t.tx;
    a.tiles_y = (a.ny + t.ty - 1) / t.ty;
    a.zchunk = t.zchunk;
    a.nzc = (a.nz + t.zchunk - 1) / t.zchunk;
}

// Launch configuration for a grid; SP_TILE=TXxTYxRY[xZC] overrides it for
// tuning.  Returns false (with the error set) for a configuration that is
// not compiled in.
bool tiles_for(const sp_grid *g, sp::TileCfg *out, const char *who, int mode = sp::MODE_WAVE) {
    sp::TileCfg t = sp::choose_tiles(g->nx, g->ny, g->nz, g->dtype, mode);
    // Optional override for tuning: SP_TILE=TXxTYxRY[xZC]
    if (const char *e = std::getenv("SP_TILE")) {
        int tx = 0, ty = 0, ry = 0, zc = 0;
        const int n = std::sscanf(e, "%dx%dx%dx%d", &tx, &ty, &ry, &zc);
        if (n >= 3) {
            t.tx = tx;
            t.ty = ty;
            t.ry = ry;
        }
        if (n == 4 && zc > 0) t.zchunk = std::min(zc, g->nz);
    }
    if (g->dtype != SP_F32 && t.zchunk > sp::MAX_ZCHUNK_SCALED) t.zchunk = sp::MAX_ZCHUNK_SCALED;
    if (!sp::tile_supported(t, mode)) {
        fail(SP_EINVAL, "%s: tile configuration %dx%dx%d is not compiled in", who, t.tx, t.ty, t.ry);
        return false;
    }
    if (sp::log_on()) {
        const int64_t blocks = (int64_t)((g->nx + t.tx - 1) / t.tx) * ((g->ny + t.ty - 1) / t.ty) *
                               ((g->nz + t.zchunk - 1) / t.zchunk);
        sp::log_line("%s: %dx%dx%d dtype %d mode %d -> tile %dx%dx%d, z-chunk %d, %lld blocks", who,
                     g->nx, g->ny, g->nz, g->dtype, mode, t.tx, t.ty, t.ry, t.zchunk, (long long)blocks);
    }
    *out = t;
    return true;
}

}  // namespace

extern "C" {

const char *sp_last_error(void) { return g_err; }

const char *sp_version(void) { return "libstencil 0.1 (gfx950)"; }

int sp_grid_init(int nx, int ny, int nz, int halo, int dtype, sp_grid *out) {
    if (!out) return fail(SP_EINVAL, "sp_grid_init: out is NULL");
    if (halo != SP_HALO) return fail(SP_EINVAL, "sp_grid_init: halo must be %d, got %d", SP_HALO, halo);
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(SP_EINVAL, "sp_grid_init: dims must be >= 1 (got %d x %d x %d)", nx, ny, nz);
    if (nx > (1 << 24) || ny > (1 << 24) || nz > (1 << 24))
        return fail(SP_EINVAL, "sp_grid_init: dims too large");
    int eb;
    switch (dtype) {
        case SP_F32: eb = 4; break;
        case SP_F16:
        case SP_BF16: eb = 2; break;
        default: return fail(SP_EINVAL, "sp_grid_init: unknown dtype %d", dtype);
    }
    sp_grid g;
    std::memset(&g, 0, sizeof g);
    const int64_t align = 128 / eb;           // elements per 128-byte line
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.halo = halo;
    g.dtype = dtype;
    g.elem_bytes = eb;
    g.pitch_x = align + round_up(nx, align);  // lead pad holds left halo and previous row's right halo
    g.pitch_y = (int64_t)ny + 2 * SP_HALO;
    g.planes = (int64_t)nz + 2 * SP_HALO;
    g.origin = ((int64_t)SP_HALO * g.pitch_y + SP_HALO) * g.pitch_x + align;
    g.elems = g.planes * g.pitch_y * g.pitch_x + g.pitch_x;
    g.bytes = round_up(g.elems * eb, 256);
    *out = g;
    return ok();
}

int sp_grid_init_2d(int nx, int ny, int halo, int dtype, sp_grid *out) {
    if (int e = sp_grid_init(nx, ny, 1, halo, dtype, out)) return e;
    sp_grid &g = *out;
    g.planes = 1;
    g.origin = (int64_t)SP_HALO * g.pitch_x + 128 / g.elem_bytes;
    g.elems = g.pitch_y * g.pitch_x + g.pitch_x;
    g.bytes = round_up(g.elems * g.elem_bytes, 256);
    return ok();
}

int sp_apply(const sp_grid *g, const sp_stencil *st, int sweeps, void *u, void *v, int *result_in,
             void *stream) {
    const char *who = "sp_apply";
    if (int e = check_grid(g, who, true)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "%s: FP32 grids only", who);
    if (!st || !st->w || !u || !v || !result_in) return fail(SP_EINVAL, "%s: NULL argument", who);
    if (st->shape != SP_STAR && st->shape != SP_BOX)
        return fail(SP_EINVAL, "%s: unknown stencil shape %d", who, st->shape);
    if (st->ndim != 2 && st->ndim != 3) return fail(SP_EINVAL, "%s: ndim must be 2 or 3", who);
    if (st->radius < 1 || st->radius > SP_HALO)
        return fail(SP_EINVAL, "%s: radius must be 1..%d, got %d", who, SP_HALO, st->radius);
    if (st->ndim == 3 && g->planes == 1) return fail(SP_EINVAL, "%s: a 3D stencil needs a 3D grid", who);
    if (sweeps < 0) return fail(SP_EINVAL, "%s: sweeps < 0", who);
    if (!aligned16(u) || !aligned16(v)) return fail(SP_EINVAL, "%s: pointers must be 16-byte aligned", who);
    if (overlaps(u, v, g->bytes)) return fail(SP_EINVAL, "%s: u and v overlap", who);
    if (g->pitch_x * g->pitch_y >= ((int64_t)1 << 31))
        return fail(SP_EUNSUPPORTED, "%s: planes of 2^31 or more elements", who);
    const int r = st->radius, D = 2 * r + 1, n = st->ndim == 3 ? D * D * D : D * D;
    float w[9 * 9 * 9];
    for (int i = 0; i < n; ++i) {
        const double x = st->w[i];
        if (!std::isfinite(x)) return fail(SP_EINVAL, "%s: weight %d is not finite", who, i);
        int k = i, dx = k % D - r, dy, dz = 0;
        k /= D;
        dy = k % D - r;
        if (st->ndim == 3) dz = k / D - r;
        const int off_axis = (dx != 0) + (dy != 0) + (dz != 0) > 1;
        if (st->shape == SP_STAR && off_axis && x != 0.0)
            return fail(SP_EINVAL, "%s: star weights must be zero off the axes (index %d)", who, i);
        w[i] = (float)x;
    }
    sp::SuiteArgs a;
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    a.sy = g->pitch_x;
    a.sz = g->pitch_x * g->pitch_y;
    float *bufs[2] = {static_cast<float *>(u) + g->origin, static_cast<float *>(v) + g->origin};
    hipStream_t s = static_cast<hipStream_t>(stream);
    int in = 0;
    for (int k = 0; k < sweeps; ++k) {
        a.u = bufs[in];
        a.out = bufs[1 - in];
        hipError_t err = sp::launch_suite(st->shape, st->ndim, r, w, a, s);
        if (err != hipSuccess) return fail(SP_EDEVICE, "%s: launch failed: %s", who, hipGetErrorString(err));
        in = 1 - in;
    }
    *result_in = in;
    return ok();
}

int sp_stencil_apply(const sp_grid *g, const sp_coeffs *c, int sweeps, void *u, void *v,
                     int *result_in, void *stream) {
    if (int e = check_grid(g, "sp_stencil_apply")) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "sp_stencil_apply: FP32 grids only");
    if (!c || !u || !v || !result_in) return fail(SP_EINVAL, "sp_stencil_apply: NULL argument");
    if (sweeps < 0) return fail(SP_EINVAL, "sp_stencil_apply: sweeps < 0");
    if (!aligned16(u) || !aligned16(v)) return fail(SP_EINVAL, "sp_stencil_apply: pointers must be 16-byte aligned");
    if (overlaps(u, v, g->bytes)) return fail(SP_EINVAL, "sp_stencil_apply: u and v overlap");
    sp::SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    a.sy = g->pitch_x;
    a.sz = g->pitch_x * g->pitch_y;
    a.c = to_f32(c);
    sp::TileCfg t;
    if (!tiles_for(g, &t, "sp_stencil_apply", sp::MODE_APPLY)) return SP_EINVAL;
    fill_tiling(a, t);
    float *bufs[2] = {static_cast<float *>(u) + g->origin, static_cast<float *>(v) + g->origin};
    hipStream_t s = static_cast<hipStream_t>(stream);
    int in = 0;
    for (int k = 0; k < sweeps; ++k) {
        a.u = bufs[in];
        a.out = bufs[1 - in];
        hipError_t err = sp::launch_sweep(sp::MODE_APPLY, SP_F32, t, a, s);
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "sp_stencil_apply: launch failed: %s", hipGetErrorString(err));
        in = 1 - in;
    }
    *result_in = in;
    return ok();
}

int64_t sp_wave_meta_bytes(const sp_grid *g) {
    if (!g || g->dtype == SP_F32) return 0;
    const int64_t nslab = (g->nz + SP_SLAB - 1) / SP_SLAB;
    return 4 * 2 * nslab * (int64_t)sizeof(float);
}

}  // extern "C"

namespace sp {

// Validation and argument setup shared by the leapfrog entry points.
int prep_wave(const char *who, const sp_grid *g, const sp_coeffs *c, double dt, double dx,
              const sp_grid *gv, const float *v, const sp_sources *src, const sp_receivers *rec,
              sp::SweepArgs *a, sp::TileCfg *t) {
    if (int e = check_grid(g, who)) return e;
    if (int e = check_grid(gv, who)) return e;
    if (gv->dtype != SP_F32 || gv->nx != g->nx || gv->ny != g->ny || gv->nz != g->nz)
        return fail(SP_EINVAL, "%s: v must be an FP32 grid of the same shape", who);
    if (!c || !v) return fail(SP_EINVAL, "%s: NULL argument", who);
    if (!(dt > 0) || !(dx > 0)) return fail(SP_EINVAL, "%s: dt and dx must be > 0", who);
    if (!aligned16(v)) return fail(SP_EINVAL, "%s: pointers must be 16-byte aligned", who);
    // the 16-bit leapfrog addresses a plane with 32-bit byte offsets (its
    // FP32 v plane included)
    if (g->dtype != SP_F32 && gv->pitch_x * gv->pitch_y >= ((int64_t)1 << 30))
        return fail(SP_EUNSUPPORTED, "%s: FP16/BF16 storage needs planes of fewer than 2^30 elements", who);
    int nsrc = 0;
    if (src) {
        if (src->n < 0 || src->n > SP_MAX_SOURCES)
            return fail(SP_EINVAL, "%s: %d sources (max %d)", who, src->n, SP_MAX_SOURCES);
        nsrc = src->n;
        if (nsrc > 0 && !src->amp) return fail(SP_EINVAL, "%s: source amplitudes are NULL", who);
        if (nsrc > 0 && src->amp_stride < nsrc) return fail(SP_EINVAL, "%s: amp_stride < n", who);
        for (int s = 0; s < nsrc; ++s) {
            const int *p = src->xyz[s];
            if (p[0] < 0 || p[0] >= g->nx || p[1] < 0 || p[1] >= g->ny || p[2] < 0 || p[2] >= g->nz)
                return fail(SP_EINVAL, "%s: source %d outside the interior", who, s);
        }
    }
    if (rec) {
        if (rec->n < 0) return fail(SP_EINVAL, "%s: negative receiver count", who);
        if (rec->n > 0 && (!rec->xyz || !rec->traces))
            return fail(SP_EINVAL, "%s: receiver arrays are NULL", who);
        if (rec->n > 0 && rec->trace_stride < rec->n)
            return fail(SP_EINVAL, "%s: trace_stride < n", who);
    }
    if (!tiles_for(g, t, who)) return SP_EINVAL;
    std::memset(a, 0, sizeof *a);
    a->nx = g->nx;
    a->ny = g->ny;
    a->nz = g->nz;
    a->sy = g->pitch_x;
    a->sz = g->pitch_x * g->pitch_y;
    a->vsy = gv->pitch_x;
    a->vsz = gv->pitch_x * gv->pitch_y;
    a->v = v + gv->origin;
    a->m_scale = (float)((dt / dx) * (dt / dx));
    a->c = to_f32(c);
    a->src.n = nsrc;
    a->src.dt2 = (float)(dt * dt);
    for (int s = 0; s < nsrc; ++s) {
        a->src.x[s] = src->xyz[s][0];
        a->src.y[s] = src->xyz[s][1];
        a->src.z[s] = src->xyz[s][2];
    }
    fill_tiling(*a, *t);
    return SP_OK;
}

void step_args(SweepArgs &a, const sp_grid *g, void *cur, void *prev, void *out, float *meta,
               int64_t n, const float *amp, int64_t amp_stride) {
    const int64_t eb = g->elem_bytes;
    a.u = static_cast<char *>(cur) + g->origin * eb;
    a.prev = static_cast<char *>(prev) + g->origin * eb;
    a.out = static_cast<char *>(out) + g->origin * eb;
    if (meta) {
        const int nslab = (g->nz + SP_SLAB - 1) / SP_SLAB;
        auto slot = [&](int64_t k) { return meta + ((k % 4 + 4) % 4) * 2 * nslab; };
        a.meta.nslab = nslab;
        a.meta.s_u = slot(n);
        a.meta.a_u = reinterpret_cast<const uint32_t *>(slot(n) + nslab);
        a.meta.s_prev = slot(n - 1);
        a.meta.a_prev = reinterpret_cast<const uint32_t *>(slot(n - 1) + nslab);
        a.meta.s_out = slot(n + 1);
        a.meta.a_out = reinterpret_cast<uint32_t *>(slot(n + 1) + nslab);
        a.meta.s_clear = slot(n + 2);
        a.meta.a_clear = reinterpret_cast<uint32_t *>(slot(n + 2) + nslab);
    }
    if (a.src.n > 0) a.src.amp = amp + n * amp_stride;
}

}  // namespace sp

using sp::prep_wave;

extern "C" {

int sp_wave_step(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                 const float *v, sp_wave_state *st, int nsteps, const sp_sources *src,
                 const sp_receivers *rec, void *stream) {
    sp::SweepArgs a;
    sp::TileCfg t;
    if (int e = prep_wave("sp_wave_step", g, c, dt, dx, gv, v, src, rec, &a, &t)) return e;
    if (!st || !st->cur || !st->prev) return fail(SP_EINVAL, "sp_wave_step: NULL state");
    if (g->dtype == SP_F32 && st->meta) return fail(SP_EINVAL, "sp_wave_step: meta must be NULL for FP32 grids");
    if (g->dtype != SP_F32 && (!st->meta || !aligned16(st->meta)))
        return fail(SP_EINVAL, "sp_wave_step: FP16/BF16 grids need a 16-byte aligned meta block");
    if (nsteps < 0) return fail(SP_EINVAL, "sp_wave_step: nsteps < 0");
    if (!aligned16(st->cur) || !aligned16(st->prev))
        return fail(SP_EINVAL, "sp_wave_step: pointers must be 16-byte aligned");
    if (overlaps(st->cur, st->prev, g->bytes)) return fail(SP_EINVAL, "sp_wave_step: cur and prev overlap");
    if (overlaps(st->cur, g->bytes, v, gv->bytes) || overlaps(st->prev, g->bytes, v, gv->bytes))
        return fail(SP_EINVAL, "sp_wave_step: v overlaps a wavefield");
    if (st->step < 0) return fail(SP_EINVAL, "sp_wave_step: negative step counter");
    const int nsrc = a.src.n;
    const int nrec = rec ? rec->n : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t step0 = st->step;
    const int64_t eb = g->elem_bytes;
    const int nslab = (g->nz + SP_SLAB - 1) / SP_SLAB;
    float *meta = static_cast<float *>(st->meta);
    auto slot_s = [&](int64_t k) { return meta + ((k % 4 + 4) % 4) * 2 * nslab; };
    for (int k = 0; k < nsteps; ++k) {
        char *prev = static_cast<char *>(st->prev) + g->origin * eb;
        const int64_t n = st->step;
        sp::step_args(a, g, st->cur, st->prev, st->prev, meta, n, nsrc ? src->amp : nullptr,
                      nsrc ? src->amp_stride : 0);
        hipError_t err = sp::launch_sweep(sp::MODE_WAVE, g->dtype, t, a, s);
        if (err == hipSuccess && nrec > 0)
            err = sp::launch_record(g->dtype, prev, meta ? slot_s(n + 1) : nullptr, a.sy, a.sz,
                                    g->nx, g->ny, g->nz, rec->xyz, nrec,
                                    rec->traces + (st->step - step0) * rec->trace_stride, s);
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "sp_wave_step: launch failed at step %lld: %s",
                        (long long)st->step, hipGetErrorString(err));
        std::swap(st->cur, st->prev);
        st->step += 1;
    }
    return ok();
}

int sp_wave_step_fused(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                       const float *v, sp_wave_state *st, int nsteps, void **spare,
                       const sp_sources *src, const sp_receivers *rec, void *stream) {
    const char *who = "sp_wave_step_fused";
    sp::SweepArgs a;
    sp::TileCfg t;
    if (int e = prep_wave(who, g, c, dt, dx, gv, v, src, rec, &a, &t)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "%s: FP32 grids only", who);
    if (!st || !st->cur || !st->prev || st->meta) return fail(SP_EINVAL, "%s: bad state", who);
    if (!spare || !spare[0] || !spare[1]) return fail(SP_EINVAL, "%s: NULL spare field", who);
    if (nsteps < 0 || st->step < 0) return fail(SP_EINVAL, "%s: negative step count", who);
    void *f[4] = {st->cur, st->prev, spare[0], spare[1]};
    for (int i = 0; i < 4; ++i) {
        if (!aligned16(f[i])) return fail(SP_EINVAL, "%s: pointers must be 16-byte aligned", who);
        if (overlaps(f[i], v, g->bytes)) return fail(SP_EINVAL, "%s: v overlaps a wavefield", who);
        for (int j = 0; j < i; ++j)
            if (overlaps(f[i], f[j], g->bytes)) return fail(SP_EINVAL, "%s: wavefields overlap", who);
    }

    sp::TileCfg tb = sp::choose_tiles_tb2(g->nx, g->ny, g->nz);
    // Optional override for tuning: SP_TILE_FUSED=RXxRR[xZC] (region extent)
    if (const char *e = std::getenv("SP_TILE_FUSED")) {
        int rx = 0, rr = 0, zc = 0;
        const int n = std::sscanf(e, "%dx%dx%d", &rx, &rr, &zc);
        if (n >= 2) {
            tb.tx = rx;
            tb.ty = rr;
            tb.zchunk = sp::tb2_zchunk(tb, g->nx, g->ny, g->nz);
        }
        if (n == 3 && zc > 0) tb.zchunk = std::min(zc, g->nz);
    }
    if (!sp::tb2_supported(tb))
        return fail(SP_EINVAL, "%s: region %dx%d is not compiled in", who, tb.tx, tb.ty);
    sp::Tb2Args b;
    std::memset(&b, 0, sizeof b);
    b.v = a.v;
    b.nx = g->nx;
    b.ny = g->ny;
    b.nz = g->nz;
    b.sy = a.sy;
    b.sz = a.sz;
    b.vsy = a.vsy;
    b.vsz = a.vsz;
    b.m_scale = a.m_scale;
    b.c = a.c;
    b.src = a.src;
    b.tiles_x = (g->nx + tb.tx - 9) / (tb.tx - 8);
    b.tiles_y = (g->ny + tb.ty - 9) / (tb.ty - 8);
    b.zchunk = tb.zchunk;
    b.nzc = (g->nz + tb.zchunk - 1) / tb.zchunk;

    const int nsrc = a.src.n;
    const int nrec = rec ? rec->n : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t step0 = st->step;
    const int64_t org = g->origin;
    auto at = [&](void *p) { return static_cast<float *>(p) + org; };
    for (int k = 0; k + 1 < nsteps; k += 2) {
        const int64_t n = st->step;
        b.u = at(st->cur);
        b.prev = at(st->prev);
        b.out1 = at(spare[0]);
        b.out2 = at(spare[1]);
        if (nsrc) {
            b.src.amp = src->amp + n * src->amp_stride;
            b.amp1 = src->amp + (n + 1) * src->amp_stride;
        }
        hipError_t err = sp::launch_tb2(tb, b, s);
        for (int h = 0; h < 2 && err == hipSuccess && nrec > 0; ++h)
            err = sp::launch_record(SP_F32, h ? b.out2 : b.out1, nullptr, a.sy, a.sz, g->nx, g->ny,
                                    g->nz, rec->xyz, nrec,
                                    rec->traces + (n + h - step0) * rec->trace_stride, s);
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "%s: launch failed at step %lld: %s", who, (long long)n,
                        hipGetErrorString(err));
        void *old_cur = st->cur, *old_prev = st->prev;
        st->prev = spare[0];
        st->cur = spare[1];
        spare[0] = old_prev;
        spare[1] = old_cur;
        st->step += 2;
    }
    if (nsteps % 2) {
        sp_receivers r1;
        if (nrec > 0) {
            r1 = *rec;
            r1.traces = rec->traces + (st->step - step0) * rec->trace_stride;
        }
        return sp_wave_step(g, c, dt, dx, gv, v, st, 1, src, nrec > 0 ? &r1 : nullptr, stream);
    }
    return ok();
}

int sp_pml_profile(const sp_grid *gv, int width, double eta_max, float *eta, void *stream) {
    if (int e = check_grid(gv, "sp_pml_profile")) return e;
    if (gv->dtype != SP_F32) return fail(SP_EINVAL, "sp_pml_profile: eta must be an FP32 grid");
    if (!eta || !aligned16(eta)) return fail(SP_EINVAL, "sp_pml_profile: eta NULL or misaligned");
    if (width < 1) return fail(SP_EINVAL, "sp_pml_profile: width must be >= 1");
    if (!(eta_max >= 0) || !std::isfinite(eta_max))
        return fail(SP_EINVAL, "sp_pml_profile: eta_max must be finite and >= 0");
    hipError_t err = sp::launch_pml_profile(eta + gv->origin, gv->pitch_x, gv->pitch_x * gv->pitch_y,
                                            gv->nx, gv->ny, gv->nz, width, (float)eta_max,
                                            static_cast<hipStream_t>(stream));
    if (err != hipSuccess) return fail(SP_EDEVICE, "sp_pml_profile: launch failed: %s", hipGetErrorString(err));
    return ok();
}

// The shell's slabs reach the multi-box kernel as one by-value argument.
static_assert(sizeof(sp::BoxSet) <= 4096, "BoxSet exceeds the 4 KB kernel-argument limit");

int sp_wave_step_pml(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                     const float *v, sp_wave_state *st, int nsteps, const sp_pml *pml,
                     const sp_sources *src, const sp_receivers *rec, void *stream) {
    const char *who = "sp_wave_step_pml";
    sp::SweepArgs a;
    sp::TileCfg t;
    if (int e = prep_wave(who, g, c, dt, dx, gv, v, src, rec, &a, &t)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "%s: FP32 grids only", who);
    if (g->pitch_x != gv->pitch_x || g->pitch_y != gv->pitch_y || g->origin != gv->origin)
        return fail(SP_EINVAL, "%s: g and gv must have the same layout", who);
    if (!st || !st->cur || !st->prev || st->meta) return fail(SP_EINVAL, "%s: bad state", who);
    if (!pml || !pml->eta || !pml->psi) return fail(SP_EINVAL, "%s: NULL layer argument", who);
    if (nsteps < 0 || st->step < 0) return fail(SP_EINVAL, "%s: negative step count", who);
    if (!aligned16(st->cur) || !aligned16(st->prev) || !aligned16(pml->eta) || !aligned16(pml->psi))
        return fail(SP_EINVAL, "%s: pointers must be 16-byte aligned", who);
    if (overlaps(st->cur, st->prev, g->bytes)) return fail(SP_EINVAL, "%s: cur and prev overlap", who);
    for (const void *f : {static_cast<const void *>(v), static_cast<const void *>(pml->eta),
                          static_cast<const void *>(pml->psi)})
        if (overlaps(st->cur, f, g->bytes) || overlaps(st->prev, f, g->bytes))
            return fail(SP_EINVAL, "%s: a wavefield overlaps v, eta or psi", who);
    if (overlaps(pml->psi, v, g->bytes) || overlaps(pml->psi, pml->eta, g->bytes))
        return fail(SP_EINVAL, "%s: psi overlaps v or eta", who);
    if (!(pml->alpha >= 0) || !std::isfinite(pml->alpha))
        return fail(SP_EINVAL, "%s: alpha must be finite and >= 0", who);
    const int W = pml->width, nx = g->nx, ny = g->ny, nz = g->nz;
    const int dec = pml->decomposition;
    if (dec != SP_PML_UNIFIED && dec != SP_PML_SEVEN && dec != SP_PML_TWO)
        return fail(SP_EINVAL, "%s: unknown decomposition %d", who, dec);
    const bool seven = dec != SP_PML_UNIFIED;   // SEVEN and TWO share the box layout
    if (seven && (W < 4 || W % 4 != 0 || 2 * W >= nx || 2 * W >= ny || 2 * W >= nz))
        return fail(SP_EINVAL, "%s: the region maps need W %% 4 == 0, W >= 4 and 2W < n (W = %d)",
                    who, W);

    // Boxes [x0, x1) x [y0, y1) x [z0, z1), each swept by k_star25 on a
    // sub-grid whose pointers are offset to the box corner (its halo being
    // the neighbouring cells of the full grid).  x0 must stay a multiple of 4
    // (16-byte rows), so the inner box ends at a multiple of 4 and the high x
    // slab takes the remainder: its extra cells have eta = 0 and the layer
    // update reduces to the leapfrog there.
    struct Box {
        int mode;
        bool wide;                 // a z or y slab (the full x extent)
        sp::SweepArgs a;
        sp::TileCfg t;
        int64_t off;
    };
    Box boxes[7];
    int nb = 0;
    auto add = [&](int x0, int x1, int y0, int y1, int z0, int z1, int mode, bool wide) {
        Box &b = boxes[nb++];
        b.mode = mode;
        b.wide = wide;
        b.a = a;
        b.a.nx = x1 - x0;
        b.a.ny = y1 - y0;
        b.a.nz = z1 - z0;
        b.off = (int64_t)z0 * a.sz + (int64_t)y0 * a.sy + x0;
        b.a.v = a.v + b.off;
        b.a.eta = pml->eta + gv->origin + b.off;
        b.a.psi = pml->psi + g->origin + b.off;
        b.a.dt = (float)dt;
        b.a.alpha_dt = (float)(pml->alpha * dt);
        for (int q = 0; q < b.a.src.n; ++q) {   // sources outside the box never match a point
            b.a.src.x[q] -= x0;
            b.a.src.y[q] -= y0;
            b.a.src.z[q] -= z0;
        }
        b.t = sp::choose_tiles(b.a.nx, b.a.ny, b.a.nz, SP_F32, mode);
        if (dec == SP_PML_TWO && mode == sp::MODE_PML) {
            // the shell as one launch of 512-thread blocks (one per CU):
            // the z and y slabs on 256x8x1 tiles, the x slabs on 32x64x1
            b.t.tx = wide ? 256 : 32;
            b.t.ty = wide ? 8 : 64;
            b.t.ry = 1;
            b.t.zchunk = sp::occupancy_zchunk((int64_t)((b.a.nx + b.t.tx - 1) / b.t.tx) *
                                                  ((b.a.ny + b.t.ty - 1) / b.t.ty),
                                              b.a.nz, 256);
        }
        fill_tiling(b.a, b.t);
    };
    if (!seven) {
        add(0, nx, 0, ny, 0, nz, sp::MODE_PML, true);
    } else {
        const int xe = W + 4 * ((nx - 2 * W) / 4);
        add(W, xe, W, ny - W, W, nz - W, sp::MODE_WAVE, true);
        add(0, nx, 0, ny, 0, W, sp::MODE_PML, true);
        add(0, nx, 0, ny, nz - W, nz, sp::MODE_PML, true);
        add(0, nx, 0, W, W, nz - W, sp::MODE_PML, true);
        add(0, nx, ny - W, ny, W, nz - W, sp::MODE_PML, true);
        add(0, W, W, ny - W, W, nz - W, sp::MODE_PML, false);
        add(xe, nx, W, ny - W, W, nz - W, sp::MODE_PML, false);
    }
    const int nrec = rec ? rec->n : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t step0 = st->step;
    for (int k = 0; k < nsteps; ++k) {
        const int64_t n = st->step;
        float *cur = static_cast<float *>(st->cur) + g->origin;
        float *prev = static_cast<float *>(st->prev) + g->origin;
        const float *amp = a.src.n ? src->amp + n * src->amp_stride : nullptr;
        hipError_t err = hipSuccess;
        for (int q = 0; q < nb; ++q) {
            Box &b = boxes[q];
            b.a.u = cur + b.off;
            b.a.prev = prev + b.off;
            b.a.out = prev + b.off;
            b.a.src.amp = amp;
        }
        if (dec == SP_PML_TWO) {
            // inner box, then the six slabs of the shell in one launch
            err = sp::launch_sweep(boxes[0].mode, SP_F32, boxes[0].t, boxes[0].a, s);
            sp::BoxSet shell;
            shell.n = nb - 1;
            shell.first[0] = 0;
            for (int q = 1; q < nb; ++q) {
                const sp::SweepArgs &ba = boxes[q].a;
                shell.a[q - 1] = ba;
                shell.wide[q - 1] = boxes[q].wide ? 1 : 0;
                shell.first[q] = shell.first[q - 1] + ba.tiles_x * ba.tiles_y * ba.nzc;
            }
            if (err == hipSuccess) err = sp::launch_sweep_boxes(sp::MODE_PML, shell, s);
        } else {
            for (int q = 0; q < nb && err == hipSuccess; ++q)
                err = sp::launch_sweep(boxes[q].mode, SP_F32, boxes[q].t, boxes[q].a, s);
        }
        if (err == hipSuccess && nrec > 0)
            err = sp::launch_record(SP_F32, prev, nullptr, a.sy, a.sz, nx, ny, nz, rec->xyz, nrec,
                                    rec->traces + (n - step0) * rec->trace_stride, s);
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "%s: launch failed at step %lld: %s", who, (long long)n,
                        hipGetErrorString(err));
        std::swap(st->cur, st->prev);
        st->step += 1;
    }
    return ok();
}

int sp_wave_run_states(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                       const sp_grid *gv, const float *v, void *const *states, int64_t n0,
                       int nsteps, const sp_sources *src, const sp_receivers *rec, void *stream) {
    sp::SweepArgs a;
    sp::TileCfg t;
    if (int e = prep_wave("sp_wave_run_states", g, c, dt, dx, gv, v, src, rec, &a, &t)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "sp_wave_run_states: FP32 grids only");
    if (nsteps < 0 || n0 < 0) return fail(SP_EINVAL, "sp_wave_run_states: negative nsteps or n0");
    if (!states) return fail(SP_EINVAL, "sp_wave_run_states: states is NULL");
    for (int i = 0; i < nsteps + 2; ++i) {
        if (!states[i] || !aligned16(states[i]))
            return fail(SP_EINVAL, "sp_wave_run_states: state %d NULL or misaligned", i);
        if (overlaps(states[i], v, g->bytes)) return fail(SP_EINVAL, "sp_wave_run_states: v overlaps a state");
        for (int j = (i > 2 ? i - 2 : 0); j < i; ++j)
            if (overlaps(states[i], states[j], g->bytes))
                return fail(SP_EINVAL, "sp_wave_run_states: states %d and %d overlap", j, i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nrec = rec ? rec->n : 0;
    for (int i = 0; i < nsteps; ++i) {
        a.prev = static_cast<const float *>(states[i]) + g->origin;
        a.u = static_cast<const float *>(states[i + 1]) + g->origin;
        float *out = static_cast<float *>(states[i + 2]) + g->origin;
        a.out = out;
        if (a.src.n > 0) a.src.amp = src->amp + (n0 + i) * src->amp_stride;
        hipError_t err = sp::launch_sweep(sp::MODE_WAVE, SP_F32, t, a, s);
        if (err == hipSuccess && nrec > 0)
            err = sp::launch_record(SP_F32, out, nullptr, a.sy, a.sz, g->nx, g->ny, g->nz,
                                    rec->xyz, nrec, rec->traces + i * rec->trace_stride, s);
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "sp_wave_run_states: launch failed: %s", hipGetErrorString(err));
    }
    return ok();
}

int sp_wave_adjoint_step(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                         const sp_grid *gv, const float *v, sp_wave_state *adj,
                         const void *const *u_hist, int nsteps, const sp_sources *src,
                         const sp_receivers *rec, double *G, void *stream) {
    sp::SweepArgs a;
    sp::TileCfg t;
    if (int e = prep_wave("sp_wave_adjoint_step", g, c, dt, dx, gv, v, src, rec, &a, &t)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "sp_wave_adjoint_step: FP32 grids only");
    if (!adj || !adj->cur || !adj->prev || !G || !u_hist)
        return fail(SP_EINVAL, "sp_wave_adjoint_step: NULL argument");
    if (adj->meta) return fail(SP_EINVAL, "sp_wave_adjoint_step: meta must be NULL");
    if (nsteps < 0) return fail(SP_EINVAL, "sp_wave_adjoint_step: nsteps < 0");
    if (adj->step < nsteps) return fail(SP_EINVAL, "sp_wave_adjoint_step: step counter below 1");
    if (!aligned16(adj->cur) || !aligned16(adj->prev) || (reinterpret_cast<uintptr_t>(G) & 31u))
        return fail(SP_EINVAL, "sp_wave_adjoint_step: misaligned pointer");
    if (overlaps(adj->cur, adj->prev, g->bytes)) return fail(SP_EINVAL, "sp_wave_adjoint_step: adjoint fields overlap");
    for (int i = 0; i < nsteps; ++i) {
        if (!u_hist[i] || !aligned16(u_hist[i]))
            return fail(SP_EINVAL, "sp_wave_adjoint_step: u_hist[%d] NULL or misaligned", i);
        if (overlaps(u_hist[i], adj->cur, g->bytes) || overlaps(u_hist[i], adj->prev, g->bytes))
            return fail(SP_EINVAL, "sp_wave_adjoint_step: u_hist[%d] overlaps an adjoint field", i);
    }
    const int nrec = rec ? rec->n : 0;
    const sp::SrcList fwd_src = a.src;      // forward sources: gradient term only
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float inj_scale = (float)((dt / dx) * (dt / dx));   // m g = dt^2 v^2 g / dx^2
    // One fused sweep per step (propagation and gradient, two register
    // queues per thread) plus a receiver kernel, on one-row tiles; the tile
    // override may name a configuration without it, which then takes three
    // launches (propagation, receivers, gradient sweep).
    sp::TileCfg tf;
    if (!tiles_for(g, &tf, "sp_wave_adjoint_step", sp::MODE_ADJ)) return SP_EINVAL;
    if (tf.ry == 1 && tf.tx * tf.ty / 4 <= 512) {
        sp::SweepArgs fa = a;
        fill_tiling(fa, tf);
        fa.src = fwd_src;
        fa.dx2 = (float)(dx * dx);
        fa.gacc = G + g->origin;
        for (int i = 0; i < nsteps; ++i) {
            const int64_t k = adj->step;
            fa.u = static_cast<float *>(adj->cur) + g->origin;       // nu^{k+1}
            fa.prev = static_cast<float *>(adj->prev) + g->origin;   // nu^{k+2} -> nu^k
            fa.out = const_cast<void *>(fa.prev);
            fa.u2 = static_cast<const float *>(u_hist[i]) + g->origin;
            if (fa.src.n > 0) fa.src.amp = src->amp + (k - 1) * src->amp_stride;
            hipError_t err = sp::launch_sweep(sp::MODE_ADJ, SP_F32, tf, fa, s);
            if (err == hipSuccess && nrec > 0)
                err = sp::launch_inject_grad(fa, rec->xyz, nrec, rec->traces + (k - 1) * rec->trace_stride,
                                             inj_scale, s);
            if (err != hipSuccess)
                return fail(SP_EDEVICE, "sp_wave_adjoint_step: launch failed at k=%lld: %s",
                            (long long)k, hipGetErrorString(err));
            std::swap(adj->cur, adj->prev);
            adj->step -= 1;
        }
        return ok();
    }
    for (int i = 0; i < nsteps; ++i) {
        const int64_t k = adj->step;
        float *nu1 = static_cast<float *>(adj->cur) + g->origin;    // nu^{k+1}
        float *nu2 = static_cast<float *>(adj->prev) + g->origin;   // nu^{k+2} -> nu^k
        a.src.n = 0;
        a.u = nu1;
        a.prev = nu2;
        a.out = nu2;
        hipError_t err = sp::launch_sweep(sp::MODE_WAVE, SP_F32, t, a, s);
        if (err == hipSuccess && nrec > 0)
            err = sp::launch_inject(nu2, a.sy, a.sz, a.v, a.vsy, a.vsz, g->nx, g->ny, g->nz,
                                    rec->xyz, nrec, rec->traces + (k - 1) * rec->trace_stride,
                                    inj_scale, s);
        if (err == hipSuccess) {
            sp::SweepArgs ga = a;
            ga.src = fwd_src;
            if (ga.src.n > 0) ga.src.amp = src->amp + (k - 1) * src->amp_stride;
            ga.u = static_cast<const float *>(u_hist[i]) + g->origin;
            ga.prev = nu2;
            ga.out = nullptr;
            ga.gacc = G + g->origin;
            ga.dx2 = (float)(dx * dx);
            err = sp::launch_sweep(sp::MODE_GRAD, SP_F32, t, ga, s);
        }
        if (err != hipSuccess)
            return fail(SP_EDEVICE, "sp_wave_adjoint_step: launch failed at k=%lld: %s",
                        (long long)k, hipGetErrorString(err));
        std::swap(adj->cur, adj->prev);
        adj->step -= 1;
    }
    return ok();
}

int sp_grad_finish(const sp_grid *gv, const float *v, const double *G, float *out, void *stream) {
    if (int e = check_grid(gv, "sp_grad_finish")) return e;
    if (gv->dtype != SP_F32) return fail(SP_EINVAL, "sp_grad_finish: v must be an FP32 grid");
    if (!v || !G || !out) return fail(SP_EINVAL, "sp_grad_finish: NULL argument");
    if (overlaps(out, v, gv->bytes)) return fail(SP_EINVAL, "sp_grad_finish: out overlaps v");
    hipError_t err = sp::launch_grad_finish(G + gv->origin, v + gv->origin, out + gv->origin,
                                            gv->pitch_x, gv->pitch_x * gv->pitch_y, gv->nx,
                                            gv->ny, gv->nz, static_cast<hipStream_t>(stream));
    if (err != hipSuccess) return fail(SP_EDEVICE, "sp_grad_finish: %s", hipGetErrorString(err));
    return ok();
}

int sp_decode(const sp_grid *g, const void *field, const void *meta, int64_t k, float *out,
              void *stream) {
    if (int e = check_grid(g, "sp_decode")) return e;
    if (!field || !out) return fail(SP_EINVAL, "sp_decode: NULL argument");
    const float *scale = nullptr;
    if (g->dtype != SP_F32) {
        if (!meta) return fail(SP_EINVAL, "sp_decode: FP16/BF16 fields need their slab records");
        const int64_t nslab = (g->nz + SP_SLAB - 1) / SP_SLAB;
        scale = static_cast<const float *>(meta) + ((k % 4 + 4) % 4) * 2 * nslab;
    }
    const int64_t n = (int64_t)g->nx * g->ny * g->nz;
    const auto f0 = reinterpret_cast<uintptr_t>(field), o0 = reinterpret_cast<uintptr_t>(out);
    if (o0 < f0 + (uintptr_t)g->bytes && f0 < o0 + (uintptr_t)(n * (int64_t)sizeof(float)))
        return fail(SP_EINVAL, "sp_decode: out overlaps the field");
    hipError_t err = sp::launch_unpack(g->dtype, static_cast<const char *>(field) + g->origin * g->elem_bytes,
                                       scale, out, g->pitch_x, g->pitch_x * g->pitch_y, g->nx, g->ny,
                                       g->nz, static_cast<hipStream_t>(stream));
    if (err != hipSuccess) return fail(SP_EDEVICE, "sp_decode: %s", hipGetErrorString(err));
    return ok();
}

}  // extern "C"

namespace {

// Validation and arguments shared by the two energy entry points.
int energy_prep(const char *who, const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                const sp_grid *gv, const float *v, const void *u0, const void *u1, double *out,
                sp::SweepArgs *a, sp::TileCfg *t, int *nblk) {
    if (int e = prep_wave(who, g, c, dt, dx, gv, v, nullptr, nullptr, a, t)) return e;
    if (g->dtype != SP_F32) return fail(SP_EUNSUPPORTED, "%s: FP32 grids only", who);
    if (!u0 || !u1 || !out) return fail(SP_EINVAL, "%s: NULL argument", who);
    if (!aligned16(u0) || !aligned16(u1) || (reinterpret_cast<uintptr_t>(out) & 7u))
        return fail(SP_EINVAL, "%s: misaligned pointer", who);
    a->u = static_cast<const float *>(u0) + g->origin;
    a->prev = static_cast<const float *>(u1) + g->origin;
    *nblk = a->tiles_x * a->tiles_y * a->nzc;
    return SP_OK;
}

// MODE_ENERGY sweep writing one FP64 partial per block into `partial`, then
// their sum in block order into *out.  Every partial is written before it
// is read, so `partial` needs no clearing.
int energy_launch(const char *who, sp::SweepArgs &a, const sp::TileCfg &t, int nblk,
                  double *partial, double *out, void *stream) {
    a.gacc = partial;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err = sp::launch_sweep(sp::MODE_ENERGY, SP_F32, t, a, s);
    if (err == hipSuccess) err = sp::launch_sum(partial, nblk, out, s);
    if (err != hipSuccess) return fail(SP_EDEVICE, "%s: %s", who, hipGetErrorString(err));
    return ok();
}

// The allocation-free energy keeps its per-block partial sums in this
// file-scope device array instead of a caller workspace.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// the name `scratch` is only a stand-in for the symbol: its device address
// is looked up once per device (scratch_for_device) and used instead.
constexpr int kScratchPartials = 1 << 16;   // 512 KiB of FP64 partial sums
static __device__ __align__(256) double scratch[kScratchPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];         // device address of `scratch`, per device

// Device address of the current device's `scratch`; the stream must belong
// to the current device (the launch and the address must agree).
int scratch_for_device(const char *who, void *stream, double **out) {
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return fail(SP_EDEVICE, "%s: %s", who, hipGetErrorString(err));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SP_EUNSUPPORTED, "%s: device ordinal %d (max %d)", who, dev, kMaxDevices - 1);
    if (stream) {
        hipDevice_t sdev = -1;
        err = hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev);
        if (err != hipSuccess) return fail(SP_EDEVICE, "%s: %s", who, hipGetErrorString(err));
        if (sdev != dev)
            return fail(SP_EINVAL, "%s: the stream belongs to device %d, the current device is %d",
                        who, (int)sdev, dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p)
            return fail(SP_EDEVICE, "%s: no device address for the scratch array: %s", who,
                        hipGetErrorString(err));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SP_OK;
}

}  // namespace

extern "C" {

int64_t sp_energy_ws_bytes(const sp_grid *g) {
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return 0;
    // upper bound over every compiled tile shape (smallest: 64 x 8) and z-chunk
    return (int64_t)((g->nx + 63) / 64) * ((g->ny + 7) / 8) * g->nz * (int64_t)sizeof(double);
}

int sp_energy(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
              const float *v, const void *u0, const void *u1, double *out, void *ws, void *stream) {
    sp::SweepArgs a;
    sp::TileCfg t;
    int nblk = 0;
    if (int e = energy_prep("sp_energy", g, c, dt, dx, gv, v, u0, u1, out, &a, &t, &nblk)) return e;
    if (!ws) return fail(SP_EINVAL, "sp_energy: NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return fail(SP_EINVAL, "sp_energy: misaligned pointer");
    if ((int64_t)nblk * 8 > sp_energy_ws_bytes(g)) return fail(SP_ENOMEM, "sp_energy: workspace too small");
    return energy_launch("sp_energy", a, t, nblk, static_cast<double *>(ws), out, stream);
}

int64_t sp_energy_noalloc_max_partials(void) { return kScratchPartials; }

int sp_energy_noalloc(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                      const float *v, const void *u0, const void *u1, double *out, void *stream) {
    sp::SweepArgs a;
    sp::TileCfg t;
    int nblk = 0;
    const char *who = "sp_energy_noalloc";
    if (int e = energy_prep(who, g, c, dt, dx, gv, v, u0, u1, out, &a, &t, &nblk)) return e;
    if (nblk > kScratchPartials)
        return fail(SP_ENOMEM, "%s: the sweep needs %d partial sums, the static scratch holds %d",
                    who, nblk, kScratchPartials);
    double *partial = nullptr;
    if (int e = scratch_for_device(who, stream, &partial)) return e;
    return energy_launch(who, a, t, nblk, partial, out, stream);
}

}  // extern "C"
