// C-ABI of libstencil: argument validation, grid layout and launch sequencing.
// Every entry point validates before enqueueing anything and reports errors
// through a status code plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace {

thread_local char g_err[512] = "";

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

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_grid(const sp_grid *g, const char *what) {
    if (!g) return fail(SP_EINVAL, "%s: grid descriptor is NULL", what);
    sp_grid ref;
    if (sp_grid_init(g->nx, g->ny, g->nz, g->halo, g->dtype, &ref) != SP_OK)
        return fail(SP_EINVAL, "%s: invalid grid descriptor (%s)", what, sp_last_error());
    if (std::memcmp(&ref, g, sizeof ref) != 0)
        return fail(SP_EINVAL, "%s: grid descriptor was not produced by sp_grid_init", what);
    return SP_OK;
}

bool overlaps(const void *a, const void *b, int64_t bytes) {
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)bytes && y < x + (uintptr_t)bytes;
}

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
bool tiles_for(const sp_grid *g, sp::TileCfg *out, const char *who) {
    sp::TileCfg t = sp::choose_tiles(g->nx, g->ny, g->nz);
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
    if (!sp::tile_supported(t)) {
        fail(SP_EINVAL, "%s: tile configuration %dx%dx%d is not compiled in", who, t.tx, t.ty, t.ry);
        return false;
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
    if (!tiles_for(g, &t, "sp_stencil_apply")) return SP_EINVAL;
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

int sp_wave_step(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                 const float *v, sp_wave_state *st, int nsteps, const sp_sources *src,
                 const sp_receivers *rec, void *stream) {
    if (int e = check_grid(g, "sp_wave_step")) return e;
    if (int e = check_grid(gv, "sp_wave_step(v)")) return e;
    if (gv->dtype != SP_F32 || gv->nx != g->nx || gv->ny != g->ny || gv->nz != g->nz)
        return fail(SP_EINVAL, "sp_wave_step: v must be an FP32 grid of the same shape");
    if (!c || !v || !st || !st->cur || !st->prev) return fail(SP_EINVAL, "sp_wave_step: NULL argument");
    if (g->dtype == SP_F32 && st->meta) return fail(SP_EINVAL, "sp_wave_step: meta must be NULL for FP32 grids");
    if (g->dtype != SP_F32 && (!st->meta || !aligned16(st->meta)))
        return fail(SP_EINVAL, "sp_wave_step: FP16/BF16 grids need a 16-byte aligned meta block");
    if (nsteps < 0) return fail(SP_EINVAL, "sp_wave_step: nsteps < 0");
    if (!(dt > 0) || !(dx > 0)) return fail(SP_EINVAL, "sp_wave_step: dt and dx must be > 0");
    if (!aligned16(st->cur) || !aligned16(st->prev) || !aligned16(v))
        return fail(SP_EINVAL, "sp_wave_step: pointers must be 16-byte aligned");
    if (overlaps(st->cur, st->prev, g->bytes)) return fail(SP_EINVAL, "sp_wave_step: cur and prev overlap");
    if (overlaps(st->cur, v, g->bytes) || overlaps(st->prev, v, g->bytes))
        return fail(SP_EINVAL, "sp_wave_step: v overlaps a wavefield");
    if (st->step < 0) return fail(SP_EINVAL, "sp_wave_step: negative step counter");
    int nsrc = 0;
    if (src) {
        if (src->n < 0 || src->n > SP_MAX_SOURCES)
            return fail(SP_EINVAL, "sp_wave_step: %d sources (max %d)", src->n, SP_MAX_SOURCES);
        nsrc = src->n;
        if (nsrc > 0 && !src->amp) return fail(SP_EINVAL, "sp_wave_step: source amplitudes are NULL");
        if (nsrc > 0 && src->amp_stride < nsrc) return fail(SP_EINVAL, "sp_wave_step: amp_stride < n");
        for (int s = 0; s < nsrc; ++s) {
            const int *p = src->xyz[s];
            if (p[0] < 0 || p[0] >= g->nx || p[1] < 0 || p[1] >= g->ny || p[2] < 0 || p[2] >= g->nz)
                return fail(SP_EINVAL, "sp_wave_step: source %d outside the interior", s);
        }
    }
    int nrec = 0;
    if (rec) {
        if (rec->n < 0) return fail(SP_EINVAL, "sp_wave_step: negative receiver count");
        nrec = rec->n;
        if (nrec > 0 && (!rec->xyz || !rec->traces)) return fail(SP_EINVAL, "sp_wave_step: receiver arrays are NULL");
        if (nrec > 0 && rec->trace_stride < nrec) return fail(SP_EINVAL, "sp_wave_step: trace_stride < n");
    }

    sp::SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    a.sy = g->pitch_x;
    a.sz = g->pitch_x * g->pitch_y;
    a.vsy = gv->pitch_x;
    a.vsz = gv->pitch_x * gv->pitch_y;
    a.v = v + gv->origin;
    a.m_scale = (float)((dt / dx) * (dt / dx));
    a.c = to_f32(c);
    a.src.n = nsrc;
    a.src.dt2 = (float)(dt * dt);
    for (int s = 0; s < nsrc; ++s) {
        a.src.x[s] = src->xyz[s][0];
        a.src.y[s] = src->xyz[s][1];
        a.src.z[s] = src->xyz[s][2];
    }
    sp::TileCfg t;
    if (!tiles_for(g, &t, "sp_wave_step")) return SP_EINVAL;
    fill_tiling(a, t);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t step0 = st->step;
    const int64_t eb = g->elem_bytes;
    const int nslab = (g->nz + SP_SLAB - 1) / SP_SLAB;
    float *meta = static_cast<float *>(st->meta);
    auto slot_s = [&](int64_t k) { return meta + ((k % 4 + 4) % 4) * 2 * nslab; };
    auto slot_a = [&](int64_t k) {
        return reinterpret_cast<uint32_t *>(meta + ((k % 4 + 4) % 4) * 2 * nslab + nslab);
    };
    for (int k = 0; k < nsteps; ++k) {
        char *cur = static_cast<char *>(st->cur) + g->origin * eb;
        char *prev = static_cast<char *>(st->prev) + g->origin * eb;
        a.u = cur;
        a.prev = prev;
        a.out = prev;
        const int64_t n = st->step;
        if (meta) {
            a.meta.nslab = nslab;
            a.meta.s_u = slot_s(n);
            a.meta.a_u = slot_a(n);
            a.meta.s_prev = slot_s(n - 1);
            a.meta.a_prev = slot_a(n - 1);
            a.meta.s_out = slot_s(n + 1);
            a.meta.a_out = slot_a(n + 1);
            a.meta.s_clear = slot_s(n + 2);
            a.meta.a_clear = slot_a(n + 2);
        }
        if (nsrc > 0) a.src.amp = src->amp + st->step * src->amp_stride;
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

}  // extern "C"
