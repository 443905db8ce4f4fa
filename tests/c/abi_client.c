/*
 * A plain C99 client of libstencil.  It includes nothing but the library's
 * header and the C API of the HIP runtime, allocates its own device fields,
 * and exchanges raw little-endian arrays with the caller through files.
 *
 *   abi_client host
 *       checks that need no GPU: version string, grid layout, argument
 *       validation and error messages.
 *   abi_client apply NX NY NZ SWEEPS IN_F32 COEFFS_F64 OUT_F32
 *       SWEEPS sweeps of the 25-point star (Eq. 3) on the interior read from
 *       IN_F32 (NZ x NY x NX, x fastest) with a zero halo; writes the
 *       interior of the grid that holds the result.
 *   abi_client wave NX NY NZ NSTEPS DT DX V_F32 COEFFS_F64 SX SY SZ AMP_F32 OUT_F32
 *       NSTEPS leapfrog steps (Eq. 2) from zero fields with one point source
 *       at (SX, SY, SZ) whose amplitude for step n is AMP_F32[n]; writes the
 *       interior of u^NSTEPS.
 *
 * COEFFS_F64 holds 13 doubles: the centre weight, then ax[4], ay[4], az[4].
 * Exit status 0 on success; any failure prints its reason and exits 1.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "stencil.h"

static int fail(const char *what, const char *why) {
    fprintf(stderr, "abi_client: %s: %s\n", what, why);
    return 1;
}

#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) return fail(what, sp_last_error());    \
    } while (0)

#define HIPCHECK(call)                                                  \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return fail(#call, hipGetErrorString(e_)); \
    } while (0)

static int read_file(const char *path, void *dst, size_t bytes) {
    FILE *f = fopen(path, "rb");
    size_t got;
    if (!f) return 0;
    got = fread(dst, 1, bytes, f);
    fclose(f);
    return got == bytes;
}

static int write_file(const char *path, const void *src, size_t bytes) {
    FILE *f = fopen(path, "wb");
    size_t put;
    if (!f) return 0;
    put = fwrite(src, 1, bytes, f);
    return fclose(f) == 0 && put == bytes;
}

static int read_coeffs(const char *path, sp_coeffs *c) {
    double w[13];
    int m;
    if (!read_file(path, w, sizeof w)) return 0;
    c->center = w[0];
    for (m = 0; m < 4; ++m) {
        c->ax[m] = w[1 + m];
        c->ay[m] = w[5 + m];
        c->az[m] = w[9 + m];
    }
    return 1;
}

/* element offset of interior cell (x, y, z) */
static int64_t cell(const sp_grid *g, int x, int y, int z) {
    return g->origin + ((int64_t)z * g->pitch_y + y) * g->pitch_x + x;
}

/* padded host image of a field: zero halo, interior from `in` */
static float *pad(const sp_grid *g, const float *in) {
    float *h = (float *)calloc((size_t)g->elems, sizeof(float));
    int x, y, z;
    if (!h) return NULL;
    for (z = 0; z < g->nz; ++z)
        for (y = 0; y < g->ny; ++y)
            for (x = 0; x < g->nx; ++x)
                h[cell(g, x, y, z)] = in[((size_t)z * g->ny + y) * g->nx + x];
    return h;
}

static void unpad(const sp_grid *g, const float *h, float *out) {
    int x, y, z;
    for (z = 0; z < g->nz; ++z)
        for (y = 0; y < g->ny; ++y)
            for (x = 0; x < g->nx; ++x)
                out[((size_t)z * g->ny + y) * g->nx + x] = h[cell(g, x, y, z)];
}

static int host_checks(void) {
    sp_grid g, h;
    sp_coeffs c;
    int where = -1;
    memset(&c, 0, sizeof c);
    CHECK(strncmp(sp_version(), "libstencil", 10) == 0, "sp_version");
    CHECK(sp_grid_init(70, 37, 23, SP_HALO, SP_F32, &g) == SP_OK, "sp_grid_init");
    CHECK(g.nx == 70 && g.ny == 37 && g.nz == 23 && g.elem_bytes == 4, "grid sizes");
    CHECK(g.pitch_y == 37 + 8 && g.planes == 23 + 8, "grid pitches");
    CHECK((g.origin * 4) % 128 == 0 && (g.pitch_x * 4) % 128 == 0, "row alignment");
    CHECK(g.bytes % 256 == 0 && g.bytes >= g.elems * 4, "grid bytes");
    CHECK(cell(&g, 0, 0, 0) - 4 * g.pitch_y * g.pitch_x - 4 * g.pitch_x - 4 >= 0, "halo origin");
    CHECK(sp_grid_init(70, 37, 23, SP_HALO, SP_F16, &h) == SP_OK && h.elem_bytes == 2, "FP16 grid");
    CHECK(sp_grid_init(70, 37, 23, 3, SP_F32, &h) == SP_EINVAL, "halo 3 refused");
    CHECK(sp_last_error()[0] != '\0', "message after a refusal");
    CHECK(sp_grid_init(0, 37, 23, SP_HALO, SP_F32, &h) == SP_EINVAL, "empty grid refused");
    CHECK(sp_stencil_apply(&g, &c, 1, NULL, NULL, &where, NULL) == SP_EINVAL, "NULL fields refused");
    CHECK(where == -1, "result flag untouched by a refused call");
    CHECK(sp_wave_meta_bytes(&g) == 0, "no metadata for FP32");
    printf("host ok\n");
    return 0;
}

static int run_apply(int argc, char **argv) {
    sp_grid g;
    sp_coeffs c;
    int nx, ny, nz, sweeps, where = -1;
    size_t n;
    float *in, *out, *h;
    void *u = NULL, *v = NULL;
    if (argc != 9) return fail("apply", "expected NX NY NZ SWEEPS IN COEFFS OUT");
    nx = atoi(argv[2]);
    ny = atoi(argv[3]);
    nz = atoi(argv[4]);
    sweeps = atoi(argv[5]);
    CHECK(sp_grid_init(nx, ny, nz, SP_HALO, SP_F32, &g) == SP_OK, "sp_grid_init");
    n = (size_t)nx * ny * nz;
    in = (float *)malloc(n * sizeof(float));
    out = (float *)malloc(n * sizeof(float));
    if (!in || !out) return fail("apply", "out of host memory");
    if (!read_file(argv[6], in, n * sizeof(float))) return fail("apply", "cannot read the input field");
    if (!read_coeffs(argv[7], &c)) return fail("apply", "cannot read the coefficients");
    h = pad(&g, in);
    if (!h) return fail("apply", "out of host memory");
    HIPCHECK(hipMalloc(&u, (size_t)g.bytes));
    HIPCHECK(hipMalloc(&v, (size_t)g.bytes));
    HIPCHECK(hipMemset(v, 0, (size_t)g.bytes));
    HIPCHECK(hipMemcpy(u, h, (size_t)(g.elems * 4), hipMemcpyHostToDevice));
    CHECK(sp_stencil_apply(&g, &c, sweeps, u, v, &where, NULL) == SP_OK, "sp_stencil_apply");
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(h, where ? v : u, (size_t)(g.elems * 4), hipMemcpyDeviceToHost));
    unpad(&g, h, out);
    if (!write_file(argv[8], out, n * sizeof(float))) return fail("apply", "cannot write the output");
    HIPCHECK(hipFree(u));
    HIPCHECK(hipFree(v));
    free(h);
    free(in);
    free(out);
    printf("apply ok: %d sweeps, result in %s\n", sweeps, where ? "v" : "u");
    return 0;
}

static int run_wave(int argc, char **argv) {
    sp_grid g;
    sp_coeffs c;
    sp_sources src;
    sp_wave_state st;
    int nx, ny, nz, nsteps;
    double dt, dx;
    size_t n;
    float *vin, *amp_h, *out, *h;
    void *a = NULL, *b = NULL, *vf = NULL, *amp = NULL;
    if (argc != 15) return fail("wave", "expected NX NY NZ NSTEPS DT DX V COEFFS SX SY SZ AMP OUT");
    nx = atoi(argv[2]);
    ny = atoi(argv[3]);
    nz = atoi(argv[4]);
    nsteps = atoi(argv[5]);
    dt = atof(argv[6]);
    dx = atof(argv[7]);
    CHECK(sp_grid_init(nx, ny, nz, SP_HALO, SP_F32, &g) == SP_OK, "sp_grid_init");
    n = (size_t)nx * ny * nz;
    vin = (float *)malloc(n * sizeof(float));
    out = (float *)malloc(n * sizeof(float));
    amp_h = (float *)malloc((size_t)(nsteps > 0 ? nsteps : 1) * sizeof(float));
    if (!vin || !out || !amp_h) return fail("wave", "out of host memory");
    if (!read_file(argv[8], vin, n * sizeof(float))) return fail("wave", "cannot read the velocity");
    if (!read_coeffs(argv[9], &c)) return fail("wave", "cannot read the coefficients");
    if (!read_file(argv[13], amp_h, (size_t)nsteps * sizeof(float))) return fail("wave", "cannot read the amplitudes");
    memset(&src, 0, sizeof src);
    src.n = 1;
    src.xyz[0][0] = atoi(argv[10]);
    src.xyz[0][1] = atoi(argv[11]);
    src.xyz[0][2] = atoi(argv[12]);
    src.amp_stride = 1;
    h = pad(&g, vin);
    if (!h) return fail("wave", "out of host memory");
    HIPCHECK(hipMalloc(&a, (size_t)g.bytes));
    HIPCHECK(hipMalloc(&b, (size_t)g.bytes));
    HIPCHECK(hipMalloc(&vf, (size_t)g.bytes));
    HIPCHECK(hipMalloc(&amp, (size_t)(nsteps > 0 ? nsteps : 1) * sizeof(float)));
    HIPCHECK(hipMemset(a, 0, (size_t)g.bytes));
    HIPCHECK(hipMemset(b, 0, (size_t)g.bytes));
    HIPCHECK(hipMemcpy(vf, h, (size_t)(g.elems * 4), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(amp, amp_h, (size_t)nsteps * sizeof(float), hipMemcpyHostToDevice));
    src.amp = (const float *)amp;
    st.cur = b;
    st.prev = a;
    st.meta = NULL;
    st.step = 0;
    CHECK(sp_wave_step(&g, &c, dt, dx, &g, (const float *)vf, &st, nsteps, &src, NULL, NULL) == SP_OK,
          "sp_wave_step");
    CHECK(st.step == nsteps, "step counter");
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(h, st.cur, (size_t)(g.elems * 4), hipMemcpyDeviceToHost));
    unpad(&g, h, out);
    if (!write_file(argv[14], out, n * sizeof(float))) return fail("wave", "cannot write the output");
    HIPCHECK(hipFree(a));
    HIPCHECK(hipFree(b));
    HIPCHECK(hipFree(vf));
    HIPCHECK(hipFree(amp));
    free(h);
    free(vin);
    free(out);
    free(amp_h);
    printf("wave ok: %d steps\n", nsteps);
    return 0;
}

int main(int argc, char **argv) {
    if (argc >= 2 && strcmp(argv[1], "host") == 0) return host_checks();
    if (argc >= 2 && strcmp(argv[1], "apply") == 0) return run_apply(argc, argv);
    if (argc >= 2 && strcmp(argv[1], "wave") == 0) return run_wave(argc, argv);
    return fail("usage", "abi_client host | apply ... | wave ...");
}
