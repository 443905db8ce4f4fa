/*
 * FP64 CPU oracle for the 25-point star stencil and the acoustic leapfrog.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the GPU library.
 *
 * Layout: every field is a dense FP64 array of (nz+8) x (ny+8) x (nx+8)
 * values, x fastest, with a 4-cell frame (the halo) on every face.  Interior
 * point (x, y, z), 0 <= x < nx etc., lives at index
 *     ((z+4) * (ny+8) + (y+4)) * (nx+8) + (x+4).
 * The halo holds the boundary values (zero for the Dirichlet problems); the
 * oracle reads it and never writes it.
 *
 * Coefficients: c[0] is the centre weight c_xyz; c[1..4] are c_x1..c_x4,
 * c[5..8] are c_y1..c_y4 and c[9..12] are c_z1..c_z4 (the paper's Eq. 3).
 *
 * The loops over z may run in parallel (OpenMP); every output point is
 * computed by one thread in a fixed order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define H 4

/* Allocation that stops with a message instead of returning NULL (the
 * full-size checks allocate several GB per field). */
static void *xcalloc(size_t n, size_t size)
{
    void *p = calloc(n, size);
    if (!p && n && size) {
        fprintf(stderr, "oracle: cannot allocate %zu x %zu bytes\n", n, size);
        abort();
    }
    return p;
}

static void *xmalloc(size_t size)
{
    void *p = malloc(size);
    if (!p && size) {
        fprintf(stderr, "oracle: cannot allocate %zu bytes\n", size);
        abort();
    }
    return p;
}

/* Progress lines on stderr every `progress_every` time steps of the long
 * runs (0: none).  Reporting only; no result depends on it. */
static int progress_every = 0;

void ref_set_progress(int every)
{
    progress_every = every > 0 ? every : 0;
}

static void progress(const char *what, int done, int total)
{
    if (progress_every > 0 && done % progress_every == 0) {
        fprintf(stderr, "oracle %s: %d of %d steps\n", what, done, total);
        fflush(stderr);
    }
}

static inline int64_t at(int nx, int ny, int x, int y, int z)
{
    return ((int64_t)(z + H) * (ny + 2 * H) + (y + H)) * (int64_t)(nx + 2 * H) + (x + H);
}

static int64_t padded_count(int nx, int ny, int nz)
{
    return (int64_t)(nx + 2 * H) * (ny + 2 * H) * (nz + 2 * H);
}

/* Eq. 3: c_xyz u(i,j,k) + sum_{m=1..4} c_xm [u(i+m)+u(i-m)] + c_ym [...] + c_zm [...] */
static double star25_at(int nx, int ny, const double *c, const double *u, int x, int y, int z)
{
    double s = c[0] * u[at(nx, ny, x, y, z)];
    for (int m = 1; m <= 4; ++m) {
        s += c[m] * (u[at(nx, ny, x + m, y, z)] + u[at(nx, ny, x - m, y, z)]);
        s += c[4 + m] * (u[at(nx, ny, x, y + m, z)] + u[at(nx, ny, x, y - m, z)]);
        s += c[8 + m] * (u[at(nx, ny, x, y, z + m)] + u[at(nx, ny, x, y, z - m)]);
    }
    return s;
}

/* out[interior] = L u, the 25-point star of Eq. 3 with the halo of u. */
void ref_laplacian(int nx, int ny, int nz, const double *c, const double *u, double *out)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                out[at(nx, ny, x, y, z)] = star25_at(nx, ny, c, u, x, y, z);
}

/*
 * Repeated sweeps, ping-ponging two grids as in the paper's star2d4r listing:
 * sweep s reads one grid and writes the other's interior, then the roles swap.
 * Returns 0 if the last result is in u, 1 if it is in v.
 */
int ref_stencil_apply(int nx, int ny, int nz, const double *c, int sweeps, double *u, double *v)
{
    double *a = u, *b = v;
    int in_v = 0;
    for (int s = 0; s < sweeps; ++s) {
        ref_laplacian(nx, ny, nz, c, a, b);
        double *t = a; a = b; b = t;
        in_v = !in_v;
    }
    return in_v;
}

/*
 * Leapfrog run (Eq. 2 with the Laplacian of Eq. 3 at unit spacing, and the
 * time loop of Algorithm 1).  For n = 0..nsteps-1:
 *     u^{n+1} = 2 u^n - u^{n-1} + m (L u^n),     m = (v dt / dx)^2,
 *     u^{n+1}[src_s] += dt^2 v[src_s]^2 amp[n][s]        (right-hand side),
 *     traces[n][r] = u^{n+1}[rec_r].
 * On entry prev = u^{-1}, cur = u^0 (padded); on return prev = u^{N-1},
 * cur = u^N.  v is interior-dense (nz, ny, nx).  Halos of prev/cur are kept.
 */
void ref_wave_run(int nx, int ny, int nz, const double *c, double dt, double dx,
                  const double *v, int nsteps,
                  int nsrc, const int32_t *src, const double *amp,
                  int nrec, const int32_t *rec, double *traces,
                  double *prev, double *cur)
{
    const int64_t np = padded_count(nx, ny, nz);
    double *lap = (double *)xcalloc((size_t)np, sizeof(double));
    double *bufs[2] = {prev, cur};
    int ip = 0, ic = 1;
    const double r = dt / dx;
    for (int n = 0; n < nsteps; ++n) {
        double *up = bufs[ip], *uc = bufs[ic];
        ref_laplacian(nx, ny, nz, c, uc, lap);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int64_t i = at(nx, ny, x, y, z);
                    double vv = v[((int64_t)z * ny + y) * nx + x];
                    double m = (vv * r) * (vv * r);
                    up[i] = 2.0 * uc[i] - up[i] + m * lap[i];
                }
        for (int s = 0; s < nsrc; ++s) {
            int x = src[3 * s], y = src[3 * s + 1], z = src[3 * s + 2];
            double vv = v[((int64_t)z * ny + y) * nx + x];
            up[at(nx, ny, x, y, z)] += dt * dt * vv * vv * amp[(int64_t)n * nsrc + s];
        }
        for (int q = 0; q < nrec; ++q) {
            int x = rec[3 * q], y = rec[3 * q + 1], z = rec[3 * q + 2];
            traces[(int64_t)n * nrec + q] = up[at(nx, ny, x, y, z)];
        }
        int t = ip; ip = ic; ic = t;
        progress("leapfrog", n + 1, nsteps);
    }
    /* the newest state is bufs[ic]; put u^N in cur and u^{N-1} in prev */
    if (bufs[ic] != cur) {
        double *tmp = (double *)xmalloc((size_t)np * sizeof(double));
        memcpy(tmp, cur, (size_t)np * sizeof(double));
        memcpy(cur, prev, (size_t)np * sizeof(double));
        memcpy(prev, tmp, (size_t)np * sizeof(double));
        free(tmp);
    }
    free(lap);
}

/*
 * Discrete energy between two consecutive states u0 = u^n, u1 = u^{n+1}:
 *     E = sum (u1 - u0)^2 / m  -  sum u1 (L u0),   m = (v dt / dx)^2.
 * Conserved by the source-free leapfrog when L is symmetric (zero halo).
 * Per-plane partial sums are added in plane order.
 */
double ref_energy(int nx, int ny, int nz, const double *c, double dt, double dx,
                  const double *v, const double *u0, const double *u1)
{
    double *part = (double *)xcalloc((size_t)nz, sizeof(double));
    const double r = dt / dx;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double s = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = at(nx, ny, x, y, z);
                double vv = v[((int64_t)z * ny + y) * nx + x];
                double m = (vv * r) * (vv * r);
                double d = u1[i] - u0[i];
                s += d * d / m - u1[i] * star25_at(nx, ny, c, u0, x, y, z);
            }
        part[z] = s;
    }
    double e = 0.0;
    for (int z = 0; z < nz; ++z) e += part[z];
    free(part);
    return e;
}

/*
 * Shared steps of the two adjoint-gradient routines below.  Both use the
 * same per-point operations in the same order, so the checkpointed routine
 * reproduces the full-storage one bit for bit.
 */

/* m = (v dt / dx)^2 on the padded grid, zero on the halo. */
static double *wave_m(int nx, int ny, int nz, double dt, double dx, const double *v)
{
    const double r = dt / dx;
    double *m = (double *)xcalloc((size_t)padded_count(nx, ny, nz), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double vv = v[((int64_t)z * ny + y) * nx + x];
                m[at(nx, ny, x, y, z)] = (vv * r) * (vv * r);
            }
    return m;
}

/* Forward step n of Eq. 2 with the source of Algorithm 1 written through m:
 *     un = 2 uc - up + m (L uc),   un[src] += m dx^2 amp[n]
 * (m dx^2 amp = dt^2 v^2 amp).  lap is scratch. */
static void fwd_step(int nx, int ny, int nz, const double *c, double dx, const double *m,
                     const double *up, const double *uc, double *un, double *lap, int n,
                     int nsrc, const int32_t *src, const double *amp)
{
    ref_laplacian(nx, ny, nz, c, uc, lap);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = at(nx, ny, x, y, z);
                un[i] = 2.0 * uc[i] - up[i] + m[i] * lap[i];
            }
    for (int s = 0; s < nsrc; ++s) {
        int64_t i = at(nx, ny, src[3 * s], src[3 * s + 1], src[3 * s + 2]);
        un[i] += m[i] * dx * dx * amp[(int64_t)n * nsrc + s];
    }
}

/* Adjoint step for time index k, then its gradient term:
 *     l0 = 2 l1 - l2 + L(m l1) + R^T res[k-1]          (lambda^k),
 *     gm += l0 (L ukm1 + dx^2 amp[k-1] e_src)        (ukm1 = u^{k-1}).
 * ml and lap are scratch. */
static void adj_step(int nx, int ny, int nz, const double *c, double dx, const double *m,
                     const double *l1, const double *l2, double *l0, const double *ukm1,
                     double *gm, double *ml, double *lap, int k, int nsrc, const int32_t *src,
                     const double *amp, int nrec, const int32_t *rec, const double *res)
{
    const int64_t np = padded_count(nx, ny, nz);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) ml[i] = m[i] * l1[i];
    ref_laplacian(nx, ny, nz, c, ml, lap);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = at(nx, ny, x, y, z);
                l0[i] = 2.0 * l1[i] - l2[i] + lap[i];
            }
    for (int q = 0; q < nrec; ++q)
        l0[at(nx, ny, rec[3 * q], rec[3 * q + 1], rec[3 * q + 2])] += res[(int64_t)(k - 1) * nrec + q];
    ref_laplacian(nx, ny, nz, c, ukm1, lap);
    for (int s = 0; s < nsrc; ++s) {
        int64_t i = at(nx, ny, src[3 * s], src[3 * s + 1], src[3 * s + 2]);
        lap[i] += dx * dx * amp[(int64_t)(k - 1) * nsrc + s];
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = at(nx, ny, x, y, z);
                gm[i] += l0[i] * lap[i];
            }
}

/* dJ/dv = dJ/dm 2 m / v on the interior (interior-dense output). */
static void grad_to_v(int nx, int ny, int nz, const double *v, const double *m, const double *gm,
                      double *grad_v)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = at(nx, ny, x, y, z);
                double vv = v[((int64_t)z * ny + y) * nx + x];
                grad_v[((int64_t)z * ny + y) * nx + x] = gm[i] * 2.0 * m[i] / vv;
            }
}

/*
 * Misfit gradient by the discrete adjoint of the leapfrog, with every forward
 * state kept in memory (for small grids).  Forward (ref_wave_run semantics)
 * from zero states:
 *     u^{n+1} = 2u^n - u^{n-1} + m (L u^n + dx^2 amp[n] e_src),  n = 0..N-1
 * (so that m dx^2 amp = dt^2 v^2 amp is the injected value), traces
 * d^n = R u^{n+1}.  Misfit J = 1/2 sum_n sum_r (R u^{n+1} - obs[n])^2.
 * Adjoint, lambda^{N+1} = lambda^{N+2} = 0, for k = N..1:
 *     lambda^k = 2 lambda^{k+1} - lambda^{k+2} + L(m lambda^{k+1}) + R^T r^k,
 *     r^k = R u^k - obs[k-1].
 * Gradient: dJ/dm = sum_{n=0}^{N-1} lambda^{n+1} (L u^n + dx^2 amp[n] e_src),
 *           dJ/dv = dJ/dm * 2 m / v   (dt, dx held fixed).
 * Returns J; grad_v is interior-dense (nz, ny, nx).
 */
double ref_adjoint_grad(int nx, int ny, int nz, const double *c, double dt, double dx,
                        const double *v, int nsteps,
                        int nsrc, const int32_t *src, const double *amp,
                        int nrec, const int32_t *rec, const double *obs,
                        double *grad_v)
{
    const int64_t np = padded_count(nx, ny, nz);
    const int N = nsteps;
    double *m = wave_m(nx, ny, nz, dt, dx, v);
    /* all states u^{-1}..u^N: u[n+1] is u^n */
    double *u = (double *)xcalloc((size_t)np * (N + 2), sizeof(double));
    double *lap = (double *)xcalloc((size_t)np, sizeof(double));
#define U(n) (u + (int64_t)((n) + 1) * np)
    for (int n = 0; n < N; ++n)
        fwd_step(nx, ny, nz, c, dx, m, U(n - 1), U(n), U(n + 1), lap, n, nsrc, src, amp);
    /* residuals and misfit */
    double *res = (double *)xcalloc((size_t)N * (nrec > 0 ? nrec : 1), sizeof(double));
    double J = 0.0;
    for (int k = 1; k <= N; ++k)
        for (int q = 0; q < nrec; ++q) {
            double d = U(k)[at(nx, ny, rec[3 * q], rec[3 * q + 1], rec[3 * q + 2])]
                       - obs[(int64_t)(k - 1) * nrec + q];
            res[(int64_t)(k - 1) * nrec + q] = d;
            J += 0.5 * d * d;
        }
    /* adjoint sweep */
    double *l1 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^{k+1} */
    double *l2 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^{k+2} */
    double *l0 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^k     */
    double *ml = (double *)xcalloc((size_t)np, sizeof(double));
    double *gm = (double *)xcalloc((size_t)np, sizeof(double));
    for (int k = N; k >= 1; --k) {
        adj_step(nx, ny, nz, c, dx, m, l1, l2, l0, U(k - 1), gm, ml, lap, k, nsrc, src, amp,
                 nrec, rec, res);
        double *t = l2; l2 = l1; l1 = l0; l0 = t;
    }
    grad_to_v(nx, ny, nz, v, m, gm, grad_v);
#undef U
    free(m); free(u); free(lap); free(res); free(l1); free(l2); free(l0); free(ml); free(gm);
    return J;
}

/*
 * The same misfit gradient with checkpointing, for grids whose N states do
 * not fit in memory: the forward pass keeps only the pair (u^{n0-1}, u^{n0})
 * at every segment start n0 = 0, C, 2C, ... (C = ckpt, about sqrt(N) for the
 * least memory), and the residuals.  The adjoint then walks the segments
 * from the last to the first; for each it recomputes u^{n0+1} .. u^{n0+L-1}
 * from the segment's pair (L = min(C, N - n0)) with the same forward step,
 * and takes the adjoint steps k = n0+L .. n0+1, which need u^{k-1}.
 * Memory: 2 N/C + C + 8 padded fields instead of N + 8.  Every state and
 * every adjoint step is computed by the same operations as in
 * ref_adjoint_grad, so the results are bit-identical to it.
 * traces (optional, may be NULL): the forward traces R u^{n+1}, [N][nrec].
 * Returns J; grad_v is interior-dense (nz, ny, nx).
 */
double ref_adjoint_grad_ckpt(int nx, int ny, int nz, const double *c, double dt, double dx,
                             const double *v, int nsteps,
                             int nsrc, const int32_t *src, const double *amp,
                             int nrec, const int32_t *rec, const double *obs,
                             int ckpt, double *traces, double *grad_v)
{
    const int64_t np = padded_count(nx, ny, nz);
    const int N = nsteps;
    const int C = ckpt < 1 ? 1 : ckpt;
    const int nseg = N > 0 ? (N + C - 1) / C : 0;
    double *m = wave_m(nx, ny, nz, dt, dx, v);
    double *lap = (double *)xcalloc((size_t)np, sizeof(double));
    /* segment-start pairs: pair[2j] = u^{jC-1}, pair[2j+1] = u^{jC} */
    double *pair = (double *)xcalloc((size_t)np * 2 * (nseg > 0 ? nseg : 1), sizeof(double));
    /* segment ring: ring[i] = u^{n0-1+i}, i = 0..C */
    double *ring = (double *)xcalloc((size_t)np * (C + 1), sizeof(double));
    double *res = (double *)xcalloc((size_t)N * (nrec > 0 ? nrec : 1), sizeof(double));
#define RING(i) (ring + (int64_t)(i) * np)
#define PAIR(j, h) (pair + ((int64_t)2 * (j) + (h)) * np)
    /* forward pass from zero states: three rotating buffers in the ring */
    double J = 0.0;
    {
        double *b[3] = {RING(0), RING(1), RING(2 <= C ? 2 : 0)};
        double *extra = NULL;
        if (C < 2) {                    /* C = 1: the ring has two fields only */
            extra = (double *)xcalloc((size_t)np, sizeof(double));
            b[2] = extra;
        }
        double *up = b[0], *uc = b[1], *un = b[2];
        for (int n = 0; n < N; ++n) {
            if (n % C == 0) {
                memcpy(PAIR(n / C, 0), up, (size_t)np * sizeof(double));
                memcpy(PAIR(n / C, 1), uc, (size_t)np * sizeof(double));
            }
            fwd_step(nx, ny, nz, c, dx, m, up, uc, un, lap, n, nsrc, src, amp);
            for (int q = 0; q < nrec; ++q) {
                double t = un[at(nx, ny, rec[3 * q], rec[3 * q + 1], rec[3 * q + 2])];
                double d = t - obs[(int64_t)n * nrec + q];
                if (traces) traces[(int64_t)n * nrec + q] = t;
                res[(int64_t)n * nrec + q] = d;
                J += 0.5 * d * d;
            }
            double *t = up; up = uc; uc = un; un = t;
            progress("adjoint, forward pass", n + 1, N);
        }
        free(extra);
    }
    /* adjoint pass, segments last to first */
    double *l1 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^{k+1} */
    double *l2 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^{k+2} */
    double *l0 = (double *)xcalloc((size_t)np, sizeof(double)); /* lambda^k     */
    double *ml = (double *)xcalloc((size_t)np, sizeof(double));
    double *gm = (double *)xcalloc((size_t)np, sizeof(double));
    for (int j = nseg - 1; j >= 0; --j) {
        const int n0 = j * C;
        const int L = N - n0 < C ? N - n0 : C;
        memcpy(RING(0), PAIR(j, 0), (size_t)np * sizeof(double));
        memcpy(RING(1), PAIR(j, 1), (size_t)np * sizeof(double));
        for (int i = 0; i + 1 < L; ++i)     /* u^{n0+i+1} from u^{n0+i-1}, u^{n0+i} */
            fwd_step(nx, ny, nz, c, dx, m, RING(i), RING(i + 1), RING(i + 2), lap, n0 + i,
                     nsrc, src, amp);
        for (int k = n0 + L; k >= n0 + 1; --k) {
            adj_step(nx, ny, nz, c, dx, m, l1, l2, l0, RING(k - n0), gm, ml, lap, k, nsrc, src,
                     amp, nrec, rec, res);
            double *t = l2; l2 = l1; l1 = l0; l0 = t;
            progress("adjoint, backward pass", N - k + 1, N);
        }
    }
    grad_to_v(nx, ny, nz, v, m, gm, grad_v);
#undef RING
#undef PAIR
    free(m); free(lap); free(pair); free(ring); free(res);
    free(l1); free(l2); free(l0); free(ml); free(gm);
    return J;
}

/*
 * Damping profile of the absorbing layer, on the padded array (frame
 * included): for a layer of W cells on every face,
 *     eta = eta_max * sum over axes (d_a / W)^2,
 *     d_a = max(0, W - 1 - a, a - (n_a - W)),  a = -4 .. n_a + 3,
 * the depth of index a into the layer (0 on the layer's innermost cells and
 * on the inner box, growing into the halo frame).
 */
void ref_pml_profile(int nx, int ny, int nz, int width, double eta_max, double *eta)
{
    const double W = (double)width;
    for (int z = -H; z < nz + H; ++z)
        for (int y = -H; y < ny + H; ++y)
            for (int x = -H; x < nx + H; ++x) {
                const int a[3] = {x, y, z}, n[3] = {nx, ny, nz};
                double s = 0.0;
                for (int k = 0; k < 3; ++k) {
                    int d = 0;
                    if (width - 1 - a[k] > d) d = width - 1 - a[k];
                    if (a[k] - (n[k] - width) > d) d = a[k] - (n[k] - width);
                    s += ((double)d / W) * ((double)d / W);
                }
                eta[at(nx, ny, x, y, z)] = eta_max * s;
            }
}

int ref_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing only; results do not
 * depend on it, each loop being over independent z-planes). */
void ref_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/*
 * Stencil suite of the paper's accuracy study (Sec. 6, the star/box kernels
 * of radius 1..4 in 2D and 3D; Eq. 3's 25-point star is star3d4r with
 * symmetric weights).  Plain definition, for every interior point:
 *     out(x, y, z) = sum over offsets (dz, dy, dx) in [-r, r]^ndim of
 *                    w[dz][dy][dx] * in(x + dx, y + dy, z + dz),
 * with w a dense (2r+1)^ndim array, x offset fastest (index
 * ((dz + r) * (2r+1) + (dy + r)) * (2r+1) + (dx + r); dz absent for ndim 2).
 * Star kernels are the members whose off-axis weights are zero.  For ndim 2
 * every z-plane is an independent 2D grid.
 *
 * Layout here: (nz + 2 hz) x (ny + 8) x (nx + 8) values, x fastest, with a
 * 4-cell xy frame and a z frame of hz = 4 planes for ndim 3, none for
 * ndim 2.  The frame is read, never written.
 */
void ref_stencil_general(int nx, int ny, int nz, int ndim, int r, const double *w,
                         const double *in, double *out)
{
    const int hz = ndim == 3 ? H : 0;
    const int64_t px = nx + 2 * H, py = ny + 2 * H;
    const int n = 2 * r + 1;
    const int rz = ndim == 3 ? r : 0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int dz = -rz; dz <= rz; ++dz)
                    for (int dy = -r; dy <= r; ++dy)
                        for (int dx = -r; dx <= r; ++dx) {
                            const int64_t wi = ((int64_t)(dz + rz) * n + (dy + r)) * n + (dx + r);
                            const int64_t ui = ((int64_t)(z + dz + hz) * py + (y + dy + H)) * px +
                                               (x + dx + H);
                            s += w[wi] * in[ui];
                        }
                out[((int64_t)(z + hz) * py + (y + H)) * px + (x + H)] = s;
            }
}

/*
 * Leapfrog with an absorbing perfectly-matched-type layer (the inner + PML
 * regions of the paper's Sec. 2.2; the paper names the PML but does not
 * give its equations).  The reading taken: complex stretching of all three
 * coordinates by the same position-dependent factor 1 + eta/(i w), which
 * turns the wave equation into
 *     (d/dt + eta)^2 u = V^2 (lap u + phi),
 *     (d/dt + eta + alpha) phi = -grad eta . grad u,
 * (with alpha = 0 exactly the PML in 1D).  The frequency shift alpha > 0 in
 * the auxiliary equation, as in frequency-shifted (convolutional) PMLs,
 * removes a slowly growing zero-frequency mode that the unshifted isotropic
 * form develops in long runs.  Centred differences in time, with psi =
 * dx^2 phi held at half steps, eta in 1/s, a = eta dt, b = a + alpha dt:
 *     psi^{n+1/2} = [ (1 - b/2) psi^{n-1/2} - dt G^n ] / (1 + b/2)
 *     u^{n+1} = [ (2 - a^2) u^n - (1 - a) u^{n-1}
 *                 + m (L u^n + (psi^{n-1/2} + psi^{n+1/2}) / 2) ] / (1 + a)
 *     G^n = 1/4 sum over axes (eta(+1) - eta(-1)) (u^n(+1) - u^n(-1))
 * (the 7-point star of grad eta . grad u in index units); then the sources
 * of Algorithm 1 and the receivers as in ref_wave_run.  Where eta and its
 * neighbours are 0 (and psi is 0) this is the plain leapfrog.
 * eta: padded like the fields (its frame is read); psi: padded, interior
 * used, updated in place.  prev/cur as in ref_wave_run.
 */
void ref_wave_pml_run(int nx, int ny, int nz, const double *c, double dt, double dx,
                      const double *v, const double *eta, double alpha, int nsteps,
                      int nsrc, const int32_t *src, const double *amp,
                      int nrec, const int32_t *rec, double *traces,
                      double *prev, double *cur, double *psi)
{
    const int64_t np = padded_count(nx, ny, nz);
    double *lap = (double *)xcalloc((size_t)np, sizeof(double));
    double *bufs[2] = {prev, cur};
    int ip = 0, ic = 1;
    const double r = dt / dx;
    const int64_t sx = 1, sy = nx + 2 * H, sz = (int64_t)(nx + 2 * H) * (ny + 2 * H);
    for (int n = 0; n < nsteps; ++n) {
        double *up = bufs[ip], *uc = bufs[ic];
        ref_laplacian(nx, ny, nz, c, uc, lap);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t i = at(nx, ny, x, y, z);
                    const double vv = v[((int64_t)z * ny + y) * nx + x];
                    const double m = (vv * r) * (vv * r);
                    const double a = eta[i] * dt;
                    const double G = 0.25 * ((eta[i + sx] - eta[i - sx]) * (uc[i + sx] - uc[i - sx]) +
                                             (eta[i + sy] - eta[i - sy]) * (uc[i + sy] - uc[i - sy]) +
                                             (eta[i + sz] - eta[i - sz]) * (uc[i + sz] - uc[i - sz]));
                    const double b = a + alpha * dt;
                    const double pnew = ((1.0 - 0.5 * b) * psi[i] - dt * G) / (1.0 + 0.5 * b);
                    up[i] = ((2.0 - a * a) * uc[i] - (1.0 - a) * up[i] +
                             m * (lap[i] + 0.5 * (psi[i] + pnew))) / (1.0 + a);
                    psi[i] = pnew;
                }
        for (int s = 0; s < nsrc; ++s) {
            int x = src[3 * s], y = src[3 * s + 1], z = src[3 * s + 2];
            double vv = v[((int64_t)z * ny + y) * nx + x];
            up[at(nx, ny, x, y, z)] += dt * dt * vv * vv * amp[(int64_t)n * nsrc + s];
        }
        for (int q = 0; q < nrec; ++q) {
            int x = rec[3 * q], y = rec[3 * q + 1], z = rec[3 * q + 2];
            traces[(int64_t)n * nrec + q] = up[at(nx, ny, x, y, z)];
        }
        int t = ip; ip = ic; ic = t;
    }
    if (bufs[ic] != cur) {
        double *tmp = (double *)xmalloc((size_t)np * sizeof(double));
        memcpy(tmp, cur, (size_t)np * sizeof(double));
        memcpy(cur, prev, (size_t)np * sizeof(double));
        memcpy(prev, tmp, (size_t)np * sizeof(double));
        free(tmp);
    }
    free(lap);
}
