/*
 * libstencil: 25-point star stencil and acoustic leapfrog on gfx950 (MI355X).
 *
 * The operations are those of the paper "StencilPy" (arXiv 2309.04671):
 *   - the 25-point star-shaped high-order stencil of Sec. 2.2, Eq. 3
 *     (radius 4 along x, y and z around a centre point),
 *   - the constant-density acoustic isotropic leapfrog of Sec. 2.2, Eq. 2
 *     (u^{n+1} = 2u^n - u^{n-1} + dt^2 V^2 lap u^n + dt^2 V^2 f^n),
 *   - the time loop of Algorithm 1 (update every point, then add the source),
 * plus the discrete adjoint of that leapfrog for a receiver misfit, wavefield
 * storage in FP16/BF16 with per-slab scales, and a continuous-batching shot
 * queue.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: SP_OK (0) or an SP_E* code; sp_last_error() returns a
 *    thread-local message.  Arguments are validated before anything is
 *    enqueued, so an SP_EINVAL / SP_EUNSUPPORTED / SP_ENOMEM return leaves
 *    every buffer and state untouched.  SP_EDEVICE from a failed launch
 *    part-way through a multi-step call leaves the state (pointers and step
 *    counter) at the last step that was enqueued.
 *  - Every data pointer is a DEVICE pointer owned by the caller, unless the
 *    comment says HOST.  The library never allocates device memory outside
 *    a caller-provided workspace or arena; sp_energy_noalloc instead uses a
 *    static per-device array that is part of the loaded library.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    compute calls are asynchronous on that stream; a device fault surfaces at
 *    the next synchronisation.
 *  - Axes: x is contiguous (the paper's i), then y (j), then z (k, depth; the
 *    streaming axis).  Interior indices run 0..n-1; the halo is 4 cells wide
 *    on every face (the stencil radius; the paper's "order").  The library
 *    reads halo cells and never writes them: callers set them (zero for the
 *    Dirichlet boundary) once after allocation.
 */
#ifndef SP_STENCIL_H
#define SP_STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SP_OK           0
#define SP_EINVAL       1  /* bad argument (shape, halo, pointer, alignment, aliasing) */
#define SP_EUNSUPPORTED 2  /* valid request the library does not implement */
#define SP_EDEVICE      3  /* HIP runtime error */
#define SP_ENOMEM       4  /* caller workspace / arena too small */
#define SP_EBUDGET      5  /* shot can never fit the queue's HBM budget */
#define SP_EPENDING     6  /* poll: shot not finished yet */
#define SP_ENUMERIC     7  /* non-finite value detected */

/* storage types */
#define SP_F32  0
#define SP_F16  1
#define SP_BF16 2

#define SP_HALO 4            /* the only supported halo width (radius 4) */
#define SP_MAX_SOURCES 16    /* sources per wave_step call */
#define SP_SLAB 16           /* planes per z-slab for FP16/BF16 scales */

/*
 * Grid descriptor: where each cell of a halo-padded field lives.
 * Cell (x, y, z), -4 <= x < nx+4 (same for y, z), is element
 *     origin + z * pitch_y * pitch_x + y * pitch_x + x
 * of an allocation of `bytes` bytes.  Interior x = 0 of every row is
 * 128-byte aligned; the 4 right-halo cells of a row share the (otherwise
 * unused) lead padding of the next row.  Element offsets of different cells
 * are distinct.
 */
typedef struct {
    int32_t nx, ny, nz;     /* interior points */
    int32_t halo;           /* = SP_HALO */
    int32_t dtype;          /* SP_F32 / SP_F16 / SP_BF16 */
    int32_t elem_bytes;     /* 4 or 2 */
    int64_t pitch_x;        /* elements per padded row */
    int64_t pitch_y;        /* rows per padded plane (ny + 8) */
    int64_t planes;         /* padded planes (nz + 8) */
    int64_t origin;         /* element offset of interior (0, 0, 0) */
    int64_t elems;          /* elements to allocate */
    int64_t bytes;          /* bytes to allocate (multiple of 256) */
} sp_grid;

/* Fill `out` for an nx x ny x nz interior.  halo must be 4.  Host-only. */
int sp_grid_init(int nx, int ny, int nz, int halo, int dtype, sp_grid *out);

/*
 * 2D grid: one plane of nx x ny interior points with the 4-cell frame in x
 * and y only (nz = 1, planes = 1, no z halo); cell (x, y) is element
 *     origin + y * pitch_x + x.
 * Only the 2D stencils of sp_apply accept it.  halo must be 4.  Host-only.
 */
int sp_grid_init_2d(int nx, int ny, int halo, int dtype, sp_grid *out);

/*
 * Stencil weights of Eq. 3 at unit spacing: centre c_xyz and c_xm, c_ym, c_zm
 * for m = 1..4.  Given in FP64; the kernels use them rounded once to FP32.
 */
typedef struct {
    double center;
    double ax[4], ay[4], az[4];
} sp_coeffs;

/*
 * sp_stencil_apply -- `sweeps` sweeps of the star stencil (Eq. 3), FP32 only.
 * Sweep s reads one grid and writes the other's interior, then the two swap
 * roles, as in the paper's star2d4r listing (Sec. 5): after an odd number of
 * sweeps the result is in v, after an even number in u; *result_in is set to
 * 1 or 0 accordingly (HOST int).  u and v: allocations of g->bytes, distinct.
 * sweeps >= 0 (0 is a no-op with *result_in = 0).
 */
int sp_stencil_apply(const sp_grid *g, const sp_coeffs *c, int sweeps,
                     void *u, void *v, int *result_in, void *stream);

/*
 * Stencil suite (the star- and box-shaped kernels of radius 1..4 in 2D and 3D
 * of the paper's accuracy study, Sec. 6; Eq. 3 is star3d4r with symmetric
 * weights):
 *     out(p) = sum over offsets k in [-r, r]^ndim of w[k] * u(p + k)
 * on every interior point, reading u's halo (zero for the Dirichlet frame).
 * w is a HOST array of (2r+1)^ndim FP64 weights, x offset fastest: the
 * weight of offset (dx, dy, dz) is w[((dz + r) * (2r+1) + dy + r) * (2r+1)
 * + dx + r] (no dz term for ndim 2).  A star's weights must be zero off the
 * three (two) axis lines through the centre.  The kernels use the weights
 * rounded once to FP32.
 */
#define SP_STAR 0
#define SP_BOX  1
typedef struct {
    int32_t shape;          /* SP_STAR or SP_BOX */
    int32_t ndim;           /* 2 or 3 */
    int32_t radius;         /* 1 .. 4 (<= the halo) */
    const double *w;        /* HOST weights, see above */
} sp_stencil;

/*
 * sp_apply -- `sweeps` sweeps of a suite stencil on FP32 grids, ping-ponging
 * u and v exactly like sp_stencil_apply (*result_in: 1 if the result is in
 * v, 0 if in u; HOST int).  ndim 3 needs a 3D grid (sp_grid_init); ndim 2
 * takes a 2D grid (sp_grid_init_2d) or a 3D grid, whose interior planes are
 * then independent 2D grids.  u and v: allocations of g->bytes, distinct,
 * 16-byte aligned.  SP_EINVAL for a bad shape, radius, weight array or grid.
 */
int sp_apply(const sp_grid *g, const sp_stencil *s, int sweeps, void *u, void *v,
             int *result_in, void *stream);

/*
 * Wavefield state of the leapfrog.  cur = u^n, prev = u^{n-1}; a step writes
 * u^{n+1} over prev and swaps the two pointers, so on return cur is the
 * newest state.  `step` (= n) counts steps taken; it indexes the source
 * amplitudes and the FP16/BF16 records.  `meta` must be NULL for FP32.
 *
 * FP16/BF16 storage: a stored value q of a point in z-slab k (planes
 * 16k .. 16k+15) stands for q * s_k, s_k a power of two per field and slab.
 * `meta` points at sp_wave_meta_bytes() DEVICE bytes holding 4 slots; field
 * u^j uses slot j mod 4 (u^{-1}: slot 3).  Slot layout, nslab = ceil(nz/16):
 *     float    scale[nslab];   s_k
 *     uint32_t amax[nslab];    IEEE bits of max |q| * s_k over slab k
 * FP16/BF16 storage needs planes of fewer than 2^30 elements (pitch_x x
 * pitch_y of the FP32 v grid; SP_EUNSUPPORTED otherwise).
 * Zero-fill the block before the first step from zero fields; to start from
 * non-zero fields, fill slots 0 (u^0) and 3 (u^{-1}) consistently.  Step n
 * chooses s_k of u^{n+1} before computing it:
 *     B_k = 8 max(amax(u^n) slabs k-1..k+1, amax(u^{n-1}) slab k)
 *           + sum over sources in slab k of |dt^2 v^2 amp|  (FP32),
 *     s_k = 2^(ceil(log2 B_k) - 15)  (1 if B_k = 0; the exponent clamped
 *           to [-110, 110], so s_k and 1/s_k stay normal FP32 numbers),
 * which keeps |q| <= 2^15 inside the stability limit; values are rounded to
 * nearest even.  Halo planes are decoded with the nearest slab's scale.
 */
typedef struct {
    void *cur;
    void *prev;
    void *meta;
    int64_t step;
} sp_wave_state;

/* Bytes of the FP16/BF16 metadata block for grid g (0 for FP32). Host-only. */
int64_t sp_wave_meta_bytes(const sp_grid *g);

/*
 * Point sources (Eq. 2 right-hand side, added after the update as in
 * Algorithm 1): after step n computes u^{n+1},
 *     u^{n+1}[x_s] += dt^2 * v[x_s]^2 * amp[n * amp_stride + s].
 * xyz is a HOST array (copied by value); amp is DEVICE FP32, indexed by the
 * state's step counter.  n <= SP_MAX_SOURCES; points must lie in the interior.
 */
typedef struct {
    int32_t n;
    int32_t xyz[SP_MAX_SOURCES][3];
    const float *amp;
    int64_t amp_stride;
} sp_sources;

/*
 * Receivers: after step n (and its source injection)
 *     traces[(n - step0) * trace_stride + r] = u^{n+1}[x_r],
 * where step0 is the state's step counter on entry.  xyz is DEVICE int32
 * [n][3]; points outside the interior record 0.  traces is DEVICE FP32.
 */
typedef struct {
    int32_t n;
    const int32_t *xyz;
    float *traces;
    int64_t trace_stride;
} sp_receivers;

/*
 * sp_wave_step -- `nsteps` leapfrog steps (Eq. 2 with Eq. 3 at spacing dx):
 *     u^{n+1} = 2u^n - u^{n-1} + m * (L u^n),   m = (v * dt / dx)^2,
 * then sources, then receivers.  v is an FP32 field on its own grid
 * descriptor gv (same nx, ny, nz, dtype SP_F32).  src and rec may be NULL.
 * The state's pointers are swapped once per step and its step counter
 * advanced, before the call returns (the work itself is asynchronous).
 */
int sp_wave_step(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                 const sp_grid *gv, const float *v, sp_wave_state *st, int nsteps,
                 const sp_sources *src, const sp_receivers *rec, void *stream);

/*
 * sp_wave_step_fused -- the same `nsteps` steps as sp_wave_step (FP32 grids
 * only), two per sweep over the grid: temporal blocking, which the paper
 * lists among the tuning dimensions of its GPU tilings.  Each sweep reads
 * u^n, u^{n-1} and v once and writes u^{n+1} and u^{n+2} (20 B per point
 * for two steps instead of 32); an odd last step runs the single-step
 * sweep.  Results, sources and receivers are those of sp_wave_step.
 *
 * spare is a HOST array of two DEVICE fields on grid g, distinct from each
 * other and from the state's fields, with zero halos (allocate them zeroed);
 * their interiors are overwritten.  On return the state points at the two
 * newest fields and spare[0], spare[1] at the other two.
 */
int sp_wave_step_fused(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                       const sp_grid *gv, const float *v, sp_wave_state *st, int nsteps,
                       void **spare, const sp_sources *src, const sp_receivers *rec,
                       void *stream);

/*
 * sp_wave_run_states -- leapfrog steps that keep every state (FP32 grids
 * only): the recompute primitive of checkpointed adjoints.  states is a HOST
 * array of nsteps+2 DEVICE field pointers (grid g): states[0] = u^{n0-1} and
 * states[1] = u^{n0} on entry; step i writes u^{n0+i+1} into states[i+2]
 * (same update, sources and receivers as sp_wave_step, with n = n0 + i;
 * traces row i).  All pointers must be distinct allocations.
 */
int sp_wave_run_states(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                       const sp_grid *gv, const float *v, void *const *states, int64_t n0,
                       int nsteps, const sp_sources *src, const sp_receivers *rec,
                       void *stream);

/*
 * sp_wave_adjoint_step -- `nsteps` steps of the discrete adjoint of the
 * leapfrog of Eq. 2 (Sec. 2.2; time loop of Algorithm 1: update, then the
 * source) for a misfit L(traces), in the scaled variable nu = m * lambda
 * (FP32 grids only).  The adjoint is derived from the discrete update, not
 * given by the paper: transposing u^{n+1} = 2u^n - u^{n-1} + m L u^n + m dx^2
 * f^n e_src over all steps gives the backward recurrence for lambda, and
 * since L is symmetric (zero halo) nu = m lambda follows the same leapfrog
 * as the forward field.  With g_k = dL/dtraces row k (the receiver samples of
 * u^{k+1}), one adjoint step for time index k (k = N .. 1) computes
 *     nu^k = 2 nu^{k+1} - nu^{k+2} + m * (L nu^{k+1}) + m * R^T g_{k-1}
 * and accumulates, in FP64,
 *     G += nu^k * (L u^{k-1} + dx^2 f^{k-1} e_src),
 * where f are the forward source amplitudes.  After the step for k = 1,
 * dL/dv = 2 G / v (sp_grad_finish); dt and dx are held fixed.
 *   adj: adj->cur = nu^{k+1}, adj->prev = nu^{k+2}, adj->step = k on entry
 *        (zero fields and step = N to start); nu^k is written over prev,
 *        the pointers swapped and step decremented per step.
 *   u_hist: HOST array of nsteps DEVICE pointers, u_hist[i] = u^{k-1-i}.
 *   rec: receivers; rec->traces is READ (dL/dtraces, row k-1 at
 *        rec->traces + (k-1) * trace_stride).  Receiver points add (duplicates sum).
 *   src: the forward sources (amplitude row k-1 is read); may be NULL.
 *   G: DEVICE FP64 array laid out like grid g's elements (g->elems doubles,
 *      same element offsets); only interior elements are read or written.
 */
int sp_wave_adjoint_step(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                         const sp_grid *gv, const float *v, sp_wave_state *adj,
                         const void *const *u_hist, int nsteps, const sp_sources *src,
                         const sp_receivers *rec, double *G, void *stream);

/* out = 2 G / v on the interior; out is an FP32 field on grid gv (G on the
 * same element layout, FP64). */
int sp_grad_finish(const sp_grid *gv, const float *v, const double *G, float *out,
                   void *stream);

/*
 * sp_decode -- the interior of a wavefield as plain FP32 values: out is a
 * DEVICE FP32 array [nz][ny][nx] (x fastest, no halo) receiving q * s_k for
 * every interior point of `field` (grid g), where s_k is the slab scale of
 * field u^k read from slot k mod 4 of `meta` (FP16/BF16; exact, the scales
 * being powers of two).  For FP32 grids meta and k are ignored and the
 * values are copied.  out must not overlap the field.
 */
int sp_decode(const sp_grid *g, const void *field, const void *meta, int64_t k, float *out,
              void *stream);

/*
 * sp_energy -- discrete energy of the leapfrog of Eq. 2 (Sec. 2.2) between
 * u0 = u^n and u1 = u^{n+1} (FP32 grids), accumulated in FP64:
 *     E = sum (u1 - u0)^2 / m - sum u1 * (L u0),   m = (v dt / dx)^2,
 * with L the star of Eq. 3.  Taking the inner product of the Eq. 2 update
 * with (u^{n+1} - u^{n-1}) / m shows that the source-free leapfrog conserves
 * E exactly when L is symmetric (zero halo).  Writes one double to *out
 * (DEVICE, 8-byte aligned).  ws: DEVICE workspace of sp_energy_ws_bytes(g)
 * bytes (per-block partial sums, added in a fixed order, so the result is
 * deterministic).
 */
int64_t sp_energy_ws_bytes(const sp_grid *g);
int sp_energy(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
              const sp_grid *gv, const float *v, const void *u0, const void *u1,
              double *out, void *ws, void *stream);

/*
 * sp_energy_noalloc -- sp_energy without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result as sp_energy minus ws; calls no allocating routine.  The per-block
 * partial sums go to a static device array of
 * sp_energy_noalloc_max_partials() doubles (512 KiB), one per device, held
 * until the process ends; grids whose sweep needs more partial sums fail
 * with SP_ENOMEM (use sp_energy).  Every partial is written before it is
 * read, so nothing carries over from an earlier call.  All calls on one
 * device share that array: calls that overlap on one device (different
 * streams, or host threads without ordering) race.  `stream` must belong to
 * the current device (SP_EINVAL otherwise).
 */
int64_t sp_energy_noalloc_max_partials(void);
int sp_energy_noalloc(const sp_grid *g, const sp_coeffs *c, double dt, double dx,
                      const sp_grid *gv, const float *v, const void *u0, const void *u1,
                      double *out, void *stream);

/* ------------------------------------------------------------------------
 * Absorbing layer: the inner and PML regions of Sec. 2.2.
 *
 * The paper surrounds the domain with a PML whose kernel applies the
 * 25-point star plus a 7-point star to a second array, but gives no
 * equations.  The layer here stretches all coordinates by one
 * position-dependent factor, with a frequency shift alpha in the auxiliary
 * equation (stable in long runs):
 *     (d/dt + eta)^2 u = V^2 (lap u + phi),
 *     (d/dt + eta + alpha) phi = -grad eta . grad u,
 * discretised centred in time with psi = dx^2 phi at half steps
 * (a = eta dt, b = a + alpha dt, m = (v dt / dx)^2):
 *     psi^{n+1/2} = [(1 - b/2) psi^{n-1/2} - dt G] / (1 + b/2),
 *     G = 1/4 sum over axes (eta(+1) - eta(-1)) (u^n(+1) - u^n(-1)),
 *     u^{n+1} = [(2 - a^2) u^n - (1 - a) u^{n-1}
 *                + m (L u^n + (psi^{n-1/2} + psi^{n+1/2}) / 2)] / (1 + a),
 * then the sources and receivers of sp_wave_step.  Where eta and its
 * neighbours are zero this is the plain leapfrog.
 * ---------------------------------------------------------------------- */

#define SP_PML_UNIFIED 0   /* the layer kernel over the whole interior */
#define SP_PML_SEVEN   1   /* inner box by the leapfrog kernel, 6 slabs by the layer kernel */
#define SP_PML_TWO     2   /* inner box by the leapfrog kernel, the shell by one layer launch */

typedef struct {
    int32_t width;          /* W: layer cells on every face (SEVEN, TWO: W % 4 == 0, 4 <= W, 2W < n) */
    int32_t decomposition;  /* SP_PML_UNIFIED, SP_PML_SEVEN or SP_PML_TWO (the paper's
                               region maps: one region, seven boxes, inner box + shell) */
    double alpha;           /* frequency shift of the auxiliary equation (1/s), >= 0 */
    const float *eta;       /* DEVICE FP32 field on gv's layout, frame included: damping (1/s).
                               SEVEN and TWO require eta = 0 on the inner box [W, n-W) and on the
                               cells next to it, as sp_pml_profile makes it */
    float *psi;             /* DEVICE FP32 field on g's layout: psi, zero before the first step */
} sp_pml;

/* Fill eta (an FP32 field on gv, frame included) with the layer profile
 *     eta = eta_max * sum over axes (d_a / W)^2,
 *     d_a = max(0, W - 1 - a, a - (n_a - W)),
 * zero on the inner box and on its neighbouring cells. */
int sp_pml_profile(const sp_grid *gv, int width, double eta_max, float *eta, void *stream);

/* nsteps leapfrog steps with the absorbing layer (FP32 grids only).  Same
 * state, sources and receivers as sp_wave_step; g and gv must have the
 * same layout. */
int sp_wave_step_pml(const sp_grid *g, const sp_coeffs *c, double dt, double dx, const sp_grid *gv,
                     const float *v, sp_wave_state *st, int nsteps, const sp_pml *pml,
                     const sp_sources *src, const sp_receivers *rec, void *stream);

/* ------------------------------------------------------------------------
 * Continuous-batching shot queue.
 *
 * Forward-modelling requests ("shots": one grid, velocity model, sources,
 * receivers and step count each, FP32 or FP16/BF16 storage) are admitted
 * while the queue's resident HBM budget and slot count allow, and advanced
 * together in chunks of chunk_steps leapfrog steps: every step of a chunk
 * is one batched kernel launch per (storage type, tile shape) covering the
 * tiles of every resident shot, plus one batched receiver launch, and the
 * chunk is replayed from a captured HIP graph while the set of resident
 * shots is unchanged.  Requests that arrive while others run are admitted
 * at the next chunk boundary as slots and memory free up.  Each shot
 * computes exactly what sp_wave_step computes for it alone (same kernels,
 * same per-point arithmetic), so its results do not depend on the mix.
 * A shot whose leapfrog computes an infinity or a NaN at any interior point
 * (a blown-up run: unstable dt, an infinite amplitude) ends at the close of
 * that chunk as SP_SHOT_FAILED with error SP_ENUMERIC; its memory returns to
 * the arena and the other shots run on unaffected.
 * ---------------------------------------------------------------------- */

#define SP_QUEUE_EAGER 1   /* launch chunks directly instead of through captured graphs */
#define SP_QUEUE_FAKE  2   /* host logic only: no device work; chunks finish at once */

#define SP_SHOT_QUEUED  0
#define SP_SHOT_RUNNING 1
#define SP_SHOT_DONE    2
#define SP_SHOT_FAILED  3

typedef struct {
    void *arena;            /* DEVICE buffer owned by the caller (any pointer if SP_QUEUE_FAKE) */
    int64_t arena_bytes;
    int64_t budget_bytes;   /* resident shot bytes admitted at once; 0: the arena minus its control part */
    int32_t max_slots;      /* shots resident at once (>= 1) */
    int32_t chunk_steps;    /* steps per batched chunk (>= 1) */
    int32_t flags;          /* SP_QUEUE_* */
    void *stream;           /* hipStream_t on which the caller produced the shot inputs */
} sp_queue_cfg;

typedef struct {
    int32_t nx, ny, nz;     /* interior points */
    int32_t dtype;          /* wavefield storage: SP_F32, SP_F16 or SP_BF16 */
    int32_t nsteps;         /* leapfrog steps (>= 1) */
    double dt, dx;
    sp_coeffs coeffs;
    const float *v;         /* DEVICE interior-dense FP32 [nz][ny][nx]; copied in at admission */
    int32_t nsrc;           /* <= SP_MAX_SOURCES */
    int32_t src_xyz[SP_MAX_SOURCES][3];
    const float *src_amp;   /* DEVICE FP32 [nsteps][nsrc]; read while the shot runs */
    int32_t nrec;
    const int32_t *rec_xyz; /* DEVICE int32 [nrec][3]; read while the shot runs */
    float *traces;          /* DEVICE FP32 [nsteps][nrec]: row n = u^{n+1} at the receivers */
    float *final_out;       /* optional DEVICE FP32 [nz][ny][nx]: u^nsteps (decoded) */
} sp_shot_desc;

typedef struct {
    int32_t state;          /* SP_SHOT_* */
    int32_t error;          /* SP_* code of a failed shot (SP_ENUMERIC: non-finite values) */
    int64_t steps_done;
    double t_submit, t_admit, t_done;   /* seconds on the host's steady clock */
} sp_shot_status;

typedef struct sp_queue sp_queue;

/* Resident arena bytes of one shot (two wavefields, v, slab records), or -1
 * for an invalid description.  Host-only. */
int64_t sp_shot_bytes(const sp_shot_desc *d);

/* Start a queue and its worker thread.  The arena must outlive the queue. */
int sp_queue_create(const sp_queue_cfg *cfg, sp_queue **out);

/* Enqueue a shot; *ticket identifies it.  SP_EBUDGET if it can never fit.
 * The description's device buffers must stay valid until the shot is
 * finished (v: until it is admitted). */
int sp_submit(sp_queue *q, const sp_shot_desc *d, uint64_t *ticket);

/* Status of a shot: SP_OK once it is DONE or FAILED (its traces and final
 * field are then complete in device memory), SP_EPENDING while queued or
 * running, SP_EINVAL for an unknown ticket. */
int sp_poll(sp_queue *q, uint64_t ticket, sp_shot_status *st);

/* Block until every shot submitted so far has finished. */
int sp_queue_drain(sp_queue *q);

/* Finish the running shots, fail the queued ones, stop the worker, free. */
int sp_queue_destroy(sp_queue *q);

/* Thread-local message for the last error on this thread ("" if none). */
const char *sp_last_error(void);

/* Library version string. */
const char *sp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SP_STENCIL_H */
