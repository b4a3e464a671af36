/*
 * bpm.h — C ABI of the MI355X two-beam FFT beam-propagation library
 * (libbpm_hip.so, gfx950).
 *
 * The library marches the slowly varying envelopes psi+ (transmitted) and psi-
 * (reflected) of an X-ray field through a deformed crystal with the two-beam
 * split-step FFT BPM: each z-step propagates both envelopes in Fourier space
 * with their shifted propagators and then couples them in real space through
 * the susceptibility harmonics, the crystal-shape mask and the strain phase
 * (paper Sec. 2, Eq. (4), Eq. (6)-(12); bent crystals Eq. (14); dislocations
 * Eq. (15)).
 *
 * Conventions shared by every call
 *   x_j = x0_um + j*dx_um (j = 0..nx-1), periodic window; z_n = n*dz_um.
 *   Step n couples with the mask and strain sampled at (x_j, z_n), after the
 *   propagation of that step (Eq. (12): propagate, then multiply by the
 *   harmonics).
 *   Envelope storage: interleaved complex (re, im).  A solve's device state is
 *   psi+[nx] followed by psi-[nx], in the plan's precision (complex128 for
 *   BPM_F64, complex64 for BPM_F32).  Host-side buffers are always complex128.
 *   R = sum_{j in [det_lo, det_hi)} |psi-_j(nz)|^2 / sum_j |psi+_j(0)|^2 and
 *   T likewise for psi+ (both accumulated in FP64; 0 if the incident power is 0).
 *
 * Errors: every call returns a bpm_status; no exception crosses the ABI.  On
 * failure bpm_last_error() returns a thread-local message.  A plan or batch is
 * used by one thread at a time; the server API is thread-safe.
 */
#ifndef BPM_H
#define BPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bpm_status {
    BPM_OK = 0,
    BPM_E_INVALID = 1,     /* bad argument, descriptor or NULL pointer */
    BPM_E_NOMEM = 2,       /* host or device allocation failed */
    BPM_E_DEVICE = 3,      /* HIP runtime error, or no gfx950 device */
    BPM_E_BUDGET = 4,      /* request can never fit the server's device-memory budget */
    BPM_E_PENDING = 5,     /* ticket not finished yet */
    BPM_E_CANCELLED = 6,   /* ticket was cancelled before it finished */
    BPM_E_NOTFOUND = 7,    /* unknown ticket */
    BPM_E_UNSUPPORTED = 8, /* valid request outside what the library runs */
    BPM_E_NUMERIC = 9      /* non-finite input or result */
} bpm_status;

typedef struct bpm_complex {
    double re, im;
} bpm_complex;

typedef enum bpm_precision {
    BPM_F64 = 0, /* complex128 envelopes and arithmetic */
    BPM_F32 = 1  /* complex64 envelopes and arithmetic; FP64 for plan setup,
                    strain-phase arguments and R/T accumulation */
} bpm_precision;

typedef enum bpm_strain_kind {
    BPM_STRAIN_NONE = 0,
    /* u = c0 + c1 X + c2 Z + c3 X^2 + c4 X Z + c5 Z^2 with X = x - x_ref, Z = z - z_ref
     * (covers Eq. (14) bending, u = xz/R plate bending, uniform strain, offsets) */
    BPM_STRAIN_POLY2 = 1,
    /* straight edge dislocation, line along y, Burgers vector b along h (Eq. (15)):
     * u = b/(2 pi) * (atan2(Z, X) + X Z / (2 (1 - nu) (X^2 + Z^2))), core at (x_ref, z_ref) */
    BPM_STRAIN_EDGE_DISLOCATION = 2,
    /* u given at every grid point: u_table[n*nx + j] (um), copied at plan creation;
     * at most 2 GiB on the device (nz*nx*4 B FP32, *8 B FP64), else BPM_E_UNSUPPORTED */
    BPM_STRAIN_TABLE = 3
} bpm_strain_kind;

typedef struct bpm_strain {
    int32_t kind;            /* bpm_strain_kind */
    double x_ref_um, z_ref_um;
    double c[6];             /* POLY2 coefficients (um, dimensionless, um^-1) */
    double b_um, nu;         /* EDGE_DISLOCATION Burgers vector length, Poisson ratio */
    const double *u_table;   /* TABLE: [nz][nx] displacement along h (um) */
} bpm_strain;

/* One solve.  Geometry and asymmetry enter through the crystal mask: the caller
 * rasterises the crystal shape (slab, asymmetric trapezoid, any polygon) into
 * per-step index intervals, so every consumer sees the same binary Pi(x, z). */
typedef struct bpm_plan_desc {
    int32_t nx;              /* power of two, 64 <= nx <= 65536 */
    int32_t nz;              /* number of z-steps, >= 0 */
    double dx_um, dz_um;     /* > 0 */
    double x0_um;            /* x of sample 0 */
    double lambda_um;        /* vacuum wavelength, 0 < lambda < 2 d */
    double d_um;             /* spacing of the reflecting planes; h = 2 pi / d */
    bpm_complex chi0, chih, chihbar;  /* susceptibility harmonics 0, +h, -h (Eq. (8)) */
    int32_t nseg;            /* mask intervals per step, 1..4 */
    const int32_t *seg;      /* [nz][nseg][2] half-open [lo, hi) index intervals; lo >= hi
                                is empty; 0 <= lo, hi <= nx.  Copied at creation. */
    bpm_strain strain;
    int32_t det_lo, det_hi;  /* detector interval for R and T, 0 <= det_lo <= det_hi <= nx */
    int32_t precision;       /* bpm_precision */
    /* Splitting of each z-step (Eq. (13)).  0 or 1: Eq. (12), propagate then
     * couple with the Jacobi-Anger harmonics at z_n.  2: B(dz/2) A(dz) B(dz/2);
     * 4: B(t dz/2) A(t dz) B((1-t) dz/2) A((1-2t) dz) B((1-t) dz/2) A(t dz) B(t dz/2),
     * t = 1/(2 - 2^(1/3)).  For 2 and 4 a coupling sub-step B(b dz) is the
     * exponential of the two-beam coupling generator (which composes, so the
     * orders hold); it uses the mask row of step n and the strain at its own
     * height z_n + (a_1 + ... + a_i) dz (TABLE strain: row n). */
    int32_t split_order;
    /* 3D envelopes (the paper's 3D form, Eq. (4) with a 2D transverse transform):
     * ny = 0 or 1 is the x-z problem described above.  ny > 1 (a power of two,
     * 16 <= ny <= 256, with nx a power of two, 256 <= nx <= 1024; other sizes
     * return BPM_E_UNSUPPORTED) marches envelopes psi[ny][nx] (row i at
     * y_i = i*dy_um, periodic) through the 2D transform over (x, y) and the
     * propagator exp(i dzh (S(qx +/- s, qy) - c)), S(p, r) = sqrt(1 - p^2 - r^2).
     * Then seg is [nz][ny][nseg][2] (intervals along x per step and row), a
     * TABLE strain is [nz][ny][nx], POLY2 and EDGE_DISLOCATION do not depend
     * on y, R/T sum the detector interval [det_lo, det_hi) of every row, and
     * every state and host buffer holds ny*nx samples per beam. */
    int32_t ny;
    double dy_um;
} bpm_plan_desc;

typedef struct bpm_plan bpm_plan;
typedef struct bpm_batch bpm_batch;
typedef struct bpm_server bpm_server;

typedef struct bpm_plan_info {
    int32_t nx, nz, precision;
    int32_t threads_per_solve;   /* workgroup size of the march kernel */
    size_t state_bytes;          /* device bytes of one solve's envelope pair */
    size_t device_bytes;         /* device bytes held by the plan (tables, mask) */
    double cell_steps;           /* nx * nz * 2 */
} bpm_plan_info;

/* --- plans ------------------------------------------------------------------
 * bpm_plan_create validates the descriptor, copies every array it points to,
 * and builds the plan's device tables (propagators, coupling scalars) with FP64
 * setup kernels on the current device (plan setup of Eq. (12)'s p+-, Eq. (9)-(10)).
 * Errors: BPM_E_INVALID (nx not a power of two in [64, 65536], nz < 0, a spacing
 * or wavelength <= 0, lambda >= 2d, non-finite values, bad intervals, unknown
 * kinds, a coupling sub-step too long for its series: |A^2 chih chihbar| > 100
 * or |A chi0| > 700 with A = b k dz / (2 cos theta_B) and b the largest
 * splitting weight), BPM_E_UNSUPPORTED (nx too large for the library at this precision),
 * BPM_E_NOMEM, BPM_E_DEVICE.  *out is NULL on failure. */
bpm_status bpm_plan_create(const bpm_plan_desc *desc, bpm_plan **out);
void bpm_plan_destroy(bpm_plan *plan);
bpm_status bpm_plan_info_get(const bpm_plan *plan, bpm_plan_info *info);

/* Blocking march from host buffers (each nx complex128).  psi_m0 may be NULL
 * (zero reflected envelope).  Outputs psi_p_out, psi_m_out, R, T may each be
 * NULL.  Output buffers may alias the inputs.  Eq. (12) applied nz times. */
bpm_status bpm_propagate(bpm_plan *plan, const bpm_complex *psi_p0, const bpm_complex *psi_m0,
                         bpm_complex *psi_p_out, bpm_complex *psi_m_out, double *R, double *T);

/* Asynchronous march on device buffers owned by the caller, enqueued on
 * `stream` (a hipStream_t; NULL = default stream).  d_in and d_out each hold
 * one solve's state (psi+ then psi-, plan precision); they may be equal.
 * d_RT receives R, T (2 doubles) or may be NULL.
 * A plan of a staged size (FP32 nx >= 32768, FP64 nx >= 16384) or of 3D
 * envelopes marched this way (and by bpm_propagate) is spread over the whole
 * device: per coupling sub-step one launch over its rows and one over its
 * columns, z-steps replayed from a recorded graph of 32 steps (recorded on the
 * first call with nz >= 32).  Its envelopes equal a batch's one-workgroup march
 * bitwise; R and T are the same sums grouped per workgroup.  The plan keeps the
 * march's control block and partial sums, so calls on one plan must not
 * overlap (a plan is single-threaded); to march many solves at once use a
 * batch. */
bpm_status bpm_propagate_device(bpm_plan *plan, void *stream, const void *d_in, void *d_out,
                                double *d_RT);

/* bpm_propagate_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same march and arguments, bitwise the same results, but the
 * call allocates nothing and records no graph.  A wide-lane plan (staged size
 * or 3D envelopes) keeps its control block and per-workgroup partial sums in
 * a static device array of the library (16 KiB per device, held until the
 * process ends) instead of plan memory, and launches every z-step directly.
 * Every call on a device shares that array: calls that overlap on one device
 * race (as calls on one plan do).  BPM_E_INVALID for a NULL pointer,
 * BPM_E_UNSUPPORTED if a plan would need more scratch than the array holds,
 * BPM_E_DEVICE if its device address cannot be taken.  The plan itself is
 * created (and allocated) beforehand with bpm_plan_create. */
bpm_status bpm_propagate_device_noalloc(bpm_plan *plan, void *stream, const void *d_in, void *d_out,
                                        double *d_RT);

/* Far field (the far-field images of the paper's Sec. 7): the exit envelopes of
 * `plan` propagated through vacuum over distance_um along z in one FFT-based
 * step, each envelope about its own carrier (its own propagator, no coupling):
 * the field on the plane distance_um beyond the crystal's exit plane.  d_in and
 * d_out hold one solve's state as for bpm_propagate_device (may be equal),
 * enqueued on `stream`.  The library keeps one vacuum plan per plan for the
 * last distance used (created on first use; a new distance rebuilds it and
 * waits for the device).  BPM_E_INVALID for a NULL pointer or a distance that
 * is not finite and > 0. */
bpm_status bpm_far_field(bpm_plan *plan, double distance_um, void *stream, const void *d_in, void *d_out);

/* --- batches (many solves in one launch) ------------------------------------
 * A batch groups plans (any mix of nx, nz, wavelength, crystal, strain) into
 * one kernel launch per precision; solves are ordered longest first so the
 * hardware dispatcher balances uneven work.  The plans must outlive the batch.
 * bpm_batch_layout returns each solve's byte offset in the packed device
 * state buffer (offsets[n]) and the buffer's total size.  bpm_batch_run marches
 * every solve: state in d_in (packed), results to d_out (may equal d_in), R/T
 * of solve i to d_RT[2i], d_RT[2i+1] (may be NULL). */
bpm_status bpm_batch_create(bpm_plan *const *plans, int32_t n, bpm_batch **out);
bpm_status bpm_batch_layout(const bpm_batch *batch, size_t *offsets, size_t *total_bytes);
bpm_status bpm_batch_run(bpm_batch *batch, void *stream, const void *d_in, void *d_out,
                         double *d_RT);
void bpm_batch_destroy(bpm_batch *batch);

/* Time-domain assembly (the time-dependent method of Sec. 8).  The batch holds
 * M spectral components of one pulse (M a power of two, 128 <= M <= 2048),
 * ordered by ascending frequency at equal spacing, all on one x grid (same nx,
 * dx, x0) and precision, each marched to its exit plane z = L_m = nz_m dz_m;
 * d_state is the batch's packed state after bpm_batch_run.  Writes
 *   out[b][j][k] = sum_m psi_{b,m}(x_j) exp(i k_m c_m L_m) exp(-2 pi i m k / M)
 * for beams b = +, -, samples j and time samples k (t_k = k T / M,
 * T = 2 pi / frequency spacing): the field's time trace at the exit plane up
 * to a common phase per k.  exp(i k_m c_m L_m), c_m = sqrt(1 - (lambda_m/2d)^2),
 * restores the carrier phase along z the reduced propagator drops (FP64,
 * reduced exactly).  d_out: caller-owned [2][nx][M] complex in the batch
 * precision (8 B FP32, 16 B FP64).  Enqueued on `stream`.  BPM_E_INVALID for
 * another M or mixed grids. */
bpm_status bpm_td_assemble(bpm_batch *batch, void *stream, const void *d_state, void *d_out);

/* --- serving (continuous batching) ------------------------------------------
 * The paper evaluates independent realisations of the march (incidence angles,
 * photon energies, configurations) in parallel (Sec. 3); a server does so for a
 * stream of requests on one device.
 * A server owns a device-memory budget and a pool of solve slots.  A worker
 * thread advances all admitted solves together in rounds: per precision one
 * stream and one launch that takes every size and strain class side by side
 * (sizes below 1024 launch separately).  An FP32 nx = 16384 solve with a
 * polynomial strain advances chunk_steps z-steps per round; every other
 * (precision, size, strain class) the steps that take the same time at its
 * measured per-workgroup rate (at least 1), so no round waits long for one
 * class.  While a round runs, an admission thread builds the plans and
 * entrance states of requests admitted in arrival order whose state and tables
 * fit the budget; after it, finished solves are retired (their device blocks
 * return to the library's block cache rather than to the runtime) and the new
 * ones join the next round.  Per-solve arithmetic does not depend on what else
 * is in the launch, so a result is the same alone and in the mix.
 * Solves of a staged size or 3D envelopes with a long march ahead (an estimated
 * one-workgroup time of more than 0.5 s for their remaining steps; at most 4 at
 * a time, and only while at most 64 other solves are in the rounds: under load
 * the one-workgroup march does more work per second) move, at a round boundary,
 * to the wide lane of
 * bpm_propagate_device instead, 2*chunk_steps z-steps per round spread over the
 * device on a stream of their own; their envelopes are the same bitwise, R and
 * T the same sums grouped per workgroup. */
typedef struct bpm_server_desc {
    size_t hbm_budget_bytes;   /* device bytes the server may hold for admitted solves */
    int32_t max_slots;         /* max solves in flight */
    int32_t chunk_steps;       /* z-steps per round of an FP32 nx = 16384 bent solve (>= 1); other classes
                                  advance the steps that take the same time at their measured rate */
} bpm_server_desc;

typedef struct bpm_request {
    const bpm_plan_desc *plan;      /* copied at submit */
    const bpm_complex *psi_p0;      /* nx complex128, copied at submit */
    const bpm_complex *psi_m0;      /* may be NULL */
    bpm_complex *psi_p_out;         /* may be NULL; written before the ticket completes */
    bpm_complex *psi_m_out;         /* may be NULL */
} bpm_request;

typedef struct bpm_result {
    int32_t status;                 /* bpm_status of the solve */
    double R, T;
    double t_submit, t_admit, t_done;   /* seconds on the server's monotonic clock */
} bpm_result;

typedef struct bpm_server_stats {
    int64_t submitted, admitted, completed, cancelled, failed;
    int64_t launches;
    double cell_steps_done;
    size_t bytes_in_use, peak_bytes;
    int64_t wide;   /* solves marched in the wide lane (long staged-size / 3D solves, see bpm_server_create) */
    int64_t rounds;          /* rounds the march worker ran */
    int64_t active_max;      /* most solves marching in one round, waiting ones included */
    double t_device_wait_s;  /* worker time spent waiting for rounds to finish */
    double t_host_s;         /* worker time between rounds: retiring, freeing, building and launching */
} bpm_server_stats;

bpm_status bpm_server_create(const bpm_server_desc *desc, bpm_server **out);
/* Copies n requests and returns one ticket each.  BPM_E_BUDGET if a request can
 * never fit the budget (its ticket is still issued and completes with that
 * status); BPM_E_INVALID for a bad descriptor (no ticket issued for it). */
bpm_status bpm_batch_submit(bpm_server *server, const bpm_request *reqs, int32_t n,
                            uint64_t *tickets);
/* BPM_E_PENDING until done; then fills *out and returns BPM_OK (the solve's own
 * status is out->status).  A completed ticket can be polled repeatedly. */
bpm_status bpm_poll(bpm_server *server, uint64_t ticket, bpm_result *out);
/* Cancels a waiting or running ticket (it completes with BPM_E_CANCELLED). */
bpm_status bpm_cancel(bpm_server *server, uint64_t ticket);
bpm_status bpm_server_stats_get(bpm_server *server, bpm_server_stats *out);
/* Blocks until every submitted ticket has completed (or timeout_s elapses:
 * BPM_E_PENDING). */
bpm_status bpm_server_drain(bpm_server *server, double timeout_s);
void bpm_server_destroy(bpm_server *server);

/* --- schedules and autotuning ----------------------------------------------------
 * A batch marches each group of solves that share (precision, nx, strain class;
 * strain classes: none, POLY2, dislocation/table) with one kernel family:
 *   BPM_SCHED_UNIFORM  the per-size kernel: nx/16 threads per solve for nx up to
 *                      16384 FP32 / 8192 FP64, the staged kernel above;
 *   BPM_SCHED_MIXED    the mixed-size kernel: 512 (or 256) threads, nx/512
 *                      samples per thread (nx 1024..16384 FP32, ..8192 FP64);
 *   BPM_SCHED_ANY      the any-size kernel of the server: 512 threads, register-
 *                      resident sizes as MIXED, staged sizes with 512 threads
 *                      (nx >= 1024).
 * BPM_SCHED_DEFAULT is UNIFORM (and MIXED for a group of several sizes that the
 * mixed kernel takes).  The process-wide schedule table, consulted when a batch
 * is created, overrides the default per (precision, nx, strain class); 3D
 * envelopes and bpm_propagate keep their own kernels.  Schedules change the
 * samples per thread, so results change within rounding, not in value. */
typedef enum bpm_schedule {
    BPM_SCHED_DEFAULT = 0,
    BPM_SCHED_UNIFORM = 1,
    BPM_SCHED_MIXED = 2,
    BPM_SCHED_ANY = 3
} bpm_schedule;

typedef struct bpm_tune_result {
    int32_t schedule;   /* the fastest candidate, now in the table */
    int32_t nsolves, nsteps;
    double ms[4];       /* time of one batch march per candidate (index = schedule); 0 = not a candidate */
} bpm_tune_result;

/* Times every schedule that can march nx at `precision` on a synthetic batch of
 * nsolves solves (a crystal filling the window, strain of strain_kind: none, a
 * 1 m bend, a dislocation, or a zero table) over nsteps z-steps (one untimed run,
 * then the median of three), enters the fastest into the schedule table and
 * reports all.  A more general family (uniform, then mixed, then any) is
 * entered only when it is more than 1 % faster than the more specialised pick,
 * so timings within noise keep the specialised kernel.  Blocks; needs 1 <= nsolves <= 4096, 1 <= nsteps <= 100000.
 * BPM_E_INVALID for bad arguments, BPM_E_NOMEM / BPM_E_DEVICE on failure. */
bpm_status bpm_autotune(int32_t precision, int32_t nx, int32_t strain_kind, int32_t nsolves, int32_t nsteps,
                        bpm_tune_result *out);
/* Table entry for (precision, nx, strain kind): BPM_SCHED_DEFAULT removes it.
 * BPM_E_INVALID for a bad key or a schedule that cannot march nx. */
bpm_status bpm_schedule_set(int32_t precision, int32_t nx, int32_t strain_kind, int32_t schedule);
/* The table entry (BPM_SCHED_DEFAULT when none), or -1 for a bad key. */
int32_t bpm_schedule_get(int32_t precision, int32_t nx, int32_t strain_kind);
/* Write the table to a text file (one entry per line: precision log2(nx) strain
 * class schedule) / merge such a file into the table.  Loading checks every
 * line first and changes nothing on error (BPM_E_INVALID, message in
 * bpm_last_error). */
bpm_status bpm_schedule_save(const char *path);
bpm_status bpm_schedule_load(const char *path);

/* --- misc -------------------------------------------------------------------- */
const char *bpm_status_str(bpm_status s);
const char *bpm_last_error(void);
/* Largest nx the library marches at a precision (LDS/register-resident lane). */
int32_t bpm_max_nx(int32_t precision);

#ifdef __cplusplus
}
#endif
#endif
