// bpm_internal.hpp — structures shared by the host library and the gfx950 kernels.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace bpm {

enum Prec : int32_t { PREC_F64 = 0, PREC_F32 = 1 };
enum StrainKind : int32_t { STRAIN_NONE = 0, STRAIN_POLY2 = 1, STRAIN_EDGE = 2, STRAIN_TABLE = 3 };

// Strain classes compiled as separate kernels (one straight-line coupling each).
// SC_POLY1 is a polynomial phase without its X^2 term (c3 = 0, as a bend
// u = X Z / R): the FP32 per-size kernels have a copy for it, every other
// kernel takes it as SC_POLY2 (same results: the X^2 factor it leaves out is
// then exactly one).  strain_class() never returns it; march_class() does.
enum StrainClass : int { SC_NONE = 0, SC_POLY2 = 1, SC_GENERAL = 2, SC_POLY1 = 3 };
__host__ __device__ constexpr int strain_class(int kind)
{
    return kind == STRAIN_NONE ? SC_NONE : kind == STRAIN_POLY2 ? SC_POLY2 : SC_GENERAL;
}
__host__ __device__ constexpr int march_class(int kind, double c3)
{
    return strain_class(kind) == SC_POLY2 && c3 == 0.0 ? SC_POLY1 : strain_class(kind);
}

// Splitting of one z-step (Eq. (13)): the product A(a_1 dz) B(b_1 dz) ...
// A(a_m dz) B(b_m dz), applied from the left.  Order 1 is Eq. (12) (a = b = 1);
// order 2 is a = (0, 1), b = (1/2, 1/2); order 4 is a = (0, t, 1-2t, t),
// b = (t/2, (1-t)/2, (1-t)/2, t/2) with t = 1/(2 - 2^(1/3)).  Returns m (0 for
// an order this library does not know).
__host__ __device__ inline int split_sequence(int order, double *a, double *b)
{
    if (order == 0 || order == 1) {
        a[0] = 1.0, b[0] = 1.0;
        return 1;
    }
    if (order == 2) {
        a[0] = 0.0, a[1] = 1.0;
        b[0] = 0.5, b[1] = 0.5;
        return 2;
    }
    if (order == 4) {
        const double t = 1.0 / (2.0 - cbrt(2.0));
        a[0] = 0.0, a[1] = t, a[2] = 1.0 - 2.0 * t, a[3] = t;
        b[0] = 0.5 * t, b[1] = 0.5 * (1.0 - t), b[2] = 0.5 * (1.0 - t), b[3] = 0.5 * t;
        return 4;
    }
    return 0;
}
// Propagator tables a splitting needs: one per distinct nonzero a_i, in order
// of first use; table[i] is the table of sub-step i (-1 when a_i = 0).
__host__ __device__ inline int split_tables(int order, int *table, double *afrac)
{
    double a[4], b[4];
    const int m = split_sequence(order, a, b);
    int nt = 0;
    for (int i = 0; i < m; ++i) {
        table[i] = -1;
        if (a[i] == 0.0) continue;
        for (int k = 0; k < nt; ++k)
            if (afrac[k] == a[i]) table[i] = k;
        if (table[i] < 0) {
            afrac[nt] = a[i];
            table[i] = nt++;
        }
    }
    return nt;
}
constexpr int kMaxSub = 4;

// One coupling sub-step of a z-step: its coefficients, its height (in steps,
// from z_n) and the propagator table applied before it (-1: none).
struct SubStep {
    double d0x, d0y;          // a0 - 1     (harmonic 0, minus one)
    double apx, apy;          // a+         (harmonic +1, pairs with chi_h)
    double amx, amy;          // a-         (harmonic -1, pairs with chi_hbar)
    double zoff;
    int32_t table, pad;
};

// Per-plan scalars, produced on the device by the FP64 setup kernel.
struct PlanScalars {
    double k, h, s, c, dzh;   // 2pi/lambda, 2pi/d, h/(2k), sqrt(1-s^2), k*dz
    int32_t nsub, order;      // coupling sub-steps per z-step, splitting order
    SubStep sub[kMaxSub];
};

// Inputs of the setup kernel (host-filled).
struct PlanParams {
    int32_t nx, split_order;
    double dx, dz, lambda, d;
    double chi0x, chi0y, chihx, chihy, chihbx, chihby;
    int32_t ny, pad;          // ny > 1: 3D envelopes [ny][nx]
    double dy;
};

// 3D envelopes: nx = 2^k3DLog2NxMin..2^k3DLog2NxMax (one wave per x row, nx/64
// samples per thread and beam), ny = 2^k3DLog2NyMin..2^k3DLog2NyMax.
constexpr int k3DLog2NxMin = 8, k3DLog2NxMax = 10, k3DLog2NyMin = 4, k3DLog2NyMax = 8;
// bytes of one propagator table entry (P - 1)/N, both precisions: FP32 keeps
// it as hi + lo pairs of floats, FP64 as (re, im)
constexpr size_t kPropEntryBytes = 16;
// launch kind of a 3D group: kLaunch3D + 16 (log2 nx - k3DLog2NxMin) + log2 ny
constexpr int kLaunch3D = 100;
constexpr int kind_3d(int log2nx, int log2ny) { return kLaunch3D + 16 * (log2nx - k3DLog2NxMin) + log2ny; }
constexpr int kind3d_log2nx(int kind) { return k3DLog2NxMin + (kind - kLaunch3D) / 16; }
constexpr int kind3d_log2ny(int kind) { return (kind - kLaunch3D) % 16; }
constexpr bool is_kind_3d(int kind)
{
    return kind >= kLaunch3D && kind3d_log2nx(kind) <= k3DLog2NxMax && kind3d_log2ny(kind) >= k3DLog2NyMin &&
           kind3d_log2ny(kind) <= k3DLog2NyMax;
}

// Flags of one solve in one launch.
enum SolveFlags : int32_t {
    SF_FIRST = 1,   // launch starts at z-step 0: compute the incident power
    SF_LAST = 2     // launch ends at z-step nz: write R and T
};

// One solve inside one launch.  Host-built, copied to the device once per batch.
struct SolveDesc {
    int32_t log2n, nz, nseg, strain_kind;
    int32_t det_lo, det_hi, step0, nsteps;   // run z-steps [step0, step0 + nsteps)
    int32_t flags;
    int32_t opaque_zero;                     // always 0 (keeps per-step table reads in the loop)
    int32_t rt_index;                        // R,T go to RT[2*rt_index], -1 = none
    int32_t disl_m;                          // EDGE: b/d when it is a whole number 1..8 (else 0)
    const PlanScalars *sc;
    const void *prop;        // [2][nx] (P - 1)/nx in solve precision
    const void *tw;          // twiddle table of the (nx, elements-per-thread, precision) schedule
    const int32_t *seg;      // [nz][nseg][2]
    const void *utab;        // STRAIN_TABLE: [nz][nx] u/d reduced to [-1/2, 1/2), solve precision
    double *pin;             // incident power (written when SF_FIRST, read when SF_LAST)
    double x0, dx, dz, inv_d;
    double x_ref, z_ref;
    double c[6];             // POLY2 coefficients
    double disl_k, disl_q;   // EDGE: b/(2 pi d), 1/(2 (1 - nu))
    uint64_t in_off, out_off;  // byte offsets of the state in the launch's in/out buffers
};

// Staged (four-step) lane: 2^staged_log2e samples per thread and beam, rows of
// one wave (2^(6 + log2e) points); its own kernel runs staged_log2th threads
// per solve, the any-size kernel 2^kStagedAnyLog2Th.  staged_prefetch: the
// kernels keep the next round's state loads in flight while a round computes
// (FP32: with 512 threads the register budget holds the second set of samples;
// 1024 threads without it waited for every round's loads, 4 % slower).
constexpr int kStagedAnyLog2Th = 9;
constexpr int staged_log2e(int prec) { return 3; }
constexpr int staged_log2c(int prec) { return 6 + staged_log2e(prec); }
constexpr int staged_log2th(int prec) { return 9; }
constexpr bool staged_prefetch(int prec) { return prec == PREC_F32; }
// 3D envelopes: rows of nx = 2^log2nx samples, nx/64 per thread and beam.
// Threads per solve: FP32 1024 for rows of 512 or fewer samples without the
// dislocation / table coupling, else 512 (that coupling's per-row mask and
// strain reads spill in a 1024-thread workgroup's register budget, and so do
// 16 samples per thread; 512 threads march the 3D batch 12 % faster); FP64
// 512, and 256 for rows of 1024 (16 FP64 samples per beam need more than the
// 256 registers a 512-thread workgroup leaves each lane).
constexpr int staged3d_log2th(int prec, int sc, int log2nx)
{
    if (prec == PREC_F64) return log2nx >= 10 ? 8 : 9;
    return sc != SC_GENERAL && log2nx <= 9 ? 10 : 9;
}

// Wide lane: one staged-size or 3D solve spread over the device, two launches
// (row phase, column phase) per coupling sub-step.  The control block carries
// what changes from call to call, so recorded step graphs stay valid.
struct WideCtl {
    int32_t base, pad;   // z-step of the graph's step k = 0
    const char *in;      // entrance state (entry phase)
    char *out;           // the solve's state
};
enum WidePhase { WIDE_ENTRY = 0, WIDE_ROWS = 1, WIDE_COLS = 2 };
struct WideArgs {
    const SolveDesc *desc;   // one descriptor (state at in/out offsets of the control block's buffers)
    const WideCtl *ctl;
    int k, i;                // step base + k, sub-step i
    double *part;            // [3][blocks] partial sums: incident power, |psi+|^2, |psi-|^2
};
struct WideShape {
    int row_blocks, col_blocks;
    size_t lds_bytes;
};
// launch one phase of a wide march (kind: log2 nx of a staged size or
// kind_3d(log2 nx, log2 ny)); shape (may be NULL) receives the grid sizes
hipError_t launch_wide(int prec, int kind, int sc, int phase, const WideArgs &a, hipStream_t s, WideShape *shape);
hipError_t launch_wide_finish(const SolveDesc *desc, const double *part, int nblk, double *rt, hipStream_t s);
// the control block's step base and buffers, and the descriptor's step range and flags
hipError_t launch_wide_ctl(WideCtl *ctl, SolveDesc *desc, int base, const char *in, char *out, int step0, int nsteps,
                           int flags, hipStream_t s);
// does a plan of this kind have a wide form
bool wide_kind(int prec, int kind);

// Elements per thread (log2) used for a given nx by the uniform-size kernels.
constexpr int uniform_log2e(int log2n) { return log2n >= 8 ? 4 : (log2n >= 7 ? 3 : 2); }

// Launchers (bpm_setup.hip).  All return hipSuccess or the launch error.
// d_sc or d_prop may be NULL to skip that part; d_prop receives the table of a
// sub-step of afrac*dz over `cells` = nx (or nx*ny for 3D, [ky][kx] order)
// entries per beam; log2r > 0 stores the propagator of a staged size in
// [k1][k2] order (R = 2^log2r).
// lift: FP32 propagator entries in the lifting form of the staged 2D kernels
hipError_t launch_plan_setup(const PlanParams *d_params, PlanScalars *d_sc, void *d_prop, int prec,
                             int cells, int log2r, double afrac, bool lift, hipStream_t s);
hipError_t launch_twiddles(void *d_tw, int prec, int log2n, int log2e, hipStream_t s);
size_t twiddle_bytes(int prec, int log2n, int log2e);
// Staged sizes (four-step lane): whether log2n is one, and its twiddle table
// [row FFT | column FFT | four-step].
bool is_staged(int prec, int log2n);
// 3D envelopes: twiddle table [row FFT | column FFT] and launch shape.
size_t twiddle3d_bytes(int prec, int log2nx, int log2ny);
hipError_t launch_twiddles_3d(void *d_tw, int prec, int log2nx, int log2ny, hipStream_t s);
void march_shape_3d(int prec, int sc, int log2nx, int log2ny, int *threads, size_t *lds_bytes);
size_t staged_twiddle_bytes(int prec, int log2n);
hipError_t launch_staged_twiddles(void *d_tw, int prec, int log2n, hipStream_t s);
hipError_t launch_utab(const double *d_u, void *d_tab, int prec, size_t count, double inv_d,
                       hipStream_t s);
// March every solve of a launch.  All descs share prec and strain class `sc`
// (0 none, 1 polynomial, 2 dislocation/table); if `uniform_log2n` >= 0 they also
// share nx and use the uniform (or, for staged sizes, the staged) kernel;
// kLaunchMixed selects the mixed-size kernel (register-resident sizes from
// 2^mixed_min_log2n), kLaunchAny the kernel that takes any size from
// 2^mixed_min_log2n up to the largest.
constexpr int kLaunchMixed = -1, kLaunchAny = -2;
hipError_t launch_march(const SolveDesc *d_descs, int n, int prec, int uniform_log2n, int sc,
                        const char *in_base, char *out_base, double *rt, hipStream_t s);
// Time-domain assembly (bpm_td.hip): 2^kTdLog2MMin..2^kTdLog2MMax components.
// par holds (lambda, d, L) per component; ph receives the carriers (M complex).
constexpr int kTdLog2MMin = 7, kTdLog2MMax = 11;
hipError_t launch_td(int prec, int log2m, const char *state, const uint64_t *offs, const double *par, void *ph,
                     const void *tw, int nx, void *out, hipStream_t s);
// Launch shape of the uniform or staged kernel (threads per workgroup, dynamic LDS bytes).
void march_shape(int prec, int log2n, int *threads, size_t *lds_bytes);
// Mixed-size kernel: elements-per-thread (log2) it uses for log2n, and its shape.
int mixed_log2e(int prec, int log2n);
void mixed_shape(int prec, int *threads, size_t *lds_bytes);
int max_log2n(int prec);
int mixed_min_log2n(int prec);
int mixed_max_log2n(int prec);

}  // namespace bpm
