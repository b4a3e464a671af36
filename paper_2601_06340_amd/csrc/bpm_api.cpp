// bpm_api.cpp — the C ABI of libbpm_hip.so (plans, batches, errors).
// The serving loop lives in bpm_server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bpm.h"
#include "bpm_api_internal.hpp"
#include "bpm_internal.hpp"

using namespace bpm;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

bpm_status bpm::fail(bpm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = std::string(bpm_status_str(s)) + ": " + buf;
    return s;
}

extern "C" const char *bpm_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *bpm_status_str(bpm_status s)
{
    switch (s) {
    case BPM_OK: return "BPM_OK";
    case BPM_E_INVALID: return "BPM_E_INVALID";
    case BPM_E_NOMEM: return "BPM_E_NOMEM";
    case BPM_E_DEVICE: return "BPM_E_DEVICE";
    case BPM_E_BUDGET: return "BPM_E_BUDGET";
    case BPM_E_PENDING: return "BPM_E_PENDING";
    case BPM_E_CANCELLED: return "BPM_E_CANCELLED";
    case BPM_E_NOTFOUND: return "BPM_E_NOTFOUND";
    case BPM_E_UNSUPPORTED: return "BPM_E_UNSUPPORTED";
    case BPM_E_NUMERIC: return "BPM_E_NUMERIC";
    }
    return "BPM_E_UNKNOWN";
}

bpm_status bpm::hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(BPM_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(BPM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ device check
bpm_status bpm::ensure_device()
{
    static std::once_flag once;
    static bpm_status st = BPM_OK;
    static std::string msg;
    std::call_once(once, [] {
        int dev = 0, count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
            st = BPM_E_DEVICE;
            msg = "no HIP device";
            return;
        }
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            st = BPM_E_DEVICE;
            msg = "hipGetDeviceProperties failed";
            return;
        }
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            st = BPM_E_DEVICE;
            msg = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
        }
    });
    if (st != BPM_OK) return fail(st, "%s", msg.c_str());
    return BPM_OK;
}

// ------------------------------------------------------------------ setup stream
// Plan setup (table kernels, uploads) runs on a library-owned non-blocking
// stream per device and waits only for that stream, so creating a plan never
// waits for marches running on other streams.
static std::mutex g_setup_mu;
static std::map<int, hipStream_t> g_setup;

hipStream_t bpm::setup_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_setup_mu);
    auto it = g_setup.find(dev);
    if (it != g_setup.end()) return it->second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    g_setup[dev] = st;
    return st;
}

// ------------------------------------------------------------------ twiddle cache
// One table per (precision, nx, elements per thread), shared by every plan.
static std::mutex g_tw_mu;
static std::map<std::tuple<int, int, int>, void *> g_tw;

bpm_status bpm::twiddle_table(int prec, int log2n, int log2e, const void **out)
{
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_tuple(prec, log2n, log2e);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) {
        *out = it->second;
        return BPM_OK;
    }
    // log2e = 0 names the combined table of a staged size, -log2(nx) that of
    // 3D envelopes with log2(ny) = log2n - log2(nx)
    const size_t bytes = std::max<size_t>(log2e > 0    ? twiddle_bytes(prec, log2n, log2e)
                                          : log2e == 0 ? staged_twiddle_bytes(prec, log2n)
                                                       : twiddle3d_bytes(prec, -log2e, log2n + log2e),
                                          16);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return hip_fail(e, "twiddle table");
    hipStream_t ss = setup_stream();
    e = log2e > 0    ? launch_twiddles(p, prec, log2n, log2e, ss)
        : log2e == 0 ? launch_staged_twiddles(p, prec, log2n, ss)
                     : launch_twiddles_3d(p, prec, -log2e, log2n + log2e, ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "twiddle setup kernel");
    }
    g_tw[key] = p;
    *out = p;
    return BPM_OK;
}

// ------------------------------------------------------------------ propagator cache
// The propagator table (Eq. (12), P+- with the 1/nx fold) depends only on the
// precision, nx, dx, dz, lambda and d.  Plans that agree on these share one
// reference-counted device copy, so a batch of solves that differ in crystal,
// strain or incident beam reads a single table that stays in L2.
using PropKey = std::tuple<int, int, double, double, double, double, int, int, double>;
struct PropEntry {
    void *ptr;
    int refs;
};
static std::mutex g_prop_mu;
static std::map<PropKey, PropEntry> g_prop;

static bpm_status prop_acquire(const bpm_plan_desc &d, const PlanParams *d_params, void **out)
{
    std::lock_guard<std::mutex> lk(g_prop_mu);
    const int order = d.split_order <= 1 ? 1 : d.split_order;
    const int ny = d.ny > 1 ? d.ny : 1;
    const PropKey key{d.precision, d.nx, d.dx_um, d.dz_um, d.lambda_um, d.d_um, order, ny, ny > 1 ? d.dy_um : 0.0};
    auto it = g_prop.find(key);
    if (it != g_prop.end()) {
        ++it->second.refs;
        *out = it->second.ptr;
        return BPM_OK;
    }
    // one table per distinct propagation fraction of the splitting
    int tab[kMaxSub];
    double afrac[kMaxSub];
    const int ntab = split_tables(order, tab, afrac);
    const size_t one = 2 * (size_t)d.nx * ny * kPropEntryBytes;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, one * ntab);
    if (e != hipSuccess) return hip_fail(e, "propagator table");
    // built and finished under the lock: a second plan never sees a table in flight
    int log2n = 0;
    while ((1 << log2n) < d.nx) ++log2n;
    const int log2r = ny == 1 && is_staged(d.precision, log2n) ? log2n - staged_log2c(d.precision) : 0;
    // the staged 2D kernels read FP32 entries in the lifting form
    const bool lift = d.precision == BPM_F32 && ny == 1 && is_staged(d.precision, log2n);
    hipStream_t ss = setup_stream();
    for (int k = 0; k < ntab && e == hipSuccess; ++k)
        e = launch_plan_setup(d_params, nullptr, (char *)p + k * one, d.precision, d.nx * ny, log2r, afrac[k], lift,
                              ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "propagator setup kernel");
    }
    g_prop[key] = PropEntry{p, 1};
    *out = p;
    return BPM_OK;
}

static void prop_release(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_prop_mu);
    for (auto it = g_prop.begin(); it != g_prop.end(); ++it)
        if (it->second.ptr == p) {
            if (--it->second.refs == 0) {
                (void)hipFree(p);
                g_prop.erase(it);
            }
            return;
        }
}

// ------------------------------------------------------------------ plans
static bool is_finite(double v) { return std::isfinite(v); }
static bool is_finite(bpm_complex c) { return std::isfinite(c.re) && std::isfinite(c.im); }

// largest table (mask, strain table) one solve may hold: the kernels index
// them with 32-bit byte offsets
constexpr long long kMaxTableBytes = 0x7fffffffLL;
// bounds on one coupling sub-step (see validate_desc)
constexpr double kMaxCouplingY = 100.0, kMaxCouplingPhase = 700.0;

bpm_status bpm::validate_desc(const bpm_plan_desc *d)
{
    if (!d) return fail(BPM_E_INVALID, "NULL descriptor");
    if (d->nx < 64 || d->nx > 65536 || (d->nx & (d->nx - 1)))
        return fail(BPM_E_INVALID, "nx = %d is not a power of two in [64, 65536]", d->nx);
    if (d->nz < 0) return fail(BPM_E_INVALID, "nz = %d < 0", d->nz);
    if (!is_finite(d->dx_um) || d->dx_um <= 0 || !is_finite(d->dz_um) || d->dz_um <= 0)
        return fail(BPM_E_INVALID, "dx and dz must be finite and > 0");
    if (!is_finite(d->x0_um)) return fail(BPM_E_INVALID, "x0 is not finite");
    if (!is_finite(d->lambda_um) || d->lambda_um <= 0 || !is_finite(d->d_um) || d->d_um <= 0)
        return fail(BPM_E_INVALID, "lambda and d must be finite and > 0");
    if (!(d->lambda_um < 2.0 * d->d_um)) return fail(BPM_E_INVALID, "lambda >= 2d: no Bragg angle");
    if (!is_finite(d->chi0) || !is_finite(d->chih) || !is_finite(d->chihbar))
        return fail(BPM_E_INVALID, "susceptibilities must be finite");
    if (d->split_order == 0 || d->split_order == 1 || d->split_order == 2 || d->split_order == 4) {
        // The coupling coefficients of a sub-step (Eq. (9)-(12)) are series in
        // y = -A^2 chih chihbar and carry exp(i A chi0), A = b k dz / 2 cos(theta_B).
        // Bounding |y| keeps the 60-term series converged and free of ruinous
        // cancellation (its largest term stays below 1e7), bounding |A chi0|
        // keeps the exponential finite: every coefficient is finite, which the
        // march relies on where it weights the coupling by 0 outside the crystal.
        double a[kMaxSub], b[kMaxSub];
        const int m = split_sequence(d->split_order, a, b);
        double bmax = 0.0;
        for (int i = 0; i < m; ++i) bmax = std::max(bmax, std::fabs(b[i]));
        const double k = 2.0 * M_PI / d->lambda_um, s = M_PI / (d->d_um * k);
        const double A = bmax * k * d->dz_um / (2.0 * std::sqrt(1.0 - s * s));
        const double y = A * A * std::hypot(d->chih.re, d->chih.im) * std::hypot(d->chihbar.re, d->chihbar.im);
        const double g = A * std::hypot(d->chi0.re, d->chi0.im);
        if (!(y <= kMaxCouplingY) || !(g <= kMaxCouplingPhase))
            return fail(BPM_E_INVALID,
                        "coupling step too long: |A^2 chih chihbar| = %.3g (at most %g), |A chi0| = %.3g (at most %g); "
                        "reduce dz",
                        y, kMaxCouplingY, g, kMaxCouplingPhase);
    }
    const bool d3 = d->ny > 1;
    if (d->ny < 0) return fail(BPM_E_INVALID, "ny = %d < 0", d->ny);
    if (d3) {
        if ((d->ny & (d->ny - 1)) || d->ny < (1 << k3DLog2NyMin) || d->ny > (1 << k3DLog2NyMax))
            return fail(BPM_E_UNSUPPORTED, "3D envelopes need ny a power of two in [%d, %d], got %d", 1 << k3DLog2NyMin,
                        1 << k3DLog2NyMax, d->ny);
        if ((d->nx & (d->nx - 1)) || d->nx < (1 << k3DLog2NxMin) || d->nx > (1 << k3DLog2NxMax))
            return fail(BPM_E_UNSUPPORTED, "3D envelopes need nx a power of two in [%d, %d], got %d",
                        1 << k3DLog2NxMin, 1 << k3DLog2NxMax, d->nx);
        if (!is_finite(d->dy_um) || d->dy_um <= 0) return fail(BPM_E_INVALID, "dy must be finite and > 0");
    }
    const long long rows = (long long)d->nz * (d3 ? d->ny : 1);
    if (d->nseg < 1) return fail(BPM_E_INVALID, "nseg = %d < 1", d->nseg);
    if (d->nseg > 4) return fail(BPM_E_UNSUPPORTED, "nseg = %d: at most 4 mask intervals per step", d->nseg);
    if (d->nz > 0 && !d->seg) return fail(BPM_E_INVALID, "seg is NULL");
    if (rows * d->nseg * 8 > kMaxTableBytes)
        return fail(BPM_E_UNSUPPORTED, "mask of %lld rows x %d intervals: at most 2 GiB per solve", rows, d->nseg);
    for (long long i = 0; i < rows * d->nseg; ++i) {
        const int lo = d->seg[2 * i], hi = d->seg[2 * i + 1];
        if (lo < 0 || hi < 0 || lo > d->nx || hi > d->nx)
            return fail(BPM_E_INVALID, "mask interval %lld = [%d, %d) outside [0, %d]", i, lo, hi, d->nx);
    }
    const bpm_strain &st = d->strain;
    switch (st.kind) {
    case BPM_STRAIN_NONE: break;
    case BPM_STRAIN_POLY2:
        for (double c : st.c)
            if (!is_finite(c)) return fail(BPM_E_INVALID, "POLY2 coefficient not finite");
        if (!is_finite(st.x_ref_um) || !is_finite(st.z_ref_um)) return fail(BPM_E_INVALID, "strain origin not finite");
        break;
    case BPM_STRAIN_EDGE_DISLOCATION:
        if (!is_finite(st.b_um) || !is_finite(st.nu) || st.nu >= 1.0 || !is_finite(st.x_ref_um) || !is_finite(st.z_ref_um))
            return fail(BPM_E_INVALID, "dislocation parameters invalid (need finite b, nu < 1, core)");
        break;
    case BPM_STRAIN_TABLE:
        if (d->nz > 0 && !st.u_table) return fail(BPM_E_INVALID, "u_table is NULL");
        // the kernels read tables through 32-bit byte offsets
        if (rows * d->nx * (d->precision == BPM_F32 ? 4LL : 8LL) > kMaxTableBytes)
            return fail(BPM_E_UNSUPPORTED, "strain table of %lld x %d samples: at most 2 GiB per solve", rows, d->nx);
        for (long long i = 0; i < rows * d->nx; ++i)
            if (!is_finite(st.u_table[i])) return fail(BPM_E_INVALID, "u_table[%lld] not finite", i);
        break;
    default: return fail(BPM_E_INVALID, "unknown strain kind %d", st.kind);
    }
    if (d->det_lo < 0 || d->det_hi > d->nx || d->det_lo > d->det_hi)
        return fail(BPM_E_INVALID, "detector [%d, %d) outside [0, %d]", d->det_lo, d->det_hi, d->nx);
    if (d->precision != BPM_F64 && d->precision != BPM_F32)
        return fail(BPM_E_INVALID, "unknown precision %d", d->precision);
    if (d->split_order != 0 && d->split_order != 1 && d->split_order != 2 && d->split_order != 4)
        return fail(BPM_E_INVALID, "split_order = %d: 1 (or 0), 2 or 4", d->split_order);
    int log2n = 0;
    while ((1 << log2n) < d->nx) ++log2n;
    if (log2n > max_log2n(d->precision))
        return fail(BPM_E_UNSUPPORTED, "nx = %d above the largest size the library marches at %s (%d)", d->nx,
                    d->precision == BPM_F32 ? "FP32" : "FP64", 1 << max_log2n(d->precision));
    return BPM_OK;
}

static size_t elem_bytes(int prec) { return prec == BPM_F32 ? 8 : 16; }

void bpm_plan::release()
{
    if (far) {
        far->release();
        delete far;
        far = nullptr;
    }
    dev_free(d_sc);
    dev_free(d_params);
    prop_release(d_prop);
    dev_free(d_seg);
    dev_free(d_utab);
    dev_free(d_pin);
    dev_free(d_desc1);
    dev_free(d_state);
    dev_free(d_rt);
    if (wide_exec) (void)hipGraphExecDestroy(wide_exec);
    if (wide_graph) (void)hipGraphDestroy(wide_graph);
    dev_free(d_wide_ctl);
    dev_free(d_wide_part);
    wide_exec = nullptr;
    wide_graph = nullptr;
    d_wide_ctl = nullptr;
    d_wide_part = nullptr;
    d_sc = nullptr;
    d_params = nullptr;
    d_prop = d_utab = d_state = nullptr;
    d_seg = nullptr;
    d_pin = d_rt = nullptr;
    d_desc1 = nullptr;
}

size_t bpm_plan::state_bytes() const { return 2 * cells() * elem_bytes(desc.precision); }

void bpm_plan::fill(SolveDesc &s, int log2e, const void *tw, int flags, int step0, int nsteps, uint64_t in_off,
                    uint64_t out_off, int rt_index) const
{
    std::memset(&s, 0, sizeof s);
    s.log2n = log2n;
    s.nz = desc.nz;
    s.nseg = desc.nseg;
    s.strain_kind = desc.strain.kind;
    s.det_lo = desc.det_lo;
    s.det_hi = desc.det_hi;
    s.step0 = step0;
    s.nsteps = nsteps;
    s.flags = flags;
    s.opaque_zero = 0;
    s.rt_index = rt_index;
    s.sc = d_sc;
    s.prop = d_prop;
    s.tw = tw;
    s.seg = d_seg;
    s.utab = d_utab;
    s.pin = d_pin;
    s.x0 = desc.x0_um;
    s.dx = desc.dx_um;
    s.dz = desc.dz_um;
    s.inv_d = 1.0 / desc.d_um;
    s.x_ref = desc.strain.x_ref_um;
    s.z_ref = desc.strain.z_ref_um;
    for (int i = 0; i < 6; ++i) s.c[i] = desc.strain.c[i];
    s.disl_k = desc.strain.b_um / (2.0 * M_PI * desc.d_um);
    s.disl_q = 1.0 / (2.0 * (1.0 - desc.strain.nu));
    // a Burgers vector that is a whole number of plane spacings winds the phase
    // by whole turns: exp(i h u) then has the algebraic factor ((X + i Z)/r)^m
    const double bd = desc.strain.b_um / desc.d_um, m = std::nearbyint(bd);
    s.disl_m = (desc.strain.kind == BPM_STRAIN_EDGE_DISLOCATION && std::fabs(bd - m) <= 1e-9 * std::fabs(bd) &&
                std::fabs(m) >= 1 && std::fabs(m) <= 8) ? (int32_t)m : 0;
    s.in_off = in_off;
    s.out_off = out_off;
    (void)log2e;
}

// ------------------------------------------------------------------ device block cache
// Plan tables, masks, descriptors and solve states come from size classes of
// powers of two (256 B to 64 MiB).  A released block goes back to its class's
// free list instead of hipFree, which waits for the whole device: a server
// creating and destroying plans at hundreds per second then allocates and frees
// no device memory in its steady state.  Larger blocks, and releases that would
// take the cached total beyond kCacheCap, go to hipFree.  The caller makes sure
// no kernel still uses a block it releases (plans wait for the device first).
namespace {
constexpr int kMinClassLog2 = 8, kMaxClassLog2 = 26;
constexpr size_t kCacheCap = size_t(4) << 30;
std::mutex g_blk_mu;
std::map<void *, int> g_blk_class;   // block -> log2 of its class (-1: allocated directly)
std::vector<void *> g_blk_free[kMaxClassLog2 + 1];
size_t g_blk_cached = 0;
}  // namespace

hipError_t bpm::dev_malloc(void **p, size_t bytes)
{
    int l = kMinClassLog2;
    while (l <= kMaxClassLog2 && (size_t(1) << l) < bytes) ++l;
    if (l > kMaxClassLog2) {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_blk_mu);
            g_blk_class[*p] = -1;
        }
        return e;
    }
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        if (!g_blk_free[l].empty()) {
            *p = g_blk_free[l].back();
            g_blk_free[l].pop_back();
            g_blk_cached -= size_t(1) << l;
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, size_t(1) << l);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        g_blk_class[*p] = l;
    }
    return e;
}

void bpm::dev_free(void *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        auto it = g_blk_class.find(p);
        if (it != g_blk_class.end() && it->second >= 0 && g_blk_cached + (size_t(1) << it->second) <= kCacheCap) {
            g_blk_free[it->second].push_back(p);
            g_blk_cached += size_t(1) << it->second;
            return;
        }
        if (it != g_blk_class.end()) g_blk_class.erase(it);
    }
    (void)hipFree(p);
}

template <typename F>
static bpm_status dev_alloc(F **p, size_t bytes, const char *what)
{
    hipError_t e = dev_malloc((void **)p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) return hip_fail(e, what);
    return BPM_OK;
}

extern "C" bpm_status bpm_plan_create(const bpm_plan_desc *d, bpm_plan **out)
{
    if (!out) return fail(BPM_E_INVALID, "out is NULL");
    *out = nullptr;
    bpm_status st = validate_desc(d);
    if (st != BPM_OK) return st;
    if ((st = ensure_device()) != BPM_OK) return st;

    bpm_plan *p = new (std::nothrow) bpm_plan();
    if (!p) return fail(BPM_E_NOMEM, "host allocation");
    p->desc = *d;
    p->desc.seg = nullptr;
    p->desc.strain.u_table = nullptr;
    p->log2n = 0;
    while ((1 << p->log2n) < d->nx) ++p->log2n;
    if (d->ny > 1) {
        while ((1 << p->log2ny) < d->ny) ++p->log2ny;
        p->log2n += p->log2ny;   // 3D: log2 of the samples per beam
    }
    p->launch_kind = p->log2ny ? kind_3d(p->log2n - p->log2ny, p->log2ny) : p->log2n;
    const int prec = d->precision;
    const size_t nx = p->cells(), nz = d->nz, rows = std::max<size_t>(p->rows(), 1);   // nx: samples per beam

    auto bail = [&](bpm_status s) {
        p->release();
        delete p;
        return s;
    };
    if ((st = dev_alloc(&p->d_sc, sizeof(PlanScalars), "plan scalars")) != BPM_OK) return bail(st);
    if ((st = dev_alloc(&p->d_params, sizeof(PlanParams), "plan params")) != BPM_OK) return bail(st);
    if ((st = dev_alloc(&p->d_seg, rows * d->nseg * 2 * sizeof(int32_t), "mask")) != BPM_OK) return bail(st);
    if ((st = dev_alloc(&p->d_pin, sizeof(double), "incident power")) != BPM_OK) return bail(st);
    if ((st = dev_alloc(&p->d_rt, 2 * sizeof(double), "R/T")) != BPM_OK) return bail(st);
    int tab[kMaxSub];
    double afrac[kMaxSub];
    const int ntab = split_tables(d->split_order <= 1 ? 1 : d->split_order, tab, afrac);
    p->device_bytes = sizeof(PlanScalars) + sizeof(PlanParams) + 2 * nx * elem_bytes(prec) * ntab +
                      rows * d->nseg * 2 * sizeof(int32_t) + 3 * sizeof(double);

    PlanParams pp;
    std::memset(&pp, 0, sizeof pp);
    pp.nx = d->nx;
    pp.dx = d->dx_um;
    pp.dz = d->dz_um;
    pp.lambda = d->lambda_um;
    pp.d = d->d_um;
    pp.chi0x = d->chi0.re;
    pp.chi0y = d->chi0.im;
    pp.chihx = d->chih.re;
    pp.chihy = d->chih.im;
    pp.chihbx = d->chihbar.re;
    pp.chihby = d->chihbar.im;
    pp.split_order = d->split_order <= 1 ? 1 : d->split_order;
    pp.ny = d->ny > 1 ? d->ny : 1;
    pp.dy = d->ny > 1 ? d->dy_um : 0.0;
    hipStream_t ss = setup_stream();
    hipError_t e = hipMemcpyAsync(p->d_params, &pp, sizeof pp, hipMemcpyHostToDevice, ss);
    if (e == hipSuccess && nz > 0)
        e = hipMemcpyAsync(p->d_seg, d->seg, p->rows() * d->nseg * 2 * sizeof(int32_t), hipMemcpyHostToDevice, ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (e != hipSuccess) return bail(hip_fail(e, "plan upload"));
    e = launch_plan_setup(p->d_params, p->d_sc, nullptr, prec, d->nx, 0, 1.0, false, ss);
    if (e != hipSuccess) return bail(hip_fail(e, "plan setup kernel"));
    if ((st = prop_acquire(*d, p->d_params, &p->d_prop)) != BPM_OK) return bail(st);

    if (d->strain.kind == BPM_STRAIN_TABLE && nz > 0) {
        double *d_u = nullptr;
        if ((st = dev_alloc(&d_u, nz * nx * sizeof(double), "strain staging")) != BPM_OK) return bail(st);
        if ((st = dev_alloc(&p->d_utab, nz * nx * (prec == BPM_F32 ? 4 : 8), "strain table")) != BPM_OK) {
            dev_free(d_u);
            return bail(st);
        }
        e = hipMemcpyAsync(d_u, d->strain.u_table, nz * nx * sizeof(double), hipMemcpyHostToDevice, ss);
        if (e == hipSuccess) e = launch_utab(d_u, p->d_utab, prec, nz * nx, 1.0 / d->d_um, ss);
        if (e == hipSuccess) e = hipStreamSynchronize(ss);
        dev_free(d_u);
        if (e != hipSuccess) return bail(hip_fail(e, "strain table"));
        p->device_bytes += nz * nx * (prec == BPM_F32 ? 4 : 8);
    }
    e = hipStreamSynchronize(ss);
    if (e != hipSuccess) return bail(hip_fail(e, "plan setup"));

    const int log2e = uniform_log2e(p->log2n);
    const int tw_key = p->log2ny ? -(p->log2n - p->log2ny) : is_staged(prec, p->log2n) ? 0 : log2e;
    if ((st = twiddle_table(prec, p->log2n, tw_key, &p->tw_uniform)) != BPM_OK) return bail(st);
    if (p->log2ny)
        march_shape_3d(prec, strain_class(d->strain.kind), p->log2n - p->log2ny, p->log2ny, &p->threads,
                       &p->lds_bytes);
    else march_shape(prec, p->log2n, &p->threads, &p->lds_bytes);

    // wide lane of a staged size or 3D solve marched alone
    if (wide_kind(prec, p->launch_kind)) {
        WideShape sh{};
        const WideArgs none{};
        if ((e = launch_wide(prec, p->launch_kind, strain_class(d->strain.kind), -1, none, ss, &sh)) != hipSuccess)
            return bail(hip_fail(e, "wide lane shape"));
        p->wide_blocks = sh.col_blocks;
        if ((st = dev_alloc((void **)&p->d_wide_ctl, sizeof(WideCtl), "wide control block")) != BPM_OK) return bail(st);
        if ((st = dev_alloc((void **)&p->d_wide_part, 3 * sizeof(double) * sh.col_blocks, "wide partial sums")) !=
            BPM_OK)
            return bail(st);
    }

    // single-solve launch descriptor (state at offset 0, R/T at index 0)
    SolveDesc s;
    p->fill(s, log2e, p->tw_uniform, SF_FIRST | SF_LAST, 0, d->nz, 0, 0, 0);
    if ((st = dev_alloc(&p->d_desc1, sizeof s, "launch descriptor")) != BPM_OK) return bail(st);
    e = hipMemcpyAsync(p->d_desc1, &s, sizeof s, hipMemcpyHostToDevice, ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (e != hipSuccess) return bail(hip_fail(e, "descriptor upload"));
    *out = p;
    return BPM_OK;
}

extern "C" void bpm_plan_destroy(bpm_plan *p)
{
    if (!p) return;
    (void)hipDeviceSynchronize();
    p->release();
    delete p;
}

extern "C" bpm_status bpm_plan_info_get(const bpm_plan *p, bpm_plan_info *info)
{
    if (!p || !info) return fail(BPM_E_INVALID, "NULL argument");
    info->nx = p->desc.nx;
    info->nz = p->desc.nz;
    info->precision = p->desc.precision;
    info->threads_per_solve = p->threads;
    info->state_bytes = p->state_bytes();
    info->device_bytes = p->device_bytes;
    info->cell_steps = 2.0 * (double)p->cells() * (double)p->desc.nz;
    return BPM_OK;
}

extern "C" int32_t bpm_max_nx(int32_t precision)
{
    if (precision != BPM_F32 && precision != BPM_F64) return 0;
    return 1 << max_log2n(precision);
}

// ---- wide lane: one staged-size or 3D solve over the whole device
constexpr int kWideGraphSteps = 32;   // z-steps per recorded graph

// the launches of z-step base + k (every sub-step: row phase, column phase),
// with the control block ctl and the partial sums part
static hipError_t wide_step(const bpm_plan *p, int k, hipStream_t s, const WideCtl *ctl, double *part)
{
    double a[kMaxSub], b[kMaxSub];
    const int nsub = split_sequence(p->desc.split_order <= 1 ? 1 : p->desc.split_order, a, b);
    const bool lead = a[0] == 0.0;   // sub-step 0 couples before any propagation (entry / previous step)
    const int prec = p->desc.precision, sc = strain_class(p->desc.strain.kind);
    hipError_t e = hipSuccess;
    for (int i = lead ? 1 : 0; i < nsub && e == hipSuccess; ++i) {
        const WideArgs w{p->d_desc1, ctl, k, i, part};
        e = launch_wide(prec, p->launch_kind, sc, WIDE_ROWS, w, s, nullptr);
        if (e == hipSuccess) e = launch_wide(prec, p->launch_kind, sc, WIDE_COLS, w, s, nullptr);
    }
    return e;
}

// Record kWideGraphSteps z-steps as one graph (once per plan); without a
// graph the steps are launched one by one.
static void wide_record(bpm_plan *p)
{
    p->wide_tried = true;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < kWideGraphSteps && e == hipSuccess; ++k) e = wide_step(p, k, cs, p->d_wide_ctl, p->d_wide_part);
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
    }
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess && g) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e == hipSuccess && x) {
        p->wide_graph = g;
        p->wide_exec = x;
    } else if (g) {
        (void)hipGraphDestroy(g);
    }
    (void)hipGetLastError();
    (void)hipStreamDestroy(cs);
}

bpm_status bpm::propagate_wide(bpm_plan *p, hipStream_t s, const char *in, char *out, double *rt, int step0,
                               int nsteps, int flags, WideCtl *ctl, double *part)
{
    const int prec = p->desc.precision, sc = strain_class(p->desc.strain.kind), end = step0 + nsteps;
    // the plan's own control block and partial sums replay a recorded graph;
    // the caller's (ctl, part) are launched step by step
    const bool own = ctl == nullptr;
    if (own) {
        ctl = p->d_wide_ctl;
        part = p->d_wide_part;
        if (!p->wide_tried && nsteps >= kWideGraphSteps) wide_record(p);
    }
    const WideArgs w{p->d_desc1, ctl, 0, 0, part};
    hipError_t e = launch_wide_ctl(ctl, p->d_desc1, step0, in, out, step0, nsteps, flags, s);
    if (e == hipSuccess) e = launch_wide(prec, p->launch_kind, sc, WIDE_ENTRY, w, s, nullptr);
    int n = step0;
    for (; e == hipSuccess && own && p->wide_exec && n + kWideGraphSteps <= end; n += kWideGraphSteps) {
        if (n > step0) e = launch_wide_ctl(ctl, p->d_desc1, n, in, out, step0, nsteps, flags, s);
        if (e == hipSuccess) e = hipGraphLaunch(p->wide_exec, s);
    }
    for (; e == hipSuccess && n < end; ++n) {
        e = launch_wide_ctl(ctl, p->d_desc1, n, in, out, step0, nsteps, flags, s);
        if (e == hipSuccess) e = wide_step(p, 0, s, ctl, part);
    }
    if (e == hipSuccess) e = launch_wide_finish(p->d_desc1, part, p->wide_blocks, rt, s);
    if (e != hipSuccess) return hip_fail(e, "wide march launch");
    return BPM_OK;
}

extern "C" bpm_status bpm_propagate_device(bpm_plan *p, void *stream, const void *d_in, void *d_out, double *d_RT)
{
    if (!p || !d_in || !d_out) return fail(BPM_E_INVALID, "NULL argument");
    if (p->d_wide_ctl)
        return propagate_wide(p, (hipStream_t)stream, (const char *)d_in, (char *)d_out, d_RT ? d_RT : p->d_rt, 0,
                              p->desc.nz, SF_FIRST | SF_LAST);
    hipError_t e = launch_march(p->d_desc1, 1, p->desc.precision, p->launch_kind,
                                march_class(p->desc.strain.kind, p->desc.strain.c[3]),
                                (const char *)d_in, (char *)d_out,
                                d_RT ? d_RT : p->d_rt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "march launch");
    return BPM_OK;
}

extern "C" bpm_status bpm_far_field(bpm_plan *p, double distance_um, void *stream, const void *d_in, void *d_out)
{
    if (!p || !d_in || !d_out) return fail(BPM_E_INVALID, "NULL argument");
    if (!std::isfinite(distance_um) || distance_um <= 0.0)
        return fail(BPM_E_INVALID, "far-field distance must be finite and > 0");
    if (!p->far || p->far_um != distance_um) {
        if (p->far) {
            bpm_plan_destroy(p->far);
            p->far = nullptr;
        }
        // one vacuum step: the crystal plan's grid, wavelength and reflection
        // (the carriers), no crystal, no strain
        bpm_plan_desc v = p->desc;
        const std::vector<int32_t> empty(2 * (size_t)std::max(1, p->desc.ny), 0);   // one empty interval per row
        v.nz = 1;
        v.dz_um = distance_um;
        // no crystal anywhere: zero susceptibilities (the propagator does not
        // depend on them, and the coupling of a metres-long step is not bounded)
        v.chi0 = v.chih = v.chihbar = bpm_complex{0.0, 0.0};
        v.nseg = 1;
        v.seg = empty.data();
        std::memset(&v.strain, 0, sizeof v.strain);
        v.strain.kind = BPM_STRAIN_NONE;
        v.split_order = 1;
        v.det_lo = 0;
        v.det_hi = v.nx;
        bpm_status st = bpm_plan_create(&v, &p->far);
        if (st != BPM_OK) return st;
        p->far_um = distance_um;
    }
    return bpm_propagate_device(p->far, stream, d_in, d_out, nullptr);
}

// host complex128 <-> device state in plan precision
static void pack_state(const bpm_plan *p, const bpm_complex *a, const bpm_complex *b, std::vector<char> &buf)
{
    const size_t nx = p->cells();   // samples per beam
    buf.resize(p->state_bytes());
    if (p->desc.precision == BPM_F64) {
        double *o = (double *)buf.data();
        for (size_t j = 0; j < nx; ++j) {
            o[2 * j] = a[j].re;
            o[2 * j + 1] = a[j].im;
            o[2 * (nx + j)] = b ? b[j].re : 0.0;
            o[2 * (nx + j) + 1] = b ? b[j].im : 0.0;
        }
    } else {
        float *o = (float *)buf.data();
        for (size_t j = 0; j < nx; ++j) {
            o[2 * j] = (float)a[j].re;
            o[2 * j + 1] = (float)a[j].im;
            o[2 * (nx + j)] = b ? (float)b[j].re : 0.0f;
            o[2 * (nx + j) + 1] = b ? (float)b[j].im : 0.0f;
        }
    }
}

static void unpack_state(const bpm_plan *p, const std::vector<char> &buf, bpm_complex *a, bpm_complex *b)
{
    const size_t nx = p->cells();   // samples per beam
    for (size_t j = 0; j < nx; ++j) {
        double v[4];
        if (p->desc.precision == BPM_F64) {
            const double *o = (const double *)buf.data();
            v[0] = o[2 * j], v[1] = o[2 * j + 1], v[2] = o[2 * (nx + j)], v[3] = o[2 * (nx + j) + 1];
        } else {
            const float *o = (const float *)buf.data();
            v[0] = o[2 * j], v[1] = o[2 * j + 1], v[2] = o[2 * (nx + j)], v[3] = o[2 * (nx + j) + 1];
        }
        if (a) a[j] = {v[0], v[1]};
        if (b) b[j] = {v[2], v[3]};
    }
}

bpm_status bpm::check_input(const bpm_plan_desc &d, const bpm_complex *a, const bpm_complex *b)
{
    if (!a) return fail(BPM_E_INVALID, "psi_p0 is NULL");
    const long long cells = (long long)d.nx * (d.ny > 1 ? d.ny : 1);
    for (long long j = 0; j < cells; ++j) {
        if (!is_finite(a[j]) || (b && !is_finite(b[j])))
            return fail(BPM_E_NUMERIC, "non-finite entrance envelope at sample %lld", j);
    }
    return BPM_OK;
}

extern "C" bpm_status bpm_propagate(bpm_plan *p, const bpm_complex *psi_p0, const bpm_complex *psi_m0,
                                    bpm_complex *psi_p_out, bpm_complex *psi_m_out, double *R, double *T)
{
    if (!p) return fail(BPM_E_INVALID, "plan is NULL");
    bpm_status st = check_input(p->desc, psi_p0, psi_m0);
    if (st != BPM_OK) return st;
    if (!p->d_state && (st = dev_alloc(&p->d_state, p->state_bytes(), "state buffer")) != BPM_OK) return st;
    std::vector<char> buf;
    pack_state(p, psi_p0, psi_m0, buf);
    hipError_t e = hipMemcpy(p->d_state, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload");
    if ((st = bpm_propagate_device(p, nullptr, p->d_state, p->d_state, p->d_rt)) != BPM_OK) return st;
    double rt[2];
    e = hipMemcpy(buf.data(), p->d_state, buf.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(rt, p->d_rt, sizeof rt, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "march / download");
    unpack_state(p, buf, psi_p_out, psi_m_out);
    if (R) *R = rt[0];
    if (T) *T = rt[1];
    if (!std::isfinite(rt[0]) || !std::isfinite(rt[1])) return fail(BPM_E_NUMERIC, "non-finite R or T");
    return BPM_OK;
}

// ------------------------------------------------------------------ batches
bpm_status bpm::build_launches(bpm_plan *const *plans, int n, const std::vector<int> &rt_index,
                               const std::vector<uint64_t> &in_off, const std::vector<uint64_t> &out_off,
                               const std::vector<int> &step0, const std::vector<int> &nsteps,
                               const std::vector<int> &flags, std::vector<Launch> &launches, bool any_size,
                               int force_schedule)
{
    launches.clear();
    // launch kind of a group of one size: the schedule table's (or the forced)
    // kernel family when it can march the size, else the per-size kernel
    auto kind_of = [&](int prec, int sc, int log2n) {
        const int f = force_schedule ? force_schedule : tuned_schedule(prec, log2n, sc);
        if (f == BPM_SCHED_MIXED && schedule_fits(prec, log2n, f)) return (int)kLaunchMixed;
        if (f == BPM_SCHED_ANY && schedule_fits(prec, log2n, f)) return (int)kLaunchAny;
        return log2n;
    };
    // longest first: the hardware dispatcher then balances uneven solves
    auto cost = [&](int i) {
        const int pairs = plans[i]->desc.split_order == 4 ? 3 : 1;
        return (double)nsteps[i] * pairs * plans[i]->cells() * (plans[i]->log2n + 4);
    };
    auto emit = [&](int prec, int sc, int group_log2n, const std::vector<int> &g) -> bpm_status {
        Launch L;
        L.prec = prec;
        L.sc = sc;
        // a polynomial class whose every solve lacks the X^2 term runs as SC_POLY1
        if (sc == SC_POLY2) {
            bool lin = true;
            for (int i : g) lin = lin && march_class(plans[i]->desc.strain.kind, plans[i]->desc.strain.c[3]) == SC_POLY1;
            if (lin) L.sc = SC_POLY1;
        }
        L.uniform_log2n = group_log2n;
        std::vector<SolveDesc> descs(g.size());
        for (size_t k = 0; k < g.size(); ++k) {
            const int i = g[k];
            const bpm_plan *p = plans[i];
            const void *tw = p->tw_uniform;
            int log2e = uniform_log2e(p->log2n);
            if (group_log2n < 0 && !is_staged(prec, p->log2n)) {
                log2e = mixed_log2e(prec, p->log2n);
                bpm_status st = twiddle_table(prec, p->log2n, log2e, &tw);
                if (st != BPM_OK) return st;
            }
            p->fill(descs[k], log2e, tw, flags[i], step0[i], nsteps[i], in_off[i], out_off[i], rt_index[i]);
        }
        L.n = (int)descs.size();
        L.host = descs;
        launches.push_back(std::move(L));
        return BPM_OK;
    };
    // 3D envelopes: one launch per (precision, strain class, nx, ny)
    for (int prec : {BPM_F32, BPM_F64})
        for (int sc : {0, 1, 2})
            for (int lx = k3DLog2NxMin; lx <= k3DLog2NxMax; ++lx)
                for (int l = k3DLog2NyMin; l <= k3DLog2NyMax; ++l) {
                    std::vector<int> g;
                    for (int i = 0; i < n; ++i)
                        if (plans[i]->log2ny && plans[i]->launch_kind == kind_3d(lx, l) &&
                            plans[i]->desc.precision == prec && strain_class(plans[i]->desc.strain.kind) == sc)
                            g.push_back(i);
                    std::stable_sort(g.begin(), g.end(), [&](int a, int b) { return cost(a) > cost(b); });
                    if (!g.empty()) {
                        bpm_status st = emit(prec, sc, kind_3d(lx, l), g);
                        if (st != BPM_OK) return st;
                    }
                }
    if (any_size) {
        // every size the any-size kernel takes, of every strain class, in one
        // launch per precision (a size always meets the same kernel, whatever
        // else is launched); smaller sizes below, per size and strain class
        for (int prec : {BPM_F32, BPM_F64}) {
            std::vector<int> big;
            for (int i = 0; i < n; ++i)
                if (plans[i]->desc.precision == prec && !plans[i]->log2ny && plans[i]->log2n >= mixed_min_log2n(prec))
                    big.push_back(i);
            std::stable_sort(big.begin(), big.end(), [&](int a, int b) { return cost(a) > cost(b); });
            if (!big.empty()) {
                bpm_status st = emit(prec, SC_NONE, kLaunchAny, big);
                if (st != BPM_OK) return st;
            }
        }
    }
    for (int prec : {BPM_F32, BPM_F64})
    for (int sc : {0, 1, 2}) {
        std::vector<int> idx;
        for (int i = 0; i < n; ++i)
            if (plans[i]->desc.precision == prec && strain_class(plans[i]->desc.strain.kind) == sc &&
                !plans[i]->log2ny && !(any_size && plans[i]->log2n >= mixed_min_log2n(prec)))
                idx.push_back(i);
        if (idx.empty()) continue;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost(a) > cost(b); });
        int lo = 99, hi = -1;
        for (int i : idx) {
            lo = std::min(lo, plans[i]->log2n);
            hi = std::max(hi, plans[i]->log2n);
        }
        std::vector<std::vector<int>> groups;
        std::vector<int> group_log2n;
        if (any_size) {
            for (int l = lo; l <= hi; ++l) {
                std::vector<int> g;
                for (int i : idx)
                    if (plans[i]->log2n == l) g.push_back(i);
                if (!g.empty()) {
                    groups.push_back(g);
                    group_log2n.push_back(l);
                }
            }
        } else if (lo == hi) {
            groups.push_back(idx);
            group_log2n.push_back(kind_of(prec, sc, lo));
        } else if (lo >= mixed_min_log2n(prec) && hi <= mixed_max_log2n(prec)) {
            groups.push_back(idx);
            group_log2n.push_back(kLaunchMixed);
        } else {
            for (int l = lo; l <= hi; ++l) {
                std::vector<int> g;
                for (int i : idx)
                    if (plans[i]->log2n == l) g.push_back(i);
                if (!g.empty()) {
                    groups.push_back(g);
                    group_log2n.push_back(kind_of(prec, sc, l));
                }
            }
        }
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            bpm_status st = emit(prec, sc, group_log2n[gi], groups[gi]);
            if (st != BPM_OK) return st;
        }
    }
    return BPM_OK;
}

bpm_status bpm::upload_launches(std::vector<Launch> &launches, hipStream_t s)
{
    for (auto &L : launches) {
        if (!L.d_descs) {
            L.d_cap = L.host.size();
            hipError_t e = hipMalloc((void **)&L.d_descs, std::max<size_t>(L.d_cap, 1) * sizeof(SolveDesc));
            if (e != hipSuccess) return hip_fail(e, "descriptor buffer");
        }
        // on stream s the host copy must stay alive until the stream passes this point
        hipError_t e = s ? hipMemcpyAsync(L.d_descs, L.host.data(), L.host.size() * sizeof(SolveDesc),
                                          hipMemcpyHostToDevice, s)
                         : hipMemcpy(L.d_descs, L.host.data(), L.host.size() * sizeof(SolveDesc),
                                     hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    }
    return BPM_OK;
}

bpm_status bpm::run_launches(const std::vector<Launch> &launches, hipStream_t s, const char *in, char *out,
                             double *rt)
{
    for (const auto &L : launches) {
        hipError_t e = launch_march(L.d_descs, L.n, L.prec, L.uniform_log2n, L.sc, in, out, rt, s);
        if (e != hipSuccess) return hip_fail(e, "march launch");
    }
    return BPM_OK;
}

void bpm::free_launches(std::vector<Launch> &launches)
{
    for (auto &L : launches) (void)hipFree(L.d_descs);
    launches.clear();
}

struct bpm_batch {
    std::vector<bpm_plan *> plans;
    std::vector<size_t> offsets;
    size_t total = 0;
    std::vector<Launch> launches;
    double *d_rt_scratch = nullptr;
    // time-domain assembly (built on first use)
    uint64_t *d_td_offs = nullptr;
    double *d_td_par = nullptr;
    void *d_td_ph = nullptr;
};

extern "C" bpm_status bpm_batch_create(bpm_plan *const *plans, int32_t n, bpm_batch **out)
{
    if (!out) return fail(BPM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && !plans)) return fail(BPM_E_INVALID, "bad plan array");
    for (int i = 0; i < n; ++i)
        if (!plans[i]) return fail(BPM_E_INVALID, "plan %d is NULL", i);
    bpm_batch *b = new (std::nothrow) bpm_batch();
    if (!b) return fail(BPM_E_NOMEM, "host allocation");
    b->plans.assign(plans, plans + n);
    std::vector<int> rt(n), s0(n, 0), ns(n), fl(n, SF_FIRST | SF_LAST);
    std::vector<uint64_t> off(n);
    for (int i = 0; i < n; ++i) {
        b->offsets.push_back(b->total);
        off[i] = b->total;
        b->total += (plans[i]->state_bytes() + 255) / 256 * 256;
        rt[i] = i;
        ns[i] = plans[i]->desc.nz;
    }
    bpm_status st = build_launches(plans, n, rt, off, off, s0, ns, fl, b->launches);
    if (st == BPM_OK) st = upload_launches(b->launches);
    if (st == BPM_OK) {
        hipError_t e = hipMalloc((void **)&b->d_rt_scratch, std::max(2 * n, 2) * sizeof(double));
        if (e != hipSuccess) st = hip_fail(e, "R/T scratch");
    }
    if (st != BPM_OK) {
        free_launches(b->launches);
        delete b;
        return st;
    }
    *out = b;
    return BPM_OK;
}

extern "C" bpm_status bpm_batch_layout(const bpm_batch *b, size_t *offsets, size_t *total_bytes)
{
    if (!b) return fail(BPM_E_INVALID, "batch is NULL");
    if (offsets) std::copy(b->offsets.begin(), b->offsets.end(), offsets);
    if (total_bytes) *total_bytes = b->total;
    return BPM_OK;
}

extern "C" bpm_status bpm_batch_run(bpm_batch *b, void *stream, const void *d_in, void *d_out, double *d_RT)
{
    if (!b || !d_in || !d_out) return fail(BPM_E_INVALID, "NULL argument");
    return run_launches(b->launches, (hipStream_t)stream, (const char *)d_in, (char *)d_out,
                        d_RT ? d_RT : b->d_rt_scratch);
}

extern "C" void bpm_batch_destroy(bpm_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    free_launches(b->launches);
    (void)hipFree(b->d_rt_scratch);
    (void)hipFree(b->d_td_offs);
    (void)hipFree(b->d_td_par);
    (void)hipFree(b->d_td_ph);
    delete b;
}

extern "C" bpm_status bpm_td_assemble(bpm_batch *b, void *stream, const void *d_state, void *d_out)
{
    if (!b || !d_state || !d_out) return fail(BPM_E_INVALID, "NULL argument");
    const int M = (int)b->plans.size();
    int log2m = 0;
    while ((1 << log2m) < M) ++log2m;
    if ((1 << log2m) != M || log2m < kTdLog2MMin || log2m > kTdLog2MMax)
        return fail(BPM_E_INVALID, "time-domain assembly needs 2^%d..2^%d components, got %d", kTdLog2MMin,
                    kTdLog2MMax, M);
    const bpm_plan_desc &d0 = b->plans[0]->desc;
    for (const bpm_plan *p : b->plans) {
        const bpm_plan_desc &d = p->desc;
        if (d.nx != d0.nx || d.dx_um != d0.dx_um || d.x0_um != d0.x0_um || d.precision != d0.precision)
            return fail(BPM_E_INVALID, "time-domain assembly needs one x grid and one precision for all components");
        if (d.ny > 1) return fail(BPM_E_UNSUPPORTED, "time-domain assembly of 3D envelopes is not built");
    }
    if (!b->d_td_offs) {
        std::vector<uint64_t> offs(M);
        std::vector<double> par(3 * (size_t)M);
        for (int m = 0; m < M; ++m) {
            const bpm_plan_desc &d = b->plans[m]->desc;
            offs[m] = b->offsets[m];
            par[3 * m] = d.lambda_um;
            par[3 * m + 1] = d.d_um;
            par[3 * m + 2] = d.nz * d.dz_um;
        }
        const size_t eb = d0.precision == BPM_F32 ? 8 : 16;
        hipError_t e = hipMalloc((void **)&b->d_td_offs, M * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_td_par, par.size() * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&b->d_td_ph, M * eb);
        if (e == hipSuccess) e = hipMemcpy(b->d_td_offs, offs.data(), M * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_td_par, par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(b->d_td_offs);
            (void)hipFree(b->d_td_par);
            (void)hipFree(b->d_td_ph);
            b->d_td_offs = nullptr;
            b->d_td_par = nullptr;
            b->d_td_ph = nullptr;
            return hip_fail(e, "time-domain assembly tables");
        }
    }
    const void *tw = nullptr;
    bpm_status st = twiddle_table(d0.precision, log2m, log2m - 6, &tw);
    if (st != BPM_OK) return st;
    hipError_t e = launch_td(d0.precision, log2m, (const char *)d_state, b->d_td_offs, b->d_td_par, b->d_td_ph, tw,
                             d0.nx, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "time-domain assembly launch");
    return BPM_OK;
}
