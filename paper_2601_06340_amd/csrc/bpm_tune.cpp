// bpm_tune.cpp — the schedule table and its autotuner.
//
// A batch marches each group of solves that share (precision, nx, strain class)
// with one kernel family (bpm_schedule).  The families differ in samples per
// thread and workgroup width: the per-size kernel (nx/16 threads, or the staged
// kernel), the mixed-size kernel (512 threads, nx/512 samples per thread) and the
// any-size kernel (512 threads, staged sizes included).  Which one marches a size
// fastest depends on its register and LDS footprint against the occupancy the
// device allows, so the autotuner measures: it builds a synthetic batch of the
// size, times one batch march with every family that can take it, and enters
// the fastest into a process-wide table that batch creation consults.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "bpm.h"
#include "bpm_api_internal.hpp"
#include "bpm_internal.hpp"

using namespace bpm;

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, int> g_table;   // (precision, log2 nx, strain class) -> schedule

int log2_exact(int nx)
{
    if (nx <= 0 || (nx & (nx - 1))) return -1;
    int l = 0;
    while ((1 << l) < nx) ++l;
    return l;
}

bool valid_key(int prec, int log2n, int sc)
{
    return (prec == BPM_F32 || prec == BPM_F64) && log2n >= 6 && log2n <= max_log2n(prec) && sc >= SC_NONE &&
           sc <= SC_GENERAL;
}

bool strain_kind_ok(int kind) { return kind >= BPM_STRAIN_NONE && kind <= BPM_STRAIN_TABLE; }

}  // namespace

bool bpm::schedule_fits(int prec, int log2n, int schedule)
{
    switch (schedule) {
    case BPM_SCHED_DEFAULT:
    case BPM_SCHED_UNIFORM:
        return log2n >= 6 && log2n <= max_log2n(prec);
    case BPM_SCHED_MIXED:
        return log2n >= mixed_min_log2n(prec) && log2n <= mixed_max_log2n(prec);
    case BPM_SCHED_ANY:
        return log2n >= mixed_min_log2n(prec) && log2n <= max_log2n(prec);
    default:
        return false;
    }
}

int bpm::tuned_schedule(int prec, int log2n, int sc)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(std::make_tuple(prec, log2n, sc));
    return it == g_table.end() ? BPM_SCHED_DEFAULT : it->second;
}

extern "C" bpm_status bpm_schedule_set(int32_t precision, int32_t nx, int32_t strain_kind, int32_t schedule)
{
    const int l = log2_exact(nx);
    if (!strain_kind_ok(strain_kind) || !valid_key(precision, l, strain_class(strain_kind)))
        return fail(BPM_E_INVALID, "bad schedule key (precision %d, nx %d, strain kind %d)", precision, nx,
                    strain_kind);
    if (!schedule_fits(precision, l, schedule))
        return fail(BPM_E_INVALID, "schedule %d cannot march nx = %d at precision %d", schedule, nx, precision);
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple((int)precision, l, strain_class(strain_kind));
    if (schedule == BPM_SCHED_DEFAULT) g_table.erase(key);
    else g_table[key] = schedule;
    return BPM_OK;
}

extern "C" int32_t bpm_schedule_get(int32_t precision, int32_t nx, int32_t strain_kind)
{
    const int l = log2_exact(nx);
    if (!strain_kind_ok(strain_kind) || !valid_key(precision, l, strain_class(strain_kind))) return -1;
    return tuned_schedule(precision, l, strain_class(strain_kind));
}

extern "C" bpm_status bpm_schedule_save(const char *path)
{
    if (!path) return fail(BPM_E_INVALID, "path is NULL");
    std::map<std::tuple<int, int, int>, int> t;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        t = g_table;
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(BPM_E_INVALID, "cannot write %s", path);
    std::fprintf(f, "# bpm schedule table: precision log2nx strain_class schedule\n");
    for (const auto &kv : t)
        std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     kv.second);
    const bool ok = std::fclose(f) == 0;
    return ok ? BPM_OK : fail(BPM_E_INVALID, "cannot write %s", path);
}

extern "C" bpm_status bpm_schedule_load(const char *path)
{
    if (!path) return fail(BPM_E_INVALID, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(BPM_E_INVALID, "cannot read %s", path);
    std::vector<std::pair<std::tuple<int, int, int>, int>> rows;
    char line[256];
    int lineno = 0;
    bpm_status st = BPM_OK;
    while (st == BPM_OK && std::fgets(line, sizeof line, f)) {
        ++lineno;
        const char *c = line;
        while (*c == ' ' || *c == '\t') ++c;
        if (*c == '#' || *c == '\n' || *c == '\r' || *c == 0) continue;
        int prec, l, sc, sched;
        char extra;
        if (std::sscanf(c, "%d %d %d %d %c", &prec, &l, &sc, &sched, &extra) != 4 || !valid_key(prec, l, sc) ||
            sched == BPM_SCHED_DEFAULT || !schedule_fits(prec, l, sched))
            st = fail(BPM_E_INVALID, "%s:%d: not a schedule entry", path, lineno);
        else
            rows.push_back({std::make_tuple(prec, l, sc), sched});
    }
    std::fclose(f);
    if (st != BPM_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &r : rows) g_table[r.first] = r.second;
    return BPM_OK;
}

extern "C" bpm_status bpm_autotune(int32_t precision, int32_t nx, int32_t strain_kind, int32_t nsolves, int32_t nsteps,
                                   bpm_tune_result *out)
{
    if (!out) return fail(BPM_E_INVALID, "out is NULL");
    const int l = log2_exact(nx);
    if (!strain_kind_ok(strain_kind) || !valid_key(precision, l, strain_class(strain_kind)))
        return fail(BPM_E_INVALID, "bad schedule key (precision %d, nx %d, strain kind %d)", precision, nx,
                    strain_kind);
    if (nsolves < 1 || nsolves > 4096 || nsteps < 1 || nsteps > 100000)
        return fail(BPM_E_INVALID, "autotune needs 1 <= nsolves <= 4096 and 1 <= nsteps <= 100000");
    bpm_status st = ensure_device();
    if (st != BPM_OK) return st;
    std::memset(out, 0, sizeof *out);
    out->nsolves = nsolves;
    out->nsteps = nsteps;

    // synthetic solve: 0.95 A reflection at 30 deg, a crystal filling the window
    const double dx = 0.1, dz = 0.05, dd = 9.5e-5;
    std::vector<int32_t> seg(2 * (size_t)nsteps);
    for (int n = 0; n < nsteps; ++n) seg[2 * n] = 0, seg[2 * n + 1] = nx;
    std::vector<double> utab;
    bpm_plan_desc d{};
    d.nx = nx;
    d.nz = nsteps;
    d.dx_um = dx;
    d.dz_um = dz;
    d.lambda_um = dd;
    d.d_um = dd;
    d.chi0 = {-2e-6, 1e-8};
    d.chih = d.chihbar = {-1.5e-6, 8e-9};
    d.nseg = 1;
    d.seg = seg.data();
    d.strain.kind = strain_kind;
    d.strain.x_ref_um = 0.5 * nx * dx + 0.5 * dx;
    d.strain.z_ref_um = 0.5 * nsteps * dz + 0.5 * dz;
    if (strain_kind == BPM_STRAIN_POLY2) d.strain.c[4] = 1e-6;   // u = X Z / R, R = 1 m
    if (strain_kind == BPM_STRAIN_EDGE_DISLOCATION) d.strain.b_um = 4 * dd, d.strain.nu = 0.22;
    if (strain_kind == BPM_STRAIN_TABLE) {
        utab.assign((size_t)nsteps * nx, 0.0);
        d.strain.u_table = utab.data();
    }
    d.det_lo = 0;
    d.det_hi = nx;
    d.precision = precision;
    d.split_order = 1;
    bpm_plan *p = nullptr;
    if ((st = bpm_plan_create(&d, &p)) != BPM_OK) return st;

    // nsolves copies of a tilted Gaussian beam in one state buffer
    const size_t sb = (p->state_bytes() + 255) / 256 * 256;
    std::vector<bpm_complex> beam(nx);
    for (int j = 0; j < nx; ++j) {
        const double x = (j - 0.5 * nx) * dx, w = 0.1 * nx * dx;
        const double a = std::exp(-(x / w) * (x / w));
        beam[j] = {a * std::cos(1e-3 * j), a * std::sin(1e-3 * j)};
    }
    std::vector<char> host(sb * nsolves, 0);
    for (int i = 0; i < nsolves; ++i) {
        char *o = host.data() + sb * i;
        for (int j = 0; j < nx; ++j) {
            if (precision == BPM_F64) {
                ((double *)o)[2 * j] = beam[j].re, ((double *)o)[2 * j + 1] = beam[j].im;
            } else {
                ((float *)o)[2 * j] = (float)beam[j].re, ((float *)o)[2 * j + 1] = (float)beam[j].im;
            }
        }
    }
    char *d_state = nullptr, *d_work = nullptr;
    double *d_rt = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void **)&d_state, host.size());
    if (e == hipSuccess) e = hipMalloc((void **)&d_work, host.size());
    if (e == hipSuccess) e = hipMalloc((void **)&d_rt, 2 * sizeof(double) * nsolves);
    if (e == hipSuccess) e = hipMemcpy(d_state, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) st = hip_fail(e, "autotune buffers");

    std::vector<bpm_plan *> plans(nsolves, p);
    std::vector<int> rt(nsolves), s0(nsolves, 0), ns(nsolves, nsteps), fl(nsolves, SF_FIRST | SF_LAST);
    std::vector<uint64_t> off(nsolves);
    for (int i = 0; i < nsolves; ++i) rt[i] = i, off[i] = sb * i;
    // families from the most specialised to the most general; a later one
    // replaces the pick only when it is faster by more than the margin, so
    // timings within noise keep the specialised kernel
    constexpr float kTuneMargin = 0.01f;
    int best = BPM_SCHED_DEFAULT;
    for (int sched : {BPM_SCHED_UNIFORM, BPM_SCHED_MIXED, BPM_SCHED_ANY}) {
        if (st != BPM_OK) break;
        if (!schedule_fits(precision, l, sched)) continue;
        std::vector<Launch> ls;
        st = build_launches(plans.data(), nsolves, rt, off, off, s0, ns, fl, ls, false, sched);
        if (st == BPM_OK) st = upload_launches(ls, s);
        float ms[3] = {0, 0, 0};
        for (int r = 0; r < 4 && st == BPM_OK; ++r) {   // one untimed run, then three timed
            if ((e = hipEventRecord(ev[0], s)) == hipSuccess)
                st = run_launches(ls, s, d_state, d_work, d_rt);
            if (st == BPM_OK && (e = hipEventRecord(ev[1], s)) == hipSuccess) e = hipEventSynchronize(ev[1]);
            if (st == BPM_OK && e == hipSuccess && r > 0) e = hipEventElapsedTime(&ms[r - 1], ev[0], ev[1]);
            if (st == BPM_OK && e != hipSuccess) st = hip_fail(e, "autotune timing");
        }
        free_launches(ls);
        if (st != BPM_OK) break;
        std::sort(ms, ms + 3);
        out->ms[sched] = ms[1];
        if (best == BPM_SCHED_DEFAULT || out->ms[sched] < (1.0f - kTuneMargin) * out->ms[best]) best = sched;
    }
    if (s) (void)hipStreamSynchronize(s);
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(d_state);
    (void)hipFree(d_work);
    (void)hipFree(d_rt);
    bpm_plan_destroy(p);
    if (st != BPM_OK) return st;
    out->schedule = best;
    return bpm_schedule_set(precision, nx, strain_kind, best);
}
