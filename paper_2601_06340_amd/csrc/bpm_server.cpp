// bpm_server.cpp — continuous-batching server over the march kernels.
//
// The paper evaluates independent realisations (incidence angles, photon
// energies) in parallel (Sec. 3); this server does the same for a stream of
// requests on one device.  Two threads share the work.  The admission thread
// takes waiting requests in arrival order while the slot count and the
// device-memory budget allow and builds their plans and entrance states; plan
// setup waits only for the library's setup stream, so this overlaps the
// marches.  The march worker runs rounds: every active solve advances the
// z-steps that take as long as chunk_steps steps of an FP32 nx = 16384 bent
// solve at the measured per-workgroup rate of its (precision, size, strain
// class), in one any-size launch per precision, so solves of every size and
// strain class run side by side.  After the round it
// retires the solves that reached nz (their plans and states go back to the
// library's device block cache, not to hipFree, which would wait for the
// device), and the requests set up in the meantime join the next round.  A
// solve's arithmetic is the same kernel and schedule whatever else runs, and
// its state crosses round boundaries through HBM unchanged, so results do not
// depend on what else is running.
//
// Staged-size or 3D solves with a long march ahead (estimated one-workgroup
// time of their remaining steps above kWideMinSeconds; at most kMaxWide at a
// time, and only while at most kWideMaxRegular other solves march in the
// rounds) move to the wide lane, from the start or part way through: each
// round advances them kWideChunkFactor * chunk_steps z-steps spread over the
// device on a stream of their own, alongside the round's launches, and the
// round waits for them too.  Their envelopes are the one-workgroup march's
// bitwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "bpm.h"
#include "bpm_api_internal.hpp"
#include "bpm_internal.hpp"

using namespace bpm;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket = 0;
    bpm_plan_desc desc{};
    std::vector<int32_t> seg;
    std::vector<double> utab;
    std::vector<bpm_complex> psi_p0, psi_m0;
    bpm_complex *out_p = nullptr, *out_m = nullptr;
    size_t need = 0;          // budgeted device bytes
    std::atomic<bool> cancel{false};   // set by bpm_cancel, read by both server threads
    // running state
    bpm_plan *plan = nullptr;
    void *d_state = nullptr;
    int step = 0;
    int slot = -1;
    int wide_lane = -1;             // >= 0: marched by the wide lane on this stream of the pool
    // result
    bool done = false;
    bpm_result res{};
};

// Per-workgroup march rate of the any-size kernel in cell-steps/s, by
// precision (FP64, FP32), log2 nx (10..16; 3D by its cell count) and strain
// class (none, polynomial, dislocation/table; the dislocation with b = 4 d):
// measured on MI355X with 64 solves of each class marching side by side (one per
// compute unit), on the kernels of this source.  The
// server sizes every solve's chunk so that chunks take about the same time.
constexpr float kAnyRate[2][7][3] = {
    {{4.11e8f, 3.85e8f, 3.00e8f}, {5.40e8f, 5.35e8f, 3.87e8f}, {7.86e8f, 7.38e8f, 5.35e8f},
     {7.37e8f, 7.15e8f, 4.20e8f}, {3.89e8f, 3.65e8f, 3.13e8f}, {3.91e8f, 3.62e8f, 3.10e8f},
     {3.34e8f, 3.28e8f, 2.88e8f}},
    {{5.02e8f, 4.65e8f, 4.24e8f}, {7.06e8f, 6.65e8f, 5.75e8f}, {1.13e9f, 1.08e9f, 9.20e8f},
     {1.27e9f, 1.16e9f, 9.72e8f}, {1.20e9f, 1.17e9f, 9.14e8f}, {7.03e8f, 6.65e8f, 6.23e8f},
     {6.16e8f, 5.97e8f, 6.04e8f}}};
// the reference class: FP32, nx = 16384, polynomial strain
constexpr double kRefRate = 1.17e9;

double any_rate(const bpm_plan_desc &d)
{
    const long long cells = (long long)d.nx * (d.ny > 1 ? d.ny : 1);
    int l = 0;
    while ((1LL << l) < cells) ++l;
    l = std::min(16, std::max(10, l));
    return kAnyRate[d.precision == BPM_F32 ? 1 : 0][l - 10][strain_class(d.strain.kind)];
}

constexpr int kMaxWide = 4;              // wide-lane solves at once
constexpr double kWideMinSeconds = 0.5;  // one-workgroup march time above which a solve goes wide
constexpr int kWideChunkFactor = 2;      // wide-lane z-steps per round = factor * chunk_steps
// The wide lane is launch-rate bound: it shortens a long solve's latency when
// the device has room, but under load the one-workgroup march gets more work
// done.  A solve goes wide only while at most this many others march in the rounds.
constexpr int kWideMaxRegular = 64;

// One-workgroup march time of a request at the measured rate of its class.
double one_workgroup_seconds(const bpm_plan_desc &d)
{
    const double cells = (double)d.nx * (d.ny > 1 ? d.ny : 1);
    const double pairs = d.split_order == 4 ? 3.0 : 1.0;
    return 2.0 * cells * d.nz * pairs / any_rate(d);
}

size_t estimate_bytes(const bpm_plan_desc &d)
{
    const size_t eb = d.precision == BPM_F32 ? 8 : 16;
    int tab[kMaxSub];
    double afrac[kMaxSub];
    const int ntab = split_tables(d.split_order <= 1 ? 1 : d.split_order, tab, afrac);
    const size_t ny = d.ny > 1 ? d.ny : 1;
    size_t b = 2 * (size_t)d.nx * ny * (eb + kPropEntryBytes * ntab);    // state + propagator tables
    b += (size_t)std::max(d.nz, 1) * ny * d.nseg * 2 * sizeof(int32_t);  // mask
    if (d.strain.kind == BPM_STRAIN_TABLE) b += (size_t)d.nz * ny * d.nx * (d.precision == BPM_F32 ? 4 : 8);
    b += 4096;                                                       // scalars, descriptors
    return b;
}

}  // namespace

struct bpm_server {
    bpm_server_desc cfg{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_admit, cv_done;
    std::deque<std::shared_ptr<Request>> waiting;   // submitted, not admitted
    std::vector<std::shared_ptr<Request>> ready;     // admitted and set up, not yet marching
    std::vector<std::shared_ptr<Request>> active;    // marching (worker only)
    int admitted_slots = 0;                          // admitted and not finished
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bpm_server_stats stats{};
    std::thread worker, setup_thread;
    // worker-owned device resources
    std::map<int, hipStream_t> streams;  // one per precision
    double *d_rt = nullptr;
    // per precision: a device descriptor buffer reused from round to round and
    // its pinned host staging copy (grown when a round needs more)
    struct DescBuf {
        SolveDesc *dev = nullptr, *host = nullptr;
        size_t cap = 0;
    };
    std::map<int, DescBuf> descbuf;
    hipStream_t wide_streams[kMaxWide] = {};
    bool wide_busy[kMaxWide] = {};

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    void run_setup();
    bpm_status upload(int prec, std::vector<Launch> &ls, hipStream_t st);
    int steps_for(const Request &r) const;
    bpm_status setup(Request &r, std::vector<char> &host);
    void finish(const std::shared_ptr<Request> &r, int status);
    hipStream_t stream_for(int key);
    int retire(Request &r, int status, const double *rt);
};

hipStream_t bpm_server::stream_for(int key)
{
    auto it = streams.find(key);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    streams[key] = s;
    return s;
}

// caller holds mu
void bpm_server::finish(const std::shared_ptr<Request> &r, int status)
{
    r->res.status = status;
    r->res.t_done = now();
    r->done = true;
    if (status == BPM_OK) stats.completed++;
    else if (status == BPM_E_CANCELLED) stats.cancelled++;
    else stats.failed++;
    r->psi_p0.clear();
    r->psi_p0.shrink_to_fit();
    r->psi_m0.clear();
    r->psi_m0.shrink_to_fit();
    r->seg.clear();
    r->seg.shrink_to_fit();
    r->utab.clear();
    r->utab.shrink_to_fit();
    cv_done.notify_all();
}

// z-steps a solve advances per round: chunk_steps for an FP32 nx = 16384
// solve with polynomial strain, and for every other class the steps that take
// the same time at its measured rate (kAnyRate), so no round waits long for
// one class.  A request with no z-step (nz = 0) gets one launch of 0 steps,
// which reports R and T of its entrance state.
int bpm_server::steps_for(const Request &r) const
{
    const int left = r.desc.nz - r.step;
    if (left <= 0) return 0;
    // a z-step of a splitting runs one FFT pair per propagation sub-step
    const double fft_pairs = r.desc.split_order == 4 ? 3.0 : 1.0;
    const double cells = (double)r.desc.nx * (r.desc.ny > 1 ? r.desc.ny : 1);
    const double s = cfg.chunk_steps * (16384.0 / cells) * (any_rate(r.desc) / kRefRate) / fft_pairs;
    return (int)std::max(1.0, std::min<double>(std::floor(s), left));
}

// Device setup of one admitted request (plan tables and entrance state).  Runs
// while the previous round is on the device: plan setup waits only for the
// library's setup stream.
bpm_status bpm_server::setup(Request &r, std::vector<char> &host)
{
    r.desc.seg = r.seg.data();
    r.desc.strain.u_table = r.utab.empty() ? nullptr : r.utab.data();
    bpm_status st = bpm_plan_create(&r.desc, &r.plan);
    if (st != BPM_OK) return st;
    const size_t sb = r.plan->state_bytes(), nx = r.plan->cells();   // samples per beam
    hipError_t e = dev_malloc(&r.d_state, sb);
    if (e != hipSuccess) return hip_fail(e, "server state");
    host.resize(sb);
    for (size_t j = 0; j < nx; ++j) {
        const bpm_complex a = r.psi_p0[j];
        const bpm_complex b = r.psi_m0.empty() ? bpm_complex{0, 0} : r.psi_m0[j];
        if (r.desc.precision == BPM_F64) {
            double *o = (double *)host.data();
            o[2 * j] = a.re, o[2 * j + 1] = a.im, o[2 * (nx + j)] = b.re, o[2 * (nx + j) + 1] = b.im;
        } else {
            float *o = (float *)host.data();
            o[2 * j] = (float)a.re, o[2 * j + 1] = (float)a.im;
            o[2 * (nx + j)] = (float)b.re, o[2 * (nx + j) + 1] = (float)b.im;
        }
    }
    hipStream_t ss = setup_stream();
    e = hipMemcpyAsync(r.d_state, host.data(), sb, hipMemcpyHostToDevice, ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (e != hipSuccess) return hip_fail(e, "server state upload");
    return BPM_OK;
}

// Admission thread: takes waiting requests in arrival order while slots and
// the budget allow, builds their plans and entrance states (plan setup waits
// only for the library's setup stream, so this overlaps the marches), and
// hands them to the march worker.
void bpm_server::run_setup()
{
    std::vector<char> host;
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                for (auto it = waiting.begin(); it != waiting.end();) {
                    if ((*it)->cancel) {
                        finish(*it, BPM_E_CANCELLED);
                        it = waiting.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (!waiting.empty() && admitted_slots < cfg.max_slots &&
                    stats.bytes_in_use + waiting.front()->need <= cfg.hbm_budget_bytes) {
                    r = waiting.front();
                    waiting.pop_front();
                    stats.bytes_in_use += r->need;
                    stats.peak_bytes = std::max(stats.peak_bytes, stats.bytes_in_use);
                    admitted_slots++;
                    break;
                }
                cv_admit.wait(lk);
            }
        }
        bpm_status st = setup(*r, host);
        std::lock_guard<std::mutex> lk(mu);
        if (st != BPM_OK) {
            if (r->plan) bpm_plan_destroy(r->plan);
            r->plan = nullptr;
            dev_free(r->d_state);
            r->d_state = nullptr;
            stats.bytes_in_use -= r->need;
            admitted_slots--;
            finish(r, st);
            continue;
        }
        r->res.t_admit = now();
        stats.admitted++;
        ready.push_back(r);
        cv_work.notify_all();
    }
}

// Results of a solve that reached its end (status BPM_OK so far): exit
// envelopes to the request's buffers, R and T from rt; returns the final status.
int bpm_server::retire(Request &r, int status, const double *rt)
{
    if (status != BPM_OK) return status;
    const size_t sb = r.plan->state_bytes(), nx = r.plan->cells();
    if (r.out_p || r.out_m) {
        std::vector<char> host(sb);
        if (hipMemcpy(host.data(), r.d_state, sb, hipMemcpyDeviceToHost) != hipSuccess) return BPM_E_DEVICE;
        for (size_t j = 0; j < nx; ++j) {
            double v[4];
            if (r.desc.precision == BPM_F64) {
                const double *o = (const double *)host.data();
                v[0] = o[2 * j], v[1] = o[2 * j + 1], v[2] = o[2 * (nx + j)], v[3] = o[2 * (nx + j) + 1];
            } else {
                const float *o = (const float *)host.data();
                v[0] = o[2 * j], v[1] = o[2 * j + 1], v[2] = o[2 * (nx + j)], v[3] = o[2 * (nx + j) + 1];
            }
            if (r.out_p) r.out_p[j] = {v[0], v[1]};
            if (r.out_m) r.out_m[j] = {v[2], v[3]};
        }
    }
    r.res.R = rt[0];
    r.res.T = rt[1];
    if (!std::isfinite(r.res.R) || !std::isfinite(r.res.T)) return BPM_E_NUMERIC;
    return BPM_OK;
}

// March worker: rounds over every active solve; requests set up by the
// admission thread join at the start of the next round.
void bpm_server::run()
{
    double t_host_prev = 0.0;   // host time after the previous round's wait (its retiring)
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                for (auto &r : ready) active.push_back(r);
                ready.clear();
                if (!active.empty()) break;
                cv_work.wait(lk);
            }
        }
        const double t_round = now();

        // ---- staged / 3D solves with a long march ahead take a free wide lane
        // while the device has room (at a round boundary the state is in
        // natural order, so a solve can move there part way through)
        int regular = 0;
        for (auto &r : active) regular += r->wide_lane < 0;
        for (auto &r : active) {
            if (r->wide_lane >= 0 || !r->plan->d_wide_ctl || regular - 1 > kWideMaxRegular ||
                one_workgroup_seconds(r->desc) * (r->desc.nz - r->step) / r->desc.nz <= kWideMinSeconds)
                continue;
            for (int k = 0; k < kMaxWide && r->wide_lane < 0; ++k) {
                if (wide_busy[k]) continue;
                if (!wide_streams[k] && hipStreamCreateWithFlags(&wide_streams[k], hipStreamNonBlocking) != hipSuccess) {
                    wide_streams[k] = nullptr;
                    continue;
                }
                wide_busy[k] = true;
                r->wide_lane = k;
                regular--;
                std::lock_guard<std::mutex> lk(mu);
                stats.wide++;
            }
        }

        // ---- one round: every active solve advances steps_for() z-steps (wide
        // solves kWideChunkFactor * chunk_steps); per precision one stream and
        // one any-size launch, so solves of every size and strain class run
        // side by side, and each wide solve on its own stream.  With more
        // solves than compute units the launch runs in layers of workgroups
        // (one per unit), and the hardware dispatcher packs the uneven chunks.
        std::vector<int> adv(active.size(), 0);
        bool ok = true;
        std::vector<size_t> reg;   // solves of the any-size launches
        for (size_t i = 0; i < active.size(); ++i) {
            auto &r = active[i];
            if (r->wide_lane < 0) {
                r->slot = (int)reg.size();
                reg.push_back(i);
                continue;
            }
            adv[i] = std::min(kWideChunkFactor * cfg.chunk_steps, r->desc.nz - r->step);
            const int fl = (r->step == 0 ? SF_FIRST : 0) | (r->step + adv[i] == r->desc.nz ? SF_LAST : 0);
            if (propagate_wide(r->plan, wide_streams[r->wide_lane], (const char *)r->d_state, (char *)r->d_state,
                               r->plan->d_rt, r->step, adv[i], fl) != BPM_OK)
                ok = false;
        }
        std::map<int, std::vector<size_t>> cls;
        for (size_t i : reg) cls[active[i]->desc.precision].push_back(i);
        for (auto &kv : cls) {
            const auto &ids = kv.second;
            const int n = (int)ids.size();
            std::vector<bpm_plan *> plans(n);
            std::vector<int> rt(n), s0(n), ns(n), fl(n);
            std::vector<uint64_t> off(n);
            for (int k = 0; k < n; ++k) {
                auto &r = active[ids[k]];
                plans[k] = r->plan;
                rt[k] = r->slot;
                s0[k] = r->step;
                ns[k] = adv[ids[k]] = steps_for(*r);
                fl[k] = (r->step == 0 ? SF_FIRST : 0) | (r->step + ns[k] == r->desc.nz ? SF_LAST : 0);
                off[k] = (uint64_t)(uintptr_t)r->d_state;
            }
            hipStream_t cs = stream_for(kv.first);
            std::vector<Launch> ls;
            bpm_status st = build_launches(plans.data(), n, rt, off, off, s0, ns, fl, ls, true);
            if (st == BPM_OK) st = upload(kv.first, ls, cs);
            if (st == BPM_OK) st = run_launches(ls, cs, nullptr, nullptr, d_rt);
            for (auto &L : ls) L.d_descs = nullptr;   // they point into descbuf
            if (st != BPM_OK) ok = false;
            std::lock_guard<std::mutex> lk(mu);
            stats.launches++;
        }

        // ---- wait for the round, then retire the solves that reached nz
        const double t_launched = now();
        for (auto &kv : streams)
            if (hipStreamSynchronize(kv.second) != hipSuccess) ok = false;
        for (auto &ws : wide_streams)
            if (ws && hipStreamSynchronize(ws) != hipSuccess) ok = false;
        const double t_waited = now();
        std::vector<double> rt(2 * reg.size());
        if (!reg.empty() && ok &&
            hipMemcpy(rt.data(), d_rt, rt.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            ok = false;
        std::vector<std::shared_ptr<Request>> keep;
        bool freed = false;
        for (size_t i = 0; i < active.size(); ++i) {
            auto &r = active[i];
            const double cells = (double)r->plan->cells();   // before the plan is released
            const double steps_done = adv[i];
            r->step += adv[i];
            const bool fin = !ok || r->step >= r->desc.nz || r->cancel;
            int status = !ok ? BPM_E_DEVICE : (r->cancel && r->step < r->desc.nz ? BPM_E_CANCELLED : BPM_OK);
            if (fin && status == BPM_OK) {
                double wrt[2] = {0.0, 0.0};
                const double *prt = &wrt[0];
                if (r->wide_lane >= 0) {
                    if (hipMemcpy(wrt, r->plan->d_rt, sizeof wrt, hipMemcpyDeviceToHost) != hipSuccess)
                        status = BPM_E_DEVICE;
                } else {
                    prt = &rt[2 * r->slot];
                }
                status = retire(*r, status, prt);
            }
            if (fin) {
                bpm_plan_destroy(r->plan);   // its blocks return to the device block cache
                r->plan = nullptr;
                dev_free(r->d_state);
                r->d_state = nullptr;
                if (r->wide_lane >= 0) wide_busy[r->wide_lane] = false;
            }
            std::lock_guard<std::mutex> lk(mu);
            stats.cell_steps_done += 2.0 * cells * steps_done;
            if (fin) {
                stats.bytes_in_use -= r->need;
                admitted_slots--;
                finish(r, status);
                freed = true;
            } else {
                keep.push_back(r);
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.rounds++;
            stats.active_max = std::max<int64_t>(stats.active_max, (int64_t)active.size());
            stats.t_device_wait_s += t_waited - t_launched;
            stats.t_host_s += t_host_prev + (t_launched - t_round);
        }
        t_host_prev = 0.0;
        active.swap(keep);
        if (freed) cv_admit.notify_all();
        t_host_prev = now() - t_waited;
    }
}

// Descriptors of a round's launches on stream st: one device buffer per
// precision reused from round to round (the worker has waited for the previous
// round, so nothing still reads it), filled from pinned host memory.
bpm_status bpm_server::upload(int prec, std::vector<Launch> &ls, hipStream_t st)
{
    size_t total = 0;
    for (auto &L : ls) total += L.host.size();
    DescBuf &b = descbuf[prec];
    if (total > b.cap) {
        (void)hipFree(b.dev);
        (void)hipHostFree(b.host);
        b.dev = b.host = nullptr;
        b.cap = 0;
        const size_t cap = std::max<size_t>(2 * total, 512);
        hipError_t e = hipMalloc((void **)&b.dev, cap * sizeof(SolveDesc));
        if (e == hipSuccess) e = hipHostMalloc((void **)&b.host, cap * sizeof(SolveDesc), 0);
        if (e != hipSuccess) return hip_fail(e, "server descriptor buffers");
        b.cap = cap;
    }
    size_t off = 0;
    for (auto &L : ls) {
        std::memcpy(b.host + off, L.host.data(), L.host.size() * sizeof(SolveDesc));
        L.d_descs = b.dev + off;
        L.d_cap = L.host.size();
        off += L.host.size();
    }
    if (total == 0) return BPM_OK;
    hipError_t e = hipMemcpyAsync(b.dev, b.host, total * sizeof(SolveDesc), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    return BPM_OK;
}

extern "C" bpm_status bpm_server_create(const bpm_server_desc *d, bpm_server **out)
{
    if (!out) return fail(BPM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d || d->chunk_steps < 1 || d->max_slots < 1 || d->hbm_budget_bytes == 0)
        return fail(BPM_E_INVALID, "server needs chunk_steps >= 1, max_slots >= 1, a nonzero budget");
    bpm_status st = ensure_device();
    if (st != BPM_OK) return st;
    bpm_server *s = new (std::nothrow) bpm_server();
    if (!s) return fail(BPM_E_NOMEM, "host allocation");
    s->cfg = *d;
    s->t0 = Clock::now();
    hipError_t e = hipMalloc((void **)&s->d_rt, 2 * (size_t)d->max_slots * sizeof(double));
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server R/T buffer");
    }
    s->worker = std::thread([s] { s->run(); });
    s->setup_thread = std::thread([s] { s->run_setup(); });
    *out = s;
    return BPM_OK;
}

extern "C" bpm_status bpm_batch_submit(bpm_server *s, const bpm_request *reqs, int32_t n, uint64_t *tickets)
{
    if (!s || (n > 0 && (!reqs || !tickets)) || n < 0) return fail(BPM_E_INVALID, "bad arguments");
    bpm_status ret = BPM_OK;
    std::vector<std::shared_ptr<Request>> made;
    for (int i = 0; i < n; ++i) {
        tickets[i] = 0;
        const bpm_plan_desc *d = reqs[i].plan;
        bpm_status st = validate_desc(d);
        if (st == BPM_OK) st = check_input(*d, reqs[i].psi_p0, reqs[i].psi_m0);
        if (st != BPM_OK) {
            if (ret == BPM_OK) ret = st;
            continue;
        }
        auto r = std::make_shared<Request>();
        r->desc = *d;
        const size_t ny = d->ny > 1 ? d->ny : 1, cells = (size_t)d->nx * ny;
        r->seg.assign(d->seg, d->seg + (size_t)d->nz * ny * d->nseg * 2);
        if (d->strain.kind == BPM_STRAIN_TABLE)
            r->utab.assign(d->strain.u_table, d->strain.u_table + (size_t)d->nz * cells);
        r->psi_p0.assign(reqs[i].psi_p0, reqs[i].psi_p0 + cells);
        if (reqs[i].psi_m0) r->psi_m0.assign(reqs[i].psi_m0, reqs[i].psi_m0 + cells);
        r->out_p = reqs[i].psi_p_out;
        r->out_m = reqs[i].psi_m_out;
        r->need = estimate_bytes(*d);
        made.push_back(r);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    size_t k = 0;
    for (int i = 0; i < n; ++i) {
        if (validate_desc(reqs[i].plan) != BPM_OK || check_input(*reqs[i].plan, reqs[i].psi_p0, reqs[i].psi_m0) != BPM_OK)
            continue;
        auto r = made[k++];
        r->ticket = s->next_ticket++;
        tickets[i] = r->ticket;
        r->res.t_submit = s->now();
        s->all[r->ticket] = r;
        s->stats.submitted++;
        if (r->need > s->cfg.hbm_budget_bytes) {
            s->finish(r, BPM_E_BUDGET);
            if (ret == BPM_OK) ret = fail(BPM_E_BUDGET, "request needs %zu bytes, budget is %zu", r->need,
                                          s->cfg.hbm_budget_bytes);
            continue;
        }
        s->waiting.push_back(r);
    }
    s->cv_admit.notify_all();
    return ret;
}

extern "C" bpm_status bpm_poll(bpm_server *s, uint64_t ticket, bpm_result *out)
{
    if (!s) return fail(BPM_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(BPM_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return BPM_E_PENDING;
    if (out) *out = it->second->res;
    return BPM_OK;
}

extern "C" bpm_status bpm_cancel(bpm_server *s, uint64_t ticket)
{
    if (!s) return fail(BPM_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(BPM_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    it->second->cancel = true;
    s->cv_admit.notify_all();
    s->cv_work.notify_all();
    return BPM_OK;
}

extern "C" bpm_status bpm_server_stats_get(bpm_server *s, bpm_server_stats *out)
{
    if (!s || !out) return fail(BPM_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return BPM_OK;
}

extern "C" bpm_status bpm_server_drain(bpm_server *s, double timeout_s)
{
    if (!s) return fail(BPM_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto pred = [s] {
        for (auto &kv : s->all)
            if (!kv.second->done) return false;
        return true;
    };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, pred);
        return BPM_OK;
    }
    if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return BPM_E_PENDING;
    return BPM_OK;
}

extern "C" void bpm_server_destroy(bpm_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_admit.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->setup_thread.joinable()) s->setup_thread.join();
    for (auto &r : s->ready) s->active.push_back(r);
    for (auto &r : s->active) {
        if (r->plan) bpm_plan_destroy(r->plan);
        dev_free(r->d_state);
    }
    for (auto &ws : s->wide_streams)
        if (ws) (void)hipStreamDestroy(ws);
    for (auto &kv : s->descbuf) {
        (void)hipFree(kv.second.dev);
        (void)hipHostFree(kv.second.host);
    }
    for (auto &kv : s->streams)
        if (kv.second) (void)hipStreamDestroy(kv.second);
    (void)hipFree(s->d_rt);
    delete s;
}
