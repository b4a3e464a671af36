// bpm_api_internal.hpp — host-side objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "bpm.h"
#include "bpm_internal.hpp"

struct bpm_plan {
    bpm_plan_desc desc{};     // copy; its array pointers are cleared
    int log2n = 0;
    int threads = 0;
    size_t lds_bytes = 0;
    size_t device_bytes = 0;
    bpm::PlanScalars *d_sc = nullptr;
    bpm::PlanParams *d_params = nullptr;
    void *d_prop = nullptr;      // [2][nx] (P - 1)/nx, shared through the propagator cache
    int32_t *d_seg = nullptr;    // [nz][nseg][2]
    void *d_utab = nullptr;      // strain table (TABLE kind)
    double *d_pin = nullptr;     // incident power
    bpm::SolveDesc *d_desc1 = nullptr;  // single-solve descriptor
    const void *tw_uniform = nullptr;   // shared twiddle table
    void *d_state = nullptr;     // staging for bpm_propagate
    double *d_rt = nullptr;      // R/T scratch
    bpm_plan *far = nullptr;     // vacuum plan of bpm_far_field (one step of far_um)
    double far_um = 0.0;
    int log2ny = 0;              // 3D envelopes: log2(ny), else 0
    int launch_kind = 0;         // launch_march's size argument for this plan alone
    // wide lane (staged sizes and 3D marched alone): control block, partial
    // sums, and a recorded graph of kWideGraphSteps z-steps
    bpm::WideCtl *d_wide_ctl = nullptr;
    double *d_wide_part = nullptr;
    int wide_blocks = 0;         // column-phase workgroups (partial sums)
    hipGraph_t wide_graph = nullptr;
    hipGraphExec_t wide_exec = nullptr;
    bool wide_tried = false;     // graph recording attempted

    size_t cells() const { return (size_t)desc.nx * (log2ny ? (size_t)1 << log2ny : 1); }
    size_t rows() const { return (size_t)desc.nz * (log2ny ? (size_t)1 << log2ny : 1); }

    void release();
    size_t state_bytes() const;
    void fill(bpm::SolveDesc &s, int log2e, const void *tw, int flags, int step0, int nsteps, uint64_t in_off,
              uint64_t out_off, int rt_index) const;
};

namespace bpm {

bpm_status fail(bpm_status s, const char *fmt, ...);
bpm_status hip_fail(hipError_t e, const char *what);
bpm_status ensure_device();
bpm_status validate_desc(const bpm_plan_desc *d);
bpm_status check_input(const bpm_plan_desc &d, const bpm_complex *a, const bpm_complex *b);
bpm_status twiddle_table(int prec, int log2n, int log2e, const void **out);
// Device blocks of plans and solve states through the library's size-class
// cache: dev_free returns a block to its class (no hipFree, which waits for the
// device) unless the cache is full.  Blocks from dev_malloc go to dev_free only.
hipError_t dev_malloc(void **p, size_t bytes);
void dev_free(void *p);
// Schedule table (bpm_tune.cpp): the bpm_schedule a batch group of one
// (precision, log2 nx, strain class) runs with; BPM_SCHED_DEFAULT when none.
int tuned_schedule(int prec, int log2n, int sc);
// can `schedule` march 2^log2n at prec (2D)
bool schedule_fits(int prec, int log2n, int schedule);

// Library-owned non-blocking stream of the current device for plan setup.
hipStream_t setup_stream();
// z-steps [step0, step0 + nsteps) of a plan that has a wide form (p->d_wide_ctl
// set) over the device, enqueued on s: natural-order state in `in`, out to
// `out`; flags SF_FIRST (store the incident power) and SF_LAST (R, T to rt,
// 2 doubles) as for the march kernels.  With ctl and part NULL the plan's own
// control block and partial sums are used and 32-step blocks replay a graph
// recorded on the first long call; otherwise the caller's ctl (one WideCtl)
// and part (3 * p->wide_blocks doubles) are used and every step is launched
// directly (no graph, no allocation).
bpm_status propagate_wide(bpm_plan *p, hipStream_t s, const char *in, char *out, double *rt, int step0, int nsteps,
                          int flags, WideCtl *ctl = nullptr, double *part = nullptr);

// One kernel launch over a group of solves.
struct Launch {
    int prec = 0;
    int sc = 0;            // strain class of every solve in the launch
    int uniform_log2n = -1;
    int n = 0;
    std::vector<SolveDesc> host;
    SolveDesc *d_descs = nullptr;
    size_t d_cap = 0;
};

// Group solves into launches: per (precision, strain class), one launch when
// all share nx (the schedule table's kernel family for that size, or
// force_schedule when nonzero; by default the per-size kernel), one mixed launch
// when all sizes fit the mixed kernel, and otherwise per size.  With any_size, every solve of a size the any-size kernel
// takes, of any strain class, goes into one launch of it per precision (whatever
// the mix, so a solve's arithmetic never depends on what else is launched) and
// smaller sizes per size.  Longest solves first.
bpm_status build_launches(bpm_plan *const *plans, int n, const std::vector<int> &rt_index,
                          const std::vector<uint64_t> &in_off, const std::vector<uint64_t> &out_off,
                          const std::vector<int> &step0, const std::vector<int> &nsteps,
                          const std::vector<int> &flags, std::vector<Launch> &launches, bool any_size = false,
                          int force_schedule = 0);
// Descriptor upload: blocking when s is NULL, else ordered on stream s.
bpm_status upload_launches(std::vector<Launch> &launches, hipStream_t s = nullptr);
bpm_status run_launches(const std::vector<Launch> &launches, hipStream_t s, const char *in, char *out,
                        double *rt);
void free_launches(std::vector<Launch> &launches);

}  // namespace bpm
