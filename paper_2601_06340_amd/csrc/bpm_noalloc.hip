// bpm_noalloc.hip — the march entry point that allocates nothing.
//
// bpm_propagate_device spreads a plan of a staged size or of 3D envelopes over
// the device (the wide lane).  Its launches keep a control block and per-
// workgroup partial sums of the incident power and the detector powers in plan
// memory, and its first long call records a HIP graph of 32 z-steps.  The
// variant here keeps the control block and the partial sums in `scratch`, a
// file-scope device array of kScratchBytes held by every device the library
// runs on until the process ends, and launches every step directly: after the
// plan exists, a call makes no device allocation and records no graph.  The
// kernels and their order are the same, so the results equal
// bpm_propagate_device's bitwise.
//
// Every call on one device shares that device's array and leaves its contents
// behind.  Each call writes every entry it later reads (the control block
// first, then one set of partial sums per column workgroup), so nothing needs
// clearing; calls that overlap on one device race for it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bpm.h"
#include "bpm_api_internal.hpp"
#include "bpm_internal.hpp"

using namespace bpm;

namespace {

constexpr size_t kScratchBytes = 16384;
constexpr size_t kCtlBytes = 256;   // the control block, then the partial sums
static_assert(sizeof(WideCtl) <= kCtlBytes, "control block");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).  In host code the array's name is only a
// handle for this lookup, never an address.
bpm_status scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(BPM_E_DEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BPM_OK;
}

}  // namespace

extern "C" bpm_status bpm_propagate_device_noalloc(bpm_plan *p, void *stream, const void *d_in, void *d_out,
                                                   double *d_RT)
{
    if (!p || !d_in || !d_out) return fail(BPM_E_INVALID, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    double *rt = d_RT ? d_RT : p->d_rt;
    if (!p->d_wide_ctl) {
        // one workgroup marches the solve: no scratch, the plan's own descriptor
        hipError_t e = launch_march(p->d_desc1, 1, p->desc.precision, p->launch_kind,
                                    march_class(p->desc.strain.kind, p->desc.strain.c[3]), (const char *)d_in,
                                    (char *)d_out, rt, s);
        if (e != hipSuccess) return hip_fail(e, "march launch");
        return BPM_OK;
    }
    const size_t need = kCtlBytes + 3 * sizeof(double) * (size_t)p->wide_blocks;
    if (need > kScratchBytes)
        return fail(BPM_E_UNSUPPORTED, "the wide march needs %zu bytes of scratch, the library holds %zu", need,
                    kScratchBytes);
    void *base = nullptr;
    bpm_status st = scratch_ptr(&base);
    if (st != BPM_OK) return st;
    WideCtl *ctl = (WideCtl *)base;
    double *part = (double *)((char *)base + kCtlBytes);
    return propagate_wide(p, s, (const char *)d_in, (char *)d_out, rt, 0, p->desc.nz, SF_FIRST | SF_LAST, ctl,
                          part);
}
