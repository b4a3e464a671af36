// bpm_march_kernels.hpp — march kernels and their launch logic; the build
// instantiates each (precision, size, strain class) in its own unit.
#pragma once

#include "bpm_march.hpp"

namespace bpm {

// Waves per SIMD the LDS footprint allows (1 << LOG2TH threads per workgroup):
// the register budget is sized for that occupancy, not for an unreachable one.
template <typename T, int LOG2N, int LOG2E>
constexpr int lds_waves_per_simd()
{
    constexpr size_t bytes = LdsPlan<T, LOG2N, LOG2E>::bytes + 16 * sizeof(double);
    constexpr int wg_per_cu = (int)(kLdsMax / bytes) < 1 ? 1 : (int)(kLdsMax / bytes);
    constexpr int waves = wg_per_cu * (((1 << (LOG2N - LOG2E)) + 63) / 64);
    constexpr int per_simd = (waves + 3) / 4;
    return per_simd < 1 ? 1 : (per_simd > 8 ? 8 : per_simd);
}

// One solve per workgroup, every solve of the launch has the same nx.
template <typename T, int LOG2N, int SC>
__global__ __launch_bounds__(1 << (LOG2N - uniform_log2e(LOG2N)))
__attribute__((amdgpu_waves_per_eu(1, lds_waves_per_simd<T, LOG2N, uniform_log2e(LOG2N)>())))
void k_march_uniform(
    const SolveDesc *__restrict__ descs, int n, const char *in_base, char *out_base, double *rt)
{
    constexpr int LOG2E = uniform_log2e(LOG2N);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    const SolveDesc &d = descs[blockIdx.x];
    // FP32 with up to 256 threads (one wave per SIMD or fewer: a 512-register
    // budget): the pass twiddles stay in registers (Nx 4096 +8 %; FP64 held
    // part of them in the accumulation registers and lost 6 %)
    constexpr bool TC = LOG2N - LOG2E <= 8 && staged_prec<T>() == PREC_F32;
    March<T, LOG2N, LOG2E, SC>::template run<true, TC>(d, in_base, out_base, rt, reinterpret_cast<Cx<T> *>(smem),
                                                       red);
}

// Mixed sizes in one launch: 512 threads per workgroup, E = nx/512.
template <typename T, int SC>
__global__ __launch_bounds__(1 << kMixedLog2Th) void k_march_mixed(const SolveDesc *__restrict__ descs, int n,
                                                                    const char *in_base, char *out_base,
                                                                    double *rt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    const SolveDesc &d = descs[blockIdx.x];
    Cx<T> *lds = reinterpret_cast<Cx<T> *>(smem);
    static_for<Limits<T>::mix_lo, Limits<T>::mix_hi + 1>([&](auto l) {
        constexpr int L2 = CV(l);
        if (d.log2n == L2)
            March<T, L2, L2 - mixed_log2th(L2), SC, 1 << kMixedLog2Th>::run(d, in_base, out_base, rt, lds, red);
    });
}

// Launch every solve of a launch whose solves all have nx = 2^LOG2N.
template <typename T, int LOG2N, int SC>
hipError_t launch_uniform(const SolveDesc *d_descs, int n, const char *in_base, char *out_base, double *rt,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    constexpr int th = 1 << (LOG2N - uniform_log2e(LOG2N));
    const size_t lds = LdsPlan<T, LOG2N, uniform_log2e(LOG2N)>::bytes;
    // raised once per process (a function-local static is initialised exactly
    // once, also when several threads launch at the same time)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_march_uniform<T, LOG2N, SC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_march_uniform<T, LOG2N, SC>), dim3(n), dim3(th), lds, s, d_descs, n, in_base, out_base, rt);
    return hipGetLastError();
}

// One solve per workgroup for the staged sizes (Staged<>): one workgroup per
// compute unit (LDS), TH/256 waves per SIMD.
// (pass twiddles in registers in both precisions: FP64 spills 13 VGPRs with
// them and still marches 20 % faster)
template <typename T, int LOG2N, int SC>
using StagedK = Staged<T, LOG2N, SC, staged_log2th(staged_prec<T>()), false, staged_log2c(staged_prec<T>()),
                       staged_prefetch(staged_prec<T>()), true>;

template <typename T, int LOG2N, int SC>
__global__ __launch_bounds__(1 << staged_log2th(staged_prec<T>()))
__attribute__((amdgpu_waves_per_eu(1, (1 << staged_log2th(staged_prec<T>())) / 256)))
void k_march_staged(const SolveDesc *__restrict__ descs, int n, const char *in_base, char *out_base, double *rt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    StagedK<T, LOG2N, SC>::run(descs[blockIdx.x], in_base, out_base, rt, reinterpret_cast<Cx<T> *>(smem), red);
}

template <typename T, int LOG2N, int SC>
hipError_t launch_staged(const SolveDesc *d_descs, int n, const char *in_base, char *out_base, double *rt,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = StagedK<T, LOG2N, SC>::lds_bytes;
    // raised once per process (a function-local static is initialised exactly
    // once, also when several threads launch at the same time)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_march_staged<T, LOG2N, SC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_march_staged<T, LOG2N, SC>), dim3(n), dim3(StagedK<T, LOG2N, SC>::TH), lds, s, d_descs, n,
                       in_base, out_base, rt);
    return hipGetLastError();
}

// 3D envelopes [ny][nx], nx = 2^LOG2NX: one solve per workgroup, the staged
// lane's two phases as the 2D transform (Staged<> with D3).
// (FP32 workgroups of 512 threads with rows of 512 or fewer samples hold the
// pass twiddles in registers and keep the next round's state loads in flight
// behind the round's table loads: the paper's 3D batch 9.2e10 -> 1.06e11
// cell-steps/s; rows of 1024 have no room for them)
template <typename T, int LOG2NX, int LOG2NY, int SC>
using Stage3D = Staged<T, LOG2NX + LOG2NY, SC, staged3d_log2th(staged_prec<T>(), SC, LOG2NX), true, LOG2NX,
                       staged_prec<T>() == PREC_F32 && staged3d_log2th(staged_prec<T>(), SC, LOG2NX) == 9 &&
                           LOG2NX <= 9,
                       staged_prec<T>() == PREC_F32 && staged3d_log2th(staged_prec<T>(), SC, LOG2NX) == 9 &&
                           LOG2NX <= 9>;

template <typename T, int LOG2NX, int LOG2NY, int SC>
__global__ __launch_bounds__(1 << staged3d_log2th(staged_prec<T>(), SC, LOG2NX))
__attribute__((amdgpu_waves_per_eu(1, (1 << staged3d_log2th(staged_prec<T>(), SC, LOG2NX)) / 256)))
void k_march_3d(const SolveDesc *__restrict__ descs, int n, const char *in_base, char *out_base, double *rt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    Stage3D<T, LOG2NX, LOG2NY, SC>::run(descs[blockIdx.x], in_base, out_base, rt, reinterpret_cast<Cx<T> *>(smem),
                                        red);
}

template <typename T, int LOG2NX, int LOG2NY, int SC>
hipError_t launch_3d(const SolveDesc *d_descs, int n, const char *in_base, char *out_base, double *rt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    using S = Stage3D<T, LOG2NX, LOG2NY, SC>;
    const size_t lds = S::lds_bytes;
    // raised once per process (a function-local static is initialised exactly
    // once, also when several threads launch at the same time)
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_march_3d<T, LOG2NX, LOG2NY, SC>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_march_3d<T, LOG2NX, LOG2NY, SC>), dim3(n), dim3(S::TH), lds, s, d_descs, n, in_base,
                       out_base, rt);
    return hipGetLastError();
}

// ----------------------------------------------------------------- wide lane
// One staged-size or 3D solve over the whole device.  Every sub-step of a
// z-step is two launches: the row phase, one 64-thread workgroup per row, and
// the column phase, one 64-thread workgroup per 64/LC columns; the state stays in
// the solve's buffer (L2 / last-level cache) between them.  The per-row and
// per-column arithmetic is the one-workgroup staged march's, so the envelopes
// agree with it bitwise.  The kernels read the step base and the buffers from a
// control block, so a recorded graph of steps k = 0..K-1 (z-step base + k)
// replays for any step and any buffers.
template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
using Wide = Staged<T, LOG2N, SC, 6, D3, LOG2C>;

template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
__global__ __launch_bounds__(64) void k_wide_entry(const SolveDesc *descs, const WideCtl *ctl, double *part)
{
    using S = Wide<T, LOG2N, SC, D3, LOG2C>;
    extern __shared__ __align__(16) unsigned char smem[];
    const SolveDesc &d = descs[0];
    typename S::Ctx x;
    x.init(d, ctl->in, ctl->out, reinterpret_cast<Cx<T> *>(smem), threadIdx.x);
    const bool rt_out = (d.flags & SF_LAST) && d.rt_index >= 0;
    double pin = 0.0, sp = 0.0, sm = 0.0;
    S::entry_col(x, d, blockIdx.x * S::COLS_PER_ROUND + x.gi, 0, rt_out, pin, sp, sm);
    pin = S::RowM::block_sum(pin, nullptr, threadIdx.x);
    sp = S::RowM::block_sum(sp, nullptr, threadIdx.x);
    sm = S::RowM::block_sum(sm, nullptr, threadIdx.x);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = pin;
        part[3 * blockIdx.x + 1] = sp;
        part[3 * blockIdx.x + 2] = sm;
    }
}

template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
__global__ __launch_bounds__(64) void k_wide_rows(const SolveDesc *descs, const WideCtl *ctl, int i)
{
    using S = Wide<T, LOG2N, SC, D3, LOG2C>;
    extern __shared__ __align__(16) unsigned char smem[];
    const SolveDesc &d = descs[0];
    typename S::Ctx x;
    x.init(d, ctl->out, ctl->out, reinterpret_cast<Cx<T> *>(smem), threadIdx.x);
    S::row(x, load_sub(x.scl, i), blockIdx.x, 0, 0);
}

template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
__global__ __launch_bounds__(64) void k_wide_cols(const SolveDesc *descs, const WideCtl *ctl, int k, int i,
                                                  double *part)
{
    using S = Wide<T, LOG2N, SC, D3, LOG2C>;
    extern __shared__ __align__(16) unsigned char smem[];
    const SolveDesc &d = descs[0];
    typename S::Ctx x;
    x.init(d, ctl->out, ctl->out, reinterpret_cast<Cx<T> *>(smem), threadIdx.x);
    const int n = ctl->base + k;
    const bool rt_out = (d.flags & SF_LAST) && d.rt_index >= 0;
    double sp = 0.0, sm = 0.0;
    S::col(x, d, n, i, blockIdx.x * S::COLS_PER_ROUND + x.gi, 0, 0, rt_out, sp, sm);
    if (rt_out && i + 1 == x.scl->nsub && n + 1 == d.step0 + d.nsteps) {
        sp = S::RowM::block_sum(sp, nullptr, threadIdx.x);
        sm = S::RowM::block_sum(sm, nullptr, threadIdx.x);
        if (threadIdx.x == 0) {
            part[3 * blockIdx.x + 1] = sp;
            part[3 * blockIdx.x + 2] = sm;
        }
    }
}

template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
hipError_t launch_wide_T(int phase, const WideArgs &a, hipStream_t s, WideShape *shape)
{
    using S = Wide<T, LOG2N, SC, D3, LOG2C>;
    if (shape) {
        shape->row_blocks = S::ROW_ROUNDS;
        shape->col_blocks = S::COL_ROUNDS;
        shape->lds_bytes = S::lds_bytes;
    }
    const size_t lds = S::lds_bytes;
    switch (phase) {
    case WIDE_ENTRY:
        hipLaunchKernelGGL((k_wide_entry<T, LOG2N, SC, D3, LOG2C>), dim3(S::COL_ROUNDS), dim3(64), lds, s, a.desc,
                           a.ctl, a.part);
        break;
    case WIDE_ROWS:
        hipLaunchKernelGGL((k_wide_rows<T, LOG2N, SC, D3, LOG2C>), dim3(S::ROW_ROUNDS), dim3(64), lds, s, a.desc,
                           a.ctl, a.i);
        break;
    case WIDE_COLS:
        hipLaunchKernelGGL((k_wide_cols<T, LOG2N, SC, D3, LOG2C>), dim3(S::COL_ROUNDS), dim3(64), lds, s, a.desc,
                           a.ctl, a.k, a.i, a.part);
        break;
    default:
        return hipSuccess;
    }
    return hipGetLastError();
}

template <typename T>
size_t mixed_lds_bytes()
{
    size_t m = 0;
    static_for<Limits<T>::mix_lo, Limits<T>::mix_hi + 1>([&](auto l) {
        constexpr int L2 = CV(l);
        const size_t b = LdsPlan<T, L2, L2 - mixed_log2th(L2)>::bytes;
        if (b > m) m = b;
    });
    return m;
}

// Launch solves of different nx (all within the mixed range) in one grid.
template <typename T, int SC>
hipError_t launch_mixed(const SolveDesc *d_descs, int n, const char *in_base, char *out_base, double *rt,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = mixed_lds_bytes<T>();
    // raised once per process (a function-local static is initialised exactly
    // once, also when several threads launch at the same time)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_march_mixed<T, SC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_march_mixed<T, SC>), dim3(n), dim3(1 << kMixedLog2Th), lds, s, d_descs, n, in_base, out_base,
                       rt);
    return hipGetLastError();
}

// Any size from 2^mix_lo to 2^stg_hi and any strain class in one grid (the
// server's launches): 512 threads per workgroup, register-resident sizes as in
// the mixed kernel, the larger ones through the staged lane; each workgroup
// branches on its solve's size and strain class.
template <typename T, int SC>
__device__ __forceinline__ void march_any_sc(const SolveDesc &d, const char *in_base, char *out_base, double *rt,
                                             Cx<T> *lds, double *red)
{
    static_for<Limits<T>::mix_lo, Limits<T>::mix_hi + 1>([&](auto l) {
        constexpr int L2 = CV(l);
        if (d.log2n == L2)
            March<T, L2, L2 - mixed_log2th(L2), SC, 1 << kMixedLog2Th>::template run<false>(d, in_base, out_base, rt,
                                                                                           lds, red);
    });
    // staged sizes with the next round's loads in flight in FP32 (FP64 in this
    // kernel's 256-register budget marched 3 % slower with them)
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        if (d.log2n == CV(l))
            Staged<T, CV(l), SC, kStagedAnyLog2Th, false, staged_log2c(staged_prec<T>()),
                   staged_prec<T>() == PREC_F32>::run(d, in_base, out_base, rt, lds, red);
    });
}

// The descriptors and the resident sizes' plan scalars are read with generic
// loads here: with scalar loads (as in the other kernels) the resident sizes
// of the polynomial and dislocation classes marched up to 27 % slower, the
// kernel already spilling scalar registers.
template <typename T>
__global__ __launch_bounds__(1 << kMixedLog2Th) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_march_any(const SolveDesc *descs, int n, const char *in_base, char *out_base, double *rt)
{
    static_assert(kMixedLog2Th == kStagedAnyLog2Th, "one workgroup shape");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    const SolveDesc &d = descs[blockIdx.x];
    Cx<T> *lds = reinterpret_cast<Cx<T> *>(smem);
    const int sc = strain_class(d.strain_kind);
    if (sc == SC_NONE) march_any_sc<T, SC_NONE>(d, in_base, out_base, rt, lds, red);
    else if (sc == SC_POLY2) march_any_sc<T, SC_POLY2>(d, in_base, out_base, rt, lds, red);
    else march_any_sc<T, SC_GENERAL>(d, in_base, out_base, rt, lds, red);
}

template <typename T>
size_t any_lds_bytes()
{
    size_t m = mixed_lds_bytes<T>();
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        const size_t b = Staged<T, CV(l), SC_NONE, kStagedAnyLog2Th>::lds_bytes;
        if (b > m) m = b;
    });
    return m;
}

template <typename T>
hipError_t launch_any(const SolveDesc *d_descs, int n, const char *in_base, char *out_base, double *rt,
                      hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = any_lds_bytes<T>();
    // raised once per process (a function-local static is initialised exactly
    // once, also when several threads launch at the same time)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_march_any<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_march_any<T>), dim3(n), dim3(1 << kMixedLog2Th), lds, s, d_descs, n, in_base, out_base, rt);
    return hipGetLastError();
}

}  // namespace bpm
