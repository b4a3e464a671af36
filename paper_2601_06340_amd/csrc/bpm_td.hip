// bpm_td.hip — time-domain assembly of a batch of spectral components (Sec. 8).
#include "bpm_march.hpp"

namespace bpm {

// Carrier phase exp(i k_m c_m L_m) of component m: k c L / 2 pi = c L / lambda
// revolutions with c = sqrt(1 - (lambda / 2d)^2), reduced to one revolution in
// FP64 before the sine and cosine.
template <typename T>
__global__ void k_td_phasors(const double *par, Cx<T> *ph, int M)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) {
        const double lam = par[3 * m], d = par[3 * m + 1], L = par[3 * m + 2];
        const double s = lam / (2.0 * d);
        const double rev = sqrt(1.0 - s * s) * L / lam;
        const double fr = rev - rint(rev);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        ph[m] = {(T)cs, (T)sn};
    }
}

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {fmaT(a.x, b.x, -a.y * b.y), fmaT(a.x, b.y, a.y * b.x)};
}

// One wave per x sample: the M components of that sample (component m from the
// batch state at offs[m]), times their carriers, through an M-point forward DFT
// over m (wave-local Stockham passes of the march); out[b][x][k].
constexpr int kTdWaves = 4;

template <typename T, int LOG2M>
__global__ __launch_bounds__(64 * kTdWaves) void k_td_assemble(const char *state, const uint64_t *offs,
                                                                const Cx<T> *ph, const Tw<T> *tw, int nx,
                                                                Cx<T> *out)
{
    using MF = March<T, LOG2M, LOG2M - 6, SC_NONE, 64 * kTdWaves, 1>;
    constexpr int E = 1 << (LOG2M - 6), MM = 1 << LOG2M;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int x = blockIdx.x * kTdWaves + wv;
    Cx<T> *R = reinterpret_cast<Cx<T> *>(smem) + wv * MF::BUFM;
    Cx<T> vp[E], vm[E];
    static_for<0, E>([&](auto e) {
        const int m = lane + 64 * CV(e);
        const Cx<T> *s = reinterpret_cast<const Cx<T> *>(state + offs[m]);
        const Cx<T> c = ph[m];
        vp[e] = cmul(s[x], c);
        vm[e] = cmul(s[nx + x], c);
    });
    MF::fwd_local(vp, vm, buf_view(tw, MF::TW_ENTRIES * (uint32_t)sizeof(Tw<T>)), R, R, lane, true);
    static_for<0, E>([&](auto e) {
        const int k = lane + 64 * CV(e);
        out[(size_t)x * MM + k] = vp[e];
        out[((size_t)nx + x) * MM + k] = vm[e];
    });
}

template <typename T, int LOG2M>
static hipError_t launch_td_T(const char *state, const uint64_t *offs, const double *par, void *ph, const void *tw,
                              int nx, void *out, hipStream_t s)
{
    constexpr int M = 1 << LOG2M;
    using MF = March<T, LOG2M, LOG2M - 6, SC_NONE, 64 * kTdWaves, 1>;
    hipLaunchKernelGGL(k_td_phasors<T>, dim3((M + 255) / 256), dim3(256), 0, s, par, (Cx<T> *)ph, M);
    const size_t lds = (size_t)kTdWaves * MF::BUFM * sizeof(Cx<T>);
    // raised once per process (a function-local static is initialised exactly once)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_td_assemble<T, LOG2M>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_td_assemble<T, LOG2M>), dim3(nx / kTdWaves), dim3(64 * kTdWaves), lds, s, state, offs,
                       (const Cx<T> *)ph, (const Tw<T> *)tw, nx, (Cx<T> *)out);
    return hipGetLastError();
}

hipError_t launch_td(int prec, int log2m, const char *state, const uint64_t *offs, const double *par, void *ph,
                     const void *tw, int nx, void *out, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    static_for<kTdLog2MMin, kTdLog2MMax + 1>([&](auto l) {
        if (log2m == CV(l))
            err = prec == PREC_F32 ? launch_td_T<float, CV(l)>(state, offs, par, ph, tw, nx, out, s)
                                   : launch_td_T<double, CV(l)>(state, offs, par, ph, tw, nx, out, s);
    });
    return err;
}

}  // namespace bpm
