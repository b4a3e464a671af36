// bpm_march.hpp — gfx950 device code of the two-beam FFT BPM march.
//
// One workgroup marches one solve through all of its z-steps (paper Sec. 2,
// Eq. (12) applied nz times).  Both envelopes live in VGPRs for the whole march:
// thread t owns samples t + e*TH (e < E) of psi+ and psi-.  The FFT is a
// Stockham radix-E factorisation whose passes exchange data through LDS; the
// last forward pass and the first inverse pass stay in registers, the inverse
// runs the forward passes backwards (transposed structure), so per step the
// envelopes cross LDS 2*(passes-1) times and never touch HBM.  The propagator
// multiply and the real-space coupling (mask, strain phase) are applied to the
// register-resident data between the transforms.
//
// Precision: BPM_F64 runs everything in FP64.  BPM_F32 stores and adds in FP32,
// but every multiply by a fixed constant (FFT twiddles, in-butterfly constants)
// uses a compensated hi+lo constant, and the propagator and coupling are applied
// in the form psi + (K - 1)*psi with K - 1 small, so the rounding of these
// constants does not repeat coherently from step to step.  Strain-phase
// arguments are formed and range-reduced in FP64; the incident power and R/T are
// accumulated in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "bpm_internal.hpp"

namespace bpm {

// ----------------------------------------------------------------- helpers
// value of a std::integral_constant passed through a generic lambda
#define CV(x) (std::remove_reference_t<decltype(x)>::value)

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <typename T>
struct Cx {
    T x, y;
};

// Pointers read out of a descriptor carry no address space; these views tell
// the compiler they point to global memory (global_load with a scalar base and
// a 32-bit lane offset instead of 64-bit flat addresses per lane).
template <typename X>
using gptr = const X __attribute__((address_space(1))) *;
template <typename X>
__device__ __forceinline__ gptr<X> to_global(const void *p)
{
    return (gptr<X>)(p);
}
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Cx<float> gload(gptr<Cx<float>> p, size_t i)
{
    const f2v v = ((gptr<f2v>)p)[i];
    return {v.x, v.y};
}
__device__ __forceinline__ Cx<double> gload(gptr<Cx<double>> p, size_t i)
{
    const d2v v = ((gptr<d2v>)p)[i];
    return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// cos(2 pi k / 64), k = 0..16
__host__ __device__ constexpr double qcos(int k)
{
    return k == 0 ? 1.0 : k == 1 ? 0.99518472667219693 : k == 2 ? 0.98078528040323043
         : k == 3 ? 0.95694033573220882 : k == 4 ? 0.92387953251128674 : k == 5 ? 0.88192126434835505
         : k == 6 ? 0.83146961230254524 : k == 7 ? 0.77301045336273699 : k == 8 ? 0.70710678118654757
         : k == 9 ? 0.63439328416364549 : k == 10 ? 0.55557023301960229 : k == 11 ? 0.47139673682599781
         : k == 12 ? 0.38268343236508984 : k == 13 ? 0.29028467725446233 : k == 14 ? 0.19509032201612833
         : k == 15 ? 0.09801714032956077 : 0.0;
}
__host__ __device__ constexpr double cos64(int q)
{
    q &= 63;
    return q <= 16 ? qcos(q) : q <= 32 ? -qcos(32 - q) : q <= 48 ? -qcos(q - 32) : qcos(64 - q);
}
__host__ __device__ constexpr double sin64(int q) { return cos64(q - 16); }

// a * (c + i s) for a compile-time constant (after inlining) given in FP64.
__device__ __forceinline__ Cx<float> cmul_const(Cx<float> a, double c, double s)
{
    const float ch = (float)c, cl = (float)(c - (double)ch);
    const float sh = (float)s, sl = (float)(s - (double)sh);
    return {fmaT(a.x, ch, fmaT(-a.y, sh, fmaT(a.x, cl, -a.y * sl))),
            fmaT(a.x, sh, fmaT(a.y, ch, fmaT(a.x, sl, a.y * cl)))};
}
__device__ __forceinline__ Cx<double> cmul_const(Cx<double> a, double c, double s)
{
    return {fmaT(a.x, c, -a.y * s), fmaT(a.x, s, a.y * c)};
}
// sqrt(1/2) * (a.x*cx + ..) for the odd multiples of 45 degrees.
__device__ __forceinline__ float scale_rs2(float v)
{
    constexpr double r = 0.70710678118654757;
    constexpr float rh = (float)r, rl = (float)(r - (double)rh);
    return fmaT(v, rh, v * rl);
}
__device__ __forceinline__ double scale_rs2(double v) { return v * 0.70710678118654757; }

// a * W^q with W = exp(-2 pi i / 64), compile-time q.
template <typename T, int QE>
__device__ __forceinline__ Cx<T> mul_w64(Cx<T> a)
{
    constexpr int q = QE & 63;
    if constexpr (q == 0) return a;
    else if constexpr (q == 16) return {a.y, -a.x};
    else if constexpr (q == 32) return {-a.x, -a.y};
    else if constexpr (q == 48) return {-a.y, a.x};
    else if constexpr (q == 8) return {scale_rs2(a.x + a.y), scale_rs2(a.y - a.x)};
    else if constexpr (q == 24) return {scale_rs2(a.y - a.x), scale_rs2(-a.x - a.y)};
    else if constexpr (q == 40) return {scale_rs2(-a.x - a.y), scale_rs2(a.x - a.y)};
    else if constexpr (q == 56) return {scale_rs2(a.x - a.y), scale_rs2(a.x + a.y)};
    else return cmul_const(a, cos64(q), -sin64(q));
}

// In-register DFT of size R (forward: exp(-2 pi i ms/R); INV: conjugate, no 1/R).
// Input and output in natural order.
template <typename T, int R, bool INV>
struct Dft {
    static __device__ __forceinline__ void run(Cx<T> *a)
    {
        if constexpr (R == 1) {
        } else if constexpr (R == 2) {
            Cx<T> t = a[0];
            a[0] = cadd(t, a[1]);
            a[1] = csub(t, a[1]);
        } else if constexpr (R == 4) {
            Cx<T> s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
            Cx<T> s1 = cadd(a[1], a[3]), d1 = csub(a[1], a[3]);
            Cx<T> mid = {d1.y, -d1.x};  // -i * d1
            a[0] = cadd(s0, s1);
            a[2] = csub(s0, s1);
            if constexpr (!INV) {
                a[1] = cadd(d0, mid);
                a[3] = csub(d0, mid);
            } else {
                a[1] = csub(d0, mid);
                a[3] = cadd(d0, mid);
            }
        } else {
            // R = 4 * Q: m = m1 + 4 m2, s = s2 + Q s1
            constexpr int Q = R / 4;
            Cx<T> y[4][Q];
            static_for<0, 4>([&](auto m1) {
                static_for<0, Q>([&](auto m2) { y[m1][m2] = a[m1 + 4 * m2]; });
                Dft<T, Q, INV>::run(y[m1]);
            });
            static_for<1, 4>([&](auto m1) {
                static_for<1, Q>([&](auto s2) {
                    constexpr int e = (CV(m1) * CV(s2) * (64 / R)) & 63;
                    y[m1][s2] = mul_w64<T, INV ? (64 - e) & 63 : e>(y[m1][s2]);
                });
            });
            static_for<0, Q>([&](auto s2) {
                Cx<T> z[4] = {y[0][s2], y[1][s2], y[2][s2], y[3][s2]};
                Dft<T, 4, INV>::run(z);
                static_for<0, 4>([&](auto s1) { a[s2 + Q * s1] = z[s1]; });
            });
        }
    }
};

// ----------------------------------------------------------------- twiddles
template <typename T>
struct Tw;
template <>
struct alignas(16) Tw<float> {
    float hx, hy, lx, ly;  // w = (hx + lx) + i (hy + ly)
};
template <>
struct alignas(16) Tw<double> {
    double x, y;
};

__device__ __forceinline__ Cx<float> mul_tw(Cx<float> a, const Tw<float> &w)
{
    return {fmaT(a.x, w.hx, fmaT(-a.y, w.hy, fmaT(a.x, w.lx, -a.y * w.ly))),
            fmaT(a.x, w.hy, fmaT(a.y, w.hx, fmaT(a.x, w.ly, a.y * w.lx)))};
}
__device__ __forceinline__ Cx<float> mul_tw_conj(Cx<float> a, const Tw<float> &w)
{
    return {fmaT(a.x, w.hx, fmaT(a.y, w.hy, fmaT(a.x, w.lx, a.y * w.ly))),
            fmaT(a.y, w.hx, fmaT(-a.x, w.hy, fmaT(a.y, w.lx, -a.x * w.ly)))};
}
__device__ __forceinline__ Cx<double> mul_tw(Cx<double> a, const Tw<double> &w)
{
    return {fmaT(a.x, w.x, -a.y * w.y), fmaT(a.x, w.y, a.y * w.x)};
}
__device__ __forceinline__ Cx<double> mul_tw_conj(Cx<double> a, const Tw<double> &w)
{
    return {fmaT(a.x, w.x, a.y * w.y), fmaT(a.y, w.x, -a.x * w.y)};
}
__device__ __forceinline__ Tw<float> gload(gptr<Tw<float>> p, size_t i)
{
    const f4v v = ((gptr<f4v>)p)[i];
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Tw<double> gload(gptr<Tw<double>> p, size_t i)
{
    const d2v v = ((gptr<d2v>)p)[i];
    return {v.x, v.y};
}

// ----------------------------------------------------------------- schedule
// N = 2^LOG2N split into passes of radix E = 2^LOG2E (remainder radix last).
template <int LOG2N, int LOG2E>
struct Sched {
    static constexpr int N = 1 << LOG2N, E = 1 << LOG2E, LOG2TH = LOG2N - LOG2E, TH = 1 << LOG2TH;
    static constexpr int REM = LOG2N % LOG2E;
    static constexpr int P = (REM ? 1 : 0) + LOG2N / LOG2E;
    static constexpr int log2r(int p) { return (p == P - 1 && REM) ? REM : LOG2E; }
    static constexpr int log2L(int p)
    {
        int s = 0;
        for (int q = 0; q < p; ++q) s += log2r(q);
        return s;
    }
    static constexpr int twbase(int p)
    {
        int s = 0;
        for (int q = 0; q < p; ++q) s += (1 << log2L(q)) * ((1 << log2r(q)) - 1);
        return s;
    }
    static constexpr int twcount() { return twbase(P); }
    // LDS padding of the exchange after pass p: one slot per L*r elements
    // when the scattered writes are strided (8 <= L*r < 64).
    static constexpr int padsh(int p)
    {
        int sh = log2L(p + 1);
        return (sh >= 3 && sh < 6) ? sh : -1;
    }
    static constexpr int bufsz()
    {
        int extra = 0;
        for (int p = 0; p + 1 < P; ++p)
            if (padsh(p) >= 0 && ((N - 1) >> padsh(p)) + 1 > extra) extra = ((N - 1) >> padsh(p)) + 1;
        return N + extra;
    }
};

template <typename S, int p>
__device__ __forceinline__ int padpos(int pos)
{
    constexpr int sh = S::padsh(p);
    if constexpr (sh >= 0) return pos + (pos >> sh);
    else return pos;
}

constexpr size_t kLdsMax = 160 * 1024;

// LDS plan: NBUF buffers, BX beams per buffer.
template <typename T, int LOG2N, int LOG2E>
struct LdsPlan {
    using S = Sched<LOG2N, LOG2E>;
    static constexpr size_t beam_bytes = (size_t)S::bufsz() * sizeof(Cx<T>);
    static constexpr int NBUF = 4 * beam_bytes <= kLdsMax ? 2 : 1;
    static constexpr int BX = 2 * beam_bytes <= kLdsMax ? 2 : 1;
    static constexpr size_t bytes = (size_t)NBUF * BX * beam_bytes;
    static constexpr bool fits = beam_bytes <= kLdsMax;
};

// ----------------------------------------------------------------- march
template <typename T>
__device__ __forceinline__ T to_T(double v) { return (T)v; }

// Strain phase (revolutions) of a straight edge dislocation, line along y and b
// along h (Eq. (15)): (b/d)/(2 pi) * (atan2(Z, X) + X Z / (2 (1 - nu) r^2)).
// Kept out of line: it runs only inside the crystal of dislocation solves.
__device__ __noinline__ double edge_phase_rev(double X, double Z, double k, double q)
{
    const double r2 = __builtin_fma(X, X, Z * Z);
    double a = atan2(Z, X);
    if (r2 > 0.0) a += X * Z * q / r2;
    return k * a;
}

__device__ __forceinline__ void sincospi_T(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_T(double x, double *s, double *c) { sincospi(x, s, c); }

// exp(2 pi i v) for a phase v in revolutions: reduced to [-1/2, 1/2] in FP64,
// then evaluated in T.
template <typename T>
__device__ __forceinline__ Cx<T> phasor(double v)
{
    const double fr = v - rint(v);
    T sn, cs;
    sincospi_T((T)(2.0 * fr), &sn, &cs);
    return {cs, sn};
}

// psi+ <- psi+ + d0 psi+ + bp psi-,  psi- <- psi- + d0 psi- + bm psi+   (Eq. (12))
template <typename T>
__device__ __forceinline__ void couple(Cx<T> &vp, Cx<T> &vm, Cx<T> d0, Cx<T> bp, Cx<T> bm)
{
    const Cx<T> a = vp, b = vm;
    vp = {fmaT(bp.x, b.x, fmaT(-bp.y, b.y, fmaT(d0.x, a.x, fmaT(-d0.y, a.y, a.x)))),
          fmaT(bp.x, b.y, fmaT(bp.y, b.x, fmaT(d0.x, a.y, fmaT(d0.y, a.x, a.y))))};
    vm = {fmaT(bm.x, a.x, fmaT(-bm.y, a.y, fmaT(d0.x, b.x, fmaT(-d0.y, b.y, b.x)))),
          fmaT(bm.x, a.y, fmaT(bm.y, a.x, fmaT(d0.x, b.y, fmaT(d0.y, b.x, b.y))))};
}

template <typename T, int LOG2N, int LOG2E, int SC>
struct March {
    using S = Sched<LOG2N, LOG2E>;
    using LP = LdsPlan<T, LOG2N, LOG2E>;
    static constexpr int N = S::N, E = S::E, TH = S::TH, P = S::P, BUF = S::bufsz();

    // ---- forward pass p, in registers: twiddle, DFT_r; output s of butterfly
    // i lands in v[i + s*E/r].
    template <int p>
    static __device__ __forceinline__ void fwd_compute(Cx<T> *vp, Cx<T> *vm, gptr<Tw<T>> tw, int t)
    {
        constexpr int r = 1 << S::log2r(p), EPR = E / r, L = 1 << S::log2L(p);
        static_for<0, EPR>([&](auto i) {
            Cx<T> ap[r], am[r];
            static_for<0, r>([&](auto m) {
                ap[m] = vp[i + m * EPR];
                am[m] = vm[i + m * EPR];
            });
            if constexpr (p > 0) {
                const int j = (t + i * TH) & (L - 1);
                static_for<1, r>([&](auto m) {
                    const Tw<T> w = gload(tw, S::twbase(p) + (m - 1) * L + j);
                    ap[m] = mul_tw(ap[m], w);
                    am[m] = mul_tw(am[m], w);
                });
            }
            Dft<T, r, false>::run(ap);
            Dft<T, r, false>::run(am);
            static_for<0, r>([&](auto s) {
                vp[i + s * EPR] = ap[s];
                vm[i + s * EPR] = am[s];
            });
        });
    }

    template <int p>
    static __device__ __forceinline__ void inv_compute(Cx<T> *vp, Cx<T> *vm, gptr<Tw<T>> tw, int t)
    {
        constexpr int r = 1 << S::log2r(p), EPR = E / r, L = 1 << S::log2L(p);
        static_for<0, EPR>([&](auto i) {
            Cx<T> ap[r], am[r];
            static_for<0, r>([&](auto s) {
                ap[s] = vp[i + s * EPR];
                am[s] = vm[i + s * EPR];
            });
            Dft<T, r, true>::run(ap);
            Dft<T, r, true>::run(am);
            if constexpr (p > 0) {
                const int j = (t + i * TH) & (L - 1);
                static_for<1, r>([&](auto m) {
                    const Tw<T> w = gload(tw, S::twbase(p) + (m - 1) * L + j);
                    ap[m] = mul_tw_conj(ap[m], w);
                    am[m] = mul_tw_conj(am[m], w);
                });
            }
            static_for<0, r>([&](auto m) {
                vp[i + m * EPR] = ap[m];
                vm[i + m * EPR] = am[m];
            });
        });
    }

    // Scattered positions of pass p: butterfly b = t + i*TH (j = b mod L,
    // k = b / L) puts output s at j + s*L + k*L*r.  With the pad of one slot per
    // L*r elements the padded address is (j + k*(L*r + 1)) + s*L: one base per
    // butterfly plus compile-time offsets.
    template <int p>
    static __device__ __forceinline__ int scatter_base(int b)
    {
        constexpr int lr = S::log2r(p), ll = S::log2L(p), L = 1 << ll;
        const int j = b & (L - 1), k = b >> ll;
        if constexpr (S::padsh(p) >= 0) return j + k * ((1 << (ll + lr)) + 1);
        else return j + (k << (ll + lr));
    }
    template <int p>
    static __device__ __forceinline__ void scatter_write(Cx<T> *L0, const Cx<T> *v, int t)
    {
        constexpr int r = 1 << S::log2r(p), EPR = E / r, L = 1 << S::log2L(p);
        static_for<0, EPR>([&](auto i) {
            Cx<T> *base = L0 + scatter_base<p>(t + i * TH);
            static_for<0, r>([&](auto s) { base[s * L] = v[i + s * EPR]; });
        });
    }
    template <int p>
    static __device__ __forceinline__ void scatter_read(const Cx<T> *L0, Cx<T> *v, int t)
    {
        constexpr int r = 1 << S::log2r(p), EPR = E / r, L = 1 << S::log2L(p);
        static_for<0, EPR>([&](auto i) {
            const Cx<T> *base = L0 + scatter_base<p>(t + i * TH);
            static_for<0, r>([&](auto s) { v[i + s * EPR] = base[s * L]; });
        });
    }
    // Column positions t + e*TH; padded: (t + t>>sh) + e*(TH + TH>>sh) when
    // TH is a multiple of the pad period.
    template <int p>
    static __device__ __forceinline__ void column_write(Cx<T> *L0, const Cx<T> *v, int t)
    {
        constexpr int sh = S::padsh(p);
        if constexpr (sh < 0) {
            static_for<0, E>([&](auto e) { L0[t + e * TH] = v[e]; });
        } else if constexpr ((TH >> sh) << sh == TH) {
            Cx<T> *base = L0 + t + (t >> sh);
            static_for<0, E>([&](auto e) { base[e * (TH + (TH >> sh))] = v[e]; });
        } else {
            static_for<0, E>([&](auto e) { L0[padpos<S, p>(t + e * TH)] = v[e]; });
        }
    }
    template <int p>
    static __device__ __forceinline__ void column_read(const Cx<T> *L0, Cx<T> *v, int t)
    {
        constexpr int sh = S::padsh(p);
        if constexpr (sh < 0) {
            static_for<0, E>([&](auto e) { v[e] = L0[t + e * TH]; });
        } else if constexpr ((TH >> sh) << sh == TH) {
            const Cx<T> *base = L0 + t + (t >> sh);
            static_for<0, E>([&](auto e) { v[e] = base[e * (TH + (TH >> sh))]; });
        } else {
            static_for<0, E>([&](auto e) { v[e] = L0[padpos<S, p>(t + e * TH)]; });
        }
    }

    // exchange after forward pass p (slot p) / before inverse pass p (slot 2P-3-p)
    template <int p, bool INVDIR>
    static __device__ __forceinline__ void exchange(Cx<T> *vp, Cx<T> *vm, Cx<T> *lds, int t)
    {
        constexpr int slot = INVDIR ? 2 * P - 3 - p : p;
        constexpr int q = slot % LP::NBUF;
        if constexpr (LP::BX == 2) {
            Cx<T> *Lp = lds + (q * 2 + 0) * BUF;
            Cx<T> *Lm = lds + (q * 2 + 1) * BUF;
            if constexpr (LP::NBUF == 1) __syncthreads();
            if constexpr (!INVDIR) {
                scatter_write<p>(Lp, vp, t);
                scatter_write<p>(Lm, vm, t);
                __syncthreads();
                column_read<p>(Lp, vp, t);
                column_read<p>(Lm, vm, t);
            } else {
                column_write<p>(Lp, vp, t);
                column_write<p>(Lm, vm, t);
                __syncthreads();
                scatter_read<p>(Lp, vp, t);
                scatter_read<p>(Lm, vm, t);
            }
        } else {
            Cx<T> *L0 = lds;
            static_for<0, 2>([&](auto beam) {
                Cx<T> *v = beam == 0 ? vp : vm;
                __syncthreads();
                if constexpr (!INVDIR) scatter_write<p>(L0, v, t);
                else column_write<p>(L0, v, t);
                __syncthreads();
                if constexpr (!INVDIR) column_read<p>(L0, v, t);
                else scatter_read<p>(L0, v, t);
            });
        }
    }

    // |a|^2 sums over a thread's samples, FP64
    static __device__ __forceinline__ double block_sum(double v, double *red, int t)
    {
        constexpr int W = TH < 64 ? TH : 64;
        for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
        if constexpr (TH > 64) {
            __syncthreads();
            if ((t & 63) == 0) red[t >> 6] = v;
            __syncthreads();
            double s = 0.0;
            for (int w = 0; w < TH / 64; ++w) s += red[w];
            v = s;
        }
        return v;
    }

    static __device__ void run(const SolveDesc &d, const char *in_base, char *out_base, double *rt,
                               Cx<T> *lds, double *red)
    {
        const int t = threadIdx.x;
        const Cx<T> *in = reinterpret_cast<const Cx<T> *>(in_base + d.in_off);
        Cx<T> *out = reinterpret_cast<Cx<T> *>(out_base + d.out_off);
        const gptr<Tw<T>> tw = to_global<Tw<T>>(d.tw);
        const gptr<Cx<T>> prop = to_global<Cx<T>>(d.prop);
        const gptr<int> seg = to_global<int>(d.seg);
        const gptr<T> utab = to_global<T>(d.utab);

        Cx<T> vp[E], vm[E];
        static_for<0, E>([&](auto e) {
            vp[e] = in[t + e * TH];
            vm[e] = in[N + t + e * TH];
        });

        double pin = 0.0;
        if (d.flags & SF_FIRST) {
            double s = 0.0;
            static_for<0, E>([&](auto e) {
                const double x = (double)vp[e].x, y = (double)vp[e].y;
                s = __builtin_fma(x, x, __builtin_fma(y, y, s));
            });
            pin = block_sum(s, red, t);
            if (t == 0 && d.pin) *d.pin = pin;
        }

        const PlanScalars &sc = *d.sc;
        const Cx<T> d0 = {to_T<T>(sc.d0x), to_T<T>(sc.d0y)};
        const Cx<T> ap = {to_T<T>(sc.apx), to_T<T>(sc.apy)};
        const Cx<T> am = {to_T<T>(sc.amx), to_T<T>(sc.amy)};
        const T invN = (T)(1.0 / (double)N);
        const int kind = d.strain_kind;
        const int nseg = d.nseg;
        const double X0 = d.x0 - d.x_ref;

        const int nend = d.step0 + d.nsteps;
        for (int n = d.step0; n < nend; ++n) {
            // The tables are loop-invariant; offsetting them by a zero the compiler
            // cannot see through makes it re-read them each step (from L1/L2)
            // instead of pinning ~2*E constants per thread in the register file.
            const int oz = n & d.opaque_zero;
            const gptr<Tw<T>> twn = tw + oz;
            // a second opaque zero: the inverse passes re-read the twiddles
            // instead of keeping the forward passes' copies alive across the step
            const gptr<Tw<T>> twi = tw + ((n ^ 1) & d.opaque_zero);
            const gptr<Cx<T>> propn = prop + oz;
            // per-step opaque thread index: per-lane LDS and table offsets are
            // recomputed in the loop instead of being hoisted and spilled
            const int t = threadIdx.x + oz;
            // ---- Fourier-space propagation of both envelopes (Eq. (12) p+-)
            static_for<0, P>([&](auto pc) {
                constexpr int p = CV(pc);
                fwd_compute<p>(vp, vm, twn, t);
                if constexpr (p + 1 < P) exchange<p, false>(vp, vm, lds, t);
            });
            static_for<0, E>([&](auto e) {
                const int f = t + e * TH;
                const Cx<T> kp = gload(propn, f), km = gload(propn, N + f);
                const Cx<T> a = vp[e], b = vm[e];
                vp[e] = {fmaT(kp.x, a.x, fmaT(-kp.y, a.y, a.x * invN)),
                         fmaT(kp.x, a.y, fmaT(kp.y, a.x, a.y * invN))};
                vm[e] = {fmaT(km.x, b.x, fmaT(-km.y, b.y, b.x * invN)),
                         fmaT(km.x, b.y, fmaT(km.y, b.x, b.y * invN))};
            });
            static_for<0, P>([&](auto pp) {
                constexpr int p = P - 1 - CV(pp);
                if constexpr (p + 1 < P) exchange<p, true>(vp, vm, lds, t);
                inv_compute<p>(vp, vm, twi, t);
            });

            // ---- real-space coupling inside the crystal (Eq. (9)-(12))
            const gptr<int> sg = seg + (size_t)n * nseg * 2;
            const int lo0 = sg[0], hi0 = sg[1];
            const bool all_in = (nseg == 1) & (lo0 <= 0) & (hi0 >= N);
            auto inside_at = [&](int j) {
                bool in = all_in | ((j >= lo0) & (j < hi0));
                for (int k = 1; k < nseg; ++k) in |= (j >= sg[2 * k]) & (j < sg[2 * k + 1]);
                return in;
            };
            const double Z = n * d.dz - d.z_ref;
            if constexpr (SC == SC_NONE) {
                static_for<0, E>([&](auto e) {
                    if (inside_at(t + e * TH)) couple(vp[e], vm[e], d0, ap, am);
                });
            } else if constexpr (SC == SC_POLY2) {
                // phase (revolutions) u/d = pa + pb X + pc X^2 along this z; along a
                // thread's samples X_e = X_t + e D it is quadratic in e, so the
                // phasors follow P_{e+1} = P_e Q_e, Q_{e+1} = Q_e R with P_0, Q_0, R
                // from FP64 arguments reduced to one revolution.
                const double pa = (d.c[0] + Z * (d.c[2] + Z * d.c[5])) * d.inv_d;
                const double pb = (d.c[1] + Z * d.c[4]) * d.inv_d;
                const double pc = d.c[3] * d.inv_d;
                const double D = (double)TH * d.dx;
                const double Xt = __builtin_fma((double)t, d.dx, X0);
                Cx<T> P = phasor<T>(__builtin_fma(__builtin_fma(pc, Xt, pb), Xt, pa));
                Cx<T> Q = phasor<T>(__builtin_fma(pc, __builtin_fma(2.0 * Xt, D, D * D), pb * D));
                const Cx<T> Rr = phasor<T>(2.0 * pc * D * D);
                static_for<0, E>([&](auto e) {
                    if (inside_at(t + e * TH)) {
                        const Cx<T> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
                        const Cx<T> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
                        couple(vp[e], vm[e], d0, bp, bm);
                    }
                    if constexpr (CV(e) + 1 < E) {
                        P = {fmaT(P.x, Q.x, -P.y * Q.y), fmaT(P.x, Q.y, P.y * Q.x)};
                        Q = {fmaT(Q.x, Rr.x, -Q.y * Rr.y), fmaT(Q.x, Rr.y, Q.y * Rr.x)};
                    }
                });
            } else {
                static_for<0, E>([&](auto e) {
                    const int j = t + e * TH;
                    if (inside_at(j)) {
                        const double rev = kind == STRAIN_EDGE
                                               ? edge_phase_rev(__builtin_fma((double)j, d.dx, X0), Z, d.disl_k,
                                                                d.disl_q)
                                               : (double)utab[(size_t)n * N + j];
                        const Cx<T> P = phasor<T>(rev);
                        const Cx<T> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
                        const Cx<T> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
                        couple(vp[e], vm[e], d0, bp, bm);
                    }
                });
            }
        }

        static_for<0, E>([&](auto e) {
            out[t + e * TH] = vp[e];
            out[N + t + e * TH] = vm[e];
        });

        if ((d.flags & SF_LAST) && d.rt_index >= 0) {
            double sp = 0.0, sm = 0.0;
            static_for<0, E>([&](auto e) {
                const int j = t + e * TH;
                if (j >= d.det_lo && j < d.det_hi) {
                    const double px = vp[e].x, py = vp[e].y, mx = vm[e].x, my = vm[e].y;
                    sp = __builtin_fma(px, px, __builtin_fma(py, py, sp));
                    sm = __builtin_fma(mx, mx, __builtin_fma(my, my, sm));
                }
            });
            sp = block_sum(sp, red, t);
            sm = block_sum(sm, red, t);
            if (t == 0) {
                if (!(d.flags & SF_FIRST)) pin = d.pin ? *d.pin : 0.0;
                const double R = pin > 0.0 ? sm / pin : 0.0;
                const double Tt = pin > 0.0 ? sp / pin : 0.0;
                rt[2 * d.rt_index] = R;
                rt[2 * d.rt_index + 1] = Tt;
            }
        }
    }
};


// Sizes the march kernels are built for.  Uniform kernels: one solve per
// workgroup of nx/E threads; mixed kernel: 2^kMixedLog2Th threads, any nx in
// [2^mix_lo, 2^mix_hi] within one grid.
template <typename T>
struct Limits;
template <>
struct Limits<float> {
    static constexpr int uni_lo = 6, uni_hi = 14, mix_lo = 10, mix_hi = 14;
};
template <>
struct Limits<double> {
    static constexpr int uni_lo = 6, uni_hi = 13, mix_lo = 10, mix_hi = 13;
};
constexpr int kMixedLog2Th = 9;

}  // namespace bpm
