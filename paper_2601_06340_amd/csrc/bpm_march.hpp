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
// Plan scalars are read-only for a whole launch: read through the constant
// address space, every field is a scalar load the compiler may issue early.
using CPlanScalars = const __attribute__((address_space(4))) PlanScalars;
__device__ __forceinline__ SubStep load_sub(CPlanScalars *p, int i)
{
    SubStep s;
    s.d0x = p->sub[i].d0x;
    s.d0y = p->sub[i].d0y;
    s.apx = p->sub[i].apx;
    s.apy = p->sub[i].apy;
    s.amx = p->sub[i].amx;
    s.amy = p->sub[i].amy;
    s.zoff = p->sub[i].zoff;
    s.table = p->sub[i].table;
    s.pad = 0;
    return s;
}
// the same through a generic pointer: a reference, loaded where it is used
// (per-lane loads the compiler may keep in vector registers)
__device__ __forceinline__ const SubStep &load_sub(const PlanScalars *p, int i) { return p->sub[i]; }
// CS: the plan scalars as scalar loads (constant address space) or generic
template <bool CS>
using PlanPtr = typename std::conditional<CS, CPlanScalars *, const PlanScalars *>::type;
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
// Loads from read-only tables: a uniform base plus a 32-bit byte offset, so the
// address is the scalar base with a per-lane 32-bit offset (no 64-bit add per load).
template <typename V>
__device__ __forceinline__ V gload_at(const void __attribute__((address_space(1))) *base, uint32_t byte_off)
{
    return *(gptr<V>)((const char __attribute__((address_space(1))) *)base + byte_off);
}
__device__ __forceinline__ Cx<float> gload(gptr<Cx<float>> p, uint32_t i)
{
    const f2v v = gload_at<f2v>(p, i * (uint32_t)sizeof(f2v));
    return {v.x, v.y};
}
__device__ __forceinline__ Cx<double> gload(gptr<Cx<double>> p, uint32_t i)
{
    const d2v v = gload_at<d2v>(p, i * (uint32_t)sizeof(d2v));
    return {v.x, v.y};
}

// Tables and solve states behind buffer resources.  The resource holds the
// buffer's base address and byte size in scalar registers; an access adds a
// per-lane 32-bit byte offset and a wave-uniform byte offset (scalar), so it
// costs no vector-ALU address arithmetic, where a per-lane 64-bit global address
// costs two instructions.  Reads at or past the size return zero and writes
// there are dropped.
constexpr int kRawBufferWord3 = 0x00020000;  // untyped 32-bit elements (gfx9 family)
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u3v __attribute__((ext_vector_type(3)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
struct BufView {
    __amdgpu_buffer_rsrc_t r;
    int base;  // wave-uniform byte offset of every load
};
// (every argument is the same across the wave; reading them from the first lane
// lets the compiler keep the resource in scalar registers)
__device__ __forceinline__ BufView buf_view(const void *p, uint32_t bytes, int base = 0)
{
    const uint64_t a = (uint64_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    void *q = (void *)(lo | (hi << 32));
    return {__builtin_amdgcn_make_buffer_rsrc(q, (short)0, __builtin_amdgcn_readfirstlane((int)bytes), kRawBufferWord3),
            __builtin_amdgcn_readfirstlane(base)};
}
// (bytes is the same across the wave)
__device__ __forceinline__ BufView operator+(BufView t, int bytes)
{
    return {t.r, __builtin_amdgcn_readfirstlane(t.base + bytes)};
}
__device__ __forceinline__ float f_of(unsigned u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ double d_of(unsigned lo, unsigned hi) { return __builtin_bit_cast(double, (u2v){lo, hi}); }
// element at byte offset lane_off (per lane) + uni_off (wave-uniform)
__device__ __forceinline__ Cx<float> tload_cx(const BufView &t, Cx<float> *, int lane_off, int uni_off)
{
    const u2v v = __builtin_amdgcn_raw_buffer_load_b64(t.r, lane_off, t.base + uni_off, 0);
    return {f_of(v.x), f_of(v.y)};
}
__device__ __forceinline__ Cx<double> tload_cx(const BufView &t, Cx<double> *, int lane_off, int uni_off)
{
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(t.r, lane_off, t.base + uni_off, 0);
    return {d_of(v.x, v.y), d_of(v.z, v.w)};
}
// real entry at byte offset lane_off (per lane) + uni_off (wave-uniform)
// Propagator table entry k = (P - 1)/N.  The same k multiplies a bin at every
// z-step, so in FP32 the rounding of k would add up linearly in Nz wherever a
// field has energy at |P - 1| ~ 1; FP32 entries therefore carry k as hi + lo
// (hi the nearest float, lo the nearest float to the remainder).
template <typename T>
struct PropE;
template <>
struct alignas(16) PropE<float> {
    float hx, hy, lx, ly;
};
template <>
struct alignas(16) PropE<double> {
    double x, y;
};
static_assert(sizeof(PropE<float>) == kPropEntryBytes && sizeof(PropE<double>) == kPropEntryBytes, "table entry");
__device__ __forceinline__ PropE<float> tload_prop(const BufView &t, PropE<float> *, int lane_i, int uni_i)
{
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(t.r, lane_i * 16, t.base + uni_i * 16, 0);
    return {f_of(v.x), f_of(v.y), f_of(v.z), f_of(v.w)};
}
__device__ __forceinline__ PropE<double> tload_prop(const BufView &t, PropE<double> *, int lane_i, int uni_i)
{
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(t.r, lane_i * 16, t.base + uni_i * 16, 0);
    return {d_of(v.x, v.y), d_of(v.z, v.w)};
}
template <typename T>
__device__ __forceinline__ PropE<T> tload_prop(const BufView &t, int lane_i, int uni_i)
{
    return tload_prop(t, (PropE<T> *)nullptr, lane_i, uni_i);
}

// FP32 table entry of the staged 2D sizes: P/N = c exp(i phi) as a lifting
// rotation by phi (folded into [-pi/2, pi/2]) and a scale c = +-|P|/N (the
// sign takes the folded half turn; |P| = 1 outside the evanescent bins, so c
// is then a signed power of two): p = -tan(phi/2) rounded to float and
// u = (1 - cos phi)/(-p) as hi + lo.  With p u = 1 - cos phi to about 2^-48
// the three shears turn the bin by exactly phi; the rounding of p only makes
// the orbit an ellipse of axis ratio 1 + O(2^-24), an amplitude wobble that
// does not grow with Nz (each shear has determinant one).  Three fewer
// operations per sample than a/N + k a with k as hi + lo; the per-size and
// mixed-size kernels, which wait on the table loads of this step, were faster
// with the hi + lo entries, whose arithmetic covers more of that wait (staged
// 2D batch of Nx 32768: +2 %; per-size Nx 16384: -5 %, mixed-size pulse batch
// -20 % when they took the lifting form as well).  The 3D kernels keep hi + lo.
struct alignas(16) PropLift {
    float p, uh, ul, c;
};
static_assert(sizeof(PropLift) == kPropEntryBytes, "table entry");
__device__ __forceinline__ PropLift tload_prop(const BufView &t, PropLift *, int lane_i, int uni_i)
{
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(t.r, lane_i * 16, t.base + uni_i * 16, 0);
    return {f_of(v.x), f_of(v.y), f_of(v.z), f_of(v.w)};
}
// the entry type of the staged tables (D3: the 3D envelopes' tables)
template <typename T, bool D3>
using StagedPropE = typename std::conditional<std::is_same<T, float>::value && !D3, PropLift, PropE<T>>::type;

__device__ __forceinline__ float tload_r(const BufView &t, float *, int lane_off, int uni_off)
{
    return f_of(__builtin_amdgcn_raw_buffer_load_b32(t.r, lane_off, t.base + uni_off, 0));
}
__device__ __forceinline__ double tload_r(const BufView &t, double *, int lane_off, int uni_off)
{
    const u2v v = __builtin_amdgcn_raw_buffer_load_b64(t.r, lane_off, t.base + uni_off, 0);
    return d_of(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ T tload_r(const BufView &t, int lane_i, int uni_i)
{
    return tload_r(t, (T *)nullptr, lane_i * (int)sizeof(T), uni_i * (int)sizeof(T));
}

// complex entry i of a table of Cx<T>, split as lane index + uniform index
template <typename T>
__device__ __forceinline__ Cx<T> tload_cx(const BufView &t, int lane_i, int uni_i)
{
    return tload_cx(t, (Cx<T> *)nullptr, lane_i * (int)sizeof(Cx<T>), uni_i * (int)sizeof(Cx<T>));
}
__device__ __forceinline__ void tstore_cx(const BufView &t, Cx<float> v, int lane_i, int uni_i)
{
    const u2v w = {__builtin_bit_cast(unsigned, v.x), __builtin_bit_cast(unsigned, v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(w, t.r, lane_i * 8, t.base + uni_i * 8, 0);
}
__device__ __forceinline__ void tstore_cx(const BufView &t, Cx<double> v, int lane_i, int uni_i)
{
    const u2v a = __builtin_bit_cast(u2v, v.x), b = __builtin_bit_cast(u2v, v.y);
    const u4v w = {a.x, a.y, b.x, b.y};
    __builtin_amdgcn_raw_buffer_store_b128(w, t.r, lane_i * 16, t.base + uni_i * 16, 0);
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

// tan(pi k / 64), k = 0..16
__host__ __device__ constexpr double qtan(int k)
{
    return k == 0 ? 0
         : k == 1 ? 0.049126849769467254
         : k == 2 ? 0.098491403357164248
         : k == 3 ? 0.14833598753834742
         : k == 4 ? 0.19891236737965801
         : k == 5 ? 0.25048696019130545
         : k == 6 ? 0.3033466836073424
         : k == 7 ? 0.35780572131452409
         : k == 8 ? 0.41421356237309503
         : k == 9 ? 0.47296477589131991
         : k == 10 ? 0.53451113595079158
         : k == 11 ? 0.59937693368192368
         : k == 12 ? 0.66817863791929888
         : k == 13 ? 0.74165054627203542
         : k == 14 ? 0.82067879082866024
         : k == 15 ? 0.90634716901914703
         : 1.0;
}

// ---- rotations
// FP32 rotations by a fixed angle phi are three lifting steps
//   x += p y;  y += u x;  x += p y      (p = -tan(phi/2), u = sin(phi)),
// with |phi| <= pi/2 after taking out an exact sign s = -1 for larger angles.
// The same steps with (-p, -u) undo them exactly, so every inverse transform is
// the exact inverse (in exact arithmetic) of its forward transform and the
// rounding of p and u cannot accumulate from step to step.
__device__ __forceinline__ Cx<float> lift(Cx<float> a, float p, float u)
{
    const float x1 = fmaT(p, a.y, a.x);
    const float y1 = fmaT(u, x1, a.y);
    return {fmaT(p, y1, x1), y1};
}

// Compile-time rotation by W^q, W = exp(-2 pi i / 64) (angle -2 pi q / 64).
template <int Q>
struct Rot64 {
    static constexpr int qq = (Q & 63) > 32 ? (Q & 63) - 64 : (Q & 63);          // (-32, 32]
    static constexpr int neg = (qq > 16 || qq < -16) ? 1 : 0;                     // exact -1 taken out
    static constexpr int qr = neg ? (qq > 0 ? qq - 32 : qq + 32) : qq;            // [-16, 16]
    // angle phi = -2 pi qr / 64; p = -tan(phi/2) = tan(pi qr / 64); u = sin(phi) = -sin(2 pi qr / 64)
    static_assert(qr >= -16 && qr <= 16, "folded angle outside the tan table");
    static constexpr double p = qr >= 0 ? qtan(qr) : -qtan(-qr);
    static constexpr double u = -sin64(qr);
};

// a * W^QE, forward constants
template <typename T, int QE>
__device__ __forceinline__ Cx<T> mul_w64(Cx<T> a)
{
    constexpr int q = QE & 63;
    if constexpr (q == 0) return a;
    else if constexpr (q == 16) return {a.y, -a.x};
    else if constexpr (q == 32) return {-a.x, -a.y};
    else if constexpr (q == 48) return {-a.y, a.x};
    else if constexpr (std::is_same<T, double>::value) {
        const double c = cos64(q), s = -sin64(q);
        return {fmaT(a.x, c, -a.y * s), fmaT(a.x, s, a.y * c)};
    } else {
        using R = Rot64<q>;
        const Cx<float> r = lift(a, (float)R::p, (float)R::u);
        if constexpr (R::neg) return {-r.x, -r.y};
        else return r;
    }
}

// exact inverse of mul_w64<T, QE> (FP64: multiply by the conjugate)
template <typename T, int QE>
__device__ __forceinline__ Cx<T> mul_w64_inv(Cx<T> a)
{
    constexpr int q = QE & 63;
    if constexpr (q == 0) return a;
    else if constexpr (q == 16) return {-a.y, a.x};
    else if constexpr (q == 32) return {-a.x, -a.y};
    else if constexpr (q == 48) return {a.y, -a.x};
    else if constexpr (std::is_same<T, double>::value) {
        const double c = cos64(q), s = sin64(q);
        return {fmaT(a.x, c, -a.y * s), fmaT(a.x, s, a.y * c)};
    } else {
        using R = Rot64<q>;
        const Cx<float> b = R::neg ? Cx<float>{-a.x, -a.y} : a;
        return lift(b, (float)-R::p, (float)-R::u);
    }
}

// In-register DFTs of size R in natural order.  Forward: exp(-2 pi i ms / R)
// as R = 4 Q (inner size-Q DFTs over m2, rotations W_R^{m1 s2}, outer DFT4s).
// Inverse: the same three stages undone in reverse order (outer, rotations,
// inner), i.e. R times the exact inverse of the forward; no 1/R.
template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T> *a)
{
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
}

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
            dft4<T, INV>(a);
        } else if constexpr (!INV) {
            // m = m1 + 4 m2, s = s2 + Q s1
            constexpr int Q = R / 4;
            Cx<T> y[4][Q];
            static_for<0, 4>([&](auto m1) {
                static_for<0, Q>([&](auto m2) { y[m1][m2] = a[m1 + 4 * m2]; });
                Dft<T, Q, false>::run(y[m1]);
            });
            static_for<1, 4>([&](auto m1) {
                static_for<1, Q>([&](auto s2) {
                    y[m1][s2] = mul_w64<T, (CV(m1) * CV(s2) * (64 / R)) & 63>(y[m1][s2]);
                });
            });
            static_for<0, Q>([&](auto s2) {
                Cx<T> z[4] = {y[0][s2], y[1][s2], y[2][s2], y[3][s2]};
                dft4<T, false>(z);
                static_for<0, 4>([&](auto s1) { a[s2 + Q * s1] = z[s1]; });
            });
        } else {
            constexpr int Q = R / 4;
            Cx<T> y[4][Q];
            static_for<0, Q>([&](auto s2) {
                Cx<T> z[4] = {a[s2], a[s2 + Q], a[s2 + 2 * Q], a[s2 + 3 * Q]};
                dft4<T, true>(z);
                static_for<0, 4>([&](auto m1) { y[m1][s2] = z[m1]; });
            });
            static_for<1, 4>([&](auto m1) {
                static_for<1, Q>([&](auto s2) {
                    y[m1][s2] = mul_w64_inv<T, (CV(m1) * CV(s2) * (64 / R)) & 63>(y[m1][s2]);
                });
            });
            static_for<0, 4>([&](auto m1) {
                Dft<T, Q, true>::run(y[m1]);
                static_for<0, Q>([&](auto m2) { a[m1 + 4 * m2] = y[m1][m2]; });
            });
        }
    }
};

// Forward DFT of FP32 samples that carry pending exact signs p = +-1 (a[k]
// stands for p[k] a[k]): the FP32 twiddles of a pass leave the sign they take
// out (Tw::s) pending instead of multiplying by it.  A sum or difference of
// two pending values, x px +- y py = px (x +- (px py) y), is one FMA per
// component with px passed on; rotations by fixed angles are linear and keep
// the sign.  Since p = +-1, every result is bitwise the one Dft<float, R,
// false> gives on the multiplied-out inputs; signs known to be +1 at compile
// time fold the FMAs back into additions.
__device__ __forceinline__ void sadd(Cx<float> x, float px, Cx<float> y, float py, Cx<float> &s, Cx<float> &d,
                                     float &ps)
{
    const float t = px * py;
    s = {fmaT(t, y.x, x.x), fmaT(t, y.y, x.y)};
    d = {fmaT(-t, y.x, x.x), fmaT(-t, y.y, x.y)};
    ps = px;
}
__device__ __forceinline__ void dft4_signed(Cx<float> *a, float *p)
{
    Cx<float> s0, d0, s1, d1;
    float q0, q1;
    sadd(a[0], p[0], a[2], p[2], s0, d0, q0);
    sadd(a[1], p[1], a[3], p[3], s1, d1, q1);
    const Cx<float> mid = {d1.y, -d1.x};  // -i * d1, pending q1
    float r0, r1;
    sadd(s0, q0, s1, q1, a[0], a[2], r0);
    sadd(d0, q0, mid, q1, a[1], a[3], r1);
    p[0] = p[2] = r0;
    p[1] = p[3] = r1;
}
template <int R>
struct DftSigned {
    static __device__ __forceinline__ void run(Cx<float> *a, float *p)
    {
        if constexpr (R == 1) {
        } else if constexpr (R == 2) {
            float r;
            sadd(a[0], p[0], a[1], p[1], a[0], a[1], r);
            p[0] = p[1] = r;
        } else if constexpr (R == 4) {
            dft4_signed(a, p);
        } else {
            // the same stages as Dft<float, R, false>: m = m1 + 4 m2, s = s2 + Q s1
            constexpr int Q = R / 4;
            Cx<float> y[4][Q];
            float yp[4][Q];
            static_for<0, 4>([&](auto m1) {
                static_for<0, Q>([&](auto m2) {
                    y[m1][m2] = a[m1 + 4 * m2];
                    yp[m1][m2] = p[m1 + 4 * m2];
                });
                DftSigned<Q>::run(y[m1], yp[m1]);
            });
            static_for<1, 4>([&](auto m1) {
                static_for<1, Q>([&](auto s2) {
                    y[m1][s2] = mul_w64<float, (CV(m1) * CV(s2) * (64 / R)) & 63>(y[m1][s2]);
                });
            });
            static_for<0, Q>([&](auto s2) {
                Cx<float> z[4] = {y[0][s2], y[1][s2], y[2][s2], y[3][s2]};
                float zp[4] = {yp[0][s2], yp[1][s2], yp[2][s2], yp[3][s2]};
                dft4_signed(z, zp);
                static_for<0, 4>([&](auto s1) {
                    a[s2 + Q * s1] = z[s1];
                    p[s2 + Q * s1] = zp[s1];
                });
            });
        }
    }
};

// ----------------------------------------------------------------- twiddles
template <typename T>
struct Tw;
// FP32: lifting constants of the reduced angle and the exact sign (+1 or -1)
template <>
struct Tw<float> {
    float p, u, s;
};
// bytes of one table entry
__host__ __device__ constexpr size_t tw_bytes(int prec) { return prec == PREC_F32 ? 12 : 16; }
// FP64: the rotation as a complex number
template <>
struct alignas(16) Tw<double> {
    double x, y;
};
static_assert(sizeof(Tw<float>) == tw_bytes(PREC_F32) && sizeof(Tw<double>) == tw_bytes(PREC_F64), "table entry");

__device__ __forceinline__ Cx<float> mul_tw(Cx<float> a, const Tw<float> &w)
{
    const Cx<float> r = lift(a, w.p, w.u);
    return {r.x * w.s, r.y * w.s};
}
// exact inverse of mul_tw
__device__ __forceinline__ Cx<float> mul_tw_inv(Cx<float> a, const Tw<float> &w)
{
    return lift({a.x * w.s, a.y * w.s}, -w.p, -w.u);
}
__device__ __forceinline__ Cx<double> mul_tw(Cx<double> a, const Tw<double> &w)
{
    return {fmaT(a.x, w.x, -a.y * w.y), fmaT(a.x, w.y, a.y * w.x)};
}
__device__ __forceinline__ Cx<double> mul_tw_inv(Cx<double> a, const Tw<double> &w)
{
    return {fmaT(a.x, w.x, a.y * w.y), fmaT(a.y, w.x, -a.x * w.y)};
}
// FP32 rotations whose angle never exceeds pi/2 (their table sign is +1)
__device__ __forceinline__ Cx<float> mul_tw_nosign(Cx<float> a, const Tw<float> &w) { return lift(a, w.p, w.u); }
__device__ __forceinline__ Cx<float> mul_tw_inv_nosign(Cx<float> a, const Tw<float> &w) { return lift(a, -w.p, -w.u); }
__device__ __forceinline__ Cx<double> mul_tw_nosign(Cx<double> a, const Tw<double> &w) { return mul_tw(a, w); }
__device__ __forceinline__ Cx<double> mul_tw_inv_nosign(Cx<double> a, const Tw<double> &w) { return mul_tw_inv(a, w); }

// twiddle entry lane_i + uni_i of a table (lane index per lane, uniform index per wave)
__device__ __forceinline__ Tw<float> tload_tw(const BufView &t, Tw<float> *, int lane_i, int uni_i)
{
    const u3v v = __builtin_amdgcn_raw_buffer_load_b96(t.r, lane_i * 12, t.base + uni_i * 12, 0);
    return {f_of(v.x), f_of(v.y), f_of(v.z)};
}
__device__ __forceinline__ Tw<double> tload_tw(const BufView &t, Tw<double> *, int lane_i, int uni_i)
{
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(t.r, lane_i * 16, t.base + uni_i * 16, 0);
    return {d_of(v.x, v.y), d_of(v.z, v.w)};
}
template <typename T>
__device__ __forceinline__ Tw<T> tload_tw(const BufView &t, int lane_i, int uni_i)
{
    return tload_tw(t, (Tw<T> *)nullptr, lane_i, uni_i);
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

// Work split of one solve: TH threads in G groups of LANES threads, E samples
// per thread and beam; thread (g, l) holds sample g + G*l + TH*e of each beam.
// The FFT of N = G*M points is an M-point Stockham FFT inside every group (over
// its decimated samples, exchanging through the group's own LDS region)
// followed, when G > 1, by one radix-G pass across the groups (the last
// Stockham pass: twiddles W_N^{b*g}, then DFT_G).  Groups are either single
// waves (G = TH/64; their exchanges need no workgroup barrier, only the
// cross-group pass does) or the whole workgroup (G = 1; every exchange is a
// workgroup barrier, double-buffered when LDS allows).
template <int LOG2N, int LOG2E, bool WAVE_GROUPS>
struct Geom {
    static constexpr int N = 1 << LOG2N, E = 1 << LOG2E;
    static constexpr int LOG2TH = LOG2N - LOG2E, TH = 1 << LOG2TH;
    static constexpr int LOG2G = (WAVE_GROUPS && LOG2TH > 6) ? LOG2TH - 6 : 0, G = 1 << LOG2G;
    static constexpr int LOG2LANES = LOG2TH - LOG2G, LANES = 1 << LOG2LANES;
    static constexpr int LOG2M = LOG2N - LOG2G, M = 1 << LOG2M;
    static constexpr bool WAVE_LOCAL = LANES <= 64;  // group exchanges stay inside one wave
    using SW = Sched<LOG2M, LOG2E>;  // group-local schedule (its TH is LANES)
    static_assert(SW::TH == LANES, "group-local schedule");
    static_assert(G <= E, "the cross-group pass needs radix G <= E");
    static constexpr int BUFM = SW::bufsz();       // padded region of one group
    static constexpr int TWFINAL = SW::twcount();  // table base of the cross-group pass
};

// Wave groups for the sizes whose workgroup spans 8 or more waves; below that
// the whole-workgroup FFT needs fewer passes.
__host__ __device__ constexpr bool use_wave_groups(int log2n, int log2e) { return log2n - log2e >= 9; }

// LDS: NBUF buffer sets (2 = alternate per exchange, whole-workgroup groups
// only), BX beams per set (2 = one buffer per beam, 1 = beams in turn).
template <typename T, int LOG2N, int LOG2E>
struct LdsPlan {
    static constexpr bool WG = use_wave_groups(LOG2N, LOG2E);
    using G = Geom<LOG2N, LOG2E, WG>;
    static constexpr size_t beam_bytes = (size_t)G::G * G::BUFM * sizeof(Cx<T>);
    static constexpr int NBUF = (!G::WAVE_LOCAL && 4 * beam_bytes <= kLdsMax) ? 2 : 1;
    static constexpr int BX = 2 * NBUF * beam_bytes <= kLdsMax ? 2 : 1;
    static constexpr size_t bytes = (size_t)NBUF * BX * beam_bytes;
    static constexpr bool fits = beam_bytes <= kLdsMax;
};

// ----------------------------------------------------------------- march
template <typename T>
__device__ __forceinline__ T to_T(double v) { return (T)v; }

// most mask intervals per z-step the kernels handle
constexpr int kMaxSeg = 4;

// Strain phase (revolutions) of a straight edge dislocation, line along y and b
// along h (Eq. (15)): (b/d)/(2 pi) * (atan2(Z, X) + X Z / (2 (1 - nu) r^2)),
// with X = x - x_d, Z = z - z_d formed in FP64 by the caller.  The phase is a
// few revolutions at most, so FP32 solves evaluate it in FP32; FP64 solves in FP64.
__device__ __forceinline__ float edge_phase_rev(float X, float Z, float k, float q)
{
    const float r2 = fmaT(X, X, Z * Z);
    const float a = atan2f(Z, X) + (r2 > 0.0f ? X * Z * q / r2 : 0.0f);
    return k * a;
}
__device__ __forceinline__ double edge_phase_rev(double X, double Z, double k, double q)
{
    const double r2 = __builtin_fma(X, X, Z * Z);
    const double a = atan2(Z, X) + (r2 > 0.0 ? X * Z * q / r2 : 0.0);
    return k * a;
}

// exp(i m atan2(Z, X)) for a whole winding number m (|m| <= 8) without the
// arctangent: ((X + i Z)/r)^m, by squaring, from ir = 1/r; 1 at the core itself
// (ir = 0).
template <typename T>
__device__ __forceinline__ Cx<T> winding_phasor(T X, T Z, T ir, int m)
{
    Cx<T> w = {(T)1, (T)0};
    if (ir > (T)0) w = {X * ir, Z * ir};
    if (m < 0) w.y = -w.y;
    int k = m < 0 ? -m : m;
    Cx<T> p = {(T)1, (T)0};
    while (k) {
        if (k & 1) p = {fmaT(p.x, w.x, -p.y * w.y), fmaT(p.x, w.y, p.y * w.x)};
        w = {fmaT(w.x, w.x, -w.y * w.y), (T)2 * w.x * w.y};
        k >>= 1;
    }
    return p;
}

// 1/x to about one ulp: the hardware reciprocal in FP32, a division in FP64
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }

// v^k for k >= 1, the same k across the wave: factors of two by squaring
// first, so small powers cost only their squarings
template <typename T>
__device__ __forceinline__ Cx<T> cpow_pos(Cx<T> v, int k)
{
    while (!(k & 1)) {
        v = {fmaT(v.x, v.x, -v.y * v.y), (T)2 * v.x * v.y};
        k >>= 1;
    }
    Cx<T> p = v;
    k >>= 1;
    while (k) {
        v = {fmaT(v.x, v.x, -v.y * v.y), (T)2 * v.x * v.y};
        if (k & 1) p = {fmaT(p.x, v.x, -p.y * v.y), fmaT(p.x, v.y, p.y * v.x)};
        k >>= 1;
    }
    return p;
}

__device__ __forceinline__ void sincospi_T(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_T(double x, double *s, double *c) { sincospi(x, s, c); }

// exp(2 pi i v) for a phase v in revolutions: reduced to [-1/2, 1/2] in the
// precision of v (FP64 for large arguments), then evaluated in T.
template <typename T, typename V>
__device__ __forceinline__ Cx<T> phasor(V v)
{
    const V fr = v - rint(v);
    T sn, cs;
    sincospi_T((T)(fr + fr), &sn, &cs);
    return {cs, sn};
}
// the same with the hardware sine and cosine in FP32, which take revolutions
// (measured on MI355X against FP64 over [-1, 1] revolutions: |error| <=
// 1.3e-7, no bias, ||P| - 1| <= 1.3e-7): two instructions instead of a
// full-range library sincos
template <typename T, typename V>
__device__ __forceinline__ Cx<T> phasor_hw(V v)
{
    if constexpr (std::is_same<T, float>::value) {
        const float f = (float)(v - rint(v));
        return {__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f)};
    } else {
        return phasor<T>(v);
    }
}

// a/N + k a for a propagator table entry k = (P - 1)/N.  The two terms of
// k a are summed first and a/N (exact: N is a power of two) is added last, so
// the one rounding against the large value sees the whole increment.  Added
// one at a time, a second-order term below half an ulp (the -theta^2/2 that
// keeps |P| = 1 for a small phase theta per step) would be dropped at every
// step and the power of slowly turning bins would grow by theta^2 per step.
// FP32: the lo products innermost, so every rounding sees k to about 2^-48.
__device__ __forceinline__ Cx<float> prop_mul(Cx<float> a, const PropE<float> &k, float invN)
{
    return {fmaT(a.x, invN, fmaT(k.hx, a.x, fmaT(-k.hy, a.y, fmaT(k.lx, a.x, -k.ly * a.y)))),
            fmaT(a.y, invN, fmaT(k.hx, a.y, fmaT(k.hy, a.x, fmaT(k.lx, a.y, k.ly * a.x))))};
}
__device__ __forceinline__ Cx<double> prop_mul(Cx<double> a, const PropE<double> &k, double invN)
{
    return {fmaT(a.x, invN, fmaT(k.x, a.x, -k.y * a.y)), fmaT(a.y, invN, fmaT(k.x, a.y, k.y * a.x))};
}
// P a / N from a lifting entry: three shears x += p y, y += u x, x += p y (the
// middle increment summed from its hi and lo products before it meets y, so it
// sees u to about 2^-48; each shear adds its whole increment in one rounding),
// then the scale c (exact outside the evanescent bins)
__device__ __forceinline__ Cx<float> prop_mul(Cx<float> a, const PropLift &k, float)
{
    const float x1 = fmaT(k.p, a.y, a.x);
    const float y1 = a.y + fmaT(k.uh, x1, k.ul * x1);
    const float x2 = fmaT(k.p, y1, x1);
    return {k.c * x2, k.c * y1};
}

// psi+ <- psi+ + m (d0 psi+ + bp psi-),  psi- <- psi- + m (d0 psi- + bm psi+)
// (Eq. (12)) with m = 1 where the sample is inside the crystal and m = 0
// outside, where both envelopes keep their propagated values (pure
// propagation).  The increments are summed before the envelope itself is
// added, for the same reason as in prop_mul; m weights them in that last
// fused operation, so for m = 1 the result is the sum rounded once and for
// m = 0 the envelope itself.  The coefficients are finite by construction
// (plan creation bounds the coupling step), so 0 x increment is 0.
template <typename T>
__device__ __forceinline__ void couple(Cx<T> &vp, Cx<T> &vm, T m, Cx<T> d0, Cx<T> bp, Cx<T> bm)
{
    const Cx<T> a = vp, b = vm;
    const Cx<T> ip = {fmaT(bp.x, b.x, fmaT(-bp.y, b.y, fmaT(d0.x, a.x, -d0.y * a.y))),
                      fmaT(bp.x, b.y, fmaT(bp.y, b.x, fmaT(d0.x, a.y, d0.y * a.x)))};
    const Cx<T> im = {fmaT(bm.x, a.x, fmaT(-bm.y, a.y, fmaT(d0.x, b.x, -d0.y * b.y))),
                      fmaT(bm.x, a.y, fmaT(bm.y, a.x, fmaT(d0.x, b.y, d0.y * b.x)))};
    vp.x = fmaT(ip.x, m, vp.x);
    vp.y = fmaT(ip.y, m, vp.y);
    vm.x = fmaT(im.x, m, vm.x);
    vm.y = fmaT(im.y, m, vm.y);
}

// a value the whole wave holds, moved to scalar registers
__device__ __forceinline__ float wave_uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const u2v h = __builtin_bit_cast(u2v, v);
    return d_of((unsigned)__builtin_amdgcn_readfirstlane((int)h.x), (unsigned)__builtin_amdgcn_readfirstlane((int)h.y));
}

// Orders this wave's LDS writes before its following LDS reads (LDS executes a
// wave's instructions in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Real-space coupling of one z-step or sub-step (Eq. (9)-(13)) for the E samples
// a thread holds at j0 + JS*e.  Outside the crystal the step is pure propagation:
// those samples keep their propagated values.  SC_POLY1 (no X^2 term) has a
// phase whose second difference along a thread's samples is zero: its phasor
// steps leave out that factor, which is then exactly one.
template <typename T, int SC>
struct Coupler {
    static constexpr bool POLY = SC == SC_POLY2 || SC == SC_POLY1, LIN = SC == SC_POLY1;
    double X0;       // x0 - x_ref
    int nseg, nx;
    gptr<int> seg;
    Cx<T> rr;        // polynomial strain: phasor of the phase's second difference along a thread's samples

    // JS: sample stride between a thread's elements
    template <int JS>
    __device__ __forceinline__ void init(const SolveDesc &d, int nx_)
    {
        X0 = d.x0 - d.x_ref;
        nseg = d.nseg;
        nx = nx_;
        seg = to_global<int>(d.seg);
        if constexpr (POLY) {
            // the second difference 2 pc D^2 (D = JS dx) does not depend on z
            const double D = (double)JS * d.dx;
            const Cx<T> r = phasor_hw<T>(2.0 * (d.c[3] * d.inv_d) * D * D);
            rr = {wave_uniform(r.x), wave_uniform(r.y)};
        }
    }

    // coupling sub-step ss of z-step n (its coefficients, mask row n, strain
    // at z_n + ss.zoff dz)
    template <int E, int JS>
    __device__ __forceinline__ void apply(Cx<T> *vp, Cx<T> *vm, const SolveDesc &d, int n, int j0,
                                          const SubStep &ss) const
    {
        const Cx<T> d0 = {to_T<T>(ss.d0x), to_T<T>(ss.d0y)};
        const Cx<T> ap = {to_T<T>(ss.apx), to_T<T>(ss.apy)};
        const Cx<T> am = {to_T<T>(ss.amx), to_T<T>(ss.amy)};
        static_assert(E <= 32 && (JS & (JS - 1)) == 0, "element mask");
        constexpr int LOG2JS = __builtin_ctz(JS);
        // bit e of `inside` <=> sample j0 + JS*e lies in one of the step's
        // intervals [lo, hi): the inside elements of an interval are the
        // consecutive range ceil((lo - j0)/JS) <= e < ceil((hi - j0)/JS)
        const gptr<int> sg = seg + (size_t)n * nseg * 2;
        uint32_t inside = 0;
        static_for<0, kMaxSeg>([&](auto k) {
            if (CV(k) < nseg) {
                const int lo = sg[2 * CV(k)], hi = sg[2 * CV(k) + 1];
                const int elo = min(max((lo - j0 + JS - 1) >> LOG2JS, 0), E);
                const int ehi = min(max((hi - j0 + JS - 1) >> LOG2JS, 0), E);
                const uint32_t below_hi = ehi >= 32 ? 0xffffffffu : (1u << ehi) - 1u;
                const uint32_t below_lo = elo >= 32 ? 0xffffffffu : (1u << elo) - 1u;
                inside |= below_hi & ~below_lo;
            }
        });
        // the weight m of element e: 1 inside the crystal, 0 outside
        auto inside_at_e = [&](auto e) { return (T)((inside >> CV(e)) & 1u); };
        const double Z = (n + ss.zoff) * d.dz - d.z_ref;
        // (one straight-line copy: a wave-uniform branch to a copy without the
        // selects for all-inside waves keeps both copies' values live and spills)
        if constexpr (SC == SC_NONE) {
            static_for<0, E>([&](auto e) { couple(vp[e], vm[e], inside_at_e(e), d0, ap, am); });
        } else if constexpr (POLY) {
            // phase (revolutions) u/d = pa + pb X + pc X^2 along this z; along a
            // thread's samples X_e = X_0 + e D it is quadratic in e: with
            // P_e = exp(2 pi i u_e/d), P_{e+1} = P_e Q_e and Q_{e+1} = Q_e R, so the
            // coefficients bp_e = ap P_e and bm_e = am conj(P_e) advance by Q_e and
            // conj(Q_e); P_0, Q_0 and R from FP64 arguments reduced to one revolution.
            const double pa = (d.c[0] + Z * (d.c[2] + Z * d.c[5])) * d.inv_d;
            const double pb = (d.c[1] + Z * d.c[4]) * d.inv_d;
            const double pc = d.c[3] * d.inv_d;
            const double D = (double)JS * d.dx;
            const double Xt = __builtin_fma((double)j0, d.dx, X0);
            const Cx<T> P = phasor_hw<T>(__builtin_fma(__builtin_fma(pc, Xt, pb), Xt, pa));
            Cx<T> Q = phasor_hw<T>(__builtin_fma(pc, __builtin_fma(2.0 * Xt, D, D * D), pb * D));
            Cx<T> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
            Cx<T> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
            static_for<0, E>([&](auto e) {
                couple(vp[e], vm[e], inside_at_e(e), d0, bp, bm);
                if constexpr (CV(e) + 1 < E) {
                    bp = {fmaT(bp.x, Q.x, -bp.y * Q.y), fmaT(bp.x, Q.y, bp.y * Q.x)};
                    bm = {fmaT(bm.x, Q.x, bm.y * Q.y), fmaT(bm.y, Q.x, -bm.x * Q.y)};
                }
                if constexpr (CV(e) + 2 < E && !LIN)
                    Q = {fmaT(Q.x, rr.x, -Q.y * rr.y), fmaT(Q.x, rr.y, Q.y * rr.x)};
            });
        } else {
            // dislocation field or tabulated phase (already reduced to one
            // revolution when the plan was built)
            const bool edge = d.strain_kind == STRAIN_EDGE;
            const T dk = (T)d.disl_k, dq = (T)d.disl_q;
            // table [nz][nx]: row n, sample j0 + JS e
            const BufView utv = buf_view(d.utab, edge ? 0u : (uint32_t)d.nz * nx * (uint32_t)sizeof(T));
            const int m = d.disl_m;
            if constexpr (std::is_same<T, float>::value) {
                if (edge && m != 0 && (m & 1) == 0) {
                    // even whole winding (b = m d with m even; 0.38 nm at d = 0.95 A
                    // is m = 4): with v = (X + iZ)^2 / r^2 = (cos 2t, sin 2t),
                    // t = atan2(Z, X), exp(i h u) = v^(m/2) exp(2 pi i k q Im(v) / 2),
                    // because X Z / r^2 = sin(2t) / 2.  One reciprocal per sample,
                    // no square root, division or arctangent.
                    const int half = m < 0 ? -m / 2 : m / 2;
                    const float Zt = (float)Z, Z2 = Zt * Zt, Zx2 = Zt + Zt;
                    const float kqh = (float)(0.5 * d.disl_k * d.disl_q);
                    static_for<0, E>([&](auto e) {
                        const int j = j0 + e * JS;
                        const T in = inside_at_e(e);
                        const float X = (float)__builtin_fma((double)j, d.dx, X0);
                        const float r2 = fmaT(X, X, Z2);
                        const bool core = !(r2 > 0.0f);   // the core itself: phase 0
                        const float ir2 = core ? 0.0f : rcp_fast(r2);
                        const Cx<float> v = {core ? 1.0f : fmaT(X, X, -Z2) * ir2, (X * Zx2) * ir2};
                        Cx<float> W = cpow_pos(v, half);
                        if (m < 0) W.y = -W.y;
                        // |k q Im(v) / 2| <= |k q| / 2, under a revolution: the
                        // hardware sine and cosine (they take revolutions), no reduction
                        const float arg = kqh * v.y;
                        const Cx<float> S = {__builtin_amdgcn_cosf(arg), __builtin_amdgcn_sinf(arg)};
                        const Cx<float> P = {fmaT(W.x, S.x, -W.y * S.y), fmaT(W.x, S.y, W.y * S.x)};
                        const Cx<float> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
                        const Cx<float> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
                        couple(vp[e], vm[e], in, d0, bp, bm);
                    });
                    return;
                }
            }
            if (edge && m != 0) {
                // whole winding number: exp(i h u) = ((X + i Z)/r)^m exp(2 pi i k q X Z / r^2)
                static_for<0, E>([&](auto e) {
                    const int j = j0 + e * JS;
                    const T in = inside_at_e(e);
                    const T X = (T)__builtin_fma((double)j, d.dx, X0), Zt = (T)Z;
                    const T r2 = fmaT(X, X, Zt * Zt);
                    const T ir = r2 > (T)0 ? (T)1 / sqrt(r2) : (T)0;
                    const Cx<T> W = winding_phasor<T>(X, Zt, ir, m);
                    const Cx<T> S = phasor<T>(r2 > (T)0 ? dk * (X * Zt * dq / r2) : (T)0);
                    const Cx<T> P = {fmaT(W.x, S.x, -W.y * S.y), fmaT(W.x, S.y, W.y * S.x)};
                    const Cx<T> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
                    const Cx<T> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
                    couple(vp[e], vm[e], in, d0, bp, bm);
                });
                return;
            }
            static_for<0, E>([&](auto e) {
                const int j = j0 + e * JS;
                const T in = inside_at_e(e);
                const T rev = edge ? edge_phase_rev((T)__builtin_fma((double)j, d.dx, X0), (T)Z, dk, dq)
                                   : tload_r<T>(utv, j0, n * nx + CV(e) * JS);
                const Cx<T> P = phasor<T>(rev);
                const Cx<T> bp = {fmaT(ap.x, P.x, -ap.y * P.y), fmaT(ap.x, P.y, ap.y * P.x)};
                const Cx<T> bm = {fmaT(am.x, P.x, am.y * P.y), fmaT(am.y, P.x, -am.x * P.y)};
                couple(vp[e], vm[e], in, d0, bp, bm);
            });
        }
    }

    // 3D envelopes [NY][nx]: the E samples a thread holds are the rows y0 + YS*e
    // of column x; the mask is read per row, analytic strain does not depend on y
    template <int E, int YS, int NY>
    __device__ __forceinline__ void apply3d(Cx<T> *vp, Cx<T> *vm, const SolveDesc &d, int n, int x, int y0,
                                            const SubStep &ss) const
    {
        const Cx<T> d0 = {to_T<T>(ss.d0x), to_T<T>(ss.d0y)};
        const Cx<T> ap = {to_T<T>(ss.apx), to_T<T>(ss.apy)};
        const Cx<T> am = {to_T<T>(ss.amx), to_T<T>(ss.amy)};
        const double Z = (n + ss.zoff) * d.dz - d.z_ref;
        const double Xd = __builtin_fma((double)x, d.dx, X0);
        Cx<T> P = {(T)1, (T)0};
        if constexpr (POLY) {
            const double pa = (d.c[0] + Z * (d.c[2] + Z * d.c[5])) * d.inv_d;
            const double pb = (d.c[1] + Z * d.c[4]) * d.inv_d;
            const double pc = d.c[3] * d.inv_d;
            P = phasor<T>(__builtin_fma(__builtin_fma(pc, Xd, pb), Xd, pa));
        } else if constexpr (SC == SC_GENERAL) {
            if (d.strain_kind == STRAIN_EDGE) {
                const T X = (T)Xd, Zt = (T)Z, dk = (T)d.disl_k, dq = (T)d.disl_q;
                if (d.disl_m != 0) {
                    const T r2 = fmaT(X, X, Zt * Zt);
                    const T ir = r2 > (T)0 ? (T)1 / sqrt(r2) : (T)0;
                    const Cx<T> W = winding_phasor<T>(X, Zt, ir, d.disl_m);
                    const Cx<T> S = phasor<T>(r2 > (T)0 ? dk * (X * Zt * dq / r2) : (T)0);
                    P = {fmaT(W.x, S.x, -W.y * S.y), fmaT(W.x, S.y, W.y * S.x)};
                } else {
                    P = phasor<T>(edge_phase_rev(X, Zt, dk, dq));
                }
            }
        }
        const bool table = SC == SC_GENERAL && d.strain_kind == STRAIN_TABLE;
        // strain table [nz][NY][nx]: row n*NY + y0 + YS*e, column x
        const BufView utv = buf_view(d.utab, table ? (uint32_t)d.nz * NY * nx * (uint32_t)sizeof(T) : 0u);
        // mask rows [nz][NY][nseg] of (lo, hi) pairs: row n*NY + y0 + YS*e
        const BufView sgv = buf_view(d.seg, (uint32_t)d.nz * NY * nseg * 8u);
        const int lane_off = y0 * nseg * 8;
        static_for<0, E>([&](auto e) {
            const int uni_off = (n * NY + YS * CV(e)) * nseg * 8;
            bool in = false;
            static_for<0, kMaxSeg>([&](auto k) {
                if (CV(k) < nseg) {
                    const u2v iv = __builtin_amdgcn_raw_buffer_load_b64(sgv.r, lane_off, sgv.base + uni_off + 8 * CV(k), 0);
                    in |= (x >= (int)iv.x) & (x < (int)iv.y);
                }
            });
            const Cx<T> Pe = table ? phasor<T>(tload_r<T>(utv, y0 * nx + x, (n * NY + YS * CV(e)) * nx)) : P;
            const Cx<T> bp = {fmaT(ap.x, Pe.x, -ap.y * Pe.y), fmaT(ap.x, Pe.y, ap.y * Pe.x)};
            const Cx<T> bm = {fmaT(am.x, Pe.x, am.y * Pe.y), fmaT(am.y, Pe.x, -am.x * Pe.y)};
            couple(vp[e], vm[e], in ? (T)1 : (T)0, d0, bp, bm);
        });
    }
};

// propagator-table samples in flight ahead of the one a resident march multiplies
constexpr int kPropAhead = 5;

// One solve marched by the first TH of BLOCK threads (the rest only take part
// in the workgroup barriers).
// BXO overrides the LDS plan's beams-per-buffer choice (0 = the plan's).
template <typename T, int LOG2N, int LOG2E, int SC, int BLOCK = (1 << (LOG2N - LOG2E)), int BXO = 0>
struct March {
    using LP = LdsPlan<T, LOG2N, LOG2E>;
    using G = typename LP::G;
    using SW = typename G::SW;
    static constexpr int N = G::N, E = G::E, TH = G::TH, W = G::G, LANES = G::LANES, M = G::M;
    static constexpr int PW = SW::P, BUFM = G::BUFM;
    static constexpr int NB = LP::NBUF, BX = BXO ? BXO : LP::BX;
    // twiddle entries: the group-local passes, then the cross-group pass (radix W, sub-length M)
    static constexpr int TW_ENTRIES = G::TWFINAL + (W > 1 ? M * (W - 1) : 0);
    static_assert(G::WAVE_LOCAL || W == 1, "whole-workgroup groups");
    static_assert(BLOCK >= TH, "block");

    // ---- one Stockham pass over a set of threads: radix 2^LR, sub-length 2^LL,
    // EE samples per thread, THR threads (thread tid), twiddles at tw[twb + ...]
    template <int LR, int LL, int THR>
    static __device__ __forceinline__ void pass_fwd(Cx<T> *vp, Cx<T> *vm, const BufView &tw, int twb, int tid)
    {
        constexpr int L = 1 << LL;
        auto twf = [&](auto, auto m, int j) { return tload_tw<T>(tw, j, twb + (CV(m) - 1) * L); };
        pass_fwd_f<LR, LL, THR>(vp, vm, twf, tid);
    }
    template <int LR, int LL, int THR>
    static __device__ __forceinline__ void pass_inv(Cx<T> *vp, Cx<T> *vm, const BufView &tw, int twb, int tid)
    {
        constexpr int L = 1 << LL;
        auto twf = [&](auto, auto m, int j) { return tload_tw<T>(tw, j, twb + (CV(m) - 1) * L); };
        pass_inv_f<LR, LL, THR>(vp, vm, twf, tid);
    }
    // the same with the twiddle of element m of group i (at position j of the
    // sub-length) from tw(i, m, j)
    template <int LR, int LL, int THR, typename F>
    static __device__ __forceinline__ void pass_fwd_f(Cx<T> *vp, Cx<T> *vm, const F &twf, int tid)
    {
        constexpr int r = 1 << LR, EPR = E / r, L = 1 << LL;
        static_for<0, EPR>([&](auto i) {
            Cx<T> ap[r], am[r];
            static_for<0, r>([&](auto m) {
                ap[m] = vp[i + m * EPR];
                am[m] = vm[i + m * EPR];
            });
            if constexpr (std::is_same<T, float>::value && L > 1) {
                // the exact signs of the twiddles stay pending into the DFT
                float sp[r], sm[r];
                const int j = (tid + i * THR) & (L - 1);
                sp[0] = sm[0] = 1.0f;
                static_for<1, r>([&](auto m) {
                    const Tw<T> w = twf(i, m, j);
                    ap[m] = lift(ap[m], w.p, w.u);
                    am[m] = lift(am[m], w.p, w.u);
                    // angle 2 pi j m / (L r) < pi/2 for m <= r/4: no sign taken out
                    sp[m] = sm[m] = 4 * CV(m) <= r ? 1.0f : w.s;
                });
                DftSigned<r>::run(ap, sp);
                DftSigned<r>::run(am, sm);
                static_for<0, r>([&](auto q) {
                    ap[q] = {ap[q].x * sp[q], ap[q].y * sp[q]};   // +1 here: no instruction
                    am[q] = {am[q].x * sm[q], am[q].y * sm[q]};
                });
            } else {
                if constexpr (L > 1) {
                    const int j = (tid + i * THR) & (L - 1);
                    static_for<1, r>([&](auto m) {
                        const Tw<T> w = twf(i, m, j);
                        // angle 2 pi j m / (L r) < pi/2 for m <= r/4: no sign taken out
                        if constexpr (4 * CV(m) <= r) {
                            ap[m] = mul_tw_nosign(ap[m], w);
                            am[m] = mul_tw_nosign(am[m], w);
                        } else {
                            ap[m] = mul_tw(ap[m], w);
                            am[m] = mul_tw(am[m], w);
                        }
                    });
                }
                Dft<T, r, false>::run(ap);
                Dft<T, r, false>::run(am);
            }
            static_for<0, r>([&](auto q) {
                vp[i + q * EPR] = ap[q];
                vm[i + q * EPR] = am[q];
            });
        });
    }
    template <int LR, int LL, int THR, typename F>
    static __device__ __forceinline__ void pass_inv_f(Cx<T> *vp, Cx<T> *vm, const F &twf, int tid)
    {
        constexpr int r = 1 << LR, EPR = E / r, L = 1 << LL;
        static_for<0, EPR>([&](auto i) {
            Cx<T> ap[r], am[r];
            static_for<0, r>([&](auto q) {
                ap[q] = vp[i + q * EPR];
                am[q] = vm[i + q * EPR];
            });
            Dft<T, r, true>::run(ap);
            Dft<T, r, true>::run(am);
            if constexpr (L > 1) {
                const int j = (tid + i * THR) & (L - 1);
                static_for<1, r>([&](auto m) {
                    const Tw<T> w = twf(i, m, j);
                    if constexpr (4 * CV(m) <= r) {
                        ap[m] = mul_tw_inv_nosign(ap[m], w);
                        am[m] = mul_tw_inv_nosign(am[m], w);
                    } else {
                        ap[m] = mul_tw_inv(ap[m], w);
                        am[m] = mul_tw_inv(am[m], w);
                    }
                });
            }
            static_for<0, r>([&](auto m) {
                vp[i + m * EPR] = ap[m];
                vm[i + m * EPR] = am[m];
            });
        });
    }

    // ---- wave-local exchanges (inside one wave's region; no workgroup barrier).
    // Scattered positions of wave-local pass p: butterfly b = l + i*LANES puts
    // output s at j + s*L + k*L*r (j = b mod L, k = b / L); with one pad slot per
    // L*r elements that is (j + k*(L*r + 1)) + s*L.
    template <int p>
    static __device__ __forceinline__ int scatter_base(int b)
    {
        constexpr int lr = SW::log2r(p), ll = SW::log2L(p), L = 1 << ll;
        const int j = b & (L - 1), k = b >> ll;
        if constexpr (SW::padsh(p) >= 0) return j + k * ((1 << (ll + lr)) + 1);
        else return j + (k << (ll + lr));
    }
    template <int p>
    static __device__ __forceinline__ void scatter_write(Cx<T> *R0, const Cx<T> *v, int l)
    {
        constexpr int r = 1 << SW::log2r(p), EPR = E / r, L = 1 << SW::log2L(p);
        static_for<0, EPR>([&](auto i) {
            Cx<T> *base = R0 + scatter_base<p>(l + i * LANES);
            static_for<0, r>([&](auto q) { base[q * L] = v[i + q * EPR]; });
        });
    }
    template <int p>
    static __device__ __forceinline__ void scatter_read(const Cx<T> *R0, Cx<T> *v, int l)
    {
        constexpr int r = 1 << SW::log2r(p), EPR = E / r, L = 1 << SW::log2L(p);
        static_for<0, EPR>([&](auto i) {
            const Cx<T> *base = R0 + scatter_base<p>(l + i * LANES);
            static_for<0, r>([&](auto q) { v[i + q * EPR] = base[q * L]; });
        });
    }
    // column positions l + e*LANES, padded as (l + l>>sh) + e*(LANES + LANES>>sh)
    template <int p>
    static __device__ __forceinline__ void column_write(Cx<T> *R0, const Cx<T> *v, int l)
    {
        constexpr int sh = SW::padsh(p);
        if constexpr (sh < 0) {
            static_for<0, E>([&](auto e) { R0[l + e * LANES] = v[e]; });
        } else if constexpr ((LANES >> sh) << sh == LANES) {
            Cx<T> *base = R0 + l + (l >> sh);
            static_for<0, E>([&](auto e) { base[e * (LANES + (LANES >> sh))] = v[e]; });
        } else {
            static_for<0, E>([&](auto e) { R0[padpos<SW, p>(l + e * LANES)] = v[e]; });
        }
    }
    template <int p>
    static __device__ __forceinline__ void column_read(const Cx<T> *R0, Cx<T> *v, int l)
    {
        constexpr int sh = SW::padsh(p);
        if constexpr (sh < 0) {
            static_for<0, E>([&](auto e) { v[e] = R0[l + e * LANES]; });
        } else if constexpr ((LANES >> sh) << sh == LANES) {
            const Cx<T> *base = R0 + l + (l >> sh);
            static_for<0, E>([&](auto e) { v[e] = base[e * (LANES + (LANES >> sh))]; });
        } else {
            static_for<0, E>([&](auto e) { v[e] = R0[padpos<SW, p>(l + e * LANES)]; });
        }
    }

    // ---- cross-wave transposes: wave w's region holds its M sub-transform
    // outputs at index k1 = l + LANES*e; the radix-W pass of butterfly
    // b = t + i*TH reads index b of every region.
    static __device__ __forceinline__ void write_own(Cx<T> *R0, const Cx<T> *v, int l)
    {
        static_for<0, E>([&](auto e) { R0[l + e * LANES] = v[e]; });
    }
    static __device__ __forceinline__ void read_own(const Cx<T> *R0, Cx<T> *v, int l)
    {
        static_for<0, E>([&](auto e) { v[e] = R0[l + e * LANES]; });
    }
    static __device__ __forceinline__ void read_all(const Cx<T> *B0, Cx<T> *v, int t)
    {
        constexpr int EPR = E / W;
        static_for<0, EPR>([&](auto i) {
            static_for<0, W>([&](auto m) { v[i + m * EPR] = B0[m * BUFM + t + i * TH]; });
        });
    }
    static __device__ __forceinline__ void write_all(Cx<T> *B0, const Cx<T> *v, int t)
    {
        constexpr int EPR = E / W;
        static_for<0, EPR>([&](auto i) {
            static_for<0, W>([&](auto m) { B0[m * BUFM + t + i * TH] = v[i + m * EPR]; });
        });
    }

    // Group-local exchange after forward pass p (slot p) or before inverse pass
    // p (slot 2*PW - 3 - p): forward writes scattered and reads columns, the
    // inverse the other way round.  Wave groups order their own LDS accesses;
    // whole-workgroup groups synchronise with barriers (one per exchange when
    // two buffer sets alternate, else one before the writes as well).
    template <int p, bool INVDIR>
    static __device__ __forceinline__ void gx(Cx<T> *vp, Cx<T> *vm, Cx<T> *Rp0, Cx<T> *Rm0, int l, bool active)
    {
        constexpr int slot = INVDIR ? 2 * PW - 3 - p : p;
        constexpr int off = (slot % NB) * BX * W * BUFM;
        Cx<T> *Rp = Rp0 + off;
        Cx<T> *Rm = Rm0 + off;
        auto put = [&](Cx<T> *R, const Cx<T> *v) {
            if constexpr (!INVDIR) scatter_write<p>(R, v, l);
            else column_write<p>(R, v, l);
        };
        auto get = [&](const Cx<T> *R, Cx<T> *v) {
            if constexpr (!INVDIR) column_read<p>(R, v, l);
            else scatter_read<p>(R, v, l);
        };
        if constexpr (G::WAVE_LOCAL) {
            if (active) {
                if constexpr (BX == 2) {
                    put(Rp, vp);
                    put(Rm, vm);
                    wave_lds_sync();
                    get(Rp, vp);
                    get(Rm, vm);
                } else {
                    put(Rp, vp);
                    wave_lds_sync();
                    get(Rp, vp);
                    wave_lds_sync();
                    put(Rp, vm);
                    wave_lds_sync();
                    get(Rp, vm);
                    wave_lds_sync();
                }
            }
        } else if constexpr (BX == 2) {
            if constexpr (NB == 1) __syncthreads();
            if (active) {
                put(Rp, vp);
                put(Rm, vm);
            }
            __syncthreads();
            if (active) {
                get(Rp, vp);
                get(Rm, vm);
            }
        } else {
            __syncthreads();
            if (active) put(Rp, vp);
            __syncthreads();
            if (active) get(Rp, vp);
            __syncthreads();
            if (active) put(Rp, vm);
            __syncthreads();
            if (active) get(Rp, vm);
        }
    }

    // The cross-group pass's twiddles of thread t (element m of group i at
    // index i*(W-1) + m-1).
    static __device__ __forceinline__ void load_cross_tw(Tw<T> *w, const BufView &tw, int t)
    {
        constexpr int r = W, EPR = E / r, L = M;
        static_for<0, EPR>([&](auto i) {
            const int j = (t + CV(i) * TH) & (L - 1);
            static_for<1, r>([&](auto m) {
                w[CV(i) * (r - 1) + CV(m) - 1] = tload_tw<T>(tw, j, G::TWFINAL + (CV(m) - 1) * L);
            });
        });
    }
    static __device__ __forceinline__ auto cross_tw_f(const Tw<T> *w)
    {
        return [w](auto i, auto m, int) { return w[CV(i) * (W - 1) + CV(m) - 1]; };
    }

    // Group-local forward FFT of M points (radix-E Stockham passes with the
    // group's exchanges through its LDS region Rp/Rm); natural-order samples
    // l + LANES*e in, bins l + LANES*e out.
    static __device__ __forceinline__ void fwd_local(Cx<T> *vp, Cx<T> *vm, const BufView &tw, Cx<T> *Rp, Cx<T> *Rm,
                                                     int l, bool active)
    {
        static_for<0, PW>([&](auto pc) {
            constexpr int p = CV(pc);
            if (active) pass_fwd<SW::log2r(p), SW::log2L(p), LANES>(vp, vm, tw, SW::twbase(p), l);
            if constexpr (p + 1 < PW) gx<p, false>(vp, vm, Rp, Rm, l, active);
        });
    }
    // its exact inverse: the same passes in reverse order with the same tables
    static __device__ __forceinline__ void inv_local(Cx<T> *vp, Cx<T> *vm, const BufView &tw, Cx<T> *Rp, Cx<T> *Rm,
                                                     int l, bool active)
    {
        static_for<0, PW>([&](auto pp) {
            constexpr int p = PW - 1 - CV(pp);
            if constexpr (p + 1 < PW) gx<p, true>(vp, vm, Rp, Rm, l, active);
            if (active) pass_inv<SW::log2r(p), SW::log2L(p), LANES>(vp, vm, tw, SW::twbase(p), l);
        });
    }

    // ---- the group-local passes' twiddles of one lane, held in registers: they
    // depend only on the lane's position (element m of group i of pass p at
    // position j = (l + i LANES) mod L), so a kernel that runs many transforms
    // per lane loads them once instead of after every LDS exchange
    static constexpr int cache_off(int p)
    {
        int o = 0;
        for (int q = 0; q < p; ++q)
            if (SW::log2L(q) > 0) o += (E >> SW::log2r(q)) * ((1 << SW::log2r(q)) - 1);
        return o;
    }
    static constexpr int CACHE_N = cache_off(PW) > 0 ? cache_off(PW) : 1;
    struct TwCache {
        Tw<T> v[CACHE_N];
    };
    static __device__ __forceinline__ void load_cache(TwCache &c, const BufView &tw, int l)
    {
        static_for<0, PW>([&](auto pc) {
            constexpr int p = CV(pc), LR = SW::log2r(p), r = 1 << LR, L = 1 << SW::log2L(p), EPR = E / r;
            if constexpr (L > 1) {
                static_for<0, EPR>([&](auto i) {
                    const int j = (l + CV(i) * LANES) & (L - 1);
                    static_for<1, r>([&](auto m) {
                        c.v[cache_off(p) + CV(i) * (r - 1) + CV(m) - 1] =
                            tload_tw<T>(tw, j, SW::twbase(p) + (CV(m) - 1) * L);
                    });
                });
            }
        });
    }
    static __device__ __forceinline__ void fwd_local(Cx<T> *vp, Cx<T> *vm, const TwCache &c, Cx<T> *Rp, Cx<T> *Rm,
                                                     int l, bool active)
    {
        static_for<0, PW>([&](auto pc) {
            constexpr int p = CV(pc), r = 1 << SW::log2r(p);
            auto twf = [&](auto i, auto m, int) { return c.v[cache_off(p) + CV(i) * (r - 1) + CV(m) - 1]; };
            if (active) pass_fwd_f<SW::log2r(p), SW::log2L(p), LANES>(vp, vm, twf, l);
            if constexpr (p + 1 < PW) gx<p, false>(vp, vm, Rp, Rm, l, active);
        });
    }
    static __device__ __forceinline__ void inv_local(Cx<T> *vp, Cx<T> *vm, const TwCache &c, Cx<T> *Rp, Cx<T> *Rm,
                                                     int l, bool active)
    {
        static_for<0, PW>([&](auto pp) {
            constexpr int p = PW - 1 - CV(pp), r = 1 << SW::log2r(p);
            auto twf = [&](auto i, auto m, int) { return c.v[cache_off(p) + CV(i) * (r - 1) + CV(m) - 1]; };
            if constexpr (p + 1 < PW) gx<p, true>(vp, vm, Rp, Rm, l, active);
            if (active) pass_inv_f<SW::log2r(p), SW::log2L(p), LANES>(vp, vm, twf, l);
        });
    }

    // |a|^2 sums over the block, FP64, fixed order
    static __device__ __forceinline__ double block_sum(double v, double *red, int t)
    {
        constexpr int WB = BLOCK < 64 ? BLOCK : 64;
        for (int off = WB / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WB);
        if constexpr (BLOCK > 64) {
            __syncthreads();
            if ((t & 63) == 0) red[t >> 6] = v;
            __syncthreads();
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s += red[w];
            v = s;
        }
        return v;
    }

    // CS: read the plan scalars as scalar loads (false: generic loads, which the
    // any-size kernel marches faster with; its inlined sizes and strain
    // classes leave no scalar registers to hold them).  TC: hold the
    // group-local passes' twiddles of this thread in registers for the march.
    template <bool CS = true, bool TC = false>
    static __device__ void run(const SolveDesc &d, const char *in_base, char *out_base, double *rt,
                               Cx<T> *lds, double *red)
    {
        const int t0 = threadIdx.x;
        const bool active = (BLOCK == TH) || (t0 < TH);
        const Cx<T> *in = reinterpret_cast<const Cx<T> *>(in_base + d.in_off);
        Cx<T> *out = reinterpret_cast<Cx<T> *>(out_base + d.out_off);
        const BufView tw = buf_view(d.tw, TW_ENTRIES * (uint32_t)sizeof(Tw<T>));
        const PropE<T> *prop = reinterpret_cast<const PropE<T> *>(d.prop);
        // sample index of element e of this thread: j0 + TH*e
        const int w0 = t0 >> G::LOG2LANES, l0 = t0 & (LANES - 1);
        const int j00 = w0 + W * l0;
        Cx<T> *bufp = lds;
        Cx<T> *bufm = lds + (BX == 2 ? W * BUFM : 0);

        struct NoCache {};
        typename std::conditional<TC, TwCache, NoCache>::type tcache;
        if constexpr (TC) load_cache(tcache, tw, l0);
        Cx<T> vp[E], vm[E];
        if (active) {
            static_for<0, E>([&](auto e) {
                vp[e] = in[j00 + e * TH];
                vm[e] = in[N + j00 + e * TH];
            });
        } else {
            static_for<0, E>([&](auto e) { vp[e] = vm[e] = Cx<T>{(T)0, (T)0}; });
        }

        double pin = 0.0;
        if (d.flags & SF_FIRST) {
            double s = 0.0;
            static_for<0, E>([&](auto e) {
                const double x = (double)vp[e].x, y = (double)vp[e].y;
                s = __builtin_fma(x, x, __builtin_fma(y, y, s));
            });
            pin = block_sum(s, red, t0);
            if (t0 == 0 && d.pin) *d.pin = pin;
        }

        Coupler<T, SC> cpl;
        cpl.template init<TH>(d, N);
        const T invN = (T)(1.0 / (double)N);

        // plan scalars, read-only for the whole launch
        const PlanPtr<CS> scl = (PlanPtr<CS>)(d.sc);
        const int nsub = scl->nsub;
        const int nend = d.step0 + d.nsteps;
        for (int n = d.step0; n < nend; ++n)
        for (int i = 0; i < nsub; ++i) {
            // one sub-step of the splitting: the propagation of its table (none
            // for a leading coupling), then its coupling
            decltype(auto) ss = load_sub(scl, i);   // a value (CS) or a reference
            // Opaque zeros (the compiler cannot see they are zero): the tables
            // and per-lane offsets are re-derived each sub-step instead of being
            // hoisted into registers for the whole march, and the inverse
            // passes re-read the twiddles instead of keeping the forward copies.
            const int oz = (n + i) & d.opaque_zero;
            const BufView twf = tw + oz * (int)sizeof(Tw<T>);
            const BufView twi = tw + ((n + i + 1) & d.opaque_zero) * (int)sizeof(Tw<T>);
            const BufView propn = buf_view(prop + ss.table * 2 * N, 2 * N * (uint32_t)sizeof(PropE<T>),
                                           oz * (int)sizeof(PropE<T>));
            const int t = t0 + oz;
            const int w = t >> G::LOG2LANES, l = t & (LANES - 1);
            Cx<T> *Rp = bufp + w * BUFM;
            Cx<T> *Rm = bufm + w * BUFM;

            if (ss.table >= 0) {
                // ---- forward transforms (Eq. (12): F[psi+-]); group-local passes
                if constexpr (TC) fwd_local(vp, vm, tcache, Rp, Rm, l, active);
                else fwd_local(vp, vm, twf, Rp, Rm, l, active);
                // ---- cross-group radix-W pass (wave groups only).  Its
                // twiddles are requested before the exchange: after it, every
                // wave of the workgroup leaves the same barrier and waited on
                // the L2 at once (per-size Nx 16384: 3.27 -> 3.41e11).
                Tw<T> xw[W > 1 ? E : 1];
                if constexpr (W > 1) load_cross_tw(xw, twf, t);
                if constexpr (W > 1) {
                    if (active) {
                        write_own(Rp, vp, l);
                        if constexpr (BX == 2) write_own(Rm, vm, l);
                    }
                    __syncthreads();
                    if (active) read_all(bufp, vp, t);
                    if constexpr (BX == 2) {
                        if (active) read_all(bufm, vm, t);
                    } else {
                        __syncthreads();
                        if (active) write_own(Rm, vm, l);
                        __syncthreads();
                        if (active) read_all(bufm, vm, t);
                    }
                }
                if (active) {
                    if constexpr (W > 1) pass_fwd_f<G::LOG2G, G::LOG2M, TH>(vp, vm, cross_tw_f(xw), t);
                    // ---- propagator: sample f = t + TH*e holds frequency bin f.
                    // The entries of PD samples are in flight ahead of the one
                    // multiplied (a rolling set of registers): left to itself the
                    // compiler kept one or two loads in flight and every sample
                    // waited on the L2 (per-size Nx 16384: +3.5 % with PD = 5).
                    constexpr int PD = E < kPropAhead ? E : kPropAhead;
                    PropE<T> kq[PD][2];
                    static_for<0, PD>([&](auto e) {
                        kq[CV(e)][0] = tload_prop<T>(propn, t, CV(e) * TH);
                        kq[CV(e)][1] = tload_prop<T>(propn, t, N + CV(e) * TH);
                    });
                    static_for<0, E>([&](auto e) {
                        const PropE<T> kp = kq[CV(e) % PD][0], km = kq[CV(e) % PD][1];
                        if constexpr (CV(e) + PD < E) {
                            kq[CV(e) % PD][0] = tload_prop<T>(propn, t, (CV(e) + PD) * TH);
                            kq[CV(e) % PD][1] = tload_prop<T>(propn, t, N + (CV(e) + PD) * TH);
                        }
                        const Cx<T> a = vp[e], b = vm[e];
                        vp[e] = prop_mul(a, kp, invN);
                        vm[e] = prop_mul(b, km, invN);
                    });
                    if constexpr (W > 1) pass_inv<G::LOG2G, G::LOG2M, TH>(vp, vm, twi, G::TWFINAL, t);
                }
                // ---- inverse transforms, the forward steps undone in reverse order
                if constexpr (W > 1) {
                    __syncthreads();
                    if (active) {
                        write_all(bufp, vp, t);
                        if constexpr (BX == 2) write_all(bufm, vm, t);
                    }
                    __syncthreads();
                    if (active) read_own(Rp, vp, l);
                    if constexpr (BX == 2) {
                        if (active) read_own(Rm, vm, l);
                    } else {
                        __syncthreads();
                        if (active) write_all(bufm, vm, t);
                        __syncthreads();
                        if (active) read_own(Rm, vm, l);
                    }
                }
                if constexpr (TC) inv_local(vp, vm, tcache, Rp, Rm, l, active);
                else inv_local(vp, vm, twi, Rp, Rm, l, active);
            }

            // ---- real-space coupling inside the crystal (Eq. (9)-(13))
            if (active) cpl.template apply<E, TH>(vp, vm, d, n, w + W * l, ss);
        }

        if (active) {
            static_for<0, E>([&](auto e) {
                out[j00 + e * TH] = vp[e];
                out[N + j00 + e * TH] = vm[e];
            });
        }

        if ((d.flags & SF_LAST) && d.rt_index >= 0) {
            double sp = 0.0, sm = 0.0;
            if (active) {
                static_for<0, E>([&](auto e) {
                    const int j = j00 + e * TH;
                    if (j >= d.det_lo && j < d.det_hi) {
                        const double px = vp[e].x, py = vp[e].y, mx = vm[e].x, my = vm[e].y;
                        sp = __builtin_fma(px, px, __builtin_fma(py, py, sp));
                        sm = __builtin_fma(mx, mx, __builtin_fma(my, my, sm));
                    }
                });
            }
            sp = block_sum(sp, red, t0);
            sm = block_sum(sm, red, t0);
            if (t0 == 0) {
                if (!(d.flags & SF_FIRST)) pin = d.pin ? *d.pin : 0.0;
                const double R = pin > 0.0 ? sm / pin : 0.0;
                const double Tt = pin > 0.0 ? sp / pin : 0.0;
                rt[2 * d.rt_index] = R;
                rt[2 * d.rt_index + 1] = Tt;
            }
        }
    }
};

// ----------------------------------------------------------------- staged lane
// Sizes whose two envelopes do not fit one compute unit's registers and LDS.
// N = R*C with C = 64*E (one wave per row); the transform is the four-step factorisation
//   X[k1 + R k2] = sum_n2 W_C^{n2 k2} W_N^{n2 k1} sum_n1 W_R^{n1 k1} x[C n1 + n2],
// and between its halves the field lives in the solve's own state buffer in
// the layout Y[k1][n2] at k1*C + n2, the same addresses as x[C n1 + n2] for
// n1 = k1, so entry and exit states stay in natural order.  One z-step:
//   row phase    (one wave per row k1): W_N^{n2 k1}, C-point FFT, propagator of
//                frequency k1 + R k2 (table stored in [k1][k2] order), inverse
//                C-point FFT, inverse W_N^{n2 k1};
//   column phase (R/E lanes per column n2): inverse R-point DFT, coupling at
//                x_{C n1 + n2}, then the forward R-point DFT of the next step.
// One workgroup marches one solve; the two phases are separated by workgroup
// barriers (the state stays in L2 / the last-level cache between them).
template <typename T>
constexpr int staged_prec() { return sizeof(T) == 4 ? PREC_F32 : PREC_F64; }

// both beams in one LDS buffer set per wave when all the waves' sets fit
template <typename T, int LOG2C, int LOG2E, int LOG2TH>
constexpr int staged_bx()
{
    return (size_t)(1 << LOG2TH) / 64 * 2 * Sched<LOG2C, LOG2E>::bufsz() * sizeof(Cx<T>) <= kLdsMax ? 2 : 1;
}

// D3: 3D envelopes, ny = R rows of nx = C samples: the same two phases are the
// 2D transform over (y, x) (no four-step twiddle), the propagator table is
// [ky][kx], and the coupling reads the mask per row.  Rows are always one wave
// wide, so C = 2^LOG2C_ samples take C/64 per thread (in both phases).
// PF: each wave issues its next round's state loads before the current round's
// arithmetic (one more set of E samples per beam in registers), so only the
// first round of a phase waits for the state.  TC: the row and column passes'
// twiddles of each lane are held in registers for the whole launch.
template <typename T, int LOG2N, int SC, int LOG2TH = staged_log2th(staged_prec<T>()), bool D3 = false,
          int LOG2C_ = staged_log2c(staged_prec<T>()), bool PF = false, bool TC = PF>
struct Staged {
    static constexpr int LOG2C = LOG2C_, C = 1 << LOG2C;
    static constexpr int LOG2E = LOG2C - 6, E = 1 << LOG2E;
    static constexpr int N = 1 << LOG2N;
    static constexpr int LOG2R = LOG2N - LOG2C, R = 1 << LOG2R;
    static constexpr int TH = 1 << LOG2TH, WAVES = TH / 64;
    static constexpr int BXS = staged_bx<T, LOG2C, LOG2E, LOG2TH>();
    using RowM = March<T, LOG2C, LOG2E, SC, TH, BXS>;
    using ColM = March<T, LOG2R, LOG2E, SC, TH, BXS>;
    static_assert(RowM::LANES == 64 && RowM::W == 1, "one wave per row");
    static_assert(ColM::W == 1 && ColM::LANES <= 64, "columns inside one wave");
    static constexpr int LC = ColM::LANES;            // lanes per column
    static constexpr int GPW = 64 / LC;               // columns per wave
    static constexpr int COLS_PER_ROUND = TH / LC;
    static constexpr int COL_ROUNDS = C / COLS_PER_ROUND;
    static constexpr int ROW_ROUNDS = R / WAVES;
    static_assert(COL_ROUNDS >= 1 && ROW_ROUNDS >= 1, "staged shape");
    static constexpr int ROW_SLAB = RowM::BX * RowM::BUFM;
    static constexpr int COL_SLAB = GPW * ColM::BX * ColM::BUFM;
    static constexpr int SLAB = ROW_SLAB > COL_SLAB ? ROW_SLAB : COL_SLAB;
    static constexpr size_t lds_bytes = (size_t)WAVES * SLAB * sizeof(Cx<T>);
    static_assert(lds_bytes <= kLdsMax, "staged LDS");
    // twiddle table: [row FFT | column FFT | four-step W_N^{n2 k1} at k1*C + n2]
    static constexpr int TW_COL = RowM::SW::twcount();
    static constexpr int TW_4 = TW_COL + ColM::SW::twcount();
    static constexpr int TW_TOTAL = D3 ? TW_4 : TW_4 + N;

    // samples base + stride*e of both beams (beam - at +N) of a state [2][N]
    static __device__ __forceinline__ void load(Cx<T> *vp, Cx<T> *vm, const BufView &src, int base, int stride)
    {
        static_for<0, E>([&](auto e) {
            vp[e] = tload_cx<T>(src, base, e * stride);
            vm[e] = tload_cx<T>(src, base, N + e * stride);
        });
    }
    static __device__ __forceinline__ void store(const BufView &dst, const Cx<T> *vp, const Cx<T> *vm, int base,
                                                 int stride)
    {
        static_for<0, E>([&](auto e) {
            tstore_cx(dst, vp[e], base, e * stride);
            tstore_cx(dst, vm[e], base, N + e * stride);
        });
    }
    // |psi+|^2 and |psi-|^2 over the detector interval, samples base + stride*e
    // (3D: the interval of x = sample mod C in every row)
    static __device__ __forceinline__ void det_sums(const Cx<T> *vp, const Cx<T> *vm, const SolveDesc &d, int base,
                                                    int stride, double &sp, double &sm)
    {
        static_for<0, E>([&](auto e) {
            const int j = D3 ? ((base + e * stride) & (C - 1)) : base + e * stride;
            if (j >= d.det_lo && j < d.det_hi) {
                const double px = vp[e].x, py = vp[e].y, mx = vm[e].x, my = vm[e].y;
                sp = __builtin_fma(px, px, __builtin_fma(py, py, sp));
                sm = __builtin_fma(mx, mx, __builtin_fma(my, my, sm));
            }
        });
    }

    // coupling of the column held by (lane lc of) column c: samples C*(lc + LC*e) + c
    static __device__ __forceinline__ void couple_at(const Coupler<T, SC> &cpl, Cx<T> *vp, Cx<T> *vm,
                                                     const SolveDesc &d, int n, int lc, int c, const SubStep &ss)
    {
        if constexpr (D3) cpl.template apply3d<E, LC, R>(vp, vm, d, n, c, lc, ss);
        else cpl.template apply<E, LC * C>(vp, vm, d, n, lc * C + c, ss);
    }

    // Per-wave view of one solve: buffers, this wave's LDS slab, its column
    // (gi) and lane within the column (lc), and the coupling context.
    struct Ctx {
        BufView in, st, tw;
        const StagedPropE<T, D3> *prop;
        Cx<T> *CRp, *CRm, *RRp, *RRm;
        Coupler<T, SC> cpl;
        int lane, gi, lc;
        T invN;
        CPlanScalars *scl;   // read-only for the launch: scalar loads
        bool lead;   // sub-step 0 is a leading coupling (no propagation before it)
        // TC: the row and column passes' twiddles of this lane in registers
        struct NoCache {};
        typename std::conditional<TC, typename RowM::TwCache, NoCache>::type rc;
        typename std::conditional<TC, typename ColM::TwCache, NoCache>::type cc;

        __device__ __forceinline__ void init(const SolveDesc &d, const char *in_base, char *out_base, Cx<T> *slab,
                                             int lane_)
        {
            constexpr uint32_t SB = 2 * N * (uint32_t)sizeof(Cx<T>);
            in = buf_view(in_base + d.in_off, SB);
            st = buf_view(out_base + d.out_off, SB);   // the solve's state [2][N]
            tw = buf_view(d.tw, TW_TOTAL * (uint32_t)sizeof(Tw<T>));
            prop = reinterpret_cast<const StagedPropE<T, D3> *>(d.prop);
            lane = lane_;
            gi = lane / LC;
            lc = lane % LC;
            CRp = slab + gi * (ColM::BX * ColM::BUFM);
            CRm = CRp + (ColM::BX == 2 ? ColM::BUFM : 0);
            RRp = slab;
            RRm = slab + (RowM::BX == 2 ? RowM::BUFM : 0);
            cpl.template init<LC * C>(d, D3 ? C : N);
            invN = (T)(1.0 / (double)N);
            scl = (CPlanScalars *)(d.sc);
            lead = scl->sub[0].table < 0;
            if constexpr (TC) {
                RowM::load_cache(rc, tw, lane);
                ColM::load_cache(cc, tw + TW_COL * (int)sizeof(Tw<T>), lc);
            }
        }
    };
    static constexpr int TWB = (int)sizeof(Tw<T>);

    // Entry of column c (this wave's group of lanes): natural-order samples in,
    // the incident power, a leading coupling, the forward column DFT, state out
    // as Y (with no z-step to run, the detector sums of the entrance state).
    static __device__ __forceinline__ void entry_col(const Ctx &x, const SolveDesc &d, int c, int oz, bool rt_out,
                                                     double &pin_part, double &sp, double &sm)
    {
        Cx<T> vp[E], vm[E];
        load(vp, vm, x.in, x.lc * C + c, LC * C);
        if (d.flags & SF_FIRST) {
            static_for<0, E>([&](auto e) {
                const double a = (double)vp[e].x, b = (double)vp[e].y;
                pin_part = __builtin_fma(a, a, __builtin_fma(b, b, pin_part));
            });
        }
        if (d.nsteps > 0) {
            if (x.lead) couple_at(x.cpl, vp, vm, d, d.step0, x.lc, c, load_sub(x.scl, 0));
            ColM::fwd_local(vp, vm, x.tw + (TW_COL + oz) * TWB, x.CRp, x.CRm, x.lc, true);
        } else if (rt_out) {
            det_sums(vp, vm, d, x.lc * C + c, LC * C, sp, sm);
        }
        store(x.st, vp, vm, x.lc * C + c, LC * C);
    }

    // Row phase of row k1 (one wave): propagation in Fourier space of sub-step
    // ss (Eq. (12)-(13)); oz, oi are opaque zeros.
    static __device__ __forceinline__ void row_load(const Ctx &x, int k1, int oz, Cx<T> *vp, Cx<T> *vm)
    {
        load(vp, vm, x.st, k1 * C + x.lane + oz, 64);
    }
    static __device__ __forceinline__ void row(const Ctx &x, const SubStep &ss, int k1, int oz, int oi)
    {
        Cx<T> vp[E], vm[E];
        row_load(x, k1, oz, vp, vm);
        row_run(x, ss, k1, oz, oi, vp, vm);
    }
    // the row phase of row k1 on its loaded samples
    // A row round's tables, its four-step twiddles and its propagator entries
    // (bin k2 = lane + 64 e of row k1 is frequency k1 + R k2), all requested
    // before the first is used and, with state loads in flight (PF), before the
    // next round's state loads: loads complete in issue order, so a wait for a
    // table issued after those would wait for them as well.  Requested one
    // sample at a time after the row transform, each entry waited on the L2
    // with two waves per SIMD to cover it (dislocation batch of Nx 32768:
    // 1.445e11 -> 1.634e11 cell-steps/s with the entries requested together
    // after the transform, 1.73e11 with every table ahead of the state loads).
    // Without state loads in flight (FP64) the entries are requested after the
    // row transform: held across it they spilled.
    using PE = StagedPropE<T, D3>;
    struct RowTables {
        Tw<T> w4[D3 ? 1 : E];
        PE kp[PF ? E : 1], km[PF ? E : 1];
    };
    static __device__ __forceinline__ void row_tables(const Ctx &x, const SubStep &ss, int k1, int oz, RowTables &tb)
    {
        const int rb = k1 * C + x.lane + oz;
        if constexpr (!D3) {
            static_for<0, E>([&](auto e) { tb.w4[e] = tload_tw<T>(x.tw, rb, TW_4 + e * 64); });
        }
        if constexpr (PF) load_prop_row(x, ss, k1, oz, tb.kp, tb.km);
    }
    static __device__ __forceinline__ void load_prop_row(const Ctx &x, const SubStep &ss, int k1, int oz, PE *kp,
                                                         PE *km)
    {
        const BufView pr = buf_view(x.prop + ss.table * 2 * N, 2 * N * (uint32_t)sizeof(PE), oz * (int)sizeof(PE));
        const int f = k1 * C + x.lane;
        static_for<0, E>([&](auto e) {
            kp[e] = tload_prop(pr, (PE *)nullptr, f, e * 64);
            km[e] = tload_prop(pr, (PE *)nullptr, f, N + e * 64);
        });
    }
    static __device__ __forceinline__ void row_run(const Ctx &x, const SubStep &ss, int k1, int oz, int oi, Cx<T> *vp,
                                                   Cx<T> *vm)
    {
        RowTables tb;
        row_tables(x, ss, k1, oz, tb);
        row_run_t(x, ss, k1, oz, oi, vp, vm, tb);
    }
    static __device__ __forceinline__ void row_run_t(const Ctx &x, const SubStep &ss, int k1, int oz, int oi, Cx<T> *vp,
                                                     Cx<T> *vm, const RowTables &tb)
    {
        const int rb = k1 * C + x.lane + oz;
        if constexpr (!D3) {
            static_for<0, E>([&](auto e) {
                vp[e] = mul_tw(vp[e], tb.w4[e]);
                vm[e] = mul_tw(vm[e], tb.w4[e]);
            });
        }
        if constexpr (TC) RowM::fwd_local(vp, vm, x.rc, x.RRp, x.RRm, x.lane, true);
        else RowM::fwd_local(vp, vm, x.tw + oz * TWB, x.RRp, x.RRm, x.lane, true);
        const T invN = x.invN;
        if constexpr (PF) {
            static_for<0, E>([&](auto e) {
                const Cx<T> a = vp[e], b = vm[e];
                vp[e] = prop_mul(a, tb.kp[e], invN);
                vm[e] = prop_mul(b, tb.km[e], invN);
            });
        } else {
            PE kp[E], km[E];
            load_prop_row(x, ss, k1, oz, kp, km);
            static_for<0, E>([&](auto e) {
                const Cx<T> a = vp[e], b = vm[e];
                vp[e] = prop_mul(a, kp[e], invN);
                vm[e] = prop_mul(b, km[e], invN);
            });
        }
        if constexpr (TC) RowM::inv_local(vp, vm, x.rc, x.RRp, x.RRm, x.lane, true);
        else RowM::inv_local(vp, vm, x.tw + oi * TWB, x.RRp, x.RRm, x.lane, true);
        const int rbi = k1 * C + x.lane + oi;
        if constexpr (!D3) {
            // TC: the round's four-step twiddles stay in registers for the inverse
            static_for<0, E>([&](auto e) {
                Tw<T> w;
                if constexpr (TC) w = tb.w4[e];
                else w = tload_tw<T>(x.tw, rbi, TW_4 + e * 64);
                vp[e] = mul_tw_inv(vp[e], w);
                vm[e] = mul_tw_inv(vm[e], w);
            });
        }
        store(x.st, vp, vm, rb - oz, 64);
    }

    // Column phase of column c for sub-step i of z-step n: inverse column DFT,
    // coupling (Eq. (9)-(13)), then, unless the march ends here, the next step's
    // leading coupling and forward column DFT; at the end the detector sums.
    static __device__ __forceinline__ void col_load(const Ctx &x, int c, int oz, Cx<T> *vp, Cx<T> *vm)
    {
        load(vp, vm, x.st, x.lc * C + c + oz, LC * C);
    }
    static __device__ __forceinline__ void col(const Ctx &x, const SolveDesc &d, int n, int i, int c, int oz,
                                               int of, bool rt_out, double &sp, double &sm)
    {
        Cx<T> vp[E], vm[E];
        col_load(x, c, oz, vp, vm);
        col_run(x, d, n, i, c, oz, of, rt_out, sp, sm, vp, vm);
    }
    // the column phase of column c on its loaded samples
    static __device__ __forceinline__ void col_run(const Ctx &x, const SolveDesc &d, int n, int i, int c, int oz,
                                                   int of, bool rt_out, double &sp, double &sm, Cx<T> *vp,
                                                   Cx<T> *vm)
    {
        const int nsub = x.scl->nsub;
        const bool step_end = i + 1 == nsub;
        const bool last = step_end && n + 1 == d.step0 + d.nsteps;
        if constexpr (TC) ColM::inv_local(vp, vm, x.cc, x.CRp, x.CRm, x.lc, true);
        else ColM::inv_local(vp, vm, x.tw + (TW_COL + oz) * TWB, x.CRp, x.CRm, x.lc, true);
        couple_at(x.cpl, vp, vm, d, n, x.lc, c, load_sub(x.scl, i));
        if (!last) {
            if (step_end && x.lead) couple_at(x.cpl, vp, vm, d, n + 1, x.lc, c, load_sub(x.scl, 0));
            if constexpr (TC) ColM::fwd_local(vp, vm, x.cc, x.CRp, x.CRm, x.lc, true);
            else ColM::fwd_local(vp, vm, x.tw + (TW_COL + of) * TWB, x.CRp, x.CRm, x.lc, true);
        } else if (rt_out) {
            det_sums(vp, vm, d, x.lc * C + c, LC * C, sp, sm);
        }
        store(x.st, vp, vm, x.lc * C + c, LC * C);
    }

    // One workgroup marches the solve: entry, then per sub-step the row phase
    // and the column phase, separated by workgroup barriers.
    static __device__ void run(const SolveDesc &d, const char *in_base, char *out_base, double *rt,
                               Cx<T> *lds, double *red)
    {
        const int t0 = threadIdx.x;
        const int wv = t0 >> 6;
        Ctx x;
        x.init(d, in_base, out_base, lds + wv * SLAB, t0 & 63);
        const int nend = d.step0 + d.nsteps;
        const bool rt_out = (d.flags & SF_LAST) && d.rt_index >= 0;
        double sp = 0.0, sm = 0.0, pin_part = 0.0;

#pragma unroll 1
        for (int cr = 0; cr < COL_ROUNDS; ++cr)
            entry_col(x, d, cr * COLS_PER_ROUND + wv * GPW + x.gi, cr & d.opaque_zero, rt_out, pin_part, sp, sm);
        double pin = 0.0;
        if (d.flags & SF_FIRST) {
            pin = RowM::block_sum(pin_part, red, t0);
            if (t0 == 0 && d.pin) *d.pin = pin;
        }

        const int nsub = x.scl->nsub;
        for (int n = d.step0; n < nend; ++n)
        for (int i = x.lead ? 1 : 0; i < nsub; ++i) {
            const SubStep ss = load_sub(x.scl, i);
            __syncthreads();
            if constexpr (!PF) {
#pragma unroll 1
                for (int rr = 0; rr < ROW_ROUNDS; ++rr)
                    row(x, ss, rr * WAVES + wv, (n + i + rr) & d.opaque_zero, (n + i + rr + 1) & d.opaque_zero);
                __syncthreads();
#pragma unroll 1
                for (int cr = 0; cr < COL_ROUNDS; ++cr)
                    col(x, d, n, i, cr * COLS_PER_ROUND + wv * GPW + x.gi, (n + i + cr) & d.opaque_zero,
                        (n + i + cr + 1) & d.opaque_zero, rt_out, sp, sm);
            } else {
                // each round's state loads are issued before the previous
                // round's arithmetic, so only the first round of a phase waits
                Cx<T> np[E], nm[E];
                row_load(x, wv, (n + i) & d.opaque_zero, np, nm);
#pragma unroll 1
                for (int rr = 0; rr < ROW_ROUNDS; ++rr) {
                    Cx<T> vp[E], vm[E];
                    static_for<0, E>([&](auto e) {
                        vp[e] = np[e];
                        vm[e] = nm[e];
                    });
                    RowTables tb;
                    row_tables(x, ss, rr * WAVES + wv, (n + i + rr) & d.opaque_zero, tb);
                    if (rr + 1 < ROW_ROUNDS)
                        row_load(x, (rr + 1) * WAVES + wv, (n + i + rr + 1) & d.opaque_zero, np, nm);
                    row_run_t(x, ss, rr * WAVES + wv, (n + i + rr) & d.opaque_zero, (n + i + rr + 1) & d.opaque_zero,
                              vp, vm, tb);
                }
                __syncthreads();
                col_load(x, wv * GPW + x.gi, (n + i) & d.opaque_zero, np, nm);
#pragma unroll 1
                for (int cr = 0; cr < COL_ROUNDS; ++cr) {
                    Cx<T> vp[E], vm[E];
                    static_for<0, E>([&](auto e) {
                        vp[e] = np[e];
                        vm[e] = nm[e];
                    });
                    if (cr + 1 < COL_ROUNDS)
                        col_load(x, (cr + 1) * COLS_PER_ROUND + wv * GPW + x.gi, (n + i + cr + 1) & d.opaque_zero,
                                 np, nm);
                    col_run(x, d, n, i, cr * COLS_PER_ROUND + wv * GPW + x.gi, (n + i + cr) & d.opaque_zero,
                            (n + i + cr + 1) & d.opaque_zero, rt_out, sp, sm, vp, vm);
                }
            }
        }

        if (rt_out) {
            sp = RowM::block_sum(sp, red, t0);
            sm = RowM::block_sum(sm, red, t0);
            if (t0 == 0) {
                if (!(d.flags & SF_FIRST)) pin = d.pin ? *d.pin : 0.0;
                rt[2 * d.rt_index] = pin > 0.0 ? sm / pin : 0.0;
                rt[2 * d.rt_index + 1] = pin > 0.0 ? sp / pin : 0.0;
            }
        }
    }
};

// Sizes the march kernels are built for.  Uniform kernels: one solve per
// workgroup of nx/E threads; mixed kernel: 2^kMixedLog2Th threads, any nx in
// [2^mix_lo, 2^mix_hi] within one grid; staged kernels: nx in [2^stg_lo, 2^stg_hi].
template <typename T>
struct Limits;
template <>
struct Limits<float> {
    static constexpr int uni_lo = 6, uni_hi = 14, mix_lo = 10, mix_hi = 14, stg_lo = 15, stg_hi = 16;
};
template <>
struct Limits<double> {
    static constexpr int uni_lo = 6, uni_hi = 13, mix_lo = 10, mix_hi = 13, stg_lo = 14, stg_hi = 16;
};
constexpr int kMixedLog2Th = 9;
// threads a size uses inside the mixed kernel's 512-thread workgroups (the
// cross-wave radix must not exceed the samples per thread)
__host__ __device__ constexpr int mixed_log2th(int log2n) { return log2n >= 12 ? 9 : 8; }

}  // namespace bpm
