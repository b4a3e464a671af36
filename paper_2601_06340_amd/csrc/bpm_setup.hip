// bpm_setup.hip — FP64 plan-setup kernels (propagator tables, coupling harmonics, twiddles, strain tables).
#include "bpm_march.hpp"

namespace bpm {

// ----------------------------------------------------------------- setup kernels
// FP64 plan setup: coupling harmonics and propagator tables (one launch per plan).
// Coupling coefficients of a sub-step of b*dz (Eq. (8)-(12)), all in FP64:
// A = b dzh / 2c, E = exp(i A chi0), y = -A^2 chih chihb.  form 0: the
// Jacobi-Anger harmonics, a0 = J0 E with J0 = sum y^m/(m!)^2 and
// a+- = i A chi G E with G = sum y^m/(m!(m+1)!); form 1: the exponential of the
// two-beam coupling generator, cosh/sinh series sum y^m/(2m)! and
// sum y^m/(2m+1)! in their place.  a0 - 1 is formed without cancellation.
__device__ void coupling_substep(const PlanParams &P, double A, int form, SubStep &o)
{
    // E - 1 = expm1(i A chi0)
    const double gx = -A * P.chi0y, gy = A * P.chi0x;  // i A chi0
    const double eg = exp(gx), sgy = sin(gy), shalf = sin(0.5 * gy);
    const double em1x = expm1(gx) * cos(gy) - 2.0 * shalf * shalf;
    const double em1y = eg * sgy;
    const double Ex = 1.0 + em1x, Ey = em1y;
    const double qx = P.chihx * P.chihbx - P.chihy * P.chihby;
    const double qy = P.chihx * P.chihby + P.chihy * P.chihbx;
    const double yx = -A * A * qx, yy = -A * A * qy;
    double t0x = 1.0, t0y = 0.0, t1x = 1.0, t1y = 0.0;
    double dmx = 0.0, dmy = 0.0, gxs = 1.0, gys = 0.0;   // diagonal series - 1, off-diagonal series
    for (int m = 1; m < 60; ++m) {
        const double r0 = form == 0 ? (double)m * m : (double)(2 * m - 1) * (2 * m);
        const double r1 = form == 0 ? (double)m * (m + 1) : (double)(2 * m) * (2 * m + 1);
        const double nx0 = (t0x * yx - t0y * yy) / r0, ny0 = (t0x * yy + t0y * yx) / r0;
        const double nx1 = (t1x * yx - t1y * yy) / r1, ny1 = (t1x * yy + t1y * yx) / r1;
        t0x = nx0; t0y = ny0; t1x = nx1; t1y = ny1;
        dmx += t0x; dmy += t0y; gxs += t1x; gys += t1y;
        if (fabs(t0x) + fabs(t0y) + fabs(t1x) + fabs(t1y) < 1e-20) break;
    }
    // a0 - 1 = (D - 1) E + (E - 1)
    o.d0x = (dmx * Ex - dmy * Ey) + em1x;
    o.d0y = (dmx * Ey + dmy * Ex) + em1y;
    const double gex = gxs * Ex - gys * Ey, gey = gxs * Ey + gys * Ex;
    const double cpx = -A * P.chihy, cpy = A * P.chihx;    // i A chih
    const double cmx = -A * P.chihby, cmy = A * P.chihbx;  // i A chihb
    o.apx = cpx * gex - cpy * gey;
    o.apy = cpx * gey + cpy * gex;
    o.amx = cmx * gex - cmy * gey;
    o.amy = cmx * gey + cmy * gex;
}

// FP64 plan setup.  sc != NULL: plan scalars and the coupling sub-steps of the
// splitting; prop != NULL: the propagator table (P - 1)/nx of a sub-step of
// afrac*dz.  The table of a staged size is stored in [k1][k2] order (frequency
// f = k1 + R k2 at k1*(nx/R) + k2, R = 2^log2r); log2r = 0 keeps natural order.
// lift: FP32 entries in the lifting form the staged 2D kernels read.
template <typename T>
__global__ void k_plan_setup(const PlanParams *pp, PlanScalars *sc, PropE<T> *prop, int log2r, double afrac,
                             int lift)
{
    const PlanParams P = *pp;
    const double k = 2.0 * M_PI / P.lambda;
    const double h = 2.0 * M_PI / P.d;
    const double s = h / (2.0 * k);
    const double c = sqrt(1.0 - s * s);
    const double dzh = k * P.dz;
    const int nx = P.nx;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (sc && blockIdx.x == 0 && threadIdx.x == 0) {
        sc->k = k; sc->h = h; sc->s = s; sc->c = c; sc->dzh = dzh;
        double a[kMaxSub], b[kMaxSub], af[kMaxSub];
        int tab[kMaxSub];
        const int m = split_sequence(P.split_order, a, b);
        split_tables(P.split_order, tab, af);
        sc->nsub = m;
        sc->order = P.split_order;
        // Eq. (12) couples at z_n after the propagation; the splittings put
        // sub-step i at z_n + (a_1 + ... + a_i) dz
        double acc = 0.0;
        for (int i = 0; i < m; ++i) {
            acc += a[i];
            coupling_substep(P, b[i] * dzh / (2.0 * c), P.split_order >= 2 ? 1 : 0, sc->sub[i]);
            sc->sub[i].zoff = P.split_order >= 2 ? acc : 0.0;
            sc->sub[i].table = tab[i];
        }
    }
    const int ny = P.ny > 1 ? P.ny : 1;
    const int cells = nx * ny;
    if (prop && f < cells) {
        // frequency bin (fx, fy) of entry f; 3D tables are [ky][kx]
        const int fx = ny > 1 ? f % nx : f, fy = ny > 1 ? f / nx : 0;
        const int gx = fx < nx / 2 ? fx : fx - nx, gy = fy < ny / 2 ? fy : fy - ny;
        const double q = 2.0 * M_PI * (double)gx / ((double)nx * P.dx * k);
        const double qy = ny > 1 ? 2.0 * M_PI * (double)gy / ((double)ny * P.dy * k) : 0.0;
        const double invn = 1.0 / (double)cells;
        for (int beam = 0; beam < 2; ++beam) {
            const double sg = beam == 0 ? 1.0 : -1.0;
            const double pq = q + sg * s;
            const double r = 1.0 - pq * pq - qy * qy;
            // P = mag exp(i th)
            double th, mag;
            if (r >= 0.0) {
                // S - c = -(q^2 +/- 2 s q + qy^2) / (S + c)
                const double S = sqrt(r);
                th = -afrac * dzh * (q * q + 2.0 * sg * s * q + qy * qy) / (S + c);
                mag = 1.0;
            } else {
                th = -afrac * dzh * c;
                mag = exp(-afrac * dzh * sqrt(-r));
            }
            const int pos = log2r ? (f & ((1 << log2r) - 1)) * (nx >> log2r) + (f >> log2r) : f;
            const double sh = sin(0.5 * th);
            if constexpr (std::is_same<T, float>::value) {
                if (lift) {
                    // lifting entry: th reduced to [-pi, pi], then folded into
                    // [-pi/2, pi/2] with the half turn in the sign of the scale
                    double phi = remainder(th, 2.0 * M_PI), sgn = 1.0;
                    if (phi > 0.5 * M_PI) phi -= M_PI, sgn = -1.0;
                    else if (phi < -0.5 * M_PI) phi += M_PI, sgn = -1.0;
                    const float pf = (float)(-tan(0.5 * phi));
                    const double hh = sin(0.5 * phi);
                    // u = (1 - cos phi)/(-p) = 2 sin^2(phi/2)/(-p): p u = 1 - cos phi
                    const double u = pf != 0.0f ? 2.0 * hh * hh / -(double)pf : 0.0;
                    const float uh = (float)u;
                    reinterpret_cast<PropLift *>(prop)[beam * cells + pos] = {pf, uh, (float)(u - (double)uh),
                                                                               (float)(sgn * mag * invn)};
                    continue;
                }
            }
            // k = (P - 1)/N, FP32 as hi + lo
            const double ex = (r >= 0.0 ? -2.0 * sh * sh : mag * cos(th) - 1.0) * invn, ey = mag * sin(th) * invn;
            if constexpr (std::is_same<T, float>::value) {
                const float hx = (float)ex, hy = (float)ey;
                prop[beam * cells + pos] = {hx, hy, (float)(ex - (double)hx), (float)(ey - (double)hy)};
            } else {
                prop[beam * cells + pos] = {ex, ey};
            }
        }
    }
}

// Pass radices (log2) of the (nx, E) schedule, as the march kernels run it
// (Geom): the group-local Stockham passes of M = nx / G points (radix E,
// remainder last) and, when G > 1, the radix-G pass across the G wave groups.
__host__ __device__ inline int schedule_radices(int log2n, int log2e, int *lr)
{
    const int log2th = log2n - log2e;
    const int log2w = (use_wave_groups(log2n, log2e) && log2th > 6) ? log2th - 6 : 0;
    const int log2m = log2n - log2w;
    const int rem = log2m % log2e;
    const int pw = (rem ? 1 : 0) + log2m / log2e;
    int np = 0;
    for (int p = 0; p < pw; ++p) lr[np++] = (p == pw - 1 && rem) ? rem : log2e;
    if (log2w > 0) lr[np++] = log2w;
    return np;
}

// Twiddle table: pass p (sub-length L, radix r), entry (m-1)*L + j holds the
// rotation exp(-2 pi i j m / (L r)), m = 1..r-1, j < L.  The exponent is reduced
// exactly in integers.  FP64 tables store (cos, sin); FP32 tables store the
// lifting constants p = -tan(phi/2), u = sin(phi) of the angle folded into
// [-pi/2, pi/2] and the exact sign s (= -1 when the fold took out a half turn).
// Rotation exp(-2 pi i q / M) for an integer exponent q (reduced exactly
// before any rounding).  FP64 stores (cos, sin); FP32 stores the lifting
// constants p = -tan(phi/2), u = sin(phi) of the angle folded into
// [-pi/2, pi/2] and the exact sign s (= -1 when the fold took out a half turn).
template <typename T>
__device__ Tw<T> encode_rotation(long long q, long long M)
{
    q %= M;
    if (q < 0) q += M;
    if (q > M / 2) q -= M;                  // (-M/2, M/2]
    if constexpr (std::is_same<T, float>::value) {
        float sgn = 1.0f;
        if (4 * q > M || 4 * q < -M) {      // |angle| > pi/2: take out -1
            q += q > 0 ? -M / 2 : M / 2;
            sgn = -1.0f;
        }
        const double pl = tan(M_PI * (double)q / (double)M);
        const double ul = -sinpi(2.0 * (double)q / (double)M);
        return {(float)pl, (float)ul, sgn};
    } else {
        double sn, cs;
        sincospi(-2.0 * (double)q / (double)M, &sn, &cs);
        return {cs, sn};
    }
}

// Twiddle table: pass p (sub-length L, radix r), entry (m-1)*L + j holds the
// rotation exp(-2 pi i j m / (L r)), m = 1..r-1, j < L.
template <typename T>
__global__ void k_twiddles(Tw<T> *tw, int log2n, int log2e)
{
    int lr[32];
    const int P = schedule_radices(log2n, log2e, lr);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int base = 0, ll = 0;
    for (int p = 0; p < P; ++p) {
        const int L = 1 << ll, r = 1 << lr[p];
        const int cnt = L * (r - 1);
        if (idx >= base && idx < base + cnt) {
            const int m = (idx - base) / L + 1, j = (idx - base) % L;
            tw[idx] = encode_rotation<T>((long long)j * m, (long long)L * r);
        }
        base += cnt;
        ll += lr[p];
    }
}

// Four-step twiddles of a staged size: entry k1*C + n2 = W_N^{n2 k1}.
template <typename T>
__global__ void k_twiddles4(Tw<T> *tw, int log2n, int log2c)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (1 << log2n)) {
        const long long k1 = idx >> log2c, n2 = idx & ((1 << log2c) - 1);
        tw[idx] = encode_rotation<T>(n2 * k1, 1ll << log2n);
    }
}

template <typename T>
__global__ void k_utab(const double *u, T *tab, size_t count, double inv_d)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const double rev = u[i] * inv_d;
        tab[i] = (T)(rev - rint(rev));
    }
}

// ----------------------------------------------------------------- host side
static int tw_count(int log2n, int log2e)
{
    int lr[32];
    const int P = schedule_radices(log2n, log2e, lr);
    int s = 0, ll = 0;
    for (int p = 0; p < P; ++p) {
        s += (1 << ll) * ((1 << lr[p]) - 1);
        ll += lr[p];
    }
    return s;
}

size_t twiddle_bytes(int prec, int log2n, int log2e)
{
    return (size_t)tw_count(log2n, log2e) * tw_bytes(prec);
}

hipError_t launch_twiddles(void *d_tw, int prec, int log2n, int log2e, hipStream_t s)
{
    const int cnt = tw_count(log2n, log2e);
    if (cnt == 0) return hipSuccess;
    const int bs = 256, gs = (cnt + bs - 1) / bs;
    if (prec == PREC_F32)
        hipLaunchKernelGGL(k_twiddles<float>, dim3(gs), dim3(bs), 0, s, (Tw<float> *)d_tw, log2n, log2e);
    else
        hipLaunchKernelGGL(k_twiddles<double>, dim3(gs), dim3(bs), 0, s, (Tw<double> *)d_tw, log2n, log2e);
    return hipGetLastError();
}

hipError_t launch_plan_setup(const PlanParams *d_params, PlanScalars *d_sc, void *d_prop, int prec, int cells,
                             int log2r, double afrac, bool lift, hipStream_t s)
{
    const int bs = 256, gs = d_prop ? (cells + bs - 1) / bs : 1;
    if (prec == PREC_F32)
        hipLaunchKernelGGL(k_plan_setup<float>, dim3(gs), dim3(bs), 0, s, d_params, d_sc, (PropE<float> *)d_prop, log2r,
                           afrac, lift ? 1 : 0);
    else
        hipLaunchKernelGGL(k_plan_setup<double>, dim3(gs), dim3(bs), 0, s, d_params, d_sc, (PropE<double> *)d_prop,
                           log2r, afrac, 0);
    return hipGetLastError();
}

// Staged sizes: twiddle layout [row FFT | column FFT | four-step], as Staged<> reads it.
template <typename T>
static bool staged_layout_T(int log2n, int *tw_col, int *tw_4, int *total)
{
    bool ok = false;
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        using S = Staged<T, CV(l), SC_NONE>;
        if (log2n == CV(l)) {
            *tw_col = S::TW_COL;
            *tw_4 = S::TW_4;
            *total = S::TW_TOTAL;
            ok = true;
        }
    });
    return ok;
}

// 3D twiddle table [row FFT | column FFT], as Staged<..., D3> reads it; f(S)
// is called with the Staged<> type of the (nx, ny) pair and the strain class
template <typename T, int SC, typename F>
static bool with_3d_T(int log2nx, int log2ny, F &&f)
{
    bool ok = false;
    static_for<k3DLog2NxMin, k3DLog2NxMax + 1>([&](auto lx) {
        static_for<k3DLog2NyMin, k3DLog2NyMax + 1>([&](auto ly) {
            using S = Staged<T, CV(lx) + CV(ly), SC, staged3d_log2th(staged_prec<T>(), SC, CV(lx)), true, CV(lx)>;
            if (log2nx == CV(lx) && log2ny == CV(ly)) {
                f(S{});
                ok = true;
            }
        });
    });
    return ok;
}

template <typename T>
static bool layout_3d_T(int log2nx, int log2ny, int *tw_col, int *total)
{
    return with_3d_T<T, SC_NONE>(log2nx, log2ny, [&](auto s) {
        using S = decltype(s);
        *tw_col = S::TW_COL;
        *total = S::TW_TOTAL;
    });
}

size_t twiddle3d_bytes(int prec, int log2nx, int log2ny)
{
    int a = 0, tot = 0;
    const bool ok = prec == PREC_F32 ? layout_3d_T<float>(log2nx, log2ny, &a, &tot)
                                     : layout_3d_T<double>(log2nx, log2ny, &a, &tot);
    return ok ? (size_t)tot * tw_bytes(prec) : 0;
}

hipError_t launch_twiddles_3d(void *d_tw, int prec, int log2nx, int log2ny, hipStream_t s)
{
    int tw_col = 0, tot = 0;
    const bool ok = prec == PREC_F32 ? layout_3d_T<float>(log2nx, log2ny, &tw_col, &tot)
                                     : layout_3d_T<double>(log2nx, log2ny, &tw_col, &tot);
    const int le = log2nx - 6;   // one wave per row
    if (!ok || tw_count(log2nx, le) != tw_col || tw_col + tw_count(log2ny, le) != tot) return hipErrorInvalidValue;
    char *base = static_cast<char *>(d_tw);
    hipError_t e = launch_twiddles(base, prec, log2nx, le, s);
    if (e == hipSuccess) e = launch_twiddles(base + (size_t)tw_col * tw_bytes(prec), prec, log2ny, le, s);
    return e;
}

template <typename T, int SC>
static void shape_3d_T(int log2nx, int log2ny, int *threads, size_t *lds)
{
    *threads = 0;
    *lds = 0;
    with_3d_T<T, SC>(log2nx, log2ny, [&](auto s) {
        using S = decltype(s);
        *threads = S::TH;
        *lds = S::lds_bytes;
    });
}

void march_shape_3d(int prec, int sc, int log2nx, int log2ny, int *threads, size_t *lds_bytes)
{
    if (prec == PREC_F32) {
        if (sc == SC_GENERAL) shape_3d_T<float, SC_GENERAL>(log2nx, log2ny, threads, lds_bytes);
        else shape_3d_T<float, SC_NONE>(log2nx, log2ny, threads, lds_bytes);
    } else {
        if (sc == SC_GENERAL) shape_3d_T<double, SC_GENERAL>(log2nx, log2ny, threads, lds_bytes);
        else shape_3d_T<double, SC_NONE>(log2nx, log2ny, threads, lds_bytes);
    }
}

bool is_staged(int prec, int log2n)
{
    return prec == PREC_F32 ? log2n >= Limits<float>::stg_lo : log2n >= Limits<double>::stg_lo;
}

size_t staged_twiddle_bytes(int prec, int log2n)
{
    int a = 0, b = 0, tot = 0;
    const bool ok = prec == PREC_F32 ? staged_layout_T<float>(log2n, &a, &b, &tot)
                                     : staged_layout_T<double>(log2n, &a, &b, &tot);
    return ok ? (size_t)tot * tw_bytes(prec) : 0;
}

hipError_t launch_staged_twiddles(void *d_tw, int prec, int log2n, hipStream_t s)
{
    int tw_col = 0, tw_4 = 0, tot = 0;
    const bool ok = prec == PREC_F32 ? staged_layout_T<float>(log2n, &tw_col, &tw_4, &tot)
                                     : staged_layout_T<double>(log2n, &tw_col, &tw_4, &tot);
    const int le = staged_log2e(prec), lc = staged_log2c(prec), log2r = log2n - lc;
    if (!ok || tw_count(lc, le) != tw_col || tw_col + tw_count(log2r, le) != tw_4) return hipErrorInvalidValue;
    char *base = static_cast<char *>(d_tw);
    hipError_t e = launch_twiddles(base, prec, lc, le, s);
    if (e == hipSuccess) e = launch_twiddles(base + (size_t)tw_col * tw_bytes(prec), prec, log2r, le, s);
    if (e != hipSuccess) return e;
    const int n = 1 << log2n, bs = 256;
    if (prec == PREC_F32)
        hipLaunchKernelGGL(k_twiddles4<float>, dim3((n + bs - 1) / bs), dim3(bs), 0, s,
                           (Tw<float> *)(base + (size_t)tw_4 * tw_bytes(prec)), log2n, lc);
    else
        hipLaunchKernelGGL(k_twiddles4<double>, dim3((n + bs - 1) / bs), dim3(bs), 0, s,
                           (Tw<double> *)(base + (size_t)tw_4 * tw_bytes(prec)), log2n, lc);
    return hipGetLastError();
}

hipError_t launch_utab(const double *d_u, void *d_tab, int prec, size_t count, double inv_d, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const int bs = 256;
    const size_t gs = (count + bs - 1) / bs;
    if (prec == PREC_F32)
        hipLaunchKernelGGL(k_utab<float>, dim3((unsigned)gs), dim3(bs), 0, s, d_u, (float *)d_tab, count, inv_d);
    else
        hipLaunchKernelGGL(k_utab<double>, dim3((unsigned)gs), dim3(bs), 0, s, d_u, (double *)d_tab, count, inv_d);
    return hipGetLastError();
}

}  // namespace bpm

// ----------------------------------------------------------------- march dispatch
// The kernels are instantiated one translation unit per (precision, nx) by the
// build; here only their launchers are declared.
namespace bpm {

template <typename T, int LOG2N, int SC>
hipError_t launch_uniform(const SolveDesc *, int, const char *, char *, double *, hipStream_t);
template <typename T, int SC>
hipError_t launch_mixed(const SolveDesc *, int, const char *, char *, double *, hipStream_t);
template <typename T, int LOG2N, int SC>
hipError_t launch_staged(const SolveDesc *, int, const char *, char *, double *, hipStream_t);
template <typename T>
hipError_t launch_any(const SolveDesc *, int, const char *, char *, double *, hipStream_t);
template <typename T, int LOG2NX, int LOG2NY, int SC>
hipError_t launch_3d(const SolveDesc *, int, const char *, char *, double *, hipStream_t);


template <typename T, int SC>
static hipError_t dispatch(const SolveDesc *d_descs, int n, int uniform_log2n, const char *in_base, char *out_base,
                           double *rt, hipStream_t s)
{
    if (uniform_log2n == kLaunchAny) return launch_any<T>(d_descs, n, in_base, out_base, rt, s);
    if (uniform_log2n >= kLaunch3D) {
        hipError_t err = hipErrorInvalidValue;
        static_for<k3DLog2NxMin, k3DLog2NxMax + 1>([&](auto lx) {
            static_for<k3DLog2NyMin, k3DLog2NyMax + 1>([&](auto ly) {
                if (uniform_log2n == kind_3d(CV(lx), CV(ly)))
                    err = launch_3d<T, CV(lx), CV(ly), SC>(d_descs, n, in_base, out_base, rt, s);
            });
        });
        return err;
    }
    if (uniform_log2n < 0) return launch_mixed<T, SC>(d_descs, n, in_base, out_base, rt, s);
    hipError_t err = hipErrorInvalidValue;
    static_for<Limits<T>::uni_lo, Limits<T>::uni_hi + 1>([&](auto l) {
        if (uniform_log2n == CV(l)) err = launch_uniform<T, CV(l), SC>(d_descs, n, in_base, out_base, rt, s);
    });
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        if (uniform_log2n == CV(l)) err = launch_staged<T, CV(l), SC>(d_descs, n, in_base, out_base, rt, s);
    });
    return err;
}

// ---- wide lane
template <typename T, int LOG2N, int SC, bool D3, int LOG2C>
hipError_t launch_wide_T(int, const WideArgs &, hipStream_t, WideShape *);

template <typename T, int SC>
static hipError_t wide_dispatch(int kind, int phase, const WideArgs &a, hipStream_t s, WideShape *shape)
{
    hipError_t err = hipErrorInvalidValue;
    if (kind >= kLaunch3D) {
        static_for<k3DLog2NxMin, k3DLog2NxMax + 1>([&](auto lx) {
            static_for<k3DLog2NyMin, k3DLog2NyMax + 1>([&](auto ly) {
                if (kind == kind_3d(CV(lx), CV(ly)))
                    err = launch_wide_T<T, CV(lx) + CV(ly), SC, true, CV(lx)>(phase, a, s, shape);
            });
        });
        return err;
    }
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        if (kind == CV(l))
            err = launch_wide_T<T, CV(l), SC, false, staged_log2c(staged_prec<T>())>(phase, a, s, shape);
    });
    return err;
}

template <typename T>
static hipError_t wide_dispatch_sc(int kind, int sc, int phase, const WideArgs &a, hipStream_t s, WideShape *shape)
{
    if (sc == SC_NONE) return wide_dispatch<T, SC_NONE>(kind, phase, a, s, shape);
    if (sc == SC_POLY2) return wide_dispatch<T, SC_POLY2>(kind, phase, a, s, shape);
    return wide_dispatch<T, SC_GENERAL>(kind, phase, a, s, shape);
}

hipError_t launch_wide(int prec, int kind, int sc, int phase, const WideArgs &a, hipStream_t s, WideShape *shape)
{
    if (prec == PREC_F32) return wide_dispatch_sc<float>(kind, sc, phase, a, s, shape);
    return wide_dispatch_sc<double>(kind, sc, phase, a, s, shape);
}

bool wide_kind(int prec, int kind)
{
    if (kind >= kLaunch3D) return is_kind_3d(kind);
    if (prec == PREC_F32) return kind >= Limits<float>::stg_lo && kind <= Limits<float>::stg_hi;
    return kind >= Limits<double>::stg_lo && kind <= Limits<double>::stg_hi;
}

// R and T of a wide march from its per-workgroup partial sums, summed in
// workgroup order in FP64; the incident power is stored when the march began.
__global__ void k_wide_finish(const SolveDesc *descs, const double *part, int nblk, double *rt)
{
    if (threadIdx.x != 0) return;
    const SolveDesc &d = descs[0];
    double pin = 0.0, sp = 0.0, sm = 0.0;
    for (int b = 0; b < nblk; ++b) {
        pin += part[3 * b];
        sp += part[3 * b + 1];
        sm += part[3 * b + 2];
    }
    if (d.flags & SF_FIRST) {
        if (d.pin) *d.pin = pin;
    } else {
        pin = d.pin ? *d.pin : 0.0;
    }
    if ((d.flags & SF_LAST) && d.rt_index >= 0) {
        rt[2 * d.rt_index] = pin > 0.0 ? sm / pin : 0.0;
        rt[2 * d.rt_index + 1] = pin > 0.0 ? sp / pin : 0.0;
    }
}

__global__ void k_wide_ctl(WideCtl *ctl, SolveDesc *desc, int base, const char *in, char *out, int step0, int nsteps,
                           int flags)
{
    if (threadIdx.x == 0) {
        ctl->base = base;
        ctl->in = in;
        ctl->out = out;
        desc->step0 = step0;
        desc->nsteps = nsteps;
        desc->flags = flags;
    }
}

hipError_t launch_wide_finish(const SolveDesc *desc, const double *part, int nblk, double *rt, hipStream_t s)
{
    hipLaunchKernelGGL(k_wide_finish, dim3(1), dim3(64), 0, s, desc, part, nblk, rt);
    return hipGetLastError();
}

hipError_t launch_wide_ctl(WideCtl *ctl, SolveDesc *desc, int base, const char *in, char *out, int step0, int nsteps,
                           int flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_wide_ctl, dim3(1), dim3(64), 0, s, ctl, desc, base, in, out, step0, nsteps, flags);
    return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_sc(const SolveDesc *d_descs, int n, int uniform_log2n, int sc, const char *in_base,
                              char *out_base, double *rt, hipStream_t s)
{
    if (sc == SC_NONE) return dispatch<T, SC_NONE>(d_descs, n, uniform_log2n, in_base, out_base, rt, s);
    if (sc == SC_POLY1 && std::is_same<T, float>::value && uniform_log2n >= Limits<T>::uni_lo &&
        uniform_log2n <= Limits<T>::uni_hi) {
        hipError_t err = hipErrorInvalidValue;
        static_for<Limits<float>::uni_lo, Limits<float>::uni_hi + 1>([&](auto l) {
            if (uniform_log2n == CV(l))
                err = launch_uniform<float, CV(l), SC_POLY1>(d_descs, n, in_base, out_base, rt, s);
        });
        return err;
    }
    if (sc == SC_POLY2 || sc == SC_POLY1)
        return dispatch<T, SC_POLY2>(d_descs, n, uniform_log2n, in_base, out_base, rt, s);
    return dispatch<T, SC_GENERAL>(d_descs, n, uniform_log2n, in_base, out_base, rt, s);
}

hipError_t launch_march(const SolveDesc *d_descs, int n, int prec, int uniform_log2n, int sc, const char *in_base,
                        char *out_base, double *rt, hipStream_t s)
{
    if (prec == PREC_F32) return dispatch_sc<float>(d_descs, n, uniform_log2n, sc, in_base, out_base, rt, s);
    return dispatch_sc<double>(d_descs, n, uniform_log2n, sc, in_base, out_base, rt, s);
}

template <typename T>
static void shape_T(int log2n, int *threads, size_t *lds)
{
    *threads = 0;
    *lds = 0;
    static_for<Limits<T>::uni_lo, Limits<T>::uni_hi + 1>([&](auto l) {
        constexpr int L2 = CV(l);
        if (log2n == L2) {
            *threads = 1 << (L2 - uniform_log2e(L2));
            *lds = LdsPlan<T, L2, uniform_log2e(L2)>::bytes;
        }
    });
    static_for<Limits<T>::stg_lo, Limits<T>::stg_hi + 1>([&](auto l) {
        if (log2n == CV(l)) {
            *threads = Staged<T, CV(l), SC_NONE>::TH;
            *lds = Staged<T, CV(l), SC_NONE>::lds_bytes;
        }
    });
}

template <typename T>
static size_t mixed_lds_T()
{
    size_t m = 0;
    static_for<Limits<T>::mix_lo, Limits<T>::mix_hi + 1>([&](auto l) {
        constexpr int L2 = CV(l);
        const size_t b = LdsPlan<T, L2, L2 - mixed_log2th(L2)>::bytes;
        if (b > m) m = b;
    });
    return m;
}

void march_shape(int prec, int log2n, int *threads, size_t *lds_bytes)
{
    if (prec == PREC_F32) shape_T<float>(log2n, threads, lds_bytes);
    else shape_T<double>(log2n, threads, lds_bytes);
}
void mixed_shape(int prec, int *threads, size_t *lds_bytes)
{
    *threads = 1 << kMixedLog2Th;
    *lds_bytes = prec == PREC_F32 ? mixed_lds_T<float>() : mixed_lds_T<double>();
}
int max_log2n(int prec) { return prec == PREC_F32 ? Limits<float>::stg_hi : Limits<double>::stg_hi; }
int mixed_min_log2n(int prec) { return prec == PREC_F32 ? Limits<float>::mix_lo : Limits<double>::mix_lo; }
int mixed_max_log2n(int prec) { return prec == PREC_F32 ? Limits<float>::mix_hi : Limits<double>::mix_hi; }
int mixed_log2e(int prec, int log2n) { return log2n - mixed_log2th(log2n); }

}  // namespace bpm
