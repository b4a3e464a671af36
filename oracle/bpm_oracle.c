/*
 * bpm_oracle.c — TEST INFRASTRUCTURE (see bpm_oracle.h).
 *
 * A plain FP64 transcription of the two-beam FFT BPM march, step by step in the
 * paper's order: propagate each envelope in Fourier space with its shifted
 * propagator, return to real space, then couple the two envelopes through the
 * n = 0, +/-1 harmonics of the susceptibility phase (Sec. 2, Eq. (4), (8)-(12)).
 * No blocking, fusion or reordering beyond what those equations state.
 * Built with -O2 -ffp-contract=off so every product is rounded on its own.
 */
#include "bpm_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* ---------------------------------------------------------------- DFTs ---- */

/* Twiddle table w[m] = exp(sign*2*pi*i*m/n), m < n/2, straight from cos/sin (no
 * recurrence). */
static double complex *twiddles(int n, int sign)
{
    double complex *w = malloc(sizeof(double complex) * (size_t)(n / 2 > 0 ? n / 2 : 1));
    if (!w) return NULL;
    for (int m = 0; m < n / 2; m++) {
        double ang = sign * 2.0 * M_PI * (double)m / (double)n;
        w[m] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* Iterative radix-2 Cooley-Tukey: bit-reversal permutation, then log2(n) stages of
 * butterflies using the table above. */
static void fft_with(double complex *a, int n, const double complex *w)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { double complex t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, wstep = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; k++) {
                double complex u = a[i + k];
                double complex v = a[i + k + half] * w[k * wstep];
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
    }
}

int oracle_fft(double complex *a, int n, int sign)
{
    if (!is_pow2(n)) return -1;
    double complex *w = twiddles(n, sign);
    if (!w) return -2;
    fft_with(a, n, w);
    free(w);
    return 0;
}

void oracle_dft(const double complex *in, double complex *out, int n, int sign)
{
    for (int f = 0; f < n; f++) {
        double complex acc = 0;
        for (int j = 0; j < n; j++) {
            /* reduce j*f mod n exactly before forming the angle */
            long long m = ((long long)j * f) % n;
            double ang = sign * 2.0 * M_PI * (double)m / (double)n;
            acc += in[j] * (cos(ang) + I * sin(ang));
        }
        out[f] = acc;
    }
}

/* ------------------------------------------------------------- scalars ---- */

/* Jacobi-Anger for delta_eps = chi0 + chih e^{+i k_d x} + chihb e^{-i k_d x}
 * (Eq. (8)-(10), generalised to chih != chihb): with A = dzh/(2c) and
 * y = -A^2 chih chihb,
 *   harmonic 0 : J0 = sum_m y^m/(m!)^2
 *   harmonic +1: i A chih  * G,   G = sum_m y^m/(m!(m+1)!)   (= 2 J1(w)/w)
 * Both series are even in w = 2A sqrt(chih chihb), so no square root is taken. */
void oracle_bessel_series(double complex y, double complex *j0, double complex *g)
{
    double complex t0 = 1.0, s0 = 1.0; /* y^m/(m!)^2 */
    double complex t1 = 1.0, s1 = 1.0; /* y^m/(m!(m+1)!) */
    for (int m = 1; m < 200; m++) {
        t0 = t0 * y / ((double)m * (double)m);
        t1 = t1 * y / ((double)m * (double)(m + 1));
        s0 += t0;
        s1 += t1;
        if (cabs(t0) <= 1e-18 * cabs(s0) && cabs(t1) <= 1e-18 * cabs(s1)) break;
    }
    *j0 = s0;
    *g = s1;
}

/* Exponential of the two-beam coupling generator N = i A [[0, chih], [chihb, 0]]:
 * N^2 = y I with y = -A^2 chih chihb, so exp(N) = cosh(v) I + (sinh(v)/v) N with
 * v^2 = y; both series are in y, so no square root is taken. */
void oracle_exp_series(double complex y, double complex *ch, double complex *sh)
{
    double complex t0 = 1.0, s0 = 1.0; /* y^m/(2m)! */
    double complex t1 = 1.0, s1 = 1.0; /* y^m/(2m+1)! */
    for (int m = 1; m < 200; m++) {
        t0 = t0 * y / ((double)(2 * m - 1) * (double)(2 * m));
        t1 = t1 * y / ((double)(2 * m) * (double)(2 * m + 1));
        s0 += t0;
        s1 += t1;
        if (cabs(t0) <= 1e-18 * cabs(s0) && cabs(t1) <= 1e-18 * cabs(s1)) break;
    }
    *ch = s0;
    *sh = s1;
}

static int desc_valid(const oracle_desc *d)
{
    if (!d || !is_pow2(d->nx) || d->nz < 0) return 0;
    if (!(d->dx_um > 0) || !(d->dz_um > 0) || !(d->lambda_um > 0) || !(d->d_um > 0)) return 0;
    if (!(d->lambda_um < 2.0 * d->d_um)) return 0;
    if (d->nseg < 0 || (d->nseg > 0 && d->nz > 0 && !d->seg)) return 0;
    if (d->strain_kind == ORACLE_STRAIN_TABLE && !d->u_table && d->nz > 0) return 0;
    if (d->split_order != 0 && d->split_order != 1 && d->split_order != 2 && d->split_order != 4) return 0;
    if (d->ny > 1 && (!is_pow2(d->ny) || !(d->dy_um > 0))) return 0;
    return 1;
}

int oracle_scalars_get(const oracle_desc *d, oracle_scalars *o)
{
    if (!desc_valid(d)) return -1;
    o->k = 2.0 * M_PI / d->lambda_um;
    o->h = 2.0 * M_PI / d->d_um;
    o->s = o->h / (2.0 * o->k);
    o->c = sqrt(1.0 - o->s * o->s);
    o->dzh = o->k * d->dz_um;
    return oracle_coupling(d, 1.0, 0, &o->a0, &o->ap, &o->am);
}

int oracle_coupling(const oracle_desc *d, double b, int form, double complex *a0, double complex *ap,
                    double complex *am)
{
    if (!desc_valid(d)) return -1;
    double k = 2.0 * M_PI / d->lambda_um, h = 2.0 * M_PI / d->d_um;
    double s = h / (2.0 * k), c = sqrt(1.0 - s * s);
    double complex chi0 = d->chi0_re + I * d->chi0_im;
    double complex chih = d->chih_re + I * d->chih_im;
    double complex chihb = d->chihb_re + I * d->chihb_im;
    double A = b * k * d->dz_um / (2.0 * c);
    double complex E = cexp(I * A * chi0);
    double complex y = -A * A * chih * chihb;
    double complex diag, off;
    if (form == 0) oracle_bessel_series(y, &diag, &off);
    else oracle_exp_series(y, &diag, &off);
    *a0 = diag * E;
    *ap = I * A * chih * off * E;
    *am = I * A * chihb * off * E;
    return 0;
}

int oracle_split_sequence(int order, double *a, double *b)
{
    if (order <= 1) {
        a[0] = 1.0; b[0] = 1.0;
        return 1;
    }
    if (order == 2) {
        a[0] = 0.0; a[1] = 1.0;
        b[0] = 0.5; b[1] = 0.5;
        return 2;
    }
    if (order == 4) {
        const double t = 1.0 / (2.0 - cbrt(2.0));
        a[0] = 0.0; a[1] = t; a[2] = 1.0 - 2.0 * t; a[3] = t;
        b[0] = 0.5 * t; b[1] = 0.5 * (1.0 - t); b[2] = 0.5 * (1.0 - t); b[3] = 0.5 * t;
        return 4;
    }
    return 0;
}

/* p+- = exp(i dzh (S(q +/- s) - c)) / nx on the numpy frequency grid.  The
 * difference S - c is formed without cancellation as
 * -(q^2 +/- 2 s q) / (S + c); dropping the constant -c relative to Eq. (4) only
 * multiplies both envelopes by the same global phase per step. */
int oracle_propagator(const oracle_desc *d, double complex *pp, double complex *pm)
{
    return oracle_propagator_frac(d, 1.0, pp, pm);
}

int oracle_propagator_frac(const oracle_desc *d, double a, double complex *pp, double complex *pm)
{
    oracle_scalars sc;
    if (oracle_scalars_get(d, &sc)) return -1;
    sc.dzh *= a;
    int n = d->nx;
    for (int f = 0; f < n; f++) {
        int ff = f < n / 2 ? f : f - n;
        double q = 2.0 * M_PI * (double)ff / ((double)n * d->dx_um * sc.k);
        for (int b = 0; b < 2; b++) {
            double sg = b == 0 ? 1.0 : -1.0;
            double p = q + sg * sc.s;
            double complex P;
            if (fabs(p) <= 1.0) {
                double S = sqrt(1.0 - p * p);
                double th = -sc.dzh * (q * q + 2.0 * sg * sc.s * q) / (S + sc.c);
                P = cexp(I * th);
            } else {
                P = exp(-sc.dzh * sqrt(p * p - 1.0)) * cexp(-I * sc.dzh * sc.c);
            }
            P /= (double)n;
            if (b == 0) pp[f] = P; else pm[f] = P;
        }
    }
    return 0;
}

/* ------------------------------------------------------------- strain ----- */

double oracle_strain_phase(const oracle_desc *d, int j, int n)
{
    return oracle_strain_phase_z(d, j, n, n * d->dz_um);
}

double oracle_strain_phase_z(const oracle_desc *d, int j, int n, double z)
{
    double h = 2.0 * M_PI / d->d_um;
    double x = d->x0_um + j * d->dx_um;
    double X = x - d->x_ref_um, Z = z - d->z_ref_um;
    double u = 0.0;
    switch (d->strain_kind) {
    case ORACLE_STRAIN_POLY2: {
        const double *c = d->strain_c;
        u = c[0] + c[1] * X + c[2] * Z + c[3] * X * X + c[4] * X * Z + c[5] * Z * Z;
        break;
    }
    case ORACLE_STRAIN_EDGE_DISL: {
        /* Eq. (15) for a line along y and b along h: only the arctangent and the
         * y0 z0 / (2(1-nu) r^2) terms have a component along h. */
        double r2 = X * X + Z * Z;
        double t = atan2(Z, X);
        if (r2 > 0) t += X * Z / (2.0 * (1.0 - d->disl_nu) * r2);
        u = d->disl_b_um / (2.0 * M_PI) * t;
        break;
    }
    case ORACLE_STRAIN_TABLE:
        u = d->u_table[(size_t)n * d->nx + j];
        break;
    default:
        u = 0.0;
    }
    return h * u;
}

/* ------------------------------------------------------------- march ------ */

static int inside_mask(const oracle_desc *d, int j, int n)
{
    for (int k = 0; k < d->nseg; k++) {
        const int *iv = d->seg + ((size_t)n * d->nseg + k) * 2;
        if (j >= iv[0] && j < iv[1]) return 1;
    }
    return 0;
}

/* Compensated (Kahan) sum of |a_j|^2 over [lo, hi). */
static double power_sum(const double complex *a, int lo, int hi)
{
    double s = 0.0, comp = 0.0;
    for (int j = lo; j < hi; j++) {
        double v = creal(a[j]) * creal(a[j]) + cimag(a[j]) * cimag(a[j]);
        double yv = v - comp;
        double t = s + yv;
        comp = (t - s) - yv;
        s = t;
    }
    return s;
}

/* Coupling of one (sub-)step with coefficients a0, ap, am: mask row n, strain at z. */
static void couple_step(const oracle_desc *d, double complex *psi_p, double complex *psi_m, int n, double z,
                        double complex a0, double complex ap, double complex am)
{
    for (int j = 0; j < d->nx; j++) {
        if (!inside_mask(d, j, n)) continue;
        double complex e = 1.0;
        if (d->strain_kind != ORACLE_STRAIN_NONE) {
            double phi = oracle_strain_phase_z(d, j, n, z);
            e = cos(phi) + I * sin(phi);
        }
        double complex p = psi_p[j], m = psi_m[j];
        psi_p[j] = a0 * p + ap * e * m;
        psi_m[j] = a0 * m + am * conj(e) * p;
    }
}

/* Eq. (13): every step is A(a_1 dz) B(b_1 dz) ... A(a_m dz) B(b_m dz), applied
 * from the left; B_i sits at z_n + (a_1 + ... + a_i) dz. */
static int propagate_split(const oracle_desc *d, double complex *psi_p, double complex *psi_m,
                           const double complex *wf, const double complex *wi)
{
    double a[8], b[8];
    int m = oracle_split_sequence(d->split_order, a, b);
    if (m == 0) return -1;
    int n = d->nx;
    double complex *tp[8], *tm[8], c0[8], cp[8], cm[8];
    double zoff[8], acc = 0.0;
    int rc = 0;
    for (int i = 0; i < m; i++) {
        tp[i] = tm[i] = NULL;
        acc += a[i];
        zoff[i] = acc;
        if (a[i] != 0.0) {
            tp[i] = malloc(sizeof(double complex) * (size_t)n);
            tm[i] = malloc(sizeof(double complex) * (size_t)n);
            if (!tp[i] || !tm[i]) rc = -2;
            else oracle_propagator_frac(d, a[i], tp[i], tm[i]);
        }
        oracle_coupling(d, b[i], 1, &c0[i], &cp[i], &cm[i]);
    }
    for (int step = 0; rc == 0 && step < d->nz; step++) {
        for (int i = 0; i < m; i++) {
            if (a[i] != 0.0) {
                fft_with(psi_p, n, wf);
                fft_with(psi_m, n, wf);
                for (int f = 0; f < n; f++) { psi_p[f] *= tp[i][f]; psi_m[f] *= tm[i][f]; }
                fft_with(psi_p, n, wi);
                fft_with(psi_m, n, wi);
            }
            couple_step(d, psi_p, psi_m, step, (step + zoff[i]) * d->dz_um, c0[i], cp[i], cm[i]);
        }
    }
    for (int i = 0; i < m; i++) { free(tp[i]); free(tm[i]); }
    return rc;
}

/* ------------------------------------------------------------- 3D --------- */

int oracle_propagator_2d(const oracle_desc *d, double a, double complex *pp, double complex *pm)
{
    oracle_scalars sc;
    if (oracle_scalars_get(d, &sc) || d->ny < 2) return -1;
    int nx = d->nx, ny = d->ny;
    double dzh = a * sc.dzh;
    for (int fy = 0; fy < ny; fy++) {
        int gy = fy < ny / 2 ? fy : fy - ny;
        double qy = 2.0 * M_PI * (double)gy / ((double)ny * d->dy_um * sc.k);
        for (int fx = 0; fx < nx; fx++) {
            int gx = fx < nx / 2 ? fx : fx - nx;
            double qx = 2.0 * M_PI * (double)gx / ((double)nx * d->dx_um * sc.k);
            for (int b = 0; b < 2; b++) {
                double sg = b == 0 ? 1.0 : -1.0;
                double px = qx + sg * sc.s;
                double r = 1.0 - px * px - qy * qy;
                double complex P;
                if (r >= 0.0) {
                    /* S - c = -(qx^2 +/- 2 s qx + qy^2) / (S + c) */
                    double S = sqrt(r);
                    P = cexp(-I * dzh * (qx * qx + 2.0 * sg * sc.s * qx + qy * qy) / (S + sc.c));
                } else {
                    P = exp(-dzh * sqrt(-r)) * cexp(-I * dzh * sc.c);
                }
                P /= (double)nx * (double)ny;
                if (b == 0) pp[(size_t)fy * nx + fx] = P; else pm[(size_t)fy * nx + fx] = P;
            }
        }
    }
    return 0;
}

/* 2D transform of an [ny][nx] array: every row, then every column. */
static void fft2_with(double complex *a, int nx, int ny, const double complex *wx, const double complex *wy,
                      double complex *col)
{
    for (int i = 0; i < ny; i++) fft_with(a + (size_t)i * nx, nx, wx);
    for (int j = 0; j < nx; j++) {
        for (int i = 0; i < ny; i++) col[i] = a[(size_t)i * nx + j];
        fft_with(col, ny, wy);
        for (int i = 0; i < ny; i++) a[(size_t)i * nx + j] = col[i];
    }
}

static void couple_3d(const oracle_desc *d, double complex *psi_p, double complex *psi_m, int n, double z,
                      double complex a0, double complex ap, double complex am)
{
    double h = 2.0 * M_PI / d->d_um;
    for (int i = 0; i < d->ny; i++)
        for (int j = 0; j < d->nx; j++) {
            int in = 0;
            for (int k = 0; k < d->nseg; k++) {
                const int *iv = d->seg + (((size_t)n * d->ny + i) * d->nseg + k) * 2;
                if (j >= iv[0] && j < iv[1]) in = 1;
            }
            if (!in) continue;
            double complex e = 1.0;
            if (d->strain_kind == ORACLE_STRAIN_TABLE) {
                double phi = h * d->u_table[((size_t)n * d->ny + i) * d->nx + j];
                e = cos(phi) + I * sin(phi);
            } else if (d->strain_kind != ORACLE_STRAIN_NONE) {
                double phi = oracle_strain_phase_z(d, j, n, z);
                e = cos(phi) + I * sin(phi);
            }
            size_t q = (size_t)i * d->nx + j;
            double complex p = psi_p[q], m = psi_m[q];
            psi_p[q] = a0 * p + ap * e * m;
            psi_m[q] = a0 * m + am * conj(e) * p;
        }
}

static int propagate_3d(const oracle_desc *d, double complex *psi_p, double complex *psi_m, double *R, double *T)
{
    int nx = d->nx, ny = d->ny;
    size_t N = (size_t)nx * ny;
    double a[8], b[8];
    int m = oracle_split_sequence(d->split_order, a, b);
    int form = d->split_order > 1 ? 1 : 0;
    double complex *tp[8], *tm[8], c0[8], cp[8], cm[8];
    double zoff[8], acc = 0.0;
    double complex *wfx = twiddles(nx, -1), *wix = twiddles(nx, +1);
    double complex *wfy = twiddles(ny, -1), *wiy = twiddles(ny, +1);
    double complex *col = malloc(sizeof(double complex) * (size_t)ny);
    int rc = (wfx && wix && wfy && wiy && col) ? 0 : -2;
    for (int i = 0; i < m; i++) {
        tp[i] = tm[i] = NULL;
        acc += a[i];
        zoff[i] = form ? acc : 0.0;     /* Eq. (12) couples at z_n; the splittings at their own height */
        if (a[i] != 0.0 && rc == 0) {
            tp[i] = malloc(sizeof(double complex) * N);
            tm[i] = malloc(sizeof(double complex) * N);
            if (!tp[i] || !tm[i]) rc = -2;
            else oracle_propagator_2d(d, a[i], tp[i], tm[i]);
        }
        oracle_coupling(d, b[i], form, &c0[i], &cp[i], &cm[i]);
    }
    double pin = 0.0;
    for (int i = 0; i < ny; i++) pin += power_sum(psi_p + (size_t)i * nx, 0, nx);
    for (int step = 0; rc == 0 && step < d->nz; step++)
        for (int i = 0; i < m; i++) {
            if (a[i] != 0.0) {
                fft2_with(psi_p, nx, ny, wfx, wfy, col);
                fft2_with(psi_m, nx, ny, wfx, wfy, col);
                for (size_t f = 0; f < N; f++) { psi_p[f] *= tp[i][f]; psi_m[f] *= tm[i][f]; }
                fft2_with(psi_p, nx, ny, wix, wiy, col);
                fft2_with(psi_m, nx, ny, wix, wiy, col);
            }
            couple_3d(d, psi_p, psi_m, step, (step + zoff[i]) * d->dz_um, c0[i], cp[i], cm[i]);
        }
    int lo = d->det_lo < 0 ? 0 : d->det_lo;
    int hi = d->det_hi > nx ? nx : d->det_hi;
    if (hi < lo) hi = lo;
    double r = 0.0, t = 0.0;
    for (int i = 0; i < ny; i++) {
        r += power_sum(psi_m + (size_t)i * nx, lo, hi);
        t += power_sum(psi_p + (size_t)i * nx, lo, hi);
    }
    if (R) *R = pin > 0 ? r / pin : 0.0;
    if (T) *T = pin > 0 ? t / pin : 0.0;
    for (int i = 0; i < m; i++) { free(tp[i]); free(tm[i]); }
    free(wfx); free(wix); free(wfy); free(wiy); free(col);
    return rc;
}

int oracle_propagate(const oracle_desc *d, double complex *psi_p, double complex *psi_m,
                     double *R, double *T)
{
    if (!desc_valid(d)) return -1;
    if (d->ny > 1) return propagate_3d(d, psi_p, psi_m, R, T);
    int n = d->nx;
    oracle_scalars sc;
    oracle_scalars_get(d, &sc);
    double complex *pp = malloc(sizeof(double complex) * (size_t)n);
    double complex *pm = malloc(sizeof(double complex) * (size_t)n);
    double complex *wf = twiddles(n, -1), *wi = twiddles(n, +1);
    if (!pp || !pm || !wf || !wi) { free(pp); free(pm); free(wf); free(wi); return -2; }
    oracle_propagator(d, pp, pm);
    double pin = power_sum(psi_p, 0, n);

    if (d->split_order > 1) {
        int rc = propagate_split(d, psi_p, psi_m, wf, wi);
        free(pp);
        free(pm);
        pp = pm = NULL;
        if (rc) { free(wf); free(wi); return rc; }
    }
    for (int step = 0; step < (d->split_order > 1 ? 0 : d->nz); step++) {
        /* Fourier-space propagation of each envelope about its own carrier */
        fft_with(psi_p, n, wf);
        fft_with(psi_m, n, wf);
        for (int f = 0; f < n; f++) { psi_p[f] *= pp[f]; psi_m[f] *= pm[f]; }
        fft_with(psi_p, n, wi);
        fft_with(psi_m, n, wi);
        /* real-space coupling at z_step */
        for (int j = 0; j < n; j++) {
            if (!inside_mask(d, j, step)) continue;
            double complex e = 1.0;
            if (d->strain_kind != ORACLE_STRAIN_NONE) {
                double phi = oracle_strain_phase(d, j, step);
                e = cos(phi) + I * sin(phi);
            }
            double complex p = psi_p[j], m = psi_m[j];
            psi_p[j] = sc.a0 * p + sc.ap * e * m;
            psi_m[j] = sc.a0 * m + sc.am * conj(e) * p;
        }
    }
    int lo = d->det_lo < 0 ? 0 : d->det_lo;
    int hi = d->det_hi > n ? n : d->det_hi;
    if (hi < lo) hi = lo;
    double r = 0.0, t = 0.0;
    if (pin > 0) {
        r = power_sum(psi_m, lo, hi) / pin;
        t = power_sum(psi_p, lo, hi) / pin;
    }
    if (R) *R = r;
    if (T) *T = t;
    free(pp);
    free(pm);
    free(wf);
    free(wi);
    return 0;
}

/* ------------------------------------------------------------- batch ------ */

typedef struct {
    const oracle_desc *descs;
    int n;
    double complex **psi;
    double *R, *T;
    int next;
    int status;
    pthread_mutex_t mu;
} batch_ctx;

static void *batch_worker(void *arg)
{
    batch_ctx *b = arg;
    for (;;) {
        pthread_mutex_lock(&b->mu);
        int i = b->next++;
        pthread_mutex_unlock(&b->mu);
        if (i >= b->n) break;
        int nx = b->descs[i].nx;
        int rc = oracle_propagate(&b->descs[i], b->psi[i], b->psi[i] + nx,
                                  b->R ? b->R + i : NULL, b->T ? b->T + i : NULL);
        if (rc) {
            pthread_mutex_lock(&b->mu);
            b->status = rc;
            pthread_mutex_unlock(&b->mu);
        }
    }
    return NULL;
}

int oracle_propagate_batch(const oracle_desc *descs, int n, double complex **psi,
                           double *R, double *T, int nthreads)
{
    if (n < 0 || nthreads < 1) return -1;
    batch_ctx b = {descs, n, psi, R, T, 0, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads > n) nthreads = n > 0 ? n : 1;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return -2;
    int started = 0;
    for (int i = 0; i < nthreads; i++)
        if (pthread_create(&th[i], NULL, batch_worker, &b) == 0) started++;
        else break;
    if (started == 0) batch_worker(&b);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
    return b.status;
}

/* ------------------------------------------------------------- time domain */

int oracle_td_assemble(const oracle_desc *descs, int M, const double complex *psi, double complex *out)
{
    if (M <= 0 || !descs || !psi || !out) return -1;
    int nx = descs[0].nx;
    for (int m = 0; m < M; m++)
        if (!desc_valid(&descs[m]) || descs[m].nx != nx) return -1;
    double complex *carrier = malloc(sizeof(double complex) * (size_t)M);
    double complex *w = malloc(sizeof(double complex) * (size_t)M);
    if (!carrier || !w) { free(carrier); free(w); return -2; }
    for (int m = 0; m < M; m++) {
        const oracle_desc *d = &descs[m];
        double k = 2.0 * M_PI / d->lambda_um;
        double s = d->lambda_um / (2.0 * d->d_um);
        double L = d->nz * d->dz_um;
        carrier[m] = cexp(I * k * sqrt(1.0 - s * s) * L);
    }
    for (int q = 0; q < M; q++) w[q] = cexp(-2.0 * M_PI * I * (double)q / (double)M);
    for (int b = 0; b < 2; b++)
        for (int j = 0; j < nx; j++)
            for (int k = 0; k < M; k++) {
                double complex acc = 0.0;
                for (int m = 0; m < M; m++)
                    acc += psi[((size_t)m * 2 + b) * nx + j] * carrier[m] * w[((long long)m * k) % M];
                out[((size_t)b * nx + j) * M + k] = acc;
            }
    free(carrier);
    free(w);
    return 0;
}
