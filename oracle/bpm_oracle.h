/*
 * bpm_oracle.h — TEST INFRASTRUCTURE.
 *
 * Plain, slow, FP64 CPU reference for the two-beam FFT beam-propagation march
 * (the split-step method of Eq. (4) in its two-envelope form, Eq. (12)).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load, call or link this code.  The product library never does
 * and shares no code, header or table with it.
 *
 * Conventions (the paper is silent on them; the readings are listed with the
 * tests that pin them):
 *   x_j = x0 + j*dx, j = 0..nx-1, periodic window;  z_n = n*dz, n = 0..nz-1.
 *   Forward DFT  X_f = sum_j x_j exp(-2*pi*i*j*f/nx), inverse with +i and 1/nx.
 *   Frequency of bin f: f for f < nx/2, f - nx otherwise (Nyquist negative).
 *   k = 2*pi/lambda, h = 2*pi/d, s = h/(2k) = sin(theta_B), c = sqrt(1-s^2),
 *   dzh = k*dz (the normalised step of Eq. (4)).
 *
 * One step n -> n+1 (split_order 0 or 1, Eq. (12)):
 *   psi_pm <- IDFT( DFT(psi_pm) * exp(i*dzh*(S(q +/- s) - c)) ),   S(p) = sqrt(1-p^2)
 *   inside the crystal mask at (x_j, z_n):
 *      psi_p <- a0*psi_p + ap*exp(+i*phi)*psi_m
 *      psi_m <- a0*psi_m + am*exp(-i*phi)*psi_p        (old values on the right)
 *   with phi = h*u(x_j, z_n) and a0, ap, am the n = 0, +1, -1 harmonics of
 *   exp(i*dzh*delta_eps/(2c)) (Eq. (8)-(11)).
 *
 * Higher orders (Eq. (13)): the step is the product A(a_1 dz) B(b_1 dz) ...
 * A(a_m dz) B(b_m dz), applied from the left, with A the propagation of a
 * sub-step and B the coupling of a sub-step, taken here as the exponential of
 * the two-beam coupling generator (the truncated Jacobi-Anger form does not
 * compose, B(b1) B(b2) != B(b1 + b2), and would leave every splitting first
 * order).  B_i uses the mask row of step n and the strain at
 * z_n + (a_1 + ... + a_i) dz.
 */
#ifndef BPM_ORACLE_H
#define BPM_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_STRAIN_NONE = 0,
    ORACLE_STRAIN_POLY2 = 1,       /* u = c0 + c1 X + c2 Z + c3 X^2 + c4 X Z + c5 Z^2 */
    ORACLE_STRAIN_EDGE_DISL = 2,   /* straight edge dislocation, line along y, b along h */
    ORACLE_STRAIN_TABLE = 3        /* u given at every (x_j, z_n) */
};

typedef struct oracle_desc {
    int nx, nz;
    double dx_um, dz_um, x0_um;
    double lambda_um, d_um;
    double chi0_re, chi0_im, chih_re, chih_im, chihb_re, chihb_im;
    int nseg;              /* mask intervals per step */
    const int *seg;        /* [nz][nseg][2] half-open [lo, hi) grid-index intervals */
    int strain_kind;
    double x_ref_um, z_ref_um;   /* X = x - x_ref, Z = z - z_ref */
    double strain_c[6];          /* POLY2 coefficients (um, um^-1, um^-1 ...) */
    double disl_b_um, disl_nu;   /* EDGE_DISL Burgers vector length and Poisson ratio */
    const double *u_table;       /* TABLE: [nz][nx] displacement along h (um) */
    int det_lo, det_hi;          /* detector interval for R and T */
    int split_order;             /* 0 or 1: Eq. (12); 2, 4: the splittings of Eq. (13) */
    int ny;                      /* 0 or 1: the x-z problem; > 1: 3D envelopes [ny][nx] */
    double dy_um;
} oracle_desc;

/* Plan-level scalars, exposed so that the tests can pin them. */
typedef struct oracle_scalars {
    double k, h, s, c, dzh;
    double complex a0, ap, am;
} oracle_scalars;

/* Iterative radix-2 DFT in place; sign = -1 forward, +1 inverse (unnormalised). */
int oracle_fft(double complex *a, int n, int sign);
/* Direct O(n^2) DFT, out of place. */
void oracle_dft(const double complex *in, double complex *out, int n, int sign);

/* Series for J0(w) and 2*J1(w)/w written in y = -w^2/4 (branch-free, complex y). */
void oracle_bessel_series(double complex y, double complex *j0, double complex *g);
/* Series cosh(v) = sum y^m/(2m)! and sinh(v)/v = sum y^m/(2m+1)! in y = v^2. */
void oracle_exp_series(double complex y, double complex *ch, double complex *sh);

/* Coupling coefficients of a sub-step of b*dz: form 0 = the Jacobi-Anger
 * harmonics of Eq. (9)-(10), form 1 = the exponential of the two-beam coupling
 * generator (used by the higher-order splittings). */
int oracle_coupling(const oracle_desc *d, double b, int form, double complex *a0, double complex *ap,
                    double complex *am);
/* Propagator tables of a sub-step of a*dz (a may be negative), 1/nx included. */
int oracle_propagator_frac(const oracle_desc *d, double a, double complex *pp, double complex *pm);
/* Step sequence of a splitting order: A(a_i dz) then B(b_i dz) for i = 0..count-1.
 * Returns the count (0 for an unknown order). */
int oracle_split_sequence(int order, double *a, double *b);
/* Strain phase phi = h*u at x_j and height z (TABLE: row n). */
double oracle_strain_phase_z(const oracle_desc *d, int j, int n, double z);

int oracle_scalars_get(const oracle_desc *d, oracle_scalars *out);
/* Propagator tables P+[f], P-[f] including the 1/nx of the inverse transform. */
int oracle_propagator(const oracle_desc *d, double complex *pp, double complex *pm);
/* Strain phase phi = h*u at grid point (j, n). */
double oracle_strain_phase(const oracle_desc *d, int j, int n);

/* Full march.  psi_p/psi_m hold the entrance envelopes and receive the exit ones.
 * R and T may be NULL.  Returns 0 or a negative error code. */
int oracle_propagate(const oracle_desc *d, double complex *psi_p, double complex *psi_m,
                     double *R, double *T);

/* 3D envelopes (ny > 1): psi_p and psi_m are [ny][nx]; each step propagates with
 * the 2D transform over (x, y) and exp(i dzh (S(qx +/- s, qy) - c)),
 * S(p, r) = sqrt(1 - p^2 - r^2), qy = 2 pi fy / (ny dy k), and couples at
 * (x_j, y_i, z): mask intervals along x per (step, row) [nz][ny][nseg][2],
 * POLY2 and edge-dislocation strain independent of y, TABLE strain [nz][ny][nx].
 * R and T sum the detector interval of every row.  oracle_propagate takes this
 * path when ny > 1; the 2D propagator tables are [ny][nx]. */
int oracle_propagator_2d(const oracle_desc *d, double a, double complex *pp, double complex *pm);

/* Time-domain assembly of M spectral components marched to their exit planes
 * z = L_m = nz_m dz_m (the time-dependent method of Sec. 8): for every x sample
 * and beam b,
 *   out[b][j][k] = sum_m psi[m][b][j] exp(i k_m c_m L_m) exp(-2 pi i m k / M),
 * the exponential restoring each component's carrier phase along z (the
 * constant the reduced propagator drops), k_m = 2 pi / lambda_m,
 * c_m = sqrt(1 - (lambda_m / 2 d_m)^2).  psi is [M][2][nx]; out is [2][nx][M].
 * A direct sum over m (no FFT). */
int oracle_td_assemble(const oracle_desc *descs, int M, const double complex *psi, double complex *out);

/* Many independent solves on a pool of nthreads POSIX threads (one solve per thread
 * at a time).  psi arrays are [n][2][nx] in the caller's packing: psi[i] points at
 * solve i's psi_p, followed by its psi_m. */
int oracle_propagate_batch(const oracle_desc *descs, int n, double complex **psi,
                           double *R, double *T, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
