/*
 * FP64 CPU oracle for the MR-STAT matrix-free Jacobian products.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library. It shares no code with
 * the HIP library and never assumes anything the GPU path assumes (it keeps
 * the general complex EPG states, computes every phase with cexp in FP64 and
 * never uses the real/imaginary structure of the states).
 *
 * Paper: van der Heide et al., "High resolution in-vivo MR-STAT using a
 * matrix-free and parallelized reconstruction algorithm", arXiv 1904.13244.
 * Citations below name the paper's sections, equations and algorithms.
 *
 * Parity status per routine (what pins it; the pins live in tests/):
 *   oracle_epg            isochromat brute force (S2 update, averaged over the
 *                         spoiler dephasing), Ernst transient, spin echo,
 *                         inversion recovery, central finite differences.
 *   oracle_signal_*       numpy FFT of the zero-padded image; Ex^H Ex = Nk I.
 *   oracle_jv / _jhw      explicit Jacobian built from finite differences of
 *                         the signal; adjoint identity.
 *   oracle_gn_step        dense solve of the normal equations on a tiny case;
 *                         noiseless exact recovery of the ground truth.
 *   oracle_rho_init       closed-form least-squares solution (uniform maps).
 *   oracle_steihaug_dense Galerkin solutions of successive Krylov spaces and
 *                         their monotone norms (boundary exit); the boundary
 *                         Cauchy point on an indefinite model (curvature exit).
 *   oracle_reflect        a particle bouncing between the walls, stepped in
 *                         small increments.
 *   oracle_tr_step        the ratio test from an explicit Jacobian; a model
 *                         that is exact (rho fitted alone) gives rho = 1.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops of this library use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static const double PI = 3.14159265358979323846;

static int nvox(const oracle_problem *p) { return p->nx * p->ny; }

/* ------------------------------------------------------------------------ */
/* EPG simulation of one voxel with forward-mode tangents.                   */
/*                                                                           */
/* The paper integrates isochromats (Supporting Information S2): an RF        */
/* rotation followed by T1/T2 decay and regrowth, started from equilibrium,   */
/* with tangents carried along by differentiating each update (forward-mode  */
/* algorithmic differentiation, zero initial tangents). Here the same steps   */
/* act on the extended-phase-graph states F+_k, F-_k, Z_k of a                */
/* gradient-spoiled sequence: the spoiler's dephasing becomes a shift of the  */
/* state orders, truncated at K states.                                       */
/* ------------------------------------------------------------------------ */

typedef struct { double complex fp, fm, z; } epg_state;

/* RF operator: rotation by angle a about the axis (cos phi, sin phi, 0),
 * written for (F+, F-, Z) with F = Mx + i My. dT is its derivative in a. */
static void rf_operator(double a, double phi, double complex T[3][3],
                        double complex dT[3][3])
{
    double c = cos(0.5 * a), s = sin(0.5 * a);
    double c2 = c * c, s2 = s * s, sa = sin(a), ca = cos(a);
    double dc2 = -0.5 * sa, ds2 = 0.5 * sa, dsa = ca, dca = -sa;
    double complex e1 = cexp(I * phi), e2 = cexp(2.0 * I * phi);

    T[0][0] = c2;                    T[0][1] = e2 * s2;              T[0][2] = -I * e1 * sa;
    T[1][0] = conj(e2) * s2;         T[1][1] = c2;                   T[1][2] = I * conj(e1) * sa;
    T[2][0] = -0.5 * I * conj(e1) * sa; T[2][1] = 0.5 * I * e1 * sa; T[2][2] = ca;

    dT[0][0] = dc2;                  dT[0][1] = e2 * ds2;            dT[0][2] = -I * e1 * dsa;
    dT[1][0] = conj(e2) * ds2;       dT[1][1] = dc2;                 dT[1][2] = I * conj(e1) * dsa;
    dT[2][0] = -0.5 * I * conj(e1) * dsa; dT[2][1] = 0.5 * I * e1 * dsa; dT[2][2] = dca;
}

static epg_state apply3(const double complex M[3][3], epg_state x)
{
    epg_state y;
    y.fp = M[0][0] * x.fp + M[0][1] * x.fm + M[0][2] * x.z;
    y.fm = M[1][0] * x.fp + M[1][1] * x.fm + M[1][2] * x.z;
    y.z  = M[2][0] * x.fp + M[2][1] * x.fm + M[2][2] * x.z;
    return y;
}

/* x: value states [K]; dx[q]: tangent states [K] for q = lnT1, lnT2, B1. */
typedef struct {
    int K;
    epg_state *x;
    epg_state *dx[3];
} epg_voxel;

/* RF pulse of angle a = B1 * alpha_rad; dT/dB1 = alpha_rad * dT/da. */
static void epg_rf(epg_voxel *v, double B1, double alpha_rad, double phi, int tang)
{
    double complex T[3][3], dTa[3][3];
    rf_operator(B1 * alpha_rad, phi, T, dTa);
    for (int k = 0; k < v->K; ++k) {
        epg_state old = v->x[k];
        if (tang) {
            v->dx[0][k] = apply3(T, v->dx[0][k]);
            v->dx[1][k] = apply3(T, v->dx[1][k]);
            epg_state t = apply3(T, v->dx[2][k]);
            epg_state u = apply3(dTa, old);
            v->dx[2][k].fp = t.fp + alpha_rad * u.fp;
            v->dx[2][k].fm = t.fm + alpha_rad * u.fm;
            v->dx[2][k].z  = t.z  + alpha_rad * u.z;
        }
        v->x[k] = apply3(T, old);
    }
}

/* Free relaxation over tau: transverse decay E2, longitudinal decay E1 and
 * regrowth (1 - E1) of Z_0 (the decay/regrowth update of S2). Tangents:
 * dE1/dlnT1 = (tau/T1) E1, d(1-E1)/dlnT1 = -(tau/T1) E1, dE2/dlnT2 = (tau/T2) E2. */
static void epg_relax(epg_voxel *v, double tau, double T1, double T2, int tang)
{
    if (tau <= 0.0) return;
    double E1 = exp(-tau / T1), E2 = exp(-tau / T2);
    double R = -expm1(-tau / T1);
    double dE1 = (tau / T1) * E1, dE2 = (tau / T2) * E2;
    for (int k = 0; k < v->K; ++k) {
        epg_state old = v->x[k];
        if (tang) {
            /* ln T1 */
            v->dx[0][k].fp = E2 * v->dx[0][k].fp;
            v->dx[0][k].fm = E2 * v->dx[0][k].fm;
            v->dx[0][k].z  = E1 * v->dx[0][k].z + dE1 * old.z - (k == 0 ? dE1 : 0.0);
            /* ln T2 */
            v->dx[1][k].fp = E2 * v->dx[1][k].fp + dE2 * old.fp;
            v->dx[1][k].fm = E2 * v->dx[1][k].fm + dE2 * old.fm;
            v->dx[1][k].z  = E1 * v->dx[1][k].z;
            /* B1 */
            v->dx[2][k].fp = E2 * v->dx[2][k].fp;
            v->dx[2][k].fm = E2 * v->dx[2][k].fm;
            v->dx[2][k].z  = E1 * v->dx[2][k].z;
        }
        v->x[k].fp = E2 * old.fp;
        v->x[k].fm = E2 * old.fm;
        v->x[k].z  = E1 * old.z + (k == 0 ? R : 0.0);
    }
}

/* Spoiler gradient: every order moves up by one; orders >= K are dropped and
 * the new F+_0 is the conjugate of the new F-_0. */
static void epg_shift_one(epg_state *x, int K)
{
    for (int k = K - 1; k >= 1; --k) x[k].fp = x[k - 1].fp;
    for (int k = 0; k < K - 1; ++k) x[k].fm = x[k + 1].fm;
    x[K - 1].fm = 0.0;
    x[0].fp = conj(x[0].fm);
}

static void epg_simulate_voxel(const oracle_problem *p, double lnT1, double lnT2,
                               double B1, int tang, double complex *m,
                               double complex *dm1, double complex *dm2,
                               double complex *dm3, size_t stride)
{
    const int K = p->n_states;
    epg_state *buf = (epg_state *)calloc((size_t)4 * K, sizeof(epg_state));
    epg_voxel v;
    v.K = K;
    v.x = buf;
    for (int q = 0; q < 3; ++q) v.dx[q] = buf + (size_t)(q + 1) * K;
    double T1 = exp(lnT1), T2 = exp(lnT2);

    /* Equilibrium start (S2): Z_0 = 1; all tangents zero. */
    v.x[0].z = 1.0;
    /* Ideal non-selective inversion at the start (Methods, Pulse Sequence). */
    v.x[0].z = -v.x[0].z;
    epg_relax(&v, p->t_inv, T1, T2, tang);

    for (int n = 0; n < p->n_tr; ++n) {
        double alpha = p->flip_deg[n] * PI / 180.0;
        double phi = p->rf_phase ? p->rf_phase[n] : 0.0;
        epg_rf(&v, B1, alpha, phi, tang);
        epg_relax(&v, p->te, T1, T2, tang);
        /* Receiver demodulated by the RF phase. */
        double complex dem = cexp(-I * phi);
        m[(size_t)n * stride] = v.x[0].fp * dem;
        if (tang) {
            dm1[(size_t)n * stride] = v.dx[0][0].fp * dem;
            dm2[(size_t)n * stride] = v.dx[1][0].fp * dem;
            dm3[(size_t)n * stride] = v.dx[2][0].fp * dem;
        }
        epg_relax(&v, p->tr - p->te, T1, T2, tang);
        epg_shift_one(v.x, K);
        if (tang)
            for (int q = 0; q < 3; ++q) epg_shift_one(v.dx[q], K);
    }
    free(buf);
}

/* ------------------------------------------------------------------------ */
/* Balanced isochromat model (Supporting Information S2). Each isochromat is   */
/* a vector m = (mx, my, mz). The RF of TR n rotates it by theta = B1 alpha_n  */
/* scale about k = (cos phi_n, sin phi_n, 0) (Rodrigues: m cos theta +          */
/* (k x m) sin theta + (k . m) k (1 - cos theta)); decay and regrowth over      */
/* tau multiply (mx, my) by E2 and mz by E1 and add 1 - E1 to mz. With a        */
/* balanced sequence on resonance nothing else moves the magnetisation.        */
/* Tangents in ln T1, ln T2 and B1 are carried through both updates in          */
/* forward mode (zero at the start).                                           */
/* ------------------------------------------------------------------------ */

typedef struct { double v[3]; } vec3;

static vec3 rodrigues(vec3 m, const double k[3], double c, double s)
{
    double kdm = k[0] * m.v[0] + k[1] * m.v[1] + k[2] * m.v[2];
    double cr[3] = {k[1] * m.v[2] - k[2] * m.v[1], k[2] * m.v[0] - k[0] * m.v[2],
                    k[0] * m.v[1] - k[1] * m.v[0]};
    vec3 o;
    for (int i = 0; i < 3; ++i) o.v[i] = c * m.v[i] + s * cr[i] + (1.0 - c) * kdm * k[i];
    return o;
}

/* d/dtheta of the rotated vector for fixed m: -s m + c (k x m) + s (k . m) k. */
static vec3 rodrigues_dtheta(vec3 m, const double k[3], double c, double s)
{
    double kdm = k[0] * m.v[0] + k[1] * m.v[1] + k[2] * m.v[2];
    double cr[3] = {k[1] * m.v[2] - k[2] * m.v[1], k[2] * m.v[0] - k[0] * m.v[2],
                    k[0] * m.v[1] - k[1] * m.v[0]};
    vec3 o;
    for (int i = 0; i < 3; ++i) o.v[i] = -s * m.v[i] + c * cr[i] + s * kdm * k[i];
    return o;
}

/* Decay and regrowth over tau with tangents d[0] (ln T1), d[1] (ln T2),
 * d[2] (B1). */
static void iso_relax(vec3 *m, vec3 d[3], double tau, double T1, double T2, int tang)
{
    double E1 = exp(-tau / T1), E2 = exp(-tau / T2);
    double dE1 = (tau / T1) * E1, dE2 = (tau / T2) * E2;   /* d/dlnT1 E1, d/dlnT2 E2 */
    if (tang) {
        for (int q = 0; q < 3; ++q) {
            d[q].v[0] *= E2;
            d[q].v[1] *= E2;
            d[q].v[2] *= E1;
        }
        d[0].v[2] += dE1 * (m->v[2] - 1.0);   /* d(E1 mz + 1 - E1)/dlnT1 */
        d[1].v[0] += dE2 * m->v[0];
        d[1].v[1] += dE2 * m->v[1];
    }
    m->v[0] *= E2;
    m->v[1] *= E2;
    m->v[2] = E1 * m->v[2] + (1.0 - E1);
}

void oracle_isochromat(const oracle_problem *p, double lnT1, double lnT2, double B1, double scale,
                       double complex *m, double complex *dm1, double complex *dm2,
                       double complex *dm3)
{
    const int tang = dm1 != NULL;
    double T1 = exp(lnT1), T2 = exp(lnT2);
    vec3 x = {{0.0, 0.0, 1.0}};          /* equilibrium (S2) */
    vec3 d[3] = {{{0, 0, 0}}, {{0, 0, 0}}, {{0, 0, 0}}};
    x.v[2] = -x.v[2];                    /* ideal non-selective inversion */
    iso_relax(&x, d, p->t_inv, T1, T2, tang);
    for (int n = 0; n < p->n_tr; ++n) {
        double phi = p->rf_phase ? p->rf_phase[n] : 0.0;
        double k[3] = {cos(phi), sin(phi), 0.0};
        double a = p->flip_deg[n] * PI / 180.0 * scale;   /* d theta / d B1 */
        double th = B1 * a, c = cos(th), s = sin(th);
        if (tang) {
            vec3 dB = rodrigues_dtheta(x, k, c, s);
            for (int q = 0; q < 3; ++q) d[q] = rodrigues(d[q], k, c, s);
            for (int i = 0; i < 3; ++i) d[2].v[i] += a * dB.v[i];
        }
        x = rodrigues(x, k, c, s);
        iso_relax(&x, d, p->te, T1, T2, tang);
        double complex dem = cexp(-I * phi);
        m[n] = (x.v[0] + I * x.v[1]) * dem;
        if (tang) {
            dm1[n] = (d[0].v[0] + I * d[0].v[1]) * dem;
            dm2[n] = (d[1].v[0] + I * d[1].v[1]) * dem;
            dm3[n] = (d[2].v[0] + I * d[2].v[1]) * dem;
        }
        iso_relax(&x, d, p->tr - p->te, T1, T2, tang);
    }
}

/* Voxel trains of the balanced model: the weighted sum over the isochromats
 * of the slice profile. */
static void iso_simulate_voxel(const oracle_problem *p, double lnT1, double lnT2, double B1,
                               int tang, double complex *m, double complex *dm1,
                               double complex *dm2, double complex *dm3, size_t stride)
{
    const int T = p->n_tr;
    double complex *b = (double complex *)malloc((size_t)4 * T * sizeof(double complex));
    for (int n = 0; n < T; ++n) {
        m[(size_t)n * stride] = 0.0;
        if (tang) dm1[(size_t)n * stride] = dm2[(size_t)n * stride] = dm3[(size_t)n * stride] = 0.0;
    }
    for (int q = 0; q < p->n_iso; ++q) {
        oracle_isochromat(p, lnT1, lnT2, B1, p->iso_scale[q], b, tang ? b + T : NULL, b + 2 * T, b + 3 * T);
        double w = p->iso_weight[q];
        for (int n = 0; n < T; ++n) {
            m[(size_t)n * stride] += w * b[n];
            if (tang) {
                dm1[(size_t)n * stride] += w * b[T + n];
                dm2[(size_t)n * stride] += w * b[2 * T + n];
                dm3[(size_t)n * stride] += w * b[3 * T + n];
            }
        }
    }
    free(b);
}

void oracle_epg(const oracle_problem *p, const double *theta, int with_tangents,
                double complex *trains)
{
    const int Nv = nvox(p);
    const size_t plane = (size_t)p->n_tr * Nv;
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < Nv; ++j) {
        if (p->n_iso > 0)
            iso_simulate_voxel(p, theta[j], theta[Nv + j], theta[2 * Nv + j], with_tangents,
                               trains + j, trains + plane + j, trains + 2 * plane + j,
                               trains + 3 * plane + j, (size_t)Nv);
        else
            epg_simulate_voxel(p, theta[j], theta[Nv + j], theta[2 * Nv + j], with_tangents,
                               trains + j, trains + plane + j, trains + 2 * plane + j,
                               trains + 3 * plane + j, (size_t)Nv);
    }
}

/* ------------------------------------------------------------------------ */
/* Encoding. Voxel positions x = ix - nx/2, y = iy - ny/2 (voxel units);      */
/* readout sample k has kx = (k - n_read/2)/n_read cycles per voxel, TR n     */
/* samples phase-encode line ky = (l(n) - ny/2)/ny. E = exp(-2 pi i k.r).     */
/* A non-Cartesian problem gives (kx, ky) per sample in cycles per field of   */
/* view instead; its sums are taken directly over the voxels.                 */
/* ------------------------------------------------------------------------ */

static int non_cartesian(const oracle_problem *p) { return p->kx != NULL; }

/* Readout dynamics (see oracle_problem): on when samples carry the factor
 * exp(-tau_k / T2_j) exp(-2 pi i db0_j (TE + tau_k)). */
static int readout_on(const oracle_problem *p)
{
    return p->dwell != 0.0 || p->db0 != NULL || p->db0_unit > 0.0;
}

/* Parameters per voxel: 5, or 6 with Delta B0 reconstructed. */
static int npar(const oracle_problem *p) { return p->db0_unit > 0.0 ? 6 : 5; }

/* Off-resonance of voxel j in Hz: the fitted row, the given map, or 0. */
static double db0_of(const oracle_problem *p, const double *theta, int j)
{
    if (p->db0_unit > 0.0) return theta[(size_t)5 * p->nx * p->ny + j] * p->db0_unit;
    return p->db0 ? p->db0[j] : 0.0;
}

static double readout_tau(const oracle_problem *p, int k)
{
    return (double)(k - p->n_read / 2) * p->dwell;
}

/* The factor of voxel j at sample k (1 when readout dynamics are off). */
static double complex readout_factor(const oracle_problem *p, const double *theta, int j, int k)
{
    if (!readout_on(p)) return 1.0;
    const int Nv = p->nx * p->ny;
    const double tau = readout_tau(p, k);
    const double r2 = exp(-theta[(size_t)Nv + j]);   /* 1 / T2, theta row 1 = ln T2 */
    const double f = db0_of(p, theta, j);
    return cexp(-tau * r2 - 2.0 * PI * I * f * (p->te + tau));
}

static double complex phase_x(const oracle_problem *p, int k, int ix)
{
    double kx = (double)(k - p->n_read / 2) / (double)p->n_read;
    return cexp(-2.0 * PI * I * kx * (double)(ix - p->nx / 2));
}

static double complex phase_y(const oracle_problem *p, int n, int iy)
{
    double ky = (double)(p->ky_line[n] - p->ny / 2) / (double)p->ny;
    return cexp(-2.0 * PI * I * ky * (double)(iy - p->ny / 2));
}

double complex oracle_phase(const oracle_problem *p, int n, int k, int ix, int iy)
{
    if (non_cartesian(p)) {
        size_t s = (size_t)n * p->n_read + k;
        return cexp(-2.0 * PI * I * (p->kx[s] * (double)(ix - p->nx / 2) / (double)p->nx +
                                     p->ky[s] * (double)(iy - p->ny / 2) / (double)p->ny));
    }
    double kx = (double)(k - p->n_read / 2) / (double)p->n_read;
    double ky = (double)(p->ky_line[n] - p->ny / 2) / (double)p->ny;
    return cexp(-2.0 * PI * I * (kx * (double)(ix - p->nx / 2) +
                                 ky * (double)(iy - p->ny / 2)));
}

void oracle_phases(const oracle_problem *p, int n, double complex *out)
{
    const int Nv = nvox(p);
    for (int k = 0; k < p->n_read; ++k)
        for (int j = 0; j < Nv; ++j)
            out[(size_t)k * Nv + j] = oracle_phase(p, n, k, j % p->nx, j / p->nx);
}

static double complex coil_at(const double complex *coil, int c, int Nv, int j)
{
    return coil ? coil[(size_t)c * Nv + j] : 1.0;
}

static int active(const unsigned char *mask, int j) { return mask ? mask[j] != 0 : 1; }

static double complex rho_of(const double *theta, int Nv, int j)
{
    return theta[3 * (size_t)Nv + j] + I * theta[4 * (size_t)Nv + j];
}

/* D_q[n,j] = d(rho_j m_j[n]) / d alpha_{q,j} (Theory: dr/dalpha_i involves only
 * voxel j's rho_j m_j): q<3 -> rho dm/dtheta_q, q=3 -> m, q=4 -> i m. With
 * readout dynamics the sample's derivative of rho m F is F (D_q + tau_k D'_q):
 * q=5 (Delta B0) has D_5 = -2 pi i db0_unit TE rho m here and its tau part in
 * dcol_tau. */
static double complex dcol(const oracle_problem *p, const double *theta, const double complex *trains,
                           int q, int n, int j)
{
    const int Nv = nvox(p);
    const size_t plane = (size_t)p->n_tr * Nv;
    double complex m = trains[(size_t)n * Nv + j];
    switch (q) {
    case 0: case 1: case 2:
        return rho_of(theta, Nv, j) * trains[(size_t)(q + 1) * plane + (size_t)n * Nv + j];
    case 3: return m;
    case 4: return I * m;
    default: return -2.0 * PI * I * p->db0_unit * p->te * rho_of(theta, Nv, j) * m;
    }
}

/* D'_q: the factor of tau_k in the readout dynamics' share of the derivative.
 * d/dlnT2 exp(-tau / T2) = (tau / T2) exp(-tau / T2) gives D'_1 = rho m / T2;
 * d/dtheta_5 exp(-2 pi i db0 (TE + tau)) gives D'_5 = -2 pi i db0_unit rho m;
 * the other parameters do not enter the factor. */
static double complex dcol_tau(const oracle_problem *p, const double *theta, const double complex *trains,
                               int q, int n, int j)
{
    const int Nv = nvox(p);
    const double complex rm = rho_of(theta, Nv, j) * trains[(size_t)n * Nv + j];
    if (q == 1) return rm * exp(-theta[(size_t)Nv + j]);
    if (q == 5) return -2.0 * PI * I * p->db0_unit * rm;
    return 0.0;
}

void oracle_signal_direct(const oracle_problem *p, const double *theta,
                          const double complex *coil, const unsigned char *mask,
                          const double complex *trains, double complex *s)
{
    const int Nv = nvox(p);
    const int rows = p->n_coils * p->n_tr;
#pragma omp parallel for schedule(dynamic, 1)
    for (int row = 0; row < rows; ++row) {
        int c = row / p->n_tr, n = row % p->n_tr;
        for (int k = 0; k < p->n_read; ++k) {
            double complex acc = 0.0;
            for (int j = 0; j < Nv; ++j) {
                if (!active(mask, j)) continue;
                int ix = j % p->nx, iy = j / p->nx;
                acc += coil_at(coil, c, Nv, j) * rho_of(theta, Nv, j) *
                       trains[(size_t)n * Nv + j] * oracle_phase(p, n, k, ix, iy) *
                       readout_factor(p, theta, j, k);
            }
            s[(size_t)row * p->n_read + k] = acc;
        }
    }
}

/* s_c[n,k] = sum_ix Ex[k,ix] sum_iy Ey[n,iy] x_c[n,j] for x given per voxel by
 * a weight function; shared by the signal and J v. */
typedef double complex (*voxel_value_fn)(const void *ctx, int n, int j);

/* The same sum taken directly over the voxels with the phase of each sample
 * (any trajectory). */
static void encode_direct(const oracle_problem *p, const double complex *coil,
                          const unsigned char *mask, voxel_value_fn xval,
                          const void *ctx, double complex *s)
{
    const int Nv = nvox(p), C = p->n_coils;
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < p->n_tr; ++n) {
        double complex *x = (double complex *)malloc((size_t)Nv * sizeof(double complex));
        for (int j = 0; j < Nv; ++j) x[j] = active(mask, j) ? xval(ctx, n, j) : 0.0;
        for (int c = 0; c < C; ++c)
            for (int k = 0; k < p->n_read; ++k) {
                double complex acc = 0.0;
                for (int j = 0; j < Nv; ++j)
                    if (active(mask, j))
                        acc += coil_at(coil, c, Nv, j) * x[j] *
                               oracle_phase(p, n, k, j % p->nx, j / p->nx);
                s[((size_t)c * p->n_tr + n) * p->n_read + k] = acc;
            }
        free(x);
    }
}

/* With readout dynamics every sample has its own factor per voxel:
 * s_c[n,k] = sum_j C_c[j] (x0[n,j] + tau_k x1[n,j]) F[k,j] E[n,k,j], F the
 * readout factor; x1 carries the readout decay's share of the ln T2 column
 * (zero for the signal). Direct sum. */
static void encode_readout(const oracle_problem *p, const double *theta, const double complex *coil,
                           const unsigned char *mask, voxel_value_fn x0val, voxel_value_fn x1val,
                           const void *ctx, double complex *s)
{
    const int Nv = nvox(p), C = p->n_coils;
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < p->n_tr; ++n) {
        double complex *x0 = (double complex *)malloc((size_t)Nv * sizeof(double complex));
        double complex *x1 = (double complex *)malloc((size_t)Nv * sizeof(double complex));
        for (int j = 0; j < Nv; ++j) {
            x0[j] = active(mask, j) ? x0val(ctx, n, j) : 0.0;
            x1[j] = (active(mask, j) && x1val) ? x1val(ctx, n, j) : 0.0;
        }
        for (int c = 0; c < C; ++c)
            for (int k = 0; k < p->n_read; ++k) {
                const double tau = readout_tau(p, k);
                double complex acc = 0.0;
                for (int j = 0; j < Nv; ++j)
                    if (active(mask, j))
                        acc += coil_at(coil, c, Nv, j) * (x0[j] + tau * x1[j]) *
                               readout_factor(p, theta, j, k) * oracle_phase(p, n, k, j % p->nx, j / p->nx);
                s[((size_t)c * p->n_tr + n) * p->n_read + k] = acc;
            }
        free(x0);
        free(x1);
    }
}

static void encode_separable(const oracle_problem *p, const double complex *coil,
                             const unsigned char *mask, voxel_value_fn xval,
                             const void *ctx, double complex *s)
{
    const int Nv = nvox(p), C = p->n_coils;
    if (non_cartesian(p)) {
        encode_direct(p, coil, mask, xval, ctx, s);
        return;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < p->n_tr; ++n) {
        double complex *U = (double complex *)calloc((size_t)C * p->nx, sizeof(double complex));
        for (int iy = 0; iy < p->ny; ++iy) {
            double complex ey = phase_y(p, n, iy);
            for (int ix = 0; ix < p->nx; ++ix) {
                int j = iy * p->nx + ix;
                if (!active(mask, j)) continue;
                double complex x = xval(ctx, n, j);
                for (int c = 0; c < C; ++c)
                    U[(size_t)c * p->nx + ix] += ey * coil_at(coil, c, Nv, j) * x;
            }
        }
        for (int c = 0; c < C; ++c)
            for (int k = 0; k < p->n_read; ++k) {
                double complex acc = 0.0;
                for (int ix = 0; ix < p->nx; ++ix)
                    acc += phase_x(p, k, ix) * U[(size_t)c * p->nx + ix];
                s[((size_t)c * p->n_tr + n) * p->n_read + k] = acc;
            }
        free(U);
    }
}

typedef struct {
    const oracle_problem *p;
    const double *theta;
    const double complex *trains;
    const double *v;
} xval_ctx;

static double complex xval_signal(const void *vc, int n, int j)
{
    const xval_ctx *c = (const xval_ctx *)vc;
    int Nv = nvox(c->p);
    return rho_of(c->theta, Nv, j) * c->trains[(size_t)n * Nv + j];
}

void oracle_signal_separable(const oracle_problem *p, const double *theta,
                             const double complex *coil, const unsigned char *mask,
                             const double complex *trains, double complex *s)
{
    xval_ctx c = {p, theta, trains, NULL};
    if (readout_on(p))
        encode_readout(p, theta, coil, mask, xval_signal, NULL, &c, s);
    else
        encode_separable(p, coil, mask, xval_signal, &c, s);
}

/* J v = -(d s / d alpha) v (Theory: dr/dalpha_i = -d(rho_j m_j)/dalpha_i). */
static double complex xval_jv(const void *vc, int n, int j)
{
    const xval_ctx *c = (const xval_ctx *)vc;
    int Nv = nvox(c->p);
    double complex acc = 0.0;
    for (int q = 0; q < npar(c->p); ++q)
        acc += dcol(c->p, c->theta, c->trains, q, n, j) * c->v[(size_t)q * Nv + j];
    return acc;
}

/* The readout dynamics' share of J v: sum_q D'_q v_q (the ln T2 and Delta B0
 * columns), multiplied by tau_k in the encoding. */
static double complex xval_jv_tau(const void *vc, int n, int j)
{
    const xval_ctx *c = (const xval_ctx *)vc;
    int Nv = nvox(c->p);
    double complex acc = 0.0;
    for (int q = 0; q < npar(c->p); ++q)
        acc += dcol_tau(c->p, c->theta, c->trains, q, n, j) * c->v[(size_t)q * Nv + j];
    return acc;
}

void oracle_jv(const oracle_problem *p, const double *theta,
               const double complex *coil, const unsigned char *mask,
               const double complex *trains, const double *v, double complex *out)
{
    xval_ctx c = {p, theta, trains, v};
    if (readout_on(p))
        encode_readout(p, theta, coil, mask, xval_jv, xval_jv_tau, &c, out);
    else
        encode_separable(p, coil, mask, xval_jv, &c, out);
    size_t total = (size_t)p->n_coils * p->n_tr * p->n_read;
    for (size_t i = 0; i < total; ++i) out[i] = -out[i];
}

/* V[n][j] = sum_c conj(C_c[j]) sum_k conj(E[n,k,j]) w_c[n,k] (adjoint of the
 * encoding), evaluated as the x-sum then the y-phase. V is [n_tr][Nv]. */
static void adjoint_encode(const oracle_problem *p, const double *theta, const double complex *coil,
                           const unsigned char *mask, const double complex *w,
                           double complex *V, double complex *Vtau)
{
    const int Nv = nvox(p), C = p->n_coils;
    if (readout_on(p)) {
        /* V[n][j] = sum_c conj(C_c[j]) sum_k conj(F[k,j] E[n,k,j]) w_c[n,k] and,
         * when Vtau is given, the same sum with tau_k in each term. */
#pragma omp parallel for schedule(dynamic, 1)
        for (int n = 0; n < p->n_tr; ++n)
            for (int j = 0; j < Nv; ++j) {
                double complex acc = 0.0, acct = 0.0;
                if (active(mask, j))
                    for (int c = 0; c < C; ++c) {
                        double complex sc = 0.0, sct = 0.0;
                        for (int k = 0; k < p->n_read; ++k) {
                            const double complex t = conj(readout_factor(p, theta, j, k) *
                                                          oracle_phase(p, n, k, j % p->nx, j / p->nx)) *
                                                     w[((size_t)c * p->n_tr + n) * p->n_read + k];
                            sc += t;
                            sct += readout_tau(p, k) * t;
                        }
                        acc += conj(coil_at(coil, c, Nv, j)) * sc;
                        acct += conj(coil_at(coil, c, Nv, j)) * sct;
                    }
                V[(size_t)n * Nv + j] = acc;
                if (Vtau) Vtau[(size_t)n * Nv + j] = acct;
            }
        return;
    }
    if (Vtau)   /* no readout dynamics: tau plays no part */
        for (size_t i = 0; i < (size_t)p->n_tr * Nv; ++i) Vtau[i] = 0.0;
    if (non_cartesian(p)) {
        /* Direct: V[n][j] = sum_c conj(C_c[j]) sum_k conj(E[n,k,j]) w_c[n,k]. */
#pragma omp parallel for schedule(dynamic, 1)
        for (int n = 0; n < p->n_tr; ++n)
            for (int j = 0; j < Nv; ++j) {
                double complex acc = 0.0;
                if (active(mask, j))
                    for (int c = 0; c < C; ++c) {
                        double complex sc = 0.0;
                        for (int k = 0; k < p->n_read; ++k)
                            sc += conj(oracle_phase(p, n, k, j % p->nx, j / p->nx)) *
                                  w[((size_t)c * p->n_tr + n) * p->n_read + k];
                        acc += conj(coil_at(coil, c, Nv, j)) * sc;
                    }
                V[(size_t)n * Nv + j] = acc;
            }
        return;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < p->n_tr; ++n) {
        double complex *W = (double complex *)calloc((size_t)C * p->nx, sizeof(double complex));
        for (int c = 0; c < C; ++c)
            for (int ix = 0; ix < p->nx; ++ix) {
                double complex acc = 0.0;
                for (int k = 0; k < p->n_read; ++k)
                    acc += conj(phase_x(p, k, ix)) * w[((size_t)c * p->n_tr + n) * p->n_read + k];
                W[(size_t)c * p->nx + ix] = acc;
            }
        for (int iy = 0; iy < p->ny; ++iy) {
            double complex eyc = conj(phase_y(p, n, iy));
            for (int ix = 0; ix < p->nx; ++ix) {
                int j = iy * p->nx + ix;
                double complex acc = 0.0;
                if (active(mask, j))
                    for (int c = 0; c < C; ++c)
                        acc += conj(coil_at(coil, c, Nv, j)) * W[(size_t)c * p->nx + ix];
                V[(size_t)n * Nv + j] = eyc * acc;
            }
        }
        free(W);
    }
}

/* g[q,j] = Re <dr/dalpha_{q,j}, w> = -Re sum_n conj(D_q[n,j]) V[n,j]
 * (Theory, gradient section; Algorithm 4 computes all N_p partials of a voxel
 * together). */
void oracle_jhw(const oracle_problem *p, const double *theta,
                const double complex *coil, const unsigned char *mask,
                const double complex *trains, const double complex *w, double *out)
{
    const int Nv = nvox(p);
    double complex *V = (double complex *)malloc((size_t)p->n_tr * Nv * sizeof(double complex));
    double complex *Vt = (double complex *)malloc((size_t)p->n_tr * Nv * sizeof(double complex));
    adjoint_encode(p, theta, coil, mask, w, V, Vt);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < Nv; ++j) {
        for (int q = 0; q < npar(p); ++q) {
            double complex acc = 0.0;
            if (active(mask, j))
                for (int n = 0; n < p->n_tr; ++n)   /* V' holds the tau-weighted sums */
                    acc += conj(dcol(p, theta, trains, q, n, j)) * V[(size_t)n * Nv + j] +
                           conj(dcol_tau(p, theta, trains, q, n, j)) * Vt[(size_t)n * Nv + j];
            out[(size_t)q * Nv + j] = -creal(acc);
        }
    }
    free(V);
    free(Vt);
}

void oracle_jacobian(const oracle_problem *p, const double *theta,
                     const double complex *coil, const unsigned char *mask,
                     const double complex *trains, double complex *J)
{
    const int Nv = nvox(p);
    const int rows = p->n_coils * p->n_tr * p->n_read;
    const size_t cols = (size_t)npar(p) * Nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int row = 0; row < rows; ++row) {
        int k = row % p->n_read;
        int n = (row / p->n_read) % p->n_tr;
        int c = row / (p->n_read * p->n_tr);
        for (int q = 0; q < npar(p); ++q)
            for (int j = 0; j < Nv; ++j) {
                double complex e = 0.0;
                if (active(mask, j)) {
                    int ix = j % p->nx, iy = j / p->nx;
                    double complex d = dcol(p, theta, trains, q, n, j);
                    if (readout_on(p)) d += dcol_tau(p, theta, trains, q, n, j) * readout_tau(p, k);
                    e = -coil_at(coil, c, Nv, j) * oracle_phase(p, n, k, ix, iy) *
                        readout_factor(p, theta, j, k) * d;
                }
                J[(size_t)row * cols + (size_t)q * Nv + j] = e;
            }
    }
}

static size_t data_len(const oracle_problem *p)
{
    return (size_t)p->n_coils * p->n_tr * p->n_read;
}

static size_t train_len(const oracle_problem *p)
{
    return (size_t)4 * p->n_tr * nvox(p);
}

double oracle_residual(const oracle_problem *p, const double *theta,
                       const double complex *coil, const unsigned char *mask,
                       const double complex *data, double complex *r)
{
    const size_t L = data_len(p);
    double complex *tr = (double complex *)malloc(train_len(p) * sizeof(double complex));
    double complex *s = (double complex *)malloc(L * sizeof(double complex));
    oracle_epg(p, theta, 0, tr);
    oracle_signal_separable(p, theta, coil, mask, tr, s);
    double f = 0.0;
    for (size_t i = 0; i < L; ++i) {
        double complex ri = data[i] - s[i];
        if (r) r[i] = ri;
        f += creal(ri) * creal(ri) + cimag(ri) * cimag(ri);
    }
    free(tr);
    free(s);
    return 0.5 * f;
}

/* ------------------------------------------------------------------------ */
/* Inexact Gauss-Newton (Algorithm 6 with eq. 4 solved by a fixed number of  */
/* CG iterations), globalised by backtracking on f with projection onto the  */
/* parameter box.                                                            */
/* ------------------------------------------------------------------------ */

static double dot(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void apply_masks(const oracle_problem *p, double *x, int param_mask, const unsigned char *mask)
{
    const int Nv = nvox(p);
    for (int q = 0; q < npar(p); ++q)
        for (int j = 0; j < Nv; ++j)
            if (!((param_mask >> q) & 1) || !active(mask, j)) x[(size_t)q * Nv + j] = 0.0;
}

/* Box of parameter row q (ln T1, ln T2, B1 from the options; a fitted
 * Delta B0 within +-db0_box Hz); 0 for the unbounded rows. */
static int box_of(const oracle_problem *p, const double *lo3, const double *hi3, int q,
                  double *lo, double *hi)
{
    if (q < 3) {
        *lo = lo3[q];
        *hi = hi3[q];
        return 1;
    }
    if (q == 5 && p->db0_box > 0.0) {
        *hi = p->db0_box / p->db0_unit;
        *lo = -*hi;
        return 1;
    }
    return 0;
}

/* Box projection of the reconstructed (active) bounded entries onto their
 * intervals; inactive parameters and masked voxels are left as they are. */
static void project(const oracle_problem *p, double *theta, const oracle_gn_opts *o, const unsigned char *mask)
{
    const int Nv = nvox(p);
    for (int q = 0; q < npar(p); ++q) {
        double lo, hi;
        if (!box_of(p, o->lo, o->hi, q, &lo, &hi)) continue;
        for (int j = 0; j < Nv; ++j) {
            if (!((o->param_mask >> q) & 1) || !active(mask, j)) continue;
            double *t = &theta[(size_t)q * Nv + j];
            if (*t < lo) *t = lo;
            if (*t > hi) *t = hi;
        }
    }
}

void oracle_gn_step(const oracle_problem *p, double *theta,
                    const double complex *coil, const unsigned char *mask,
                    const double complex *data, const oracle_gn_opts *o,
                    oracle_gn_report *rep)
{
    const int Nv = nvox(p);
    const size_t N = (size_t)npar(p) * Nv, L = data_len(p);
    double complex *tr = (double complex *)malloc(train_len(p) * sizeof(double complex));
    double complex *r = (double complex *)malloc(L * sizeof(double complex));
    double complex *y = (double complex *)malloc(L * sizeof(double complex));
    double *g = (double *)malloc(N * sizeof(double));
    double *step = (double *)calloc(N, sizeof(double));
    double *res = (double *)malloc(N * sizeof(double));
    double *dir = (double *)malloc(N * sizeof(double));
    double *q = (double *)malloc(N * sizeof(double));
    double *trial = (double *)malloc(N * sizeof(double));
    memset(rep, 0, sizeof(*rep));

    /* Linearise at alpha: trains, r = d - s, f, g = Re(J^H r). */
    oracle_epg(p, theta, 1, tr);
    double complex *s = y;
    oracle_signal_separable(p, theta, coil, mask, tr, s);
    double f0 = 0.0;
    for (size_t i = 0; i < L; ++i) {
        r[i] = data[i] - s[i];
        f0 += creal(r[i]) * creal(r[i]) + cimag(r[i]) * cimag(r[i]);
    }
    f0 *= 0.5;
    oracle_jhw(p, theta, coil, mask, tr, r, g);
    apply_masks(p, g, o->param_mask, mask);
    rep->f0 = f0;
    rep->gnorm = sqrt(dot(g, g, N));

    /* CG on Re(J^H J) step = -g, from step = 0 (eq. 4). */
    for (size_t i = 0; i < N; ++i) { res[i] = -g[i]; dir[i] = res[i]; }
    double rr = dot(res, res, N);
    for (int it = 0; it < o->n_cg; ++it) {
        if (rr == 0.0) break;
        oracle_jv(p, theta, coil, mask, tr, dir, y);
        oracle_jhw(p, theta, coil, mask, tr, y, q);
        apply_masks(p, q, o->param_mask, mask);
        double kappa = dot(dir, q, N);
        if (kappa <= 1e-30 * dot(dir, dir, N)) break;
        double a = rr / kappa;
        for (size_t i = 0; i < N; ++i) { step[i] += a * dir[i]; res[i] -= a * q[i]; }
        double rr_new = dot(res, res, N);
        double b = rr_new / rr;
        for (size_t i = 0; i < N; ++i) dir[i] = res[i] + b * dir[i];
        rr = rr_new;
        rep->cg_iters++;
    }

    /* Backtracking with projection; Armijo test on the projected step. */
    double t = 1.0;
    rep->f1 = f0;
    for (int k = 0; k < o->n_ls_max; ++k) {
        for (size_t i = 0; i < N; ++i) trial[i] = theta[i] + t * step[i];
        project(p, trial, o, mask);
        double ft = oracle_residual(p, trial, coil, mask, data, NULL);
        double pred = 0.0, sn = 0.0;
        for (size_t i = 0; i < N; ++i) {
            double d = trial[i] - theta[i];
            pred += g[i] * d;
            sn += d * d;
        }
        rep->ls_trials++;
        if (ft <= f0 + o->armijo_c1 * pred) {
            memcpy(theta, trial, N * sizeof(double));
            rep->accepted = 1;
            rep->f1 = ft;
            rep->t = t;
            rep->step_norm = sqrt(sn);
            break;
        }
        t *= 0.5;
    }
    free(tr); free(r); free(y); free(g); free(step); free(res); free(dir); free(q); free(trial);
}

/* ------------------------------------------------------------------------ */
/* Trust-region inexact Gauss-Newton (Methods, Reconstructions): the model   */
/* m(p) = f + g'p + 0.5 p' Re(J^H J) p is minimised approximately inside     */
/* ||p|| <= delta by Steihaug's truncated CG (Nocedal & Wright, Algorithm    */
/* 7.2); bounds are kept by reflecting the trial point at the box walls      */
/* (the reflective path of Coleman & Li); the radius follows the ratio of    */
/* actual to predicted decrease (Nocedal & Wright, Algorithm 4.1).           */
/* ------------------------------------------------------------------------ */

typedef void (*matvec_fn)(void *ctx, const double *x, double *y);

/* tau >= 0 (or the other root) with ||z + tau d|| = delta. */
static void boundary_roots(const double *z, const double *d, size_t n, double delta,
                           double *t_lo, double *t_hi)
{
    double zz = dot(z, z, n), zd = dot(z, d, n), dd = dot(d, d, n);
    double disc = sqrt(zd * zd + dd * (delta * delta - zz));
    *t_hi = (-zd + disc) / dd;
    *t_lo = (-zd - disc) / dd;
}

/* Model value g'p + 0.5 p'Bp (constant f dropped). */
static double model_value(matvec_fn B, void *ctx, const double *g, const double *p, size_t n,
                          double *tmp)
{
    B(ctx, p, tmp);
    return dot(g, p, n) + 0.5 * dot(p, tmp, n);
}

/* Steihaug CG in Nocedal & Wright's notation: z_j iterates, r_j = g + B z_j
 * the model gradient, d_j search directions, d_0 = -r_0. */
static int steihaug(matvec_fn B, void *ctx, size_t n, const double *g, double delta, int n_cg,
                    double *p, int *iters)
{
    double *z = (double *)calloc(n, sizeof(double));
    double *r = (double *)malloc(n * sizeof(double));
    double *d = (double *)malloc(n * sizeof(double));
    double *Bd = (double *)malloc(n * sizeof(double));
    double *tmp = (double *)malloc(n * sizeof(double));
    int kind = ORACLE_TR_ITERS;
    *iters = 0;
    for (size_t i = 0; i < n; ++i) { r[i] = g[i]; d[i] = -g[i]; }
    double rr = dot(r, r, n);
    if (rr == 0.0) kind = ORACLE_TR_ZERO;
    for (int j = 0; j < n_cg && kind == ORACLE_TR_ITERS; ++j) {
        B(ctx, d, Bd);
        double kappa = dot(d, Bd, n);
        if (kappa <= 0.0) {
            /* Of the two boundary points along d keep the lower model value. */
            double tl, th;
            boundary_roots(z, d, n, delta, &tl, &th);
            double *pl = (double *)malloc(n * sizeof(double));
            for (size_t i = 0; i < n; ++i) { p[i] = z[i] + th * d[i]; pl[i] = z[i] + tl * d[i]; }
            if (model_value(B, ctx, g, pl, n, tmp) < model_value(B, ctx, g, p, n, tmp))
                memcpy(p, pl, n * sizeof(double));
            free(pl);
            kind = ORACLE_TR_CURVATURE;
            break;
        }
        double alpha = rr / kappa;
        double zn2 = 0.0;
        for (size_t i = 0; i < n; ++i) { double zi = z[i] + alpha * d[i]; zn2 += zi * zi; }
        if (sqrt(zn2) >= delta) {
            double tl, th;
            boundary_roots(z, d, n, delta, &tl, &th);
            for (size_t i = 0; i < n; ++i) p[i] = z[i] + th * d[i];
            kind = ORACLE_TR_BOUNDARY;
            break;
        }
        for (size_t i = 0; i < n; ++i) { z[i] += alpha * d[i]; r[i] += alpha * Bd[i]; }
        *iters = j + 1;
        double rr_new = dot(r, r, n);
        if (rr_new == 0.0) { kind = ORACLE_TR_ZERO; break; }
        double beta = rr_new / rr;
        for (size_t i = 0; i < n; ++i) d[i] = -r[i] + beta * d[i];
        rr = rr_new;
    }
    if (kind == ORACLE_TR_ITERS || kind == ORACLE_TR_ZERO) memcpy(p, z, n * sizeof(double));
    free(z); free(r); free(d); free(Bd); free(tmp);
    return kind;
}

typedef struct { int n; const double *B; } dense_ctx;

static void dense_matvec(void *c, const double *x, double *y)
{
    const dense_ctx *dc = (const dense_ctx *)c;
    for (int i = 0; i < dc->n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < dc->n; ++k) acc += dc->B[(size_t)i * dc->n + k] * x[k];
        y[i] = acc;
    }
}

int oracle_steihaug_dense(int n, const double *B, const double *g, double delta, int n_cg,
                          double *p, int *iters)
{
    dense_ctx c = {n, B};
    return steihaug(dense_matvec, &c, (size_t)n, g, delta, n_cg, p, iters);
}

double oracle_reflect(double x, double lo, double hi)
{
    double w = hi - lo;
    if (w <= 0.0) return lo;
    if (x >= lo && x <= hi) return x;   /* inside: no wall is reached */
    double y = fmod(x - lo, 2.0 * w);
    if (y < 0.0) y += 2.0 * w;
    if (y > w) y = 2.0 * w - y;
    return lo + y;
}

/* Re(J^H J) x restricted to the active entries (masked rows and columns). */
typedef struct {
    const oracle_problem *p;
    const double *theta;
    const double complex *coil, *trains;
    const unsigned char *mask;
    int param_mask;
    double complex *y;
} normal_ctx;

static void normal_matvec(void *c, const double *x, double *out)
{
    const normal_ctx *nc = (const normal_ctx *)c;
    const int Nv = nvox(nc->p);
    double *xm = (double *)malloc((size_t)npar(nc->p) * Nv * sizeof(double));
    memcpy(xm, x, (size_t)npar(nc->p) * Nv * sizeof(double));
    apply_masks(nc->p, xm, nc->param_mask, nc->mask);
    oracle_jv(nc->p, nc->theta, nc->coil, nc->mask, nc->trains, xm, nc->y);
    oracle_jhw(nc->p, nc->theta, nc->coil, nc->mask, nc->trains, nc->y, out);
    apply_masks(nc->p, out, nc->param_mask, nc->mask);
    free(xm);
}

void oracle_tr_step(const oracle_problem *p, double *theta,
                    const double complex *coil, const unsigned char *mask,
                    const double complex *data, const oracle_tr_opts *o, double *delta,
                    oracle_tr_report *rep)
{
    const int Nv = nvox(p);
    const size_t N = (size_t)npar(p) * Nv, L = data_len(p);
    double complex *tr = (double complex *)malloc(train_len(p) * sizeof(double complex));
    double complex *r = (double complex *)malloc(L * sizeof(double complex));
    double complex *y = (double complex *)malloc(L * sizeof(double complex));
    double *g = (double *)malloc(N * sizeof(double));
    double *step = (double *)malloc(N * sizeof(double));
    double *trial = (double *)malloc(N * sizeof(double));
    double *sv = (double *)malloc(N * sizeof(double));
    memset(rep, 0, sizeof(*rep));
    rep->delta_in = *delta;

    /* Linearise: trains, r = d - s, f, g = Re(J^H r). */
    oracle_epg(p, theta, 1, tr);
    oracle_signal_separable(p, theta, coil, mask, tr, y);
    double f0 = 0.0;
    for (size_t i = 0; i < L; ++i) {
        r[i] = data[i] - y[i];
        f0 += creal(r[i]) * creal(r[i]) + cimag(r[i]) * cimag(r[i]);
    }
    f0 *= 0.5;
    oracle_jhw(p, theta, coil, mask, tr, r, g);
    apply_masks(p, g, o->param_mask, mask);
    rep->f0 = f0;
    rep->f1 = f0;
    rep->gnorm = sqrt(dot(g, g, N));

    /* Truncated CG inside the region. */
    normal_ctx nc = {p, theta, coil, tr, mask, o->param_mask, y};
    rep->exit_kind = steihaug(normal_matvec, &nc, N, g, *delta, o->n_cg, step, &rep->cg_iters);

    /* Trial point: reflect the reconstructed, bounded entries into the box. */
    for (size_t i = 0; i < N; ++i) trial[i] = theta[i] + step[i];
    for (int q = 0; q < npar(p); ++q) {
        double lo, hi;
        if (!box_of(p, o->lo, o->hi, q, &lo, &hi)) continue;
        for (int j = 0; j < Nv; ++j) {
            if (!((o->param_mask >> q) & 1) || !active(mask, j)) continue;
            double *t = &trial[(size_t)q * Nv + j];
            double rf = oracle_reflect(*t, lo, hi);
            if (rf != *t) rep->n_reflected++;
            *t = rf;
        }
    }
    for (size_t i = 0; i < N; ++i) sv[i] = trial[i] - theta[i];

    /* Predicted decrease of the model at the taken step s, and the ratio. */
    oracle_jv(p, theta, coil, mask, tr, sv, y);
    double js2 = 0.0;
    for (size_t i = 0; i < L; ++i) js2 += creal(y[i]) * creal(y[i]) + cimag(y[i]) * cimag(y[i]);
    double pred = -(dot(g, sv, N) + 0.5 * js2);
    double ft = oracle_residual(p, trial, coil, mask, data, NULL);
    double rho = (f0 - ft) / pred;
    if (!(pred > 0.0) || !isfinite(rho)) rho = -INFINITY;
    rep->pred = pred;
    rep->rho = rho;
    rep->step_norm = sqrt(dot(sv, sv, N));

    int at_boundary = rep->exit_kind == ORACLE_TR_BOUNDARY || rep->exit_kind == ORACLE_TR_CURVATURE;
    if (rho < 0.25)
        *delta = 0.25 * *delta;
    else if (rho > 0.75 && at_boundary)
        *delta = fmin(2.0 * *delta, o->delta_max);
    rep->delta_out = *delta;
    if (rho > o->eta) {
        memcpy(theta, trial, N * sizeof(double));
        rep->accepted = 1;
        rep->f1 = ft;
    }
    free(tr); free(r); free(y); free(g); free(step); free(trial); free(sv);
}

/* ------------------------------------------------------------------------ */
/* Proton density initialisation (Methods, Reconstructions): least squares   */
/* solution of M(alpha0) rho = d, by CGLS on the complex unknown rho.        */
/* With A rho = s(rho) for fixed trains: A^H w at voxel j is                  */
/* sum_n conj(m_j[n]) V[n,j] with V the adjoint encoding of w.               */
/* ------------------------------------------------------------------------ */

void oracle_rho_init(const oracle_problem *p, double *theta,
                     const double complex *coil, const unsigned char *mask,
                     const double complex *data, int n_iter)
{
    const int Nv = nvox(p);
    const size_t L = data_len(p);
    double complex *tr = (double complex *)malloc(train_len(p) * sizeof(double complex));
    double complex *res = (double complex *)malloc(L * sizeof(double complex));
    double complex *qv = (double complex *)malloc(L * sizeof(double complex));
    double complex *V = (double complex *)malloc((size_t)p->n_tr * Nv * sizeof(double complex));
    double complex *x = (double complex *)calloc(Nv, sizeof(double complex));
    double complex *sv = (double complex *)malloc(Nv * sizeof(double complex));
    double complex *pv = (double complex *)malloc(Nv * sizeof(double complex));
    double *th = (double *)malloc((size_t)npar(p) * Nv * sizeof(double));
    oracle_epg(p, theta, 0, tr);

    /* A^H w */
#define ADJ(w, out)                                                          \
    do {                                                                     \
        adjoint_encode(p, theta, coil, mask, (w), V, NULL);                  \
        for (int j = 0; j < Nv; ++j) {                                       \
            double complex acc = 0.0;                                        \
            for (int n = 0; n < p->n_tr; ++n)                                \
                acc += conj(tr[(size_t)n * Nv + j]) * V[(size_t)n * Nv + j]; \
            (out)[j] = acc;                                                  \
        }                                                                    \
    } while (0)

    memcpy(th, theta, (size_t)npar(p) * Nv * sizeof(double));
    for (size_t i = 0; i < L; ++i) res[i] = data[i];
    ADJ(res, sv);
    double gamma = 0.0;
    for (int j = 0; j < Nv; ++j) { pv[j] = sv[j]; gamma += creal(sv[j] * conj(sv[j])); }
    for (int it = 0; it < n_iter && gamma > 0.0; ++it) {
        for (int j = 0; j < Nv; ++j) { th[3 * (size_t)Nv + j] = creal(pv[j]); th[4 * (size_t)Nv + j] = cimag(pv[j]); }
        oracle_signal_separable(p, th, coil, mask, tr, qv);
        double qq = 0.0;
        for (size_t i = 0; i < L; ++i) qq += creal(qv[i] * conj(qv[i]));
        if (qq == 0.0) break;
        double a = gamma / qq;
        for (int j = 0; j < Nv; ++j) x[j] += a * pv[j];
        for (size_t i = 0; i < L; ++i) res[i] -= a * qv[i];
        ADJ(res, sv);
        double gnew = 0.0;
        for (int j = 0; j < Nv; ++j) gnew += creal(sv[j] * conj(sv[j]));
        double b = gnew / gamma;
        for (int j = 0; j < Nv; ++j) pv[j] = sv[j] + b * pv[j];
        gamma = gnew;
    }
#undef ADJ
    for (int j = 0; j < Nv; ++j) {
        theta[3 * (size_t)Nv + j] = creal(x[j]);
        theta[4 * (size_t)Nv + j] = cimag(x[j]);
    }
    free(tr); free(res); free(qv); free(V); free(x); free(sv); free(pv); free(th);
}
