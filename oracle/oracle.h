/*
 * FP64 CPU oracle for the MR-STAT matrix-free Jacobian products.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call
 * this library: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code, table or constant with the HIP
 * library.
 *
 * Every routine here is the plain definition of what the method computes,
 * written for readability, in double / double complex, with OpenMP only over
 * independent voxels or output rows (no blocking, no fusion).
 *
 * Paper: van der Heide, Sbrizzi, Luijten, van den Berg, "High resolution
 * in-vivo MR-STAT using a matrix-free and parallelized reconstruction
 * algorithm" (NMR Biomed 2019, arXiv 1904.13244).
 *
 * Conventions (the paper's statement of the problem, Theory section):
 *   voxel j = iy*nx + ix, Nv = nx*ny;
 *   parameter vector alpha in R^{5 Nv} (R^{6 Nv} with Delta B0 fitted),
 *   voxel j's parameters at j + p*Nv (parameter-major layout of the Theory
 *   section), with p = 0: ln T1 [s], 1: ln T2 [s], 2: B1 [a.u.], 3: Re rho,
 *   4: Im rho, 5: Delta B0 / db0_unit
 *   (log scaling of T1 and T2 as in the Methods / Reconstructions section);
 *   r = d - s, f = 0.5 ||r||^2, J = dr/dalpha, g = Re(J^H r).
 */
#ifndef MRSTAT_ORACLE_H
#define MRSTAT_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;        /* image grid */
    int n_tr;          /* number of TRs = readouts */
    int n_read;        /* samples per readout (os * nx) */
    int n_states;      /* EPG truncation K */
    int n_coils;       /* receive coils C */
    double tr, te;     /* seconds */
    double t_inv;      /* delay between inversion and first RF, seconds */
    const double *flip_deg;   /* [n_tr] flip angle per TR, degrees */
    const double *rf_phase;   /* [n_tr] RF phase per TR, radians */
    const int *ky_line;       /* [n_tr] phase-encode line sampled in each TR */
    /* Non-Cartesian sampling (Introduction and Discussion: the method is not
     * tied to Cartesian trajectories): when kx is not NULL, sample k of TR n
     * sits at (kx, ky)[n * n_read + k] in cycles per field of view, and the
     * encoding is evaluated as a direct sum; ky_line is then unused. */
    const double *kx, *ky;
    /* Balanced isochromat signal model (Methods, Pulse Sequence and
     * Reconstructions; Supporting Information S2): when n_iso > 0 the trains
     * come from n_iso isochromats per voxel instead of the EPG, isochromat q
     * seeing the flip angle scaled by iso_scale[q] (the slice profile) and
     * entering the voxel's magnetisation with weight iso_weight[q]; no
     * spoiling and no off-resonance (a balanced sequence on resonance). */
    int n_iso;
    const double *iso_scale, *iso_weight;
    /* Readout dynamics (Discussion: the volumetric model follows T2 decay and
     * Delta B0 phase accumulation during each readout): sample k of every
     * readout is taken at TE + tau_k, tau_k = (k - n_read / 2) dwell seconds,
     * and voxel j's transverse magnetisation carries the factor
     * exp(-tau_k / T2_j) exp(-2 pi i db0_j (TE + tau_k)) (db0 in Hz per voxel,
     * NULL = 0; the precession has the sense of the encoding phase, which a
     * gradient field adds the same way). Off when dwell == 0 and db0 == NULL.
     * For the gradient-spoiled
     * EPG model a uniform off-resonance changes the echo by that phase only
     * (the spoiler's dephasing absorbs it between pulses); the balanced
     * isochromat model is not combined with off-resonance (n_iso > 0 requires
     * db0 == NULL). The encoding is then evaluated as a direct sum. */
    double dwell;
    const double *db0;
    /* Delta B0 as a reconstructed parameter (the Discussion's extension of the
     * parameter set): when db0_unit > 0 the parameter vector has a sixth row,
     * p = 5, and voxel j's off-resonance is theta[5 Nv + j] * db0_unit Hz in
     * the readout factor above (db0 must then be NULL). The GN line search and
     * the trust region keep |theta_5| db0_unit <= db0_box Hz (no bound when
     * db0_box <= 0), as they keep ln T1, ln T2 and B1 in their box. */
    double db0_unit, db0_box;
} oracle_problem;

typedef struct {
    int n_cg;          /* CG iterations (exact count; breakdown exits only) */
    int n_ls_max;      /* backtracking trials t = 1, 1/2, ... */
    int param_mask;    /* bit p set = parameter p is reconstructed */
    double lo[3], hi[3];  /* box for ln T1, ln T2, B1 */
    double armijo_c1;
} oracle_gn_opts;

typedef struct {
    double f0, f1, gnorm, step_norm, t;
    int cg_iters, ls_trials, accepted;
} oracle_gn_report;

int oracle_num_threads(void);

/* One isochromat of the balanced model: n_tr demodulated transverse
 * magnetisations at TE (and their derivatives in ln T1, ln T2, B1 when
 * dm1 != NULL) for flip angles scaled by `scale`; the Supporting Information
 * S2 update (Rodrigues rotation about the RF axis, then decay and regrowth)
 * with forward-mode tangents. */
void oracle_isochromat(const oracle_problem *p, double lnT1, double lnT2, double B1, double scale,
                       double complex *m, double complex *dm1, double complex *dm2,
                       double complex *dm3);

/* EPG simulation with forward-mode tangents (Supporting Information S2
 * pattern, applied to the extended-phase-graph states).
 * theta: [Np][Nv] (Np = 5, or 6 with Delta B0 fitted); trains out: [4][n_tr][Nv] complex = m, dm/dlnT1, dm/dlnT2,
 * dm/dB1. If with_tangents == 0 only train 0 is written. */
void oracle_epg(const oracle_problem *p, const double *theta, int with_tangents,
                double complex *trains);

/* Encoding phase E[n,k,j] of sample k of the readout in TR n for voxel j:
 * exp(-2 pi i (kx (ix - nx/2) / nx + ky (iy - ny/2) / ny)) with (kx, ky) in
 * cycles per field of view; on the Cartesian grid kx = (k - n_read/2) nx /
 * n_read and ky = l(n) - ny/2. */
double complex oracle_phase(const oracle_problem *p, int n, int k, int ix, int iy);

/* All phases of TR n: out[k][j] = E[n,k,j], [n_read][Nv]. */
void oracle_phases(const oracle_problem *p, int n, double complex *out);

/* s_c[n,k] = sum_j C_c[j] rho_j m_j[n] E[n,k,j]: the discretised volumetric
 * signal model (eq. 1 and its discretisation), direct sum over voxels.
 * coil: [C][Nv] complex or NULL (C must be 1, sensitivity 1).
 * mask: [Nv] or NULL. s out: [C][n_tr][n_read]. */
void oracle_signal_direct(const oracle_problem *p, const double *theta,
                          const double complex *coil, const unsigned char *mask,
                          const double complex *trains, double complex *s);

/* Same sum evaluated as y-then-x separable sums (Cartesian phases factor). */
void oracle_signal_separable(const oracle_problem *p, const double *theta,
                             const double complex *coil, const unsigned char *mask,
                             const double complex *trains, double complex *s);

/* J v for real v [Np][Nv]; out [C][n_tr][n_read]. J = dr/dalpha = -ds/dalpha. */
void oracle_jv(const oracle_problem *p, const double *theta,
               const double complex *coil, const unsigned char *mask,
               const double complex *trains, const double *v, double complex *out);

/* Re(J^H w) for w [C][n_tr][n_read]; out [Np][Nv]. */
void oracle_jhw(const oracle_problem *p, const double *theta,
                const double complex *coil, const unsigned char *mask,
                const double complex *trains, const double complex *w, double *out);

/* Explicit Jacobian, row (c,n,k) major: J[(c*n_tr + n)*n_read + k][q*Nv + j]. */
void oracle_jacobian(const oracle_problem *p, const double *theta,
                     const double complex *coil, const unsigned char *mask,
                     const double complex *trains, double complex *J);

/* f = 0.5 ||d - s||^2 with s from the separable sum; r out (may be NULL). */
double oracle_residual(const oracle_problem *p, const double *theta,
                       const double complex *coil, const unsigned char *mask,
                       const double complex *data, double complex *r);

/* One inexact Gauss-Newton iteration (Algorithm 6, line-search form): theta
 * updated in place when a trial is accepted. */
void oracle_gn_step(const oracle_problem *p, double *theta,
                    const double complex *coil, const unsigned char *mask,
                    const double complex *data, const oracle_gn_opts *o,
                    oracle_gn_report *rep);

/* ------------------------------------------------------------------------
 * Trust-region form of the inexact Gauss-Newton step (Methods,
 * Reconstructions: a trust-region framework after Steihaug and Nocedal &
 * Wright's Algorithm 7.2, with reflection at the feasible bounds after
 * Coleman & Li).
 * ------------------------------------------------------------------------ */

/* How the truncated CG of the trust-region step ended. */
enum {
    ORACLE_TR_ITERS = 0,      /* the iteration count was reached inside the region */
    ORACLE_TR_BOUNDARY = 1,   /* an iterate left the region: step cut at its boundary */
    ORACLE_TR_CURVATURE = 2,  /* non-positive curvature: step to the boundary */
    ORACLE_TR_ZERO = 3        /* zero model gradient: exact minimiser of the model */
};

/* Steihaug's truncated CG for min_p g'p + 0.5 p'Bp subject to ||p|| <= delta,
 * B dense symmetric n x n (row-major), at most n_cg iterations from p = 0.
 * Returns the exit kind (ORACLE_TR_*); *iters = completed CG updates. */
int oracle_steihaug_dense(int n, const double *B, const double *g, double delta, int n_cg,
                          double *p, int *iters);

/* Reflection of x into [lo, hi]: the end point of the straight path from a
 * point inside the box that bounces off the walls (a fold with period
 * 2 (hi - lo)); lo == hi gives lo. */
double oracle_reflect(double x, double lo, double hi);

typedef struct {
    int n_cg;            /* CG iteration limit of the truncated solve */
    int param_mask;      /* bit p set = parameter p is reconstructed */
    double lo[3], hi[3]; /* box of ln T1, ln T2, B1, enforced by reflection */
    double eta;          /* acceptance: rho > eta */
    double delta_max;    /* cap of the trust radius */
} oracle_tr_opts;

typedef struct {
    double f0, f1, gnorm, step_norm, rho, pred, delta_in, delta_out;
    int cg_iters, exit_kind, accepted, n_reflected;
} oracle_tr_report;

/* One trust-region inexact Gauss-Newton iteration at trust radius *delta
 * (updated in place): Steihaug CG on Re(J^H J) p = -g within ||p|| <= delta,
 * trial = reflection of theta + p into the box, ratio
 * rho = (f(theta) - f(trial)) / (model decrease at s = trial - theta), where
 * the model decrease is -(g's + 0.5 ||J s||^2); theta = trial when
 * rho > eta; the radius is quartered when rho < 1/4 and doubled (up to
 * delta_max) when rho > 3/4 and the CG stopped at the boundary. */
void oracle_tr_step(const oracle_problem *p, double *theta,
                    const double complex *coil, const unsigned char *mask,
                    const double complex *data, const oracle_tr_opts *o, double *delta,
                    oracle_tr_report *rep);

/* Proton-density initialisation: least-squares solution of M(alpha0) rho = d
 * by CGLS (equal to LSQR in exact arithmetic), n_iter iterations from rho = 0.
 * theta's rows 0..2 are used, rows 3..4 are overwritten. */
void oracle_rho_init(const oracle_problem *p, double *theta,
                     const double complex *coil, const unsigned char *mask,
                     const double complex *data, int n_iter);

#ifdef __cplusplus
}
#endif
#endif
