/*
 * FP64 CPU oracle for one relativistic electromagnetic PIC step with the WT
 * force interpolation of Lu, Kilian, Guo, Li and Liang (arXiv:1909.09613).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is plain, slow and written to be read
 * against the paper.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  The GPU library shares no code with it.
 *
 * Conventions (the paper leaves the units of a concrete run open; this is the
 * reading used throughout):
 *   - positions are absolute, in cell units (x~_d = x_d / dx_d), periodic in
 *     every axis, canonical range [0, n_d);
 *   - momenta are u = gamma*v/c (dimensionless), gamma = sqrt(1 + |u|^2);
 *   - Maxwell with 4*pi absorbed: dE/dt = c curl B - J, dB/dt = -c curl E
 *     (Sec. "Scaling for ultra-relativistic PIC simulations", dimensionless set);
 *   - Yee staggering (Sec. 2): E_i sits half a cell off along i, B_i half a cell
 *     off along the two other axes, rho and J_i co-located with E_i's lattice
 *     (rho on integer nodes).  Array index m of a component that is staggered
 *     along d stores the value at m + 1/2 along d.
 *   - field arrays are indexed i + n0*(j + n1*k); in 2D n[2] == 1 and nothing
 *     depends on x3.
 */
#ifndef WTPIC_ORACLE_H
#define WTPIC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_WT 0   /* time-step dependent interpolation, Eq. interpolation-EB-real-mod */
#define ORC_MC 1   /* momentum-conserving interpolation, Eq. interpolation-EB-real-org */
#define ORC_YEE 0  /* standard Yee curl stencils */
#define ORC_M4 1   /* Faraday stencil modified for 4th-order dispersion, Appendix C */

typedef struct {
  int ndim;       /* 2 or 3 */
  int n[3];       /* cells per axis, n[2] == 1 in 2D */
  int order;      /* B-spline order l (1..4) */
  int scheme;     /* ORC_WT or ORC_MC */
  int solver;     /* ORC_YEE or ORC_M4 */
  double dx[3];   /* cell sizes */
  double dt;      /* time step */
  double c;       /* speed of light */
  double *E[3];   /* E^n, ncell values each */
  double *B[3];   /* B^n (integer time, see orc_field_update) */
  double *J[3];   /* J^{n+1/2}, accumulated by orc_deposit */
} orc_grid;

/* 1D kernels (Sec. 2). */
double orc_W(int l, double y);              /* centred B-spline of order l, width l+1 */
double orc_C(int l, double z);              /* integral of W_{l-1} from -inf to z */
double orc_T(int l, double a, double y);    /* WT factor T_l(y) for a = c dt / dx */
void orc_W_vec(int l, const double *y, double *out, long n);
void orc_C_vec(int l, const double *z, double *out, long n);
void orc_T_vec(int l, double a, const double *y, double *out, long n);

/* Per-particle steps. */
void orc_gather(const orc_grid *g, const double *x, double *Ep, double *Bp);
void orc_boris(double *u, const double *Ep, const double *Bp, double qm, double dt, double c);
void orc_move(const orc_grid *g, double *x, const double *u);
void orc_deposit(orc_grid *g, const double *x0, const double *x1, double Q, double vz);
void orc_wrap(const orc_grid *g, double *x);

/* Whole-species and whole-grid steps. */
void orc_zero_J(orc_grid *g);
void orc_push_species(orc_grid *g, long np, double *x, double *u, double qm, double Q);

/* Partially skipped calculation (Sec. 3): A(t) membership of a canonical
 * position for the box lo..hi (cell units, periodic), and the species step in
 * which particles outside A(t) only drift. */
int orc_perturbed(const orc_grid *g, const double *x, const double *lo, const double *hi, double t);
void orc_push_species_skip(orc_grid *g, long np, double *x, double *u, double qm, double Q, const double *lo,
                           const double *hi, double t);
void orc_faraday_half(orc_grid *g);
void orc_ampere(orc_grid *g);
void orc_field_update(orc_grid *g);

/* Diagnostics. */
void orc_rho(const orc_grid *g, long np, const double *x, double Q, double *rho);
void orc_div_E(const orc_grid *g, double *out);
void orc_field_energy(const orc_grid *g, double *UE, double *UB);
double orc_kinetic(long np, const double *u, double M, double c);

#ifdef __cplusplus
}
#endif
#endif
