/*
 * FP64 CPU oracle for one relativistic EM-PIC step with the WT scheme
 * (arXiv:1909.09613).  TEST INFRASTRUCTURE ONLY: it is loaded by the tests,
 * the smoke check and the benchmark's CPU-baseline leg, never by the GPU
 * library, and it shares no code with it.  Plain loops, FP64, no blocking.
 * See oracle.h for units and array conventions.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static long ncell_of(const orc_grid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static int wrap_index(long m, int n) {
  long r = m % n;
  if (r < 0) r += n;
  return (int)r;
}

/* ------------------------------------------------------------------------ */
/* 1D kernels                                                               */
/* ------------------------------------------------------------------------ */

/* W_l: the l-th order B-spline of width l+1 (Sec. 2, the form factor of
 * Eq. shape-real; its Fourier transform is s_l, Eq. s_l).  Evaluated with the
 * uniform B-spline recurrence (a convex combination of two order-(l-1)
 * splines shifted by +-1/2), starting from the unit box on [-1/2, 1/2). */
double orc_W(int l, double y) {
  if (l == 0) return (y >= -0.5 && y < 0.5) ? 1.0 : 0.0;
  double h = 0.5 * (l + 1);
  if (y <= -h || y >= h) return 0.0;
  return ((y + h) * orc_W(l - 1, y + 0.5) + (h - y) * orc_W(l - 1, y - 0.5)) / l;
}

/* The same recurrence in extended precision (long double).  The deposit
 * takes S1 - S0 from it: a transverse step of ~1e-4 cells changes the form
 * factor by ~1e-4, and the difference of two FP64 values of order one would
 * keep only ~1e-12 of it. */
static long double W_ext(int l, long double y) {
  if (l == 0) return (y >= -0.5L && y < 0.5L) ? 1.0L : 0.0L;
  long double h = 0.5L * (l + 1);
  if (y <= -h || y >= h) return 0.0L;
  return ((y + h) * W_ext(l - 1, y + 0.5L) + (h - y) * W_ext(l - 1, y - 0.5L)) / l;
}

/* C_l(z) = integral of W_{l-1} over (-inf, z].  Since W_l(y) is the average
 * of W_{l-1} over [y-1/2, y+1/2], summing W_l(z - 1/2 - m) over m >= 0
 * telescopes to that integral. */
double orc_C(int l, double z) {
  double h = 0.5 * l;
  if (z <= -h) return 0.0;
  if (z >= h) return 1.0;
  double s = 0.0;
  for (int m = 0;; ++m) {
    double y = z - 0.5 - m;
    if (y <= -0.5 * (l + 1)) break;
    s += orc_W(l, y);
  }
  return s;
}

/* T_l(y; a), a = c dt/dx: the inverse Fourier transform of
 * tau_l = sinc^l(k dx/2) sinc(k c dt) (Eq. tau_l).  sinc^l is the transform
 * of W_{l-1}; sinc(k c dt) is the transform of a box of width 2 c dt and unit
 * area.  Their product transforms back to W_{l-1} averaged over [y-a, y+a]. */
double orc_T(int l, double a, double y) {
  return (orc_C(l, y + a) - orc_C(l, y - a)) / (2.0 * a);
}

void orc_W_vec(int l, const double *y, double *out, long n) {
  for (long i = 0; i < n; ++i) out[i] = orc_W(l, y[i]);
}
void orc_C_vec(int l, const double *z, double *out, long n) {
  for (long i = 0; i < n; ++i) out[i] = orc_C(l, z[i]);
}
void orc_T_vec(int l, double a, const double *y, double *out, long n) {
  for (long i = 0; i < n; ++i) out[i] = orc_T(l, a, y[i]);
}

/* ------------------------------------------------------------------------ */
/* Gather: Eq. interpolation-EB-real-mod (WT) or -org (MC)                   */
/* ------------------------------------------------------------------------ */

enum { KW = 0, KT = 1 };

/* Interpolate one field component f whose lattice sits at lam[d] (0 or 1/2)
 * along axis d, with kernel kind[d] (W or T) along each axis. */
static double interp(const orc_grid *g, const double *f, const double *x, const double lam[3],
                     const int kind[3]) {
  int l = g->order;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double wt[3][16];
  for (int d = 0; d < g->ndim; ++d) {
    double a = g->c * g->dt / g->dx[d];
    double h = (kind[d] == KW) ? 0.5 * (l + 1) : 0.5 * l + a;
    double xs = x[d] - lam[d];
    lo[d] = (int)ceil(xs - h);
    hi[d] = (int)floor(xs + h);
    for (int m = lo[d]; m <= hi[d]; ++m) {
      double y = xs - m;
      wt[d][m - lo[d]] = (kind[d] == KW) ? orc_W(l, y) : orc_T(l, a, y);
    }
  }
  double s = 0.0;
  for (int m2 = lo[2]; m2 <= hi[2]; ++m2) {
    double w2 = (g->ndim == 3) ? wt[2][m2 - lo[2]] : 1.0;
    int k = wrap_index(m2, g->n[2]);
    for (int m1 = lo[1]; m1 <= hi[1]; ++m1) {
      double w1 = wt[1][m1 - lo[1]];
      int j = wrap_index(m1, g->n[1]);
      for (int m0 = lo[0]; m0 <= hi[0]; ++m0) {
        double w0 = wt[0][m0 - lo[0]];
        int i = wrap_index(m0, g->n[0]);
        s += w0 * w1 * w2 * f[i + (long)g->n[0] * (j + (long)g->n[1] * k)];
      }
    }
  }
  return s;
}

/* E_i: staggered along i, W along i and T across (WT); B_i: staggered across,
 * T along i and W across (WT).  MC uses W everywhere.  In 2D the x3 factor is
 * dropped: nothing depends on x3 and both kernels sum to one over the lattice. */
void orc_gather(const orc_grid *g, const double *x, double *Ep, double *Bp) {
  for (int i = 0; i < 3; ++i) {
    double lamE[3], lamB[3];
    int kindE[3], kindB[3];
    for (int d = 0; d < 3; ++d) {
      lamE[d] = (d == i) ? 0.5 : 0.0;
      lamB[d] = (d == i) ? 0.0 : 0.5;
      if (g->scheme == ORC_MC) {
        kindE[d] = KW;
        kindB[d] = KW;
      } else {
        kindE[d] = (d == i) ? KW : KT;
        kindB[d] = (d == i) ? KT : KW;
      }
    }
    Ep[i] = interp(g, g->E[i], x, lamE, kindE);
    Bp[i] = interp(g, g->B[i], x, lamB, kindB);
  }
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push (the push named in Sec. 1)                        */
/* ------------------------------------------------------------------------ */

/* u = gamma v / c.  du/dt = (q/m)(E + (v/c) x B)/c.  Half electric kick,
 * magnetic rotation at gamma of the half-kicked momentum, half kick. */
void orc_boris(double *u, const double *Ep, const double *Bp, double qm, double dt, double c) {
  double eps = qm * dt / (2.0 * c);
  double um[3], t[3], s[3], up[3], uq[3];
  for (int d = 0; d < 3; ++d) um[d] = u[d] + eps * Ep[d];
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int d = 0; d < 3; ++d) t[d] = eps * Bp[d] / gm;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + t2);
  /* u' = u- + u- x t */
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  /* u+ = u- + u' x s */
  uq[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
  uq[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
  uq[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
  for (int d = 0; d < 3; ++d) u[d] = uq[d] + eps * Ep[d];
}

/* x~_d <- x~_d + (c dt / dx_d) u_d / gamma on the simulated axes (unwrapped). */
void orc_move(const orc_grid *g, double *x, const double *u) {
  double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int d = 0; d < g->ndim; ++d) x[d] = x[d] + (g->c * g->dt / g->dx[d]) * (u[d] / gam);
}

/* Periodic wrap into [0, n); a value that rounds onto n maps to 0. */
void orc_wrap(const orc_grid *g, double *x) {
  for (int d = 0; d < g->ndim; ++d) {
    double n = (double)g->n[d];
    while (x[d] < 0.0) x[d] += n;
    while (x[d] >= n) x[d] -= n;
  }
}

/* ------------------------------------------------------------------------ */
/* Exact charge-conserving deposit (Esirkepov's decomposition, Sec. 1, 2)    */
/* ------------------------------------------------------------------------ */

/* Adds the current of one macro-particle of charge Q moving x0 -> x1 during
 * one step.  S0, S1 are the form factors W_l on integer nodes at the old and
 * new positions; DS = S1 - S0, formed in extended precision.  The current
 * density is the unique combination of form-factor differences obeying the
 * discrete continuity equation (rho^{n+1} - rho^n)/dt + D.J = 0 with D the
 * Gauss operator of Eq. gauss; each component is a prefix sum along its own
 * axis. */
void orc_deposit(orc_grid *g, const double *x0, const double *x1, double Q, double vz) {
  int l = g->order;
  double h = 0.5 * (l + 1);
  int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  double S0[3][16], DS[3][16];
  double Vc = 1.0;
  for (int d = 0; d < g->ndim; ++d) Vc *= g->dx[d];
  for (int d = 0; d < g->ndim; ++d) {
    double xmin = x0[d] < x1[d] ? x0[d] : x1[d];
    double xmax = x0[d] < x1[d] ? x1[d] : x0[d];
    lo[d] = (int)ceil(xmin - h);
    int hi = (int)floor(xmax + h);
    cnt[d] = hi - lo[d] + 1;
    for (int k = 0; k < cnt[d]; ++k) {
      int m = lo[d] + k;
      /* x - m is exact in extended precision; the difference keeps its
       * relative precision however short the step */
      long double s0 = W_ext(l, (long double)x0[d] - m);
      long double s1 = W_ext(l, (long double)x1[d] - m);
      S0[d][k] = (double)s0;
      DS[d][k] = (double)(s1 - s0);
    }
  }
  long n0 = g->n[0], n1 = g->n[1];
  double third = 1.0 / 3.0;
  if (g->ndim == 2) {
    double sx = -Q * g->dx[0] / (Vc * g->dt);
    double sy = -Q * g->dx[1] / (Vc * g->dt);
    double sz = Q * vz / Vc;
    /* J1 at (m0 + 1/2, m1): prefix sum of Wx = DSx (S0y + DSy/2) along x. */
    for (int k1 = 0; k1 < cnt[1]; ++k1) {
      double acc = 0.0;
      int j = wrap_index(lo[1] + k1, g->n[1]);
      for (int k0 = 0; k0 < cnt[0]; ++k0) {
        acc += DS[0][k0] * (S0[1][k1] + 0.5 * DS[1][k1]);
        int i = wrap_index(lo[0] + k0, g->n[0]);
        g->J[0][i + n0 * j] += sx * acc;
      }
    }
    /* J2 at (m0, m1 + 1/2): prefix sum of Wy = DSy (S0x + DSx/2) along y. */
    for (int k0 = 0; k0 < cnt[0]; ++k0) {
      double acc = 0.0;
      int i = wrap_index(lo[0] + k0, g->n[0]);
      for (int k1 = 0; k1 < cnt[1]; ++k1) {
        acc += DS[1][k1] * (S0[0][k0] + 0.5 * DS[0][k0]);
        int j = wrap_index(lo[1] + k1, g->n[1]);
        g->J[1][i + n0 * j] += sy * acc;
      }
    }
    /* J3 at (m0, m1): Q vz / Vc times the time average of Sx Sy along the
     * straight path, S0x S0y + (DSx S0y + S0x DSy)/2 + DSx DSy/3. */
    for (int k1 = 0; k1 < cnt[1]; ++k1) {
      int j = wrap_index(lo[1] + k1, g->n[1]);
      for (int k0 = 0; k0 < cnt[0]; ++k0) {
        int i = wrap_index(lo[0] + k0, g->n[0]);
        double wz = S0[0][k0] * S0[1][k1] + 0.5 * (DS[0][k0] * S0[1][k1] + S0[0][k0] * DS[1][k1]) +
                    third * DS[0][k0] * DS[1][k1];
        g->J[2][i + n0 * j] += sz * wz;
      }
    }
    return;
  }
  /* 3D: W_a = DS_a (S0_b S0_c + DS_b S0_c/2 + S0_b DS_c/2 + DS_b DS_c/3). */
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double sa = -Q * g->dx[a] / (Vc * g->dt);
    int kk[3];
    for (kk[b] = 0; kk[b] < cnt[b]; ++kk[b]) {
      for (kk[c] = 0; kk[c] < cnt[c]; ++kk[c]) {
        double tr = S0[b][kk[b]] * S0[c][kk[c]] + 0.5 * DS[b][kk[b]] * S0[c][kk[c]] +
                    0.5 * S0[b][kk[b]] * DS[c][kk[c]] + third * DS[b][kk[b]] * DS[c][kk[c]];
        double acc = 0.0;
        for (kk[a] = 0; kk[a] < cnt[a]; ++kk[a]) {
          acc += DS[a][kk[a]] * tr;
          int i = wrap_index(lo[0] + kk[0], g->n[0]);
          int j = wrap_index(lo[1] + kk[1], g->n[1]);
          int k = wrap_index(lo[2] + kk[2], g->n[2]);
          g->J[a][i + n0 * (j + n1 * k)] += sa * acc;
        }
      }
    }
  }
}

void orc_zero_J(orc_grid *g) {
  long nc = ncell_of(g);
  for (int d = 0; d < 3; ++d) memset(g->J[d], 0, sizeof(double) * nc);
}

/* One particle step: gather at x^n, Boris to u^{n+1/2}, move to x^{n+1},
 * deposit J^{n+1/2} from the unwrapped path, then wrap. */
static void push_one(orc_grid *g, double *xp, double *up, double qm, double Q) {
  double Ep[3], Bp[3], x0[3];
  orc_gather(g, xp, Ep, Bp);
  orc_boris(up, Ep, Bp, qm, g->dt, g->c);
  for (int d = 0; d < 3; ++d) x0[d] = xp[d];
  orc_move(g, xp, up);
  double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
  orc_deposit(g, x0, xp, Q, g->c * up[2] / gam);
  orc_wrap(g, xp);
}

/* The particle step for a whole species. */
void orc_push_species(orc_grid *g, long np, double *x, double *u, double qm, double Q) {
  for (long p = 0; p < np; ++p) push_one(g, x + 3 * p, u + 3 * p, qm, Q);
}

/* ------------------------------------------------------------------------ */
/* Partially skipped calculation (Sec. 3, "Partially skipping calculation")  */
/* ------------------------------------------------------------------------ */

/* The region perturbed at time t > 0 is the set of points closer than c t to
 * some point of the initially perturbed region A0; at t = 0 it is A0.  Here
 * A0 is the closed box lo_d <= x~_d <= hi_d (cell units, 0 <= lo_d <= hi_d <=
 * n_d) repeated periodically.  The distance to a periodic box is Euclidean in
 * physical units and separates by axis: along d it is the distance from x~_d
 * to the nearest of the intervals [lo_d + k n_d, hi_d + k n_d].  (The paper's
 * set formula repeats the y term where the z term belongs; the Euclidean
 * distance is the reading taken.)  x is a canonical position in [0, n_d).
 * Returns 1 when x lies in A(t). */
int orc_perturbed(const orc_grid *g, const double *x, const double *lo, const double *hi, double t) {
  double r2 = 0.0;
  for (int d = 0; d < g->ndim; ++d) {
    double n = (double)g->n[d];
    double best = HUGE_VAL;
    for (int k = -1; k <= 1; ++k) {
      double a = lo[d] + k * n, b = hi[d] + k * n, s = 0.0;
      if (x[d] < a) s = a - x[d];
      else if (x[d] > b) s = x[d] - b;
      if (s < best) best = s;
    }
    double s = best * g->dx[d];
    r2 = r2 + s * s;
  }
  double ct = g->c * t;
  return r2 == 0.0 || r2 < ct * ct;
}

/* The particle step with the skip: a particle outside A(t) at time t of x^n
 * follows pure drift -- its momentum is kept, it moves with the velocity of
 * that momentum -- and deposits no current; a particle inside takes the full
 * step. */
void orc_push_species_skip(orc_grid *g, long np, double *x, double *u, double qm, double Q, const double *lo,
                           const double *hi, double t) {
  for (long p = 0; p < np; ++p) {
    double *xp = x + 3 * p, *up = u + 3 * p;
    if (orc_perturbed(g, xp, lo, hi, t)) {
      push_one(g, xp, up, qm, Q);
    } else {
      orc_move(g, xp, up);
      orc_wrap(g, xp);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Maxwell solver: Yee, or the Faraday stencil of Appendix C (M4)             */
/* ------------------------------------------------------------------------ */

static long idx3(const orc_grid *g, long i, long j, long k) {
  int ii = wrap_index(i, g->n[0]), jj = wrap_index(j, g->n[1]), kk = wrap_index(k, g->n[2]);
  return ii + (long)g->n[0] * (jj + (long)g->n[1] * kk);
}

/* Staggered forward difference of E component `comp` along axis d, placed
 * half a cell forward of the E node (where the B component lives). */
static double dfwd(const orc_grid *g, const double *f, int d, long i, long j, long k) {
  long o[3] = {0, 0, 0};
  o[d] = 1;
  if (d >= g->ndim) return 0.0;
  return (f[idx3(g, i + o[0], j + o[1], k + o[2])] - f[idx3(g, i, j, k)]) / g->dx[d];
}

/* Faraday derivative along d: Yee difference, times the operator
 * A_d = 1 + sum_{e != d} beta_de delta_e^2 + delta_d delta_d^2 for M4, where
 * delta_e^2 is the second difference along e, whose symbol is
 * -2[1 - cos(k_e dx_e)] (Eq. Maxwell-A).  Coefficients: beta_de =
 * (c dt/dx_e)^2/12, delta_d = ((c dt/dx_d)^2 - 1)/12 (Appendix C). */
static double faraday_d(const orc_grid *g, const double *f, int d, long i, long j, long k) {
  double v = dfwd(g, f, d, i, j, k);
  if (g->solver != ORC_M4) return v;
  double r = v;
  for (int e = 0; e < g->ndim; ++e) {
    long o[3] = {0, 0, 0};
    o[e] = 1;
    double ce = g->c * g->dt / g->dx[e];
    double coef;
    if (e == d) {
      coef = (ce * ce - 1.0) / 12.0;
    } else {
      coef = ce * ce / 12.0;
    }
    double vp = dfwd(g, f, d, i + o[0], j + o[1], k + o[2]);
    double vm = dfwd(g, f, d, i - o[0], j - o[1], k - o[2]);
    r += coef * (vp - 2.0 * v + vm);
  }
  return r;
}

/* B <- B - (dt/2) c curl E. */
void orc_faraday_half(orc_grid *g) {
  double h = 0.5 * g->dt * g->c;
  long nc = ncell_of(g);
  double *d0 = malloc(sizeof(double) * nc), *d1 = malloc(sizeof(double) * nc),
         *d2 = malloc(sizeof(double) * nc);
  for (long k = 0; k < g->n[2]; ++k)
    for (long j = 0; j < g->n[1]; ++j)
      for (long i = 0; i < g->n[0]; ++i) {
        long m = idx3(g, i, j, k);
        /* curl_1 = d2 E3 - d3 E2 at (i, j+1/2, k+1/2) */
        d0[m] = faraday_d(g, g->E[2], 1, i, j, k) - faraday_d(g, g->E[1], 2, i, j, k);
        /* curl_2 = d3 E1 - d1 E3 at (i+1/2, j, k+1/2) */
        d1[m] = faraday_d(g, g->E[0], 2, i, j, k) - faraday_d(g, g->E[2], 0, i, j, k);
        /* curl_3 = d1 E2 - d2 E1 at (i+1/2, j+1/2, k) */
        d2[m] = faraday_d(g, g->E[1], 0, i, j, k) - faraday_d(g, g->E[0], 1, i, j, k);
      }
  for (long m = 0; m < nc; ++m) {
    g->B[0][m] -= h * d0[m];
    g->B[1][m] -= h * d1[m];
    g->B[2][m] -= h * d2[m];
  }
  free(d0);
  free(d1);
  free(d2);
}

/* Backward staggered difference of a B component along d (Ampere, unmodified). */
static double dbwd(const orc_grid *g, const double *f, int d, long i, long j, long k) {
  long o[3] = {0, 0, 0};
  o[d] = 1;
  if (d >= g->ndim) return 0.0;
  return (f[idx3(g, i, j, k)] - f[idx3(g, i - o[0], j - o[1], k - o[2])]) / g->dx[d];
}

/* E <- E + dt (c curl B - J). */
void orc_ampere(orc_grid *g) {
  double dt = g->dt, c = g->c;
  long nc = ncell_of(g);
  double *d0 = malloc(sizeof(double) * nc), *d1 = malloc(sizeof(double) * nc),
         *d2 = malloc(sizeof(double) * nc);
  for (long k = 0; k < g->n[2]; ++k)
    for (long j = 0; j < g->n[1]; ++j)
      for (long i = 0; i < g->n[0]; ++i) {
        long m = idx3(g, i, j, k);
        d0[m] = dbwd(g, g->B[2], 1, i, j, k) - dbwd(g, g->B[1], 2, i, j, k);
        d1[m] = dbwd(g, g->B[0], 2, i, j, k) - dbwd(g, g->B[2], 0, i, j, k);
        d2[m] = dbwd(g, g->B[1], 0, i, j, k) - dbwd(g, g->B[0], 1, i, j, k);
      }
  for (long m = 0; m < nc; ++m) {
    g->E[0][m] += dt * (c * d0[m] - g->J[0][m]);
    g->E[1][m] += dt * (c * d1[m] - g->J[1][m]);
    g->E[2][m] += dt * (c * d2[m] - g->J[2][m]);
  }
  free(d0);
  free(d1);
  free(d2);
}

/* B^n -> B^{n+1/2} with E^n; E^n -> E^{n+1} with J^{n+1/2}; B^{n+1/2} ->
 * B^{n+1} with E^{n+1}.  B is thereby known at integer times, the average of
 * its half-step neighbours (the cos(omega' dt/2) factor of Eq. shapeEB). */
void orc_field_update(orc_grid *g) {
  orc_faraday_half(g);
  orc_ampere(g);
  orc_faraday_half(g);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

/* rho(x_g) += (Q/Vc) W_l(x - x_g) on integer nodes (Eq. shape-real). */
void orc_rho(const orc_grid *g, long np, const double *x, double Q, double *rho) {
  int l = g->order;
  double h = 0.5 * (l + 1);
  double Vc = 1.0;
  for (int d = 0; d < g->ndim; ++d) Vc *= g->dx[d];
  for (long p = 0; p < np; ++p) {
    const double *xp = x + 3 * p;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < g->ndim; ++d) {
      lo[d] = (int)ceil(xp[d] - h);
      hi[d] = (int)floor(xp[d] + h);
    }
    for (int m2 = lo[2]; m2 <= hi[2]; ++m2)
      for (int m1 = lo[1]; m1 <= hi[1]; ++m1)
        for (int m0 = lo[0]; m0 <= hi[0]; ++m0) {
          double w = orc_W(l, xp[0] - m0) * orc_W(l, xp[1] - m1);
          if (g->ndim == 3) w *= orc_W(l, xp[2] - m2);
          rho[idx3(g, m0, m1, m2)] += Q / Vc * w;
        }
  }
}

/* D.E on integer nodes: sum_d (E_d(m + 1/2 e_d) - E_d(m - 1/2 e_d))/dx_d
 * (the Gauss operator of Eq. gauss). */
void orc_div_E(const orc_grid *g, double *out) {
  for (long k = 0; k < g->n[2]; ++k)
    for (long j = 0; j < g->n[1]; ++j)
      for (long i = 0; i < g->n[0]; ++i) {
        double s = 0.0;
        for (int d = 0; d < g->ndim; ++d) s += dbwd(g, g->E[d], d, i, j, k);
        out[idx3(g, i, j, k)] = s;
      }
}

/* U_E[d] = 1/2 sum E_d^2 Vc, U_B[d] likewise. */
void orc_field_energy(const orc_grid *g, double *UE, double *UB) {
  double Vc = 1.0;
  for (int d = 0; d < g->ndim; ++d) Vc *= g->dx[d];
  long nc = ncell_of(g);
  for (int d = 0; d < 3; ++d) {
    double se = 0.0, sb = 0.0;
    for (long m = 0; m < nc; ++m) {
      se += g->E[d][m] * g->E[d][m];
      sb += g->B[d][m] * g->B[d][m];
    }
    UE[d] = 0.5 * se * Vc;
    UB[d] = 0.5 * sb * Vc;
  }
}

/* sum M (gamma - 1) c^2 over a species of macro-mass M. */
double orc_kinetic(long np, const double *u, double M, double c) {
  double s = 0.0;
  for (long p = 0; p < np; ++p) {
    const double *up = u + 3 * p;
    double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
    s += M * (gam - 1.0) * c * c;
  }
  return s;
}
