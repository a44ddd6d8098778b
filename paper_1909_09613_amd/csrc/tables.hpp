// Per-axis interpolation tables: the B-spline W_l and the WT factor T_l as
// polynomials in the in-cell coordinate.
//
// A particle at x~ (cell units) is split as x~ = base + sigma + g with
// base = floor(x~ - sigma) and g in [0, 1).  sigma is chosen per kernel so
// that all its nodes' weights are polynomials in g on [0, 1): for W_l no knot
// falls inside, for T_l exactly one (at kappa).  Node k (k = 0..K-1) is the
// lattice index base + first + k and carries
//     w_k(g) = sum_r c[k][r] g^r + alpha[k] * max(g - kappa, 0)^l.
// The tables are built on the host from the truncated-power form of each
// kernel (tables.cpp); the same evaluator runs on the host (table tests) and
// in the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace wtpic {

constexpr int kMaxNodes = 6;   // l + 2 for l = 4
constexpr int kMaxCoef = 5;    // degree l + 1 coefficients for l = 4

template <class Real>
struct Tab {
  Real sigma;                   // lattice shift of the split
  Real one_minus_sigma;         // 1 - sigma, so that g = f + (1 - sigma) rounds once
  Real kappa;                   // interior knot in g (>= 1 when there is none)
  int first;                    // node offset from base
  int K;                        // node count
  Real c[kMaxNodes][kMaxCoef];  // polynomial coefficients, c[k][r] of g^r
  Real alpha[kMaxNodes];        // coefficient of the knot term
};

// Split a position given as (cell, in-cell offset f in [0,1)) for a table.
template <class Real>
__host__ __device__ inline void tab_split(const Tab<Real>& t, int cell, Real f, int& base, Real& g) {
  if (t.sigma == Real(0)) {  // no split (folds away for constant tables)
    base = cell;
    g = f;
  } else {
    // selects rather than a branch: both sides are one instruction
    const bool below = f < t.sigma;
    base = cell - (below ? 1 : 0);
    g = below ? f + t.one_minus_sigma : f - t.sigma;
  }
}

template <class Real>
__host__ __device__ inline Real ipow(Real x, int l) {
  Real r = x;
  for (int i = 1; i < l; ++i) r *= x;
  return r;
}

// Weights w[0..K-1] at in-frame coordinate g (L = order, K = node count).
// top, if given, holds the leading coefficients c[k][L] (a copy the caller
// keeps elsewhere, e.g. in registers).
template <int L, int K, bool KNOT, class Real>
__host__ __device__ inline void tab_eval(const Tab<Real>& t, Real g, Real* w, const Real* top = nullptr) {
  Real tk = 0;
  if (KNOT) {
    Real d = g - t.kappa;
    d = d > Real(0) ? d : Real(0);
    tk = ipow(d, L);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    Real acc = top ? top[k] : t.c[k][L];
#pragma unroll
    for (int r = L - 1; r >= 0; --r) acc = acc * g + t.c[k][r];
    if (KNOT) acc += t.alpha[k] * tk;
    w[k] = acc;
  }
}

// Weight differences w_k(e) - w_k(g) = (e - g) * sum_{r>=1} c[k][r] h_r(g, e),
// h_r = sum_{i+j=r-1} g^i e^j, written as d * (divided difference) so that a
// short step d = e - g keeps full relative precision.  Knot-free tables only.
// CONST: the table is a compile-time constant, whose zero coefficients are
// left out (a product with a zero the compiler must otherwise keep).
template <int L, bool CONST = false, class Real>
__host__ __device__ inline void tab_diff(const Tab<Real>& t, Real g, Real e, Real d, Real* dw) {
  Real h[kMaxCoef];
  h[1] = Real(1);
  Real gp = g;  // g^(r-1)
#pragma unroll
  for (int r = 2; r <= L; ++r) {
    h[r] = h[r - 1] * e + gp;
    gp *= g;
  }
#pragma unroll
  for (int k = 0; k <= L; ++k) {
    Real acc = t.c[k][L] * h[L];
#pragma unroll
    for (int r = L - 1; r >= 1; --r)
      if (!CONST || t.c[k][r] != Real(0)) acc += t.c[k][r] * h[r];
    dw[k] = d * acc;
  }
}

// The B-spline tables (kinds 0 and 1 below) depend only on l and the
// lattice, so they are built at compile time: the same truncated-power
// expansion as build_table, in double (every quantity is a small rational).
// The particle kernel uses them as literal constants.
constexpr double cx_binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
constexpr double cx_frac(double x) {
  long long i = (long long)x;
  double f = x - (double)i;
  return f < 0.0 ? f + 1.0 : f;
}
template <class Real>
constexpr Tab<Real> make_wtab(int l, int kind) {
  Tab<Real> out{};
  double fact = 1.0;
  for (int i = 2; i <= l; ++i) fact *= i;
  const double lam = (kind == 0) ? 0.5 : 0.0;
  const double sigma = cx_frac(lam - 0.5 * (l + 1));
  const double first_f = sigma - lam - 0.5 * (l - 1);
  const int first = (int)(first_f < 0.0 ? first_f - 0.5 : first_f + 0.5);
  const int K = l + 1;
  const double D = sigma - first - lam;
  double c[kMaxNodes][kMaxCoef] = {};
  for (int k = 0; k < K; ++k)
    for (int j = 0; j <= l + 1; ++j) {
      const double beta = ((j & 1) ? -1.0 : 1.0) * cx_binom(l + 1, j) / fact;
      const double kp = (j - 0.5 * (l + 1)) + k - D;  // knot in g
      if (kp <= 1e-12) {
        for (int r = 0; r <= l; ++r) {
          double p = 1.0;
          for (int q = 0; q < l - r; ++q) p *= -kp;
          c[k][r] += beta * cx_binom(l, r) * p;
        }
      }
    }
  out.sigma = Real(sigma);
  out.one_minus_sigma = Real(1.0 - sigma);
  out.kappa = Real(2.0);
  out.first = first;
  out.K = K;
  for (int k = 0; k < kMaxNodes; ++k) {
    for (int r = 0; r < kMaxCoef; ++r) out.c[k][r] = Real(c[k][r]);
    out.alpha[k] = Real(0);
  }
  return out;
}

// Host: build the table of one kernel kind for order l.
//   kind 0: W_l on the half-integer lattice (nodes at m + 1/2)
//   kind 1: W_l on the integer lattice
//   kind 2: T_l(.; a) on the integer lattice, 0 < a < 1
// Returns false (and a message) on invalid input or an internal inconsistency.
bool build_table(int l, int kind, double a, Tab<double>& out, const char** err);

template <class Real>
inline void convert_table(const Tab<double>& in, Tab<Real>& out) {
  out.sigma = Real(in.sigma);
  out.one_minus_sigma = Real(in.one_minus_sigma);
  out.kappa = Real(in.kappa);
  out.first = in.first;
  out.K = in.K;
  for (int k = 0; k < kMaxNodes; ++k) {
    for (int r = 0; r < kMaxCoef; ++r) out.c[k][r] = Real(in.c[k][r]);
    out.alpha[k] = Real(in.alpha[k]);
  }
}

}  // namespace wtpic
