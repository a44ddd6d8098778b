// Host construction of the per-axis interpolation tables (see tables.hpp).
//
// Each kernel is written as a sum of truncated powers beta * (y - t)_+^l:
//   W_l(y)   = (1/l!) sum_{j=0}^{l+1} (-1)^j C(l+1, j) (y + (l+1)/2 - j)_+^l
//              (the B-spline of order l and width l+1, Sec. 2),
//   T_l(y;a) = 1/(2a l!) sum_{j=0}^{l} (-1)^j C(l, j)
//              [(y + a + l/2 - j)_+^l - (y - a + l/2 - j)_+^l]
//              (W_{l-1} averaged over [y - a, y + a]: the inverse Fourier
//              transform of tau_l = sinc^l(k dx/2) sinc(k c dt), Eq. tau_l).
// For a node at fixed offset from the split base, every term is either
// inactive on g in [0, 1), a full polynomial there, or has its knot inside
// (only for T_l, at g = kappa).  The expansion runs in long double.
#include <cmath>

#include "tables.hpp"

namespace wtpic {

namespace {

long double binom(int n, int k) {
  long double r = 1.0L;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

long double frac(long double x) { return x - floorl(x); }

}  // namespace

bool build_table(int l, int kind, double a_in, Tab<double>& out, const char** err) {
  static const char* kBadOrder = "order must be 1..4";
  static const char* kBadKind = "table kind must be 0, 1 or 2";
  static const char* kBadA = "WT factor needs 0 < c dt/dx < 1";
  static const char* kKnots = "internal: more than one interior knot";
  static const char* kUnity = "internal: table weights do not sum to one";
  if (l < 1 || l > 4) {
    if (err) *err = kBadOrder;
    return false;
  }
  if (kind < 0 || kind > 2) {
    if (err) *err = kBadKind;
    return false;
  }
  const long double a = a_in;
  if (kind == 2 && !(a > 0.0L && a < 1.0L)) {
    if (err) *err = kBadA;
    return false;
  }
  if (kind <= 1) {
    // B-spline tables: the compile-time construction the kernels use
    out = make_wtab<double>(l, kind);
    return true;
  }
  long double fact = 1.0L;
  for (int i = 2; i <= l; ++i) fact *= i;

  // T_l on the integer lattice: a sum of truncated powers beta (y - t)_+^l
  long double beta[16], t[16];
  int nterms = 0;
  const long double sigma = frac(0.5L * l + a);
  const long double first_f = sigma - 0.5L * l - a + 1.0L;
  const int K = (a_in <= 0.5) ? l + 1 : l + 2;
  for (int j = 0; j <= l; ++j) {
    long double b = ((j & 1) ? -1.0L : 1.0L) * binom(l, j) / (2.0L * a * fact);
    beta[nterms] = b;
    t[nterms] = j - 0.5L * l - a;
    ++nterms;
    beta[nterms] = -b;
    t[nterms] = j - 0.5L * l + a;
    ++nterms;
  }
  const int first = (int)lroundl(first_f);
  const long double D = sigma - first;  // y = g + D - k for node k

  long double c[kMaxNodes][kMaxCoef] = {};
  long double alpha[kMaxNodes] = {};
  long double kappa = 2.0L;
  bool have_knot = false;
  const long double tol = 1e-12L;
  for (int k = 0; k < K; ++k) {
    for (int i = 0; i < nterms; ++i) {
      long double kp = t[i] + k - D;  // knot of this term in g
      if (kp <= tol) {
        // beta (g - kp)^l = beta sum_r C(l, r) (-kp)^(l-r) g^r
        for (int r = 0; r <= l; ++r) {
          long double p = 1.0L;
          for (int q = 0; q < l - r; ++q) p *= -kp;
          c[k][r] += beta[i] * binom(l, r) * p;
        }
      } else if (kp < 1.0L - tol) {
        if (!have_knot) {
          kappa = kp;
          have_knot = true;
        } else if (fabsl(kp - kappa) > 1e-9L) {
          if (err) *err = kKnots;
          return false;
        }
        alpha[k] += beta[i];
      }
    }
  }

  out.sigma = (double)sigma;
  out.one_minus_sigma = (double)(1.0L - sigma);
  out.kappa = (double)kappa;
  out.first = first;
  out.K = K;
  for (int k = 0; k < kMaxNodes; ++k) {
    for (int r = 0; r < kMaxCoef; ++r) out.c[k][r] = (k < K) ? (double)c[k][r] : 0.0;
    out.alpha[k] = (k < K) ? (double)alpha[k] : 0.0;
  }

  // self-check: the weights of a table sum to one at any g
  for (int s = 0; s <= 16; ++s) {
    long double g = s / 16.0L * 0.999999L;
    long double sum = 0.0L;
    for (int k = 0; k < K; ++k) {
      long double acc = 0.0L, gp = 1.0L;
      for (int r = 0; r <= l; ++r) {
        acc += c[k][r] * gp;
        gp *= g;
      }
      long double d = g - kappa;
      if (d > 0) {
        long double p = 1.0L;
        for (int q = 0; q < l; ++q) p *= d;
        acc += alpha[k] * p;
      }
      sum += acc;
    }
    if (fabsl(sum - 1.0L) > 1e-12L) {
      if (err) *err = kUnity;
      return false;
    }
  }
  return true;
}

}  // namespace wtpic
