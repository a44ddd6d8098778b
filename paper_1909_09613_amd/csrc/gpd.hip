// Gather + Boris push + Esirkepov deposit for one tile's particles per
// workgroup (gfx950, wave64, no MFMA: nothing here is a dense contraction).
//
// A workgroup owns one tile g (a rectangle of cells of one run) and the two
// particle segments (electrons, positrons) the last counting sort assigned to
// it.  The particles have drifted since that sort; the tile keeps the
// bounding box of its particles' cells (tile-relative, refreshed by every
// step), and the workgroup stages E and B on that box plus the gather reach
// into LDS, accumulates the current of the box plus the deposit reach in an
// LDS tile, and flushes that tile to the FP64 global current with one atomic
// add per node.  When a box outgrows the staging margin the tile requests a
// re-sort, which the next sort pass performs before the box can overflow.
//
// Per particle (Sec. 2 and the methods it cites):
//   gather   Eq. interpolation-EB-real-mod: along an axis on which a component
//            is staggered the B-spline W_l on the half-integer lattice, across
//            it T_l (WT) or W_l (MC) on the integer lattice.  In 2D the x3
//            factor is one (nothing depends on x3, both kernels sum to one).
//            (E1, B2) and (E2, B1) share lattice and weights in 2D and are
//            staged as pairs.
//   push     relativistic Boris: half kick, rotation, half kick.
//   move     x~ += (c dt/dx) u / gamma; FP32 keeps cell + offset in [0,1).
//   deposit  form-factor differences DS = S1 - S0 on the union of old and
//            new nodes, evaluated as step * divided difference so that short
//            transverse steps keep their precision in FP32; Esirkepov's
//            decomposition W_x = DS_x (S0_y + DS_y/2) etc., prefix sums along
//            each component's own axis.
#include <climits>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace wtpic {

namespace {

template <class Real>
struct Pair;
template <>
struct Pair<float> {
  using T = float2;
};
template <>
struct Pair<double> {
  using T = double2;
};

// A move by step (|step| < 1 cell) from in-cell offset f in [0, 1): the new
// offset t and the cell change dc in {-1, 0, 1}.  f + step lies in (-1, 2);
// its floor is dc and the remainder t (exact for f + step >= 0, one rounding
// below).  Just below the lower face that rounding can give t = 1: the
// particle then stays on the face of its old cell (t = 0, dc = 0).
template <class Real>
__device__ __forceinline__ void cell_step(Real f, Real step, Real& t, int& dc) {
  const Real x = f + step;
  const Real fl = floor(x);
  const Real r = x - fl;
  const bool up = r >= Real(1);
  t = up ? Real(0) : r;
  dc = up ? 0 : (int)fl;
}

// The periodic image in [0, n) of a cell m = c + dc reached by a step dc in
// {-1, 0, 1} from c in [0, n): m is then -1, n or already in range.  One
// unsigned compare (-1 is out of range too), and the sign bit of m selects
// n - 1 or 0.
__device__ __forceinline__ int wrap_step(int m, int n) {
  return ((unsigned)m >= (unsigned)n) ? ((m >> 31) & (n - 1)) : m;
}

// Product of two integers of magnitude below 2^23 (window indices, pitches
// and their products within a window) on the full-rate 24-bit multiplier;
// a 32-bit multiply by a variable issues at a quarter of the rate.
__device__ __forceinline__ int imul24(int a, int b) { return __mul24(a, b); }

// Sum over a 3D stencil of a staged component: weights along x, y, z are wx
// (NX nodes), wy (NY), wz (NZ); ox, oy, oz the window index of the first node;
// px, pz the window's row and plane pitch.
template <int NX, int NY, int NZ, class Real>
__device__ __forceinline__ Real gather3(const Real* Fc, int px, int pz, const Real* wx, const Real* wy,
                                        const Real* wz, int ox, int oy, int oz) {
  Real s = Real(0);
  const Real* base = Fc + (ox + imul24(px, oy) + imul24(pz, oz));
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    Real sy = Real(0);
#pragma unroll
    for (int j = 0; j < NY; ++j) {
      const Real* row = base + (px * j + pz * k);
      Real sx = Real(0);
#pragma unroll
      for (int i = 0; i < NX; ++i) sx += wx[i] * row[i];
      sy += wy[j] * sx;
    }
    s += wz[k] * sy;
  }
  return s;
}

// Weights of a B-spline table's NW nodes at g.  The cubic B-spline of the
// compile-time tables in its symmetric closed form, 11 instructions against
// 12 for the four Horner polynomials: with t = 1 - g, w0 = t^3/6,
// w1 = 2/3 - g^2 + g^3/2, w2 the same at t, w3 = g^3/6 (the coefficients of
// those tables, checked where they are built).
template <int L, int NW, bool CONSTTAB, class Real>
__device__ __forceinline__ void wtab_eval(const Tab<Real>& T, Real g, Real* w) {
  if constexpr (CONSTTAB && L == 3 && NW == 4) {
    const Real t = Real(1) - g;
    const Real g2 = g * g, t2 = t * t;
    w[0] = t2 * (t * Real(1.0 / 6.0));
    w[1] = fma(g2, fma(g, Real(0.5), Real(-1)), Real(2.0 / 3.0));
    w[2] = fma(t2, fma(t, Real(0.5), Real(-1)), Real(2.0 / 3.0));
    w[3] = g2 * (g * Real(1.0 / 6.0));
  } else {
    tab_eval<L, NW, false>(T, g, w);
  }
}

// Weight differences w_k(e) - w_k(g) = d * (divided difference), d = e - g,
// for a table's L + 1 nodes.  For the cubic B-spline of the compile-time
// tables with h2 = g + e and h3 = g^2 + g e + e^2: the differences of the
// four closed forms above are d (h3/6), d ((h2 - 1)/2 - h3/6) and
// d (h3/2 - h2) for nodes 3, 0 and 1, and node 2 takes minus their sum (the
// weights sum to one), 12 instructions against 16.
template <int L, bool CONSTTAB, class Real>
__device__ __forceinline__ void wtab_diff(const Tab<Real>& T, Real g, Real e, Real d, Real* dw) {
  if constexpr (CONSTTAB && L == 3) {
    const Real h2 = g + e;
    const Real h3 = fma(h2, e, g * g);
    const Real q = h3 * (d * Real(1.0 / 6.0));
    dw[3] = q;
    dw[0] = fma(h2 - Real(1), d * Real(0.5), -q);
    dw[1] = fma(Real(3), q, -(d * h2));
    dw[2] = -(dw[0] + dw[1]) - q;
  } else {
    tab_diff<L, CONSTTAB>(T, g, e, d, dw);
  }
}

// Whether a table holds the cubic B-spline polynomials in the node order of
// wtab_eval's closed form.
template <class Real>
constexpr bool is_cubic_bspline(const Tab<Real>& t) {
  constexpr double ref[4][4] = {{1.0 / 6, -0.5, 0.5, -1.0 / 6}, {2.0 / 3, 0.0, -1.0, 0.5},
                                {1.0 / 6, 0.5, 0.5, -0.5}, {0.0, 0.0, 0.0, 1.0 / 6}};
  for (int k = 0; k < 4; ++k)
    for (int r = 0; r < 4; ++r) {
      const double d = (double)t.c[k][r] - ref[k][r];
      if (d > 1e-6 || d < -1e-6) return false;
    }
  return true;
}

template <class Real>
__device__ __forceinline__ bool finite3(Real a, Real b, Real c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

template <class Acc>
__device__ __forceinline__ void lds_add(Acc* p, Acc v) {
  atomicAdd(p, v);
}

// Fixed-point LDS accumulation modulo 2^32.  v is in units of the tile's
// quantum plus one half, so that rounding down (one VALU conversion) rounds
// the value to the nearest integer.
__device__ __forceinline__ void lds_addq(int* p, float v) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  atomicAdd(reinterpret_cast<unsigned*>(p), (unsigned)r);
}
__device__ __forceinline__ void lds_addq(int* p, double v) {
  atomicAdd(reinterpret_cast<unsigned*>(p), (unsigned)(int)floor(v));
}

// Keeps a tile-constant integer in a vector register.  The particle loop
// uses about twenty of them next to the run's tables; left to scalar
// registers they spill, and each reload costs a vector instruction.
__device__ __forceinline__ int in_vgpr(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ float in_vgpr(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Split of a position for a table known only at run time (T_l): with
// d = f - sigma in (-1, 1), g = fract(d) and base = cell - (d < 0), one
// fract where a select between two run-time constants takes three
// instructions.  (fract returns d + 1 for d < 0, clamped below 1, and d
// itself when the table has no split, sigma = 0.)
__device__ __forceinline__ float fract_(float x) { return __builtin_amdgcn_fractf(x); }
__device__ __forceinline__ double fract_(double x) { return __builtin_amdgcn_fract(x); }
template <class Real>
__device__ __forceinline__ void split_rt(const Tab<Real>& t, int cell, Real f, int& base, Real& g) {
  const Real d = f - t.sigma;
  base = cell - (d < Real(0) ? 1 : 0);
  g = fract_(d);
}

// Element of a particle array at a byte offset from its base.  The particle
// loop addresses a tile's arrays from the tile's first particle with one
// 32-bit offset that the compiler cannot rewrite into per-array pointers:
// every access is then a scalar base plus that vector offset, one add per
// particle, instead of a 64-bit pointer per array advanced every iteration
// in vector registers.
template <class T>
__device__ __forceinline__ T& at(T* base, unsigned off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}
// (A block that stores through an offset computed in another block takes it
// through fresh_off first: the address then forms in the storing block, where
// it can still be split into the scalar base and the vector offset.)
template <class Real>
__device__ __forceinline__ unsigned part_off(int q) {
  unsigned o = (unsigned)q * (unsigned)sizeof(Real);
  asm volatile("" : "+v"(o));
  return o;
}
__device__ __forceinline__ unsigned fresh_off(unsigned o) {
  asm volatile("" : "+v"(o));
  return o;
}

// m mod n for -n <= m < n, without an integer division or a compare: the
// sign bit selects n.  A cell index and the box's periodic low end, both
// reduced to [0, n), differ by less than n.
__device__ __forceinline__ int wrap_once(int m, int n) { return m + (n & (m >> 31)); }

// 1 / sqrt(x) and 1 / x for x >= 1 (1 + |u|^2, 1 + |t|^2).  FP32: the
// hardware approximations (1 ulp).  FP64: the hardware estimates (about 23
// correct bits) refined by two Newton steps, each of which doubles the
// correct bits, to within a few ulp (the IEEE square root and division
// take about 20 instructions each; 7 and 5 here).  An infinite argument (a
// diverged particle) gives NaN, which the push reports as non-finite.
__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rsqrt(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);  // y (3 - x y^2) / 2
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);  // y (2 - x y)
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// ---- partially skipped calculation (Sec. 3) ---------------------------------
// A particle at canonical position x (cell units, [0, n) per axis) lies in
// the perturbed region at time t when its distance to the box A0 =
// [lo, hi] (nearest periodic image, Euclidean in physical units) is below
// c t, or zero (A(0) = A0).  FP64 without contraction: the decision does not
// depend on how a compiler fuses the arithmetic.
__device__ __forceinline__ double skip_ct(double t0, long long steps, double dt, double c) {
#pragma clang fp contract(off)
  const double t = t0 + (double)steps * dt;
  return c * t;
}

template <int DIM, class Real>
__device__ __forceinline__ bool skip_perturbed(const RunDev<Real>& R, const double* x, double ct) {
#pragma clang fp contract(off)
  double r2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double n = (double)R.n[d];
    double best = __builtin_huge_val();
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
      const double a = R.skip_lo[d] + k * n, b = R.skip_hi[d] + k * n;
      double sd = 0.0;
      if (x[d] < a) sd = a - x[d];
      else if (x[d] > b) sd = x[d] - b;
      best = sd < best ? sd : best;
    }
    const double sd = best * R.dxd[d];
    r2 = r2 + sd * sd;
  }
  return r2 == 0.0 || r2 < ct * ct;
}

// Nearest-image distance along one axis for any x in (-3n, 4n).
__device__ __forceinline__ double skip_axis_any(double x, double lo, double hi, double n) {
  double best = __builtin_huge_val();
  for (int k = -3; k <= 3; ++k) {
    const double a = lo + k * n, b = hi + k * n;
    const double sd = x < a ? a - x : (x > b ? x - b : 0.0);
    best = fmin(best, sd);
  }
  return best;
}

// Smallest and largest nearest-image distance along one axis over x in
// [a, b]: the gap to the nearest image, and the larger end value unless the
// point halfway round the axis from the box lies inside (then half the
// complement of the box).
__device__ __forceinline__ void skip_axis_range(double a, double b, double lo, double hi, double n, double& dmin,
                                                double& dmax) {
  dmin = __builtin_huge_val();
  for (int k = -3; k <= 3; ++k) dmin = fmin(dmin, fmax(0.0, fmax(lo + k * n - b, a - (hi + k * n))));
  const double far = 0.5 * (n - (hi - lo));
  if (b - a >= n) {
    dmax = far;
    return;
  }
  dmax = fmax(skip_axis_any(a, lo, hi, n), skip_axis_any(b, lo, hi, n));
  for (int k = -3; k <= 3; ++k) {
    const double pm = hi + far + k * n;
    if (pm >= a && pm <= b) dmax = far;
  }
}

}  // namespace

// Workgroup size and waves per SIMD of the particle kernel.  2D, and the
// plain 3D kernel up to l = 2: 512 threads held to four waves per SIMD (two
// groups per CU, at most 128 registers).  The 3D kernel with the partially
// skipped calculation: 256 threads at three waves; the plain 3D kernel for
// l >= 3 (more registers than four waves allow without heavy spilling):
// 256 threads, unconstrained.
template <int L, int DIM, bool SKIP>
struct GpdShape {
  static constexpr bool kWide = DIM == 2 || (!SKIP && L <= 2);
  static constexpr int kBlock = kWide ? 512 : 256;
  static constexpr int kWaves = kWide ? 4 : (SKIP ? 3 : 1);
};

template <class P, int L, int DIM, int KT, bool SKIP, int CP>
__device__ __forceinline__ void gpd_tile(const GpdArgs<typename P::Real>& A,
                                         const RunDev<typename P::Real>* __restrict__ runs,
                                         const int* __restrict__ tile_run, const int g,
                                         unsigned char* lds, int* sred, typename P::Real* spc) {
  using Real = typename P::Real;
  using Acc = typename P::Acc;
  using Real2 = typename Pair<Real>::T;
  constexpr int NW = L + 1;  // W nodes
  constexpr int NU = L + 2;  // union of old and new form-factor nodes
  // B-spline tables on the half-integer and the integer lattice: constants
  constexpr Tab<Real> kWh = make_wtab<Real>(L, 0);
  constexpr Tab<Real> kWi = make_wtab<Real>(L, 1);
  static_assert(L != 3 || (is_cubic_bspline(kWh) && is_cubic_bspline(kWi)), "cubic tables");
  const int tid = threadIdx.x;
  const int nth = GpdShape<L, DIM, SKIP>::kBlock;

  const int r = tile_run[g];
  const RunDev<Real>& R = runs[r];
  const int lt = g - R.tile0;
  int org[3];
  org[0] = (lt % R.ntile[0]) * A.tile[0];
  org[1] = ((lt / R.ntile[0]) % R.ntile[1]) * A.tile[1];
  org[2] = (DIM == 3) ? (lt / (R.ntile[0] * R.ntile[1])) * A.tile[2] : 0;

  int bb[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) bb[i] = A.bbox[g * 6 + i];
  int fo[3] = {0, 0, 0}, fs[3] = {1, 1, 1}, jo[3] = {0, 0, 0}, jsz[3] = {1, 1, 1};
  bool fits = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    fo[d] = bb[2 * d] + R.glo[d];
    fs[d] = bb[2 * d + 1] + R.ghi[d] - fo[d] + 1;
    jo[d] = bb[2 * d] + R.dlo[d];
    jsz[d] = bb[2 * d + 1] + R.dhi[d] - jo[d] + 1;
    fits = fits && fs[d] >= 1 && jsz[d] >= 1 && fs[d] <= A.fw[d] && jsz[d] <= A.jw[d];
  }
  const int sA = A.seg[2 * g], sB = A.seg[2 * g + 1], sC = A.seg[2 * g + 2];
  // byte offsets within the tile are 32-bit
  fits = fits && (unsigned)(sC - sA) <= 0xffffffffu / (unsigned)sizeof(Real);
  if (!fits) {
    // cannot happen while the re-sort guard holds; report and leave the tile
    if (tid == 0) {
      atomicAdd(&A.st->n_out_of_range, (unsigned long long)(sC - sA));
      atomicOr(&A.st->sort_request, 1);
    }
    return;
  }

  // partially skipped calculation: 0 every particle of the tile steps, 1
  // every one drifts, 2 decided per particle.  The classification bounds the
  // distance over the box of the particles' cells, with a relative margin so
  // that it never contradicts the per-particle decision.
  int smode = 0;
  double ct = 0.0;
  if (SKIP && R.skip_on) {
    ct = skip_ct(R.skip_t0, (long long)A.st->gpd_launches - R.skip_l0, R.dtd, R.cd);
    double rmin2 = 0.0, rmax2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double dmin, dmax;
      skip_axis_range((double)(org[d] + bb[2 * d]), (double)(org[d] + bb[2 * d + 1] + 1), R.skip_lo[d],
                      R.skip_hi[d], (double)R.n[d], dmin, dmax);
      rmin2 += (dmin * R.dxd[d]) * (dmin * R.dxd[d]);
      rmax2 += (dmax * R.dxd[d]) * (dmax * R.dxd[d]);
    }
    const double c2 = ct * ct;
    if (rmax2 == 0.0 || rmax2 < c2 * (1.0 - 1e-9))
      smode = 0;
    else if (rmin2 > c2 * (1.0 + 1e-9) + 1e-300)
      smode = 1;
    else
      smode = 2;
  }

  // windows: index x + row pitch * y + plane pitch * z (the pitches may
  // exceed the extents, so that the rows a wave reads at once spread over
  // the LDS banks)
  // (CP = 1: the pitches are the compile-time constants of FixedPitch, so
  // that the rows and planes of a stencil are immediate offsets from one
  // address)
  constexpr bool kCP = CP != 0;
  using FP = FixedPitch<DIM>;
  const int fpx = kCP ? FP::f[0] : A.fp[0];
  const int fpz = (kCP && DIM == 3) ? FP::f[1] : A.fp[1];
  const int fcap = (DIM == 3) ? fpz * A.fw[2] : fpx * A.fw[1];
  const int jpx = kCP ? FP::j[0] : A.jp[0];
  const int jpz = (kCP && DIM == 3) ? FP::j[1] : A.jp[1];
  const int jcap = (DIM == 3) ? jpz * A.jw[2] : jpx * A.jw[1];
  const long long NT = A.ncell_total;
  const Real* Fg = A.F + R.cell0;

  // Mixed precision accumulates the tile's current as 32-bit fixed point
  // (FP64 LDS atomics cost about twice as much as integer ones, FP32 LDS
  // atomics far more).  Every contribution of a particle to component c is
  // bounded by |js_c| m_c, where m_c is the particle's step |d_c| along
  // axis c (a prefix sum of S1 - S0 changes by at most the step, and the
  // path-averaged transverse shapes lie in [0, 1]), or |v3| for the
  // out-of-plane current in 2D.  A node receives contributions only from
  // particles whose cell lies within l + 3 cells of it per axis, at most
  // (l + 3)^d times the tile's largest count of particles in one cell.  The
  // quantum is chosen so that this many particles with m_c <= thr_c
  // (thr_c = 2 * the tile's largest m_c of the previous step, or of the
  // stored velocities after a sort) give a node value below 2^31 quanta;
  // the sums are taken modulo 2^32, so only the final value must fit.  A
  // component above its threshold goes to a second set of windows that
  // accumulates in FP32 with floating-point atomics instead: slow per add,
  // but such components are rare (a step more than twice the tile's largest
  // of the previous step) and keep FP32's relative precision, where a
  // fixed-point window sized for any particle (|v| < c) would round a
  // thermal-scale contribution to a thousandth.
  constexpr bool kFix = !P::kAbs;
  // cell counts (the (l+3)^d cmax bound) only in 2D: a 3D tile holds fewer
  // particles than (l+3)^3 times its densest cell, so its bound is the tile's
  // particle count, and the LDS the counts would take buys 3D tiles room
  constexpr bool kCnt = kFix && DIM == 2;
  // 3D keeps its coarse (FP32) windows in a private region of global memory
  // (only the rare components above their bound touch them), so that its LDS
  // holds larger tiles at two groups per CU
  constexpr bool kGlobCoarse = kFix && DIM == 3;
  Real qinv[3] = {Real(0), Real(0), Real(0)}, thr[3] = {Real(0), Real(0), Real(0)};
  double qd[3] = {0.0, 0.0, 0.0};
  // largest step per component in this launch (>= 0, kept as the bit
  // pattern of an FP32 value: integer max orders non-negative floats, and
  // needs no NaN canonicalisation)
  int mnew[3] = {0, 0, 0};
  if (kFix) {
    int reach = 1;
    for (int d = 0; d < DIM; ++d) reach *= L + 3;
    const double nmax = fmin((double)(sC - sA), (double)reach * (double)A.jb[4 * g + 3]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      thr[c] = Real(2) * Real(A.jb[4 * g + c]);
      const double jm = fmax(fabs(R.js[0][c]), fabs(R.js[1][c]));
      const double bnd = nmax * jm * (double)thr[c];
      if (bnd > 0.0) {
        qd[c] = bnd / 2145386496.0;  // 2^31 (1 - 2^-10): room for rounding
        qinv[c] = Real(1.0 / qd[c]);
      }
    }
  }

  // species constants of the particle loop, one row per species in LDS (a
  // particle's species is decided per lane, so its row is read with one LDS
  // load rather than selected from registers): (q/m) dt / (2c) and the
  // current scales, in fine quanta on the fixed-point path
  if (tid < 2) {
    spc[4 * tid] = R.eps[tid];
#pragma unroll
    for (int c = 0; c < 3; ++c) spc[4 * tid + 1 + c] = kFix ? Real(R.js[tid][c]) * qinv[c] : Real(R.js[tid][c]);
  }

  Real2* P1 = nullptr;
  Real2* P2 = nullptr;
  Real* P3 = nullptr;
  Real* P4 = nullptr;
  Real* F6 = nullptr;
  Acc* Jl;
  if (DIM == 2) {
    P1 = reinterpret_cast<Real2*>(lds);
    P2 = P1 + fcap;
    P3 = reinterpret_cast<Real*>(P2 + fcap);
    P4 = P3 + fcap;
    Jl = reinterpret_cast<Acc*>(P4 + fcap);
  } else {
    F6 = reinterpret_cast<Real*>(lds);
    Jl = reinterpret_cast<Acc*>(F6 + 6 * fcap);
  }
  // fixed-point path: 3 fine int windows and 3 coarse FP32 windows, then
  // (2D) the particle count per cell
  int* Qf = reinterpret_cast<int*>(Jl);
  float* Qc = kGlobCoarse ? reinterpret_cast<float*>(A.coarse + (long long)blockIdx.x * A.coarse_cap)
                          : reinterpret_cast<float*>(Qf + 3 * jcap);
  int* Cw = Qf + 6 * jcap;

  // ---- stage E, B on the window; clear the current tile ------------------
  const int nfs = (smode == 1) ? 0 : fs[0] * fs[1] * fs[2];
  for (int i = tid; i < nfs; i += nth) {
    const int w0 = i % fs[0];
    const int q = i / fs[0];
    const int w1 = q % fs[1];
    const int w2 = q / fs[1];
    const int gx = wrapi(org[0] + fo[0] + w0, R.n[0]);
    const int gy = wrapi(org[1] + fo[1] + w1, R.n[1]);
    const int gz = (DIM == 3) ? wrapi(org[2] + fo[2] + w2, R.n[2]) : 0;
    const long long gi = gx + (long long)R.n[0] * (gy + (long long)R.n[1] * gz);
    const int li = w0 + fpx * w1 + fpz * w2;
    if (DIM == 2) {
      Real2 a, b;
      a.x = Fg[0 * NT + gi];
      a.y = Fg[4 * NT + gi];
      b.x = Fg[1 * NT + gi];
      b.y = Fg[3 * NT + gi];
      P1[li] = a;
      P2[li] = b;
      P3[li] = Fg[2 * NT + gi];
      P4[li] = Fg[5 * NT + gi];
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) F6[c * fcap + li] = Fg[c * NT + gi];
    }
  }
  if (kFix) {
    for (int i = tid; i < (kCnt ? 7 : (kGlobCoarse ? 3 : 6)) * jcap; i += nth) Qf[i] = 0;
  } else {
    for (int i = tid; i < 3 * jcap; i += nth) Jl[i] = Acc(0);
  }
  if (tid < 6) sred[tid] = (tid & 1) ? INT_MIN : INT_MAX;
  if (tid >= 6 && tid < 13) sred[tid] = 0;
  __syncthreads();

  // 2D FP32: the leading coefficients of the T_l tables in vector registers,
  // so that the first Horner step of each node reads one scalar operand (an
  // instruction reads at most one) and needs no copy
  Real ttop[2][KT];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int k = 0; k < KT; ++k) ttop[d][k] = (kFix && DIM == 2) ? in_vgpr(float(R.T[d].c[k][L])) : Real(0);

  // the tile's particles, from its first one (offsets from part_off)
  PBuf<Real> B = A.buf[A.st->parity];
  B.cell += sA;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    B.pos[d] += sA;
    B.u[d] += sA;
  }
  int bmin[3] = {INT_MAX, INT_MAX, INT_MAX}, bmax[3] = {INT_MIN, INT_MIN, INT_MIN};
  int nbad = 0, noor = 0;
  const Real third = Real(1) / Real(3);
  const Real half = Real(0.5);
  // per-axis constants of the loop: the periodic image of a particle's cell
  // is rel = wrap(c - co, n) + lo, and it must lie in [rlo, rhi] for the
  // staged windows; window offsets of the half-lattice, T and union stencils
  // (kept in vector registers on the FP32 path, where scalar registers run
  // out; the FP64 path and the 512-thread 3D kernel need their vector
  // registers for their own state, within 128 for four waves per SIMD)
  auto pin = [](int x) { return (P::kAbs || (DIM == 3 && GpdShape<L, DIM, SKIP>::kWide)) ? x : in_vgpr(x); };
  int co[3], lo_[3], nn[3], rlo[3], rhi[3], hoff[3], toff[3], uoff[3], jo_[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int n = R.n[d];
    const int slack = max(0, n - 1 - (bb[2 * d + 1] - bb[2 * d]));
    const int lo = bb[2 * d] - (slack >> 1);
    co[d] = pin(wrapi(org[d] + lo, n));
    lo_[d] = pin(lo);
    nn[d] = pin(n);
    rlo[d] = pin(max(fo[d] - R.glo[d], jo[d] - R.dlo[d]));
    rhi[d] = pin(min(fo[d] + fs[d] - 1 - R.ghi[d], jo[d] + jsz[d] - 1 - R.dhi[d]));
    hoff[d] = pin(R.Wh[d].first - fo[d]);
    toff[d] = pin(R.T[d].first - fo[d]);
    uoff[d] = pin(R.Wi[d].first - jo[d]);
    jo_[d] = pin(jo[d]);
  }
  // offset along axis d in the current and count windows (their row and
  // plane pitch; compile-time constants in the 2D variant with fixed pitches)
  auto cwin = [&](int d, int r) { return d == 0 ? r : imul24(r, d == 1 ? jpx : jpz); };

  // partially skipped calculation: outside the perturbed region a particle
  // follows pure drift -- it keeps its momentum, moves with that momentum's
  // velocity (the arithmetic of the move in the loop below) and deposits no
  // current; it still counts for the box, the cell counts and the next
  // step's fixed-point bounds
  auto drift = [&](unsigned o_in, const int* c, const Real* f, const Real* xo, Real u0, Real u1, Real u2, const int* rel) {
    const unsigned o = fresh_off(o_in);
    const Real ig = fast_rsqrt(Real(1) + u0 * u0 + u1 * u1 + u2 * u2);
    const Real vd[3] = {u0 * ig, u1 * ig, u2 * ig};
    int cwi = 0, cw[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const Real step = R.a[d] * vd[d];
      int cnd;
      Real ddd;
      if (P::kAbs) {
        const Real xn = xo[d] + step;
        cnd = (int)floor(xn);
        ddd = xn - xo[d];
        Real w = xn;
        const Real nd = Real(R.n[d]);
        while (w < Real(0)) w += nd;
        while (w >= nd) w -= nd;
        at(B.pos[d], o) = w;
      } else {
        Real t;
        int dc;
        cell_step(f[d], step, t, dc);
        cnd = c[d] + dc;
        ddd = (t - f[d]) + Real(dc);
        at(B.pos[d], o) = t;
        cw[d] = wrap_step(cnd, R.n[d]);
      }
      // a drifting particle still bounds the next step's fixed-point scale
      if (kFix) mnew[d] = max(mnew[d], __float_as_int((float)fabs(ddd)));
      const int rn = rel[d] + (cnd - c[d]);
      bmin[d] = min(bmin[d], rn);
      bmax[d] = max(bmax[d], rn);
      cwi += cwin(d, rn - jo_[d]);
    }
    if (kFix && DIM == 2) mnew[2] = max(mnew[2], __float_as_int((float)fabs(vd[2])));
    if (kCnt) atomicAdd(Cw + cwi, 1);
    if (!P::kAbs) at(B.cell, o) = pack_cell<DIM>(cw[0], cw[1], cw[2]);
  };
  if (SKIP && smode == 1) {
    // every particle of the tile drifts: several particles per thread with
    // their loads issued together (this loop is bound by memory latency)
    constexpr int U = 4;
    for (int p0 = sA + tid; p0 < sC; p0 += U * nth) {
      int cc[U][3];
      Real ff[U][3], xx[U][3], uu[U][3];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const unsigned o = part_off<Real>(min(p0 + k * nth, sC - 1) - sA);
        cc[k][0] = cc[k][1] = cc[k][2] = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) ff[k][d] = xx[k][d] = Real(0);
        if (P::kAbs) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) xx[k][d] = at(B.pos[d], o);
        } else {
          unpack_cell<DIM>(at(B.cell, o), cc[k][0], cc[k][1], cc[k][2]);
#pragma unroll
          for (int d = 0; d < DIM; ++d) ff[k][d] = at(B.pos[d], o);
        }
        uu[k][0] = at(B.u[0], o);
        uu[k][1] = at(B.u[1], o);
        uu[k][2] = at(B.u[2], o);
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int p = p0 + k * nth;
        if (p >= sC) break;
        if (P::kAbs) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const Real fl = floor(xx[k][d]);
            cc[k][d] = (int)fl;
            ff[k][d] = xx[k][d] - fl;
          }
        }
        int rel[3] = {0, 0, 0};
        bool inwin = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int rr = wrap_once(cc[k][d] - co[d], nn[d]) + lo_[d];
          rel[d] = rr;
          inwin = inwin && rr >= rlo[d] && rr <= rhi[d];
        }
        if (!inwin) {
          ++noor;
          continue;
        }
        drift(part_off<Real>(p - sA), cc[k], ff[k], xx[k], uu[k][0], uu[k][1], uu[k][2], rel);
      }
    }
  }

  for (int p = (SKIP && smode == 1) ? sC : sA + tid; p < sC; p += nth) {
    const int sp = (p >= sB) ? 1 : 0;
    const unsigned o = part_off<Real>(p - sA);
    // ---- load ---------------------------------------------------------
    int c[3] = {0, 0, 0};
    Real f[3] = {Real(0), Real(0), Real(0)};
    Real xo[3] = {Real(0), Real(0), Real(0)};
    if (P::kAbs) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        xo[d] = at(B.pos[d], o);
        const Real fl = floor(xo[d]);
        c[d] = (int)fl;
        f[d] = xo[d] - fl;
      }
    } else {
      unpack_cell<DIM>(at(B.cell, o), c[0], c[1], c[2]);
#pragma unroll
      for (int d = 0; d < DIM; ++d) f[d] = at(B.pos[d], o);
    }
    Real u0 = at(B.u[0], o), u1 = at(B.u[1], o), u2 = at(B.u[2], o);
    // all six loads are in flight before anything waits on one of them (left
    // alone, the compiler sinks the offset and momentum loads below the
    // window test, a second memory round trip per particle)
    asm volatile("" ::"v"(u0), "v"(u1), "v"(u2), "v"(f[0]), "v"(f[1]), "v"(f[DIM - 1]), "v"(xo[0]));

    int rel[3] = {0, 0, 0};
    bool inwin = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // periodic image nearest the box: rel in [lo, lo + n), the box centred
      // in that range (a box as wide as the axis starts it)
      const int rr = wrap_once(c[d] - co[d], nn[d]) + lo_[d];
      rel[d] = rr;
      inwin = inwin && rr >= rlo[d] && rr <= rhi[d];
    }
    if (!inwin) {
      ++noor;
      continue;
    }
    if constexpr (SKIP) {
      bool drifting = smode == 1;
      if (smode == 2) {
        double xa[3];
#pragma unroll
        for (int d = 0; d < DIM; ++d) xa[d] = P::kAbs ? (double)xo[d] : (double)c[d] + (double)f[d];
        drifting = !skip_perturbed<DIM>(R, xa, ct);
      }
      if (drifting) {
        drift(o, c, f, xo, u0, u1, u2, rel);
        continue;
      }
    }

    // ---- weights at x^n --------------------------------------------------
    Real wh[3][NW], wt[3][KT];
    int ih[3] = {0, 0, 0}, it[3] = {0, 0, 0};
    // FP32 evaluates the B-spline tables from literal constants; FP64 loads
    // them (64-bit literals would each take registers)
    auto weights_h = [&](int d, const Tab<Real>& Th) {
      int b;
      Real gg;
      tab_split(Th, c[d], f[d], b, gg);
      wtab_eval<L, NW, kFix>(Th, gg, wh[d]);
      ih[d] = rel[d] + (b - c[d]) + hoff[d];
    };
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if constexpr (kFix) weights_h(d, kWh);
      else weights_h(d, R.Wh[d]);
      int b;
      Real gg;
      split_rt(R.T[d], c[d], f[d], b, gg);
      tab_eval<L, KT, true>(R.T[d], gg, wt[d], (kFix && DIM == 2) ? ttop[d] : nullptr);
      it[d] = rel[d] + (b - c[d]) + toff[d];
    }

    // ---- gather ------------------------------------------------------------
    Real E0, E1, E2, B0, B1, B2;
    if (DIM == 2) {
      const int rt = imul24(fpx, it[1]), rh = imul24(fpx, ih[1]);
      // (E1, B2): W along x (half lattice), T along y
      E0 = B1 = Real(0);
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        const Real2* row = P1 + (ih[0] + rt) + fpx * j;
        Real se = Real(0), sb = Real(0);
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const Real2 v = row[i];
          se += wh[0][i] * v.x;
          sb += wh[0][i] * v.y;
        }
        E0 += wt[1][j] * se;
        B1 += wt[1][j] * sb;
      }
      // (E2, B1): T along x, W along y (half lattice)
      E1 = B0 = Real(0);
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const Real2* row = P2 + (it[0] + rh) + fpx * j;
        Real se = Real(0), sb = Real(0);
#pragma unroll
        for (int i = 0; i < KT; ++i) {
          const Real2 v = row[i];
          se += wt[0][i] * v.x;
          sb += wt[0][i] * v.y;
        }
        E1 += wh[1][j] * se;
        B0 += wh[1][j] * sb;
      }
      const Real one = Real(1);
      E2 = gather3<KT, KT, 1>(P3, fpx, fpz, wt[0], wt[1], &one, it[0], it[1], 0);
      B2 = gather3<NW, NW, 1>(P4, fpx, fpz, wh[0], wh[1], &one, ih[0], ih[1], 0);
    } else {
      E0 = gather3<NW, KT, KT>(F6 + 0 * fcap, fpx, fpz, wh[0], wt[1], wt[2], ih[0], it[1], it[2]);
      E1 = gather3<KT, NW, KT>(F6 + 1 * fcap, fpx, fpz, wt[0], wh[1], wt[2], it[0], ih[1], it[2]);
      E2 = gather3<KT, KT, NW>(F6 + 2 * fcap, fpx, fpz, wt[0], wt[1], wh[2], it[0], it[1], ih[2]);
      B0 = gather3<KT, NW, NW>(F6 + 3 * fcap, fpx, fpz, wt[0], wh[1], wh[2], it[0], ih[1], ih[2]);
      B1 = gather3<NW, KT, NW>(F6 + 4 * fcap, fpx, fpz, wh[0], wt[1], wh[2], ih[0], it[1], ih[2]);
      B2 = gather3<NW, NW, KT>(F6 + 5 * fcap, fpx, fpz, wh[0], wh[1], wt[2], ih[0], ih[1], it[2]);
    }

    // ---- Boris -------------------------------------------------------------
    const Real eps = spc[4 * sp];
    const Real umx = u0 + eps * E0, umy = u1 + eps * E1, umz = u2 + eps * E2;
    const Real igm = fast_rsqrt(Real(1) + umx * umx + umy * umy + umz * umz);
    const Real tx = eps * B0 * igm, ty = eps * B1 * igm, tz = eps * B2 * igm;
    const Real s2 = Real(2) * fast_rcp(Real(1) + tx * tx + ty * ty + tz * tz);
    const Real sx = s2 * tx, sy = s2 * ty, sz = s2 * tz;
    const Real upx = umx + (umy * tz - umz * ty);
    const Real upy = umy + (umz * tx - umx * tz);
    const Real upz = umz + (umx * ty - umy * tx);
    const Real n0 = umx + (upy * sz - upz * sy) + eps * E0;
    const Real n1 = umy + (upz * sx - upx * sz) + eps * E1;
    const Real n2 = umz + (upx * sy - upy * sx) + eps * E2;
    if (!finite3(n0, n1, n2)) {
      ++nbad;
      // leave the particle where it is; its box entry keeps the window valid
      int cwi = 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        bmin[d] = min(bmin[d], rel[d]);
        bmax[d] = max(bmax[d], rel[d]);
        cwi += cwin(d, rel[d] - jo_[d]);
      }
      if (kCnt) atomicAdd(Cw + cwi, 1);
      continue;
    }
    u0 = n0;
    u1 = n1;
    u2 = n2;

    // ---- move ------------------------------------------------------------
    const Real igam = fast_rsqrt(Real(1) + u0 * u0 + u1 * u1 + u2 * u2);
    const Real vv[3] = {u0 * igam, u1 * igam, u2 * igam};
    int cn[3] = {0, 0, 0};
    Real fn[3] = {Real(0), Real(0), Real(0)}, dd[3] = {Real(0), Real(0), Real(0)};
    Real xw[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const Real step = R.a[d] * vv[d];
      if (P::kAbs) {
        const Real xn = xo[d] + step;
        const Real fl = floor(xn);
        cn[d] = (int)fl;
        fn[d] = xn - fl;
        dd[d] = xn - xo[d];
        Real w = xn;
        const Real nd = Real(R.n[d]);
        while (w < Real(0)) w += nd;
        while (w >= nd) w -= nd;
        xw[d] = w;
      } else {
        Real t;
        int dc;
        cell_step(f[d], step, t, dc);
        fn[d] = t;
        cn[d] = c[d] + dc;
        dd[d] = (t - f[d]) + Real(dc);
      }
    }

    // ---- form factors and their differences on the union stencil -----------
    Real S0u[3][NU], DSu[3][NU];
    int iu[3] = {0, 0, 0};
    bool cross[3] = {false, false, false};  // union stencil one node wider than S0
    auto form_factors = [&](int d, const Tab<Real>& Tw) {
      int b0, b1;
      Real g0, g1;
      tab_split(Tw, c[d], f[d], b0, g0);
      tab_split(Tw, cn[d], fn[d], b1, g1);
      Real s0[NW], s1[NW], dA[NW], dB[NW], a0[NU], ds[NU];
      wtab_eval<L, NW, kFix>(Tw, g0, s0);
      const int db = b1 - b0;
      cross[d] = db != 0;
      const bool shA = db < 0, shB = db > 0;
      iu[d] = rel[d] + (min(b0, b1) - c[d]) + uoff[d];
      // Node k of the union is node k of S0 unless the new stencil starts one
      // node lower (shA), then node k - 1.  A wave whose steps are all short
      // and none of which changed its stencil takes the cheapest form.
      if (__all(fabs(dd[d]) >= Real(0.0625))) {
        // every step of the wave is long: S1 - S0 directly keeps its
        // precision (rounding of order one against |step| >= 1/16)
        wtab_eval<L, NW, kFix>(Tw, g1, s1);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
          a0[k] = shA ? (k >= 1 ? s0[k - 1] : Real(0)) : (k < NW ? s0[k] : Real(0));
          const Real a1 = shB ? (k >= 1 ? s1[k - 1] : Real(0)) : (k < NW ? s1[k] : Real(0));
          ds[k] = a1 - a0[k];
        }
      } else if (!__any(db != 0)) {
        // no lane of the wave changed its stencil: one divided difference
        wtab_diff<L, kFix>(Tw, g0, g1, dd[d], dA);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
          a0[k] = k < NW ? s0[k] : Real(0);
          ds[k] = k < NW ? dA[k] : Real(0);
        }
      } else {
        // a stencil that moved splits its difference at the lattice point
        // it crossed (an end of g's range)
        const Real eA = (db == 0) ? g1 : (db > 0 ? Real(1) : Real(0));
        const Real lA = (db == 0) ? dd[d] : (db > 0 ? Real(1) - g0 : -g0);
        wtab_diff<L, kFix>(Tw, g0, eA, lA, dA);
        if (db != 0) {
          const Real sBv = (db > 0) ? Real(0) : Real(1);
          const Real lB = (db > 0) ? g1 : g1 - Real(1);
          wtab_diff<L, kFix>(Tw, sBv, g1, lB, dB);
        } else {
#pragma unroll
          for (int k = 0; k < NW; ++k) dB[k] = Real(0);
        }
#pragma unroll
        for (int k = 0; k < NU; ++k) {
          a0[k] = shA ? (k >= 1 ? s0[k - 1] : Real(0)) : (k < NW ? s0[k] : Real(0));
          const Real da = shA ? (k >= 1 ? dA[k - 1] : Real(0)) : (k < NW ? dA[k] : Real(0));
          const Real dbv = shB ? (k >= 1 ? dB[k - 1] : Real(0)) : (k < NW ? dB[k] : Real(0));
          ds[k] = da + dbv;
        }
      }
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        S0u[d][k] = a0[k];
        DSu[d][k] = ds[k];
      }
    };
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if constexpr (kFix) form_factors(d, kWi);
      else form_factors(d, R.Wi[d]);
    }

    // ---- Esirkepov current into the LDS tile -----------------------------
    // sink(c, i, v) adds v to component c at window index i; kx, ky, kz are
    // the current scales (-Q dx/(Vc dt) per axis, Q c / Vc for J3 in 2D),
    // multiplied by the tile's fixed-point scale for a component that goes
    // to a fixed-point window, and the values of component c carry the
    // offset oc (one half there, else zero).
    // Window indices are jb (the particle's first union node) plus offsets
    // that are the same for every lane (uniform, or immediates when the row
    // pitch is a compile-time constant), so a row costs one add at most.
    auto deposit = [&](auto sink, const Real kx, const Real ky, const Real kz, const Real ox, const Real oy,
                       const Real oz) {
      const int jb = iu[0] + imul24(jpx, iu[1]) + (DIM == 3 ? imul24(jpz, iu[2]) : 0);
      if (DIM == 2) {
        // Slot L+1 of an axis (and the last prefix face along it) is nonzero
        // only when the particle's stencil widened along that axis.
#pragma unroll
        for (int v = 0; v < NU; ++v) {
          if (v == L + 1 && !cross[1]) continue;
          const Real fy = kx * (S0u[1][v] + half * DSu[1][v]);
          const int ro = jpx * v;
          Real acc = ox;
#pragma unroll
          for (int u = 0; u < L; ++u) {
            acc += DSu[0][u] * fy;
            sink(0, jb + (ro + u), acc);
          }
          if (cross[0]) sink(0, jb + (ro + L), acc + DSu[0][L] * fy);
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (u == L + 1 && !cross[0]) continue;
          const Real fx = ky * (S0u[0][u] + half * DSu[0][u]);
          Real acc = oy;
#pragma unroll
          for (int v = 0; v < L; ++v) {
            acc += DSu[1][v] * fx;
            sink(1, jb + (u + jpx * v), acc);
          }
          if (cross[1]) sink(1, jb + (u + jpx * L), acc + DSu[1][L] * fx);
        }
        const Real vz = kz * vv[2];
#pragma unroll
        for (int v = 0; v < NU; ++v) {
          if (v == L + 1 && !cross[1]) continue;
          const Real Av = vz * (S0u[1][v] + half * DSu[1][v]);
          const Real Bv = vz * (half * S0u[1][v] + third * DSu[1][v]);
          const int ro = jpx * v;
#pragma unroll
          for (int u = 0; u <= L; ++u)
            sink(2, jb + (ro + u),
                 kFix ? fma(S0u[0][u], Av, fma(DSu[0][u], Bv, oz)) : S0u[0][u] * Av + DSu[0][u] * Bv);
          if (cross[0])
            sink(2, jb + (ro + L + 1), kFix ? fma(S0u[0][L + 1], Av, fma(DSu[0][L + 1], Bv, oz))
                                            : S0u[0][L + 1] * Av + DSu[0][L + 1] * Bv);
        }
      } else {
        // path averages of the transverse shapes: (S0 + DS/2) and (S0/2 + DS/3)
        // enter as S0_b (S0_c + DS_c/2) + DS_b (S0_c/2 + DS_c/3); the prefix
        // sums run over DS scaled by the component's current scale, from the
        // component's offset, so that a node's value is the running sum itself
        const Real ks[3] = {kx, ky, kz};
        Real pa[3][NU], pb[3][NU], dk[3][NU];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int k = 0; k < NU; ++k) {
            pa[d][k] = S0u[d][k] + half * DSu[d][k];
            pb[d][k] = half * S0u[d][k] + third * DSu[d][k];
            dk[d][k] = ks[d] * DSu[d][k];
          }
        // J1: prefix along x of DS_x * T_yz
#pragma unroll
        for (int w = 0; w < NU; ++w) {
#pragma unroll
          for (int v = 0; v < NU; ++v) {
            if ((v == L + 1 && !cross[1]) || (w == L + 1 && !cross[2])) continue;
            const Real tr = S0u[1][v] * pa[2][w] + DSu[1][v] * pb[2][w];
            const int ro = jpx * v + jpz * w;
            Real acc = ox;
#pragma unroll
            for (int u = 0; u <= L; ++u) {
              acc += dk[0][u] * tr;
              if (u < L || cross[0]) sink(0, jb + (ro + u), acc);
            }
          }
        }
        // J2: prefix along y of DS_y * T_xz
#pragma unroll
        for (int w = 0; w < NU; ++w) {
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            if ((u == L + 1 && !cross[0]) || (w == L + 1 && !cross[2])) continue;
            const Real tr = S0u[0][u] * pa[2][w] + DSu[0][u] * pb[2][w];
            const int co = u + jpz * w;
            Real acc = oy;
#pragma unroll
            for (int v = 0; v <= L; ++v) {
              acc += dk[1][v] * tr;
              if (v < L || cross[1]) sink(1, jb + (co + jpx * v), acc);
            }
          }
        }
        // J3: prefix along z of DS_z * T_xy
#pragma unroll
        for (int v = 0; v < NU; ++v) {
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            if ((u == L + 1 && !cross[0]) || (v == L + 1 && !cross[1])) continue;
            const Real tr = S0u[0][u] * pa[1][v] + DSu[0][u] * pb[1][v];
            const int co = u + jpx * v;
            Real acc = oz;
#pragma unroll
            for (int w = 0; w <= L; ++w) {
              acc += dk[2][w] * tr;
              if (w < L || cross[2]) sink(2, jb + (co + jpz * w), acc);
            }
          }
        }
      }
    };
    const Real ksp[3] = {spc[4 * sp + 1], spc[4 * sp + 2], spc[4 * sp + 3]};
    if (!kFix) {
      deposit([&](int c, int i, Real v) { lds_add<Acc>(Jl + c * jcap + i, Acc(v)); }, ksp[0], ksp[1], ksp[2],
              Real(0), Real(0), Real(0));
    } else {
      // a component whose step (or |v3|) exceeds the tile's bound deposits
      // into the coarse windows, so that no fine node sum can overflow; the
      // particle's other components stay in the fine windows (a kick along
      // one axis leaves the others' precision alone)
      const Real m0 = fabs(dd[0]), m1 = fabs(dd[1]), m2 = (DIM == 2) ? fabs(vv[2]) : fabs(dd[2]);
      mnew[0] = max(mnew[0], __float_as_int((float)m0));
      mnew[1] = max(mnew[1], __float_as_int((float)m1));
      mnew[2] = max(mnew[2], __float_as_int((float)m2));
      if (m0 <= thr[0] && m1 <= thr[1] && m2 <= thr[2]) {
        deposit([&](int c, int i, Real v) { lds_addq(Qf + c * jcap + i, v); }, ksp[0], ksp[1], ksp[2], half, half,
                half);
      } else {
        const bool f0 = m0 <= thr[0], f1 = m1 <= thr[1], f2 = m2 <= thr[2];
        const Real jx = Real(R.js[sp][0]), jy = Real(R.js[sp][1]), jz = Real(R.js[sp][2]);
        if constexpr (kGlobCoarse) sred[12] = 1;  // the flush reads the global coarse window
        deposit(
            [&](int c, int i, Real v) {
              if (c == 0 ? f0 : (c == 1 ? f1 : f2))
                lds_addq(Qf + c * jcap + i, v);
              else
                atomicAdd(Qc + c * jcap + i, (float)v);
            },
            f0 ? jx * qinv[0] : jx, f1 ? jy * qinv[1] : jy, f2 ? jz * qinv[2] : jz, f0 ? half : Real(0),
            f1 ? half : Real(0), f2 ? half : Real(0));
      }
    }

    // ---- store, box --------------------------------------------------------
    int cwi = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int rn = rel[d] + (cn[d] - c[d]);
      bmin[d] = min(bmin[d], rn);
      bmax[d] = max(bmax[d], rn);
      cwi += cwin(d, rn - jo_[d]);
    }
    if (kCnt) atomicAdd(Cw + cwi, 1);
    const unsigned os = fresh_off(o);
    if (P::kAbs) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) at(B.pos[d], os) = xw[d];
    } else {
      int cw[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        cw[d] = wrap_step(cn[d], R.n[d]);
        at(B.pos[d], os) = fn[d];
      }
      at(B.cell, os) = pack_cell<DIM>(cw[0], cw[1], cw[2]);
    }
    at(B.u[0], os) = u0;
    at(B.u[1], os) = u1;
    at(B.u[2], os) = u2;
  }

  // ---- box and counters: wave reduction, then one LDS atomic per wave ------
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      bmin[d] = min(bmin[d], __shfl_xor(bmin[d], off));
      bmax[d] = max(bmax[d], __shfl_xor(bmax[d], off));
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    nbad += __shfl_xor(nbad, off);
    noor += __shfl_xor(noor, off);
    if (kFix) {
#pragma unroll
      for (int c = 0; c < 3; ++c) mnew[c] = max(mnew[c], __shfl_xor(mnew[c], off));
    }
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      atomicMin(&sred[2 * d], bmin[d]);
      atomicMax(&sred[2 * d + 1], bmax[d]);
    }
    if (nbad) atomicAdd(&sred[6], nbad);
    if (noor) atomicAdd(&sred[7], noor);
    if (kFix) {
#pragma unroll
      for (int c = 0; c < 3; ++c) atomicMax(&sred[8 + c], mnew[c]);
    }
  }
  __syncthreads();
  if (kCnt) {
    // largest particle count of one cell at the new positions (particles
    // left in place by a non-finite push are counted at their cell)
    int cm = 0;
    for (int i = tid; i < jcap; i += nth) cm = max(cm, Cw[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cm = max(cm, __shfl_xor(cm, off));
    if ((tid & 63) == 0) atomicMax(&sred[11], cm);
  }

  // ---- flush the current tile ------------------------------------------------
  double* Jg = A.J + R.cell0;
  [[maybe_unused]] const bool coarse_used = kGlobCoarse && sred[12] != 0;
  const int njs = (smode == 1) ? 0 : jsz[0] * jsz[1] * jsz[2];
  for (int i = tid; i < njs; i += nth) {
    const int w0 = i % jsz[0];
    const int q = i / jsz[0];
    const int w1 = q % jsz[1];
    const int w2 = q / jsz[1];
    const int gx = wrapi(org[0] + jo[0] + w0, R.n[0]);
    const int gy = wrapi(org[1] + jo[1] + w1, R.n[1]);
    const int gz = (DIM == 3) ? wrapi(org[2] + jo[2] + w2, R.n[2]) : 0;
    const long long gi = gx + (long long)R.n[0] * (gy + (long long)R.n[1] * gz);
    const int li = w0 + jpx * w1 + jpz * w2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v;
      if constexpr (kGlobCoarse) {
        v = (double)Qf[c * jcap + li] * qd[c];
        if (coarse_used) {
          // the coarse sums were added at the L2; read them there and leave
          // the window zero for the group's next tile
          float* q = Qc + c * jcap + li;
          v += (double)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(q, 0.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else {
        v = kFix ? (double)Qf[c * jcap + li] * qd[c] + (double)Qc[c * jcap + li] : (double)Jl[c * jcap + li];
      }
      if (v != 0.0) unsafeAtomicAdd(Jg + c * NT + gi, v);
    }
  }
  if (kGlobCoarse && coarse_used) __threadfence();  // the clears land before the next tile's adds

  if (kCnt) __syncthreads();
  if (tid == 0) {
    bool need = false;
    for (int d = 0; d < 3; ++d) {
      int lo = 0, hi = 0;
      if (d < DIM) {
        lo = sred[2 * d];
        hi = sred[2 * d + 1];
        if (lo > hi) {  // no particles: keep the tile rectangle
          lo = 0;
          hi = min(A.tile[d], R.n[d] - org[d]) - 1;
        }
        need = need || (hi - lo > A.guard[d]);
        // a box that drifted a whole period keeps canonical coordinates
        const int mid = (lo + hi) >> 1;
        const int shift = R.n[d] * (mid >= 0 ? mid / R.n[d] : -((R.n[d] - 1 - mid) / R.n[d]));
        lo -= shift;
        hi -= shift;
      }
      A.bbox[g * 6 + 2 * d] = lo;
      A.bbox[g * 6 + 2 * d + 1] = hi;
    }
    if (need) atomicOr(&A.st->sort_request, 1);
    if (kFix) {
      for (int c = 0; c < 3; ++c) A.jb[4 * g + c] = __int_as_float(sred[8 + c]);
      A.jb[4 * g + 3] = kCnt ? (float)sred[11] : 3.0e38f;  // 3D: the tile count bounds
    }
    if (sred[6]) atomicAdd(&A.st->n_nonfinite, (unsigned long long)sred[6]);
    if (sred[7]) atomicAdd(&A.st->n_out_of_range, (unsigned long long)sred[7]);
  }
}

// Persistent workgroups: each takes tiles from a device queue until none are
// left, so uneven tiles (edge tiles, runs of different size) balance.  The
// queue starts at zero (set at initialisation, then rewound by the last
// group of every launch).  Waves per SIMD and group size as GpdShape gives:
// where the kernel is held to four waves per SIMD (two 512-thread groups per
// CU, at most 128 registers), a fifth register block would drop a wave and
// halve the groups a CU holds, which costs far more than a few spilled
// values (3D, l = 2: 2.90 ms against 3.10 ms for three 256-thread groups of
// 156 registers at 256x128x128).
template <class P, int L, int DIM, bool SKIP, int CP>
__global__ void __launch_bounds__((GpdShape<L, DIM, SKIP>::kBlock))
__attribute__((amdgpu_waves_per_eu(GpdShape<L, DIM, SKIP>::kWaves)))
    gpd_kernel(GpdArgs<typename P::Real> A, const RunDev<typename P::Real>* __restrict__ runs,
               const int* __restrict__ tile_run) {
  extern __shared__ __align__(16) unsigned char lds_dyn[];
  __shared__ int sred[13];
  __shared__ int next;
  __shared__ __align__(32) typename P::Real spc[8];   // per-species constants of the tile's run
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(&A.st->tile_queue, 1);
    __syncthreads();
    const int g = next;
    __syncthreads();
    if (g >= A.G) {
      // the last group to find the queue empty rewinds it for the next
      // launch (every group has taken its final ticket by then)
      if (threadIdx.x == 0 && atomicAdd(&A.st->groups_done, 1u) == gridDim.x - 1) {
        A.st->tile_queue = 0;
        A.st->groups_done = 0;
        A.st->gpd_launches += 1;
      }
      return;
    }
    const int kt = runs[tile_run[g]].KT;
    if (kt == L + 1)
      gpd_tile<P, L, DIM, L + 1, SKIP, CP>(A, runs, tile_run, g, lds_dyn, sred, spc);
    else
      gpd_tile<P, L, DIM, L + 2, SKIP, CP>(A, runs, tile_run, g, lds_dyn, sred, spc);
    __syncthreads();
  }
}

template <class P, int L, int DIM, bool SKIP, int CP>
static hipError_t launch_variant(const GpdArgs<typename P::Real>& a, size_t lds, hipStream_t s) {
  const int grid = a.G < a.max_groups ? a.G : a.max_groups;
  const void* k = reinterpret_cast<const void*>(&gpd_kernel<P, L, DIM, SKIP, CP>);
  if (lds > 64 * 1024) {
    // more than the default dynamic LDS of a launch (explicit large tiles)
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gpd_kernel<P, L, DIM, SKIP, CP>), dim3(grid), dim3(GpdShape<L, DIM, SKIP>::kBlock), lds, s,
                     a, a.runs,
                     a.tile_run);
  return hipGetLastError();
}

template <class P, int L, int DIM>
static hipError_t launch_one(const GpdArgs<typename P::Real>& a, size_t lds, hipStream_t s) {
  // the variant with the partially skipped calculation only where a run uses
  // it (its extra registers would cost the plain step occupancy); mixed
  // precision windows of the fixed pitches take the variant compiled for them
  // (in 3D up to l = 2: larger orders have larger windows)
  if constexpr (!P::kAbs && (DIM == 2 || L <= 2)) {
    using FP = FixedPitch<DIM>;
    if (a.fp[0] == FP::f[0] && a.jp[0] == FP::j[0] && (DIM == 2 || (a.fp[1] == FP::f[1] && a.jp[1] == FP::j[1])))
      return a.skip ? launch_variant<P, L, DIM, true, 1>(a, lds, s) : launch_variant<P, L, DIM, false, 1>(a, lds, s);
  }
  return a.skip ? launch_variant<P, L, DIM, true, 0>(a, lds, s) : launch_variant<P, L, DIM, false, 0>(a, lds, s);
}

// Charge density of one run for the diagnostics, tile by tile (Eq.
// shape-real: rho(m) += (Q/Vc) prod_d W_l(x_d - m_d) on integer nodes).
// Each workgroup takes tiles of the run; it adds its tile's particles into an
// FP64 LDS window over the tile's box plus the form-factor reach and then
// adds the window to the global array.  The particles must sit in their
// tiles' segments with boxes from the last step (as after any step); a
// particle outside the window (not expected) is added to global memory
// directly.
template <class P, int L, int DIM>
__global__ void __launch_bounds__(256) rho_tiles_kernel(GpdArgs<typename P::Real> A, int run, double* rho) {
  using Real = typename P::Real;
  extern __shared__ __align__(16) unsigned char lds_dyn[];
  double* W = reinterpret_cast<double*>(lds_dyn);
  const RunDev<Real>& R = A.runs[run];
  const int ntiles = R.ntile[0] * R.ntile[1] * R.ntile[2];
  const int jwx = A.jw[0], jwy = A.jw[1];
  const int jcap = jwx * jwy * (DIM == 3 ? A.jw[2] : 1);
  const PBuf<Real> B = A.buf[A.st->parity];
  const int tid = threadIdx.x;
  const double qv[2] = {R.Q[0] / R.Vc, R.Q[1] / R.Vc};
  for (int lt = blockIdx.x; lt < ntiles; lt += gridDim.x) {
    const int g = R.tile0 + lt;
    int org[3];
    org[0] = (lt % R.ntile[0]) * A.tile[0];
    org[1] = ((lt / R.ntile[0]) % R.ntile[1]) * A.tile[1];
    org[2] = (DIM == 3) ? (lt / (R.ntile[0] * R.ntile[1])) * A.tile[2] : 0;
    int jo[3] = {0, 0, 0}, jsz[3] = {1, 1, 1}, co[3] = {0, 0, 0}, lo_[3] = {0, 0, 0}, rlo[3] = {0, 0, 0},
        rhi[3] = {0, 0, 0};
    bool fits = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int blo = A.bbox[g * 6 + 2 * d], bhi = A.bbox[g * 6 + 2 * d + 1];
      jo[d] = blo + R.dlo[d];
      jsz[d] = bhi + R.dhi[d] - jo[d] + 1;
      fits = fits && jsz[d] >= 1 && jsz[d] <= A.jw[d];
      const int slack = max(0, R.n[d] - 1 - (bhi - blo));
      lo_[d] = blo - (slack >> 1);
      co[d] = wrapi(org[d] + lo_[d], R.n[d]);
      // a particle's nodes are rel + (base - cell) + first .. + L with
      // base - cell in {-1, 0}
      rlo[d] = jo[d] + 1 - R.Wi[d].first;
      rhi[d] = jo[d] + jsz[d] - 1 - L - R.Wi[d].first;
    }
    if (!fits) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) rlo[d] = INT_MAX;  // every particle takes the global path
    }
    for (int i = tid; i < jcap; i += blockDim.x) W[i] = 0.0;
    __syncthreads();
    const int sA = A.seg[2 * g], sB = A.seg[2 * g + 1], sC = A.seg[2 * g + 2];
    for (int p = sA + tid; p < sC; p += blockDim.x) {
      const int sp = (p >= sB) ? 1 : 0;
      int c[3] = {0, 0, 0};
      Real f[3] = {Real(0), Real(0), Real(0)};
      if (P::kAbs) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const Real x = B.pos[d][p];
          const Real fl = floor(x);
          c[d] = (int)fl;
          f[d] = x - fl;
        }
      } else {
        unpack_cell<DIM>(B.cell[p], c[0], c[1], c[2]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) f[d] = B.pos[d][p];
      }
      Real w[3][L + 1];
      int m[3] = {0, 0, 0}, mg[3] = {0, 0, 0};
      bool inwin = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        int b;
        Real gg;
        tab_split(R.Wi[d], c[d], f[d], b, gg);
        tab_eval<L, L + 1, false>(R.Wi[d], gg, w[d]);
        const int rel = wrap_once(c[d] - co[d], R.n[d]) + lo_[d];
        inwin = inwin && rel >= rlo[d] && rel <= rhi[d];
        m[d] = rel + (b - c[d]) + R.Wi[d].first - jo[d];  // window index of the first node
        mg[d] = b + R.Wi[d].first;                        // its lattice index
      }
      const double q = qv[sp];
      const int nz = (DIM == 3) ? L + 1 : 1;
      for (int kz = 0; kz < nz; ++kz)
#pragma unroll
        for (int ky = 0; ky <= L; ++ky) {
          double wyz = q * (double)w[1][ky];
          if (DIM == 3) wyz *= (double)w[2][kz];
#pragma unroll
          for (int kx = 0; kx <= L; ++kx) {
            const double v = wyz * (double)w[0][kx];
            if (inwin) {
              atomicAdd(W + (m[0] + kx) + jwx * ((m[1] + ky) + jwy * (m[2] + kz)), v);
            } else {
              const int gx = wrapi(mg[0] + kx, R.n[0]), gy = wrapi(mg[1] + ky, R.n[1]);
              const int gz = (DIM == 3) ? wrapi(mg[2] + kz, R.n[2]) : 0;
              unsafeAtomicAdd(rho + gx + (long long)R.n[0] * (gy + (long long)R.n[1] * gz), v);
            }
          }
        }
    }
    __syncthreads();
    const int njs = fits ? jsz[0] * jsz[1] * jsz[2] : 0;
    for (int i = tid; i < njs; i += blockDim.x) {
      const int w0 = i % jsz[0];
      const int q = i / jsz[0];
      const int w1 = q % jsz[1];
      const int w2 = q / jsz[1];
      const double v = W[w0 + jwx * (w1 + jwy * w2)];
      if (v == 0.0) continue;
      const int gx = wrapi(org[0] + jo[0] + w0, R.n[0]);
      const int gy = wrapi(org[1] + jo[1] + w1, R.n[1]);
      const int gz = (DIM == 3) ? wrapi(org[2] + jo[2] + w2, R.n[2]) : 0;
      unsafeAtomicAdd(rho + gx + (long long)R.n[0] * (gy + (long long)R.n[1] * gz), v);
    }
    __syncthreads();
  }
}

template <class P, int L, int DIM>
static hipError_t launch_rho_one(const GpdArgs<typename P::Real>& a, int run, int ntiles, double* rho, size_t lds,
                                 hipStream_t s) {
  const int grid = ntiles < 2048 ? ntiles : 2048;
  hipLaunchKernelGGL((rho_tiles_kernel<P, L, DIM>), dim3(grid), dim3(256), lds, s, a, run, rho);
  return hipGetLastError();
}

template <class P>
hipError_t launch_rho_tiles(const GpdArgs<typename P::Real>& a, int run, int ntiles, double* rho, int order,
                            int ndim, size_t lds, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ndim == 2) {
    switch (order) {
      case 1: return launch_rho_one<P, 1, 2>(a, run, ntiles, rho, lds, s);
      case 2: return launch_rho_one<P, 2, 2>(a, run, ntiles, rho, lds, s);
      case 3: return launch_rho_one<P, 3, 2>(a, run, ntiles, rho, lds, s);
      case 4: return launch_rho_one<P, 4, 2>(a, run, ntiles, rho, lds, s);
    }
  } else {
    switch (order) {
      case 1: return launch_rho_one<P, 1, 3>(a, run, ntiles, rho, lds, s);
      case 2: return launch_rho_one<P, 2, 3>(a, run, ntiles, rho, lds, s);
      case 3: return launch_rho_one<P, 3, 3>(a, run, ntiles, rho, lds, s);
      case 4: return launch_rho_one<P, 4, 3>(a, run, ntiles, rho, lds, s);
    }
  }
  return hipErrorInvalidValue;
}

template <class P, int L, int DIM>
static int occupancy_one(size_t lds, bool skip) {
  const void* k = skip ? reinterpret_cast<const void*>(&gpd_kernel<P, L, DIM, true, 0>)
                       : reinterpret_cast<const void*>(&gpd_kernel<P, L, DIM, false, 0>);
  if (lds > 64 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n = 0;
  const int block = skip ? GpdShape<L, DIM, true>::kBlock : GpdShape<L, DIM, false>::kBlock;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds);
  return (e == hipSuccess && n > 0) ? n : 1;
}

template <class P>
int gpd_groups_per_cu(int order, int ndim, size_t lds, bool skip) {
  if (ndim == 2) {
    switch (order) {
      case 1: return occupancy_one<P, 1, 2>(lds, skip);
      case 2: return occupancy_one<P, 2, 2>(lds, skip);
      case 3: return occupancy_one<P, 3, 2>(lds, skip);
      case 4: return occupancy_one<P, 4, 2>(lds, skip);
    }
  } else {
    switch (order) {
      case 1: return occupancy_one<P, 1, 3>(lds, skip);
      case 2: return occupancy_one<P, 2, 3>(lds, skip);
      case 3: return occupancy_one<P, 3, 3>(lds, skip);
      case 4: return occupancy_one<P, 4, 3>(lds, skip);
    }
  }
  return 1;
}

template <class P>
hipError_t launch_gpd(const GpdArgs<typename P::Real>& a, int order, int ndim, size_t lds, hipStream_t s) {
  if (ndim == 2) {
    switch (order) {
      case 1: return launch_one<P, 1, 2>(a, lds, s);
      case 2: return launch_one<P, 2, 2>(a, lds, s);
      case 3: return launch_one<P, 3, 2>(a, lds, s);
      case 4: return launch_one<P, 4, 2>(a, lds, s);
    }
  } else {
    switch (order) {
      case 1: return launch_one<P, 1, 3>(a, lds, s);
      case 2: return launch_one<P, 2, 3>(a, lds, s);
      case 3: return launch_one<P, 3, 3>(a, lds, s);
      case 4: return launch_one<P, 4, 3>(a, lds, s);
    }
  }
  return hipErrorInvalidValue;
}

// Each precision policy can be built as a translation unit of its own
// (WTPIC_GPD_POLICY = 32 or 64), so that the two compile in parallel.
#if !defined(WTPIC_GPD_POLICY) || WTPIC_GPD_POLICY == 32
template int gpd_groups_per_cu<F32>(int, int, size_t, bool);
template hipError_t launch_gpd<F32>(const GpdArgs<float>&, int, int, size_t, hipStream_t);
template hipError_t launch_rho_tiles<F32>(const GpdArgs<float>&, int, int, double*, int, int, size_t, hipStream_t);
#endif
#if !defined(WTPIC_GPD_POLICY) || WTPIC_GPD_POLICY == 64
template int gpd_groups_per_cu<F64>(int, int, size_t, bool);
template hipError_t launch_gpd<F64>(const GpdArgs<double>&, int, int, size_t, hipStream_t);
template hipError_t launch_rho_tiles<F64>(const GpdArgs<double>&, int, int, double*, int, int, size_t, hipStream_t);
#endif

}  // namespace wtpic
