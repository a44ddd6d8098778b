// Maxwell update (Yee leapfrog, or the Faraday stencil of Appendix C) and the
// FP64 diagnostics reductions.  These stencils are HBM-bound and small next
// to the particle kernel; every run of a context in one launch, over a table
// of 256-cell blocks that never straddle two runs.
#include "common.hpp"
#include "launch.hpp"

namespace wtpic {

namespace {

// Index on a periodic axis for -n <= m < 2n (stencil neighbours of a cell).
__device__ __forceinline__ int wrap1(int m, int n) {
  return m < 0 ? m + n : (m >= n ? m - n : m);
}

// A component of one run; a run has fewer than 2^30 cells (at least one
// particle per species per cell, fewer than 2^31 particles), so indices fit
// in 32 bits.
template <class Real>
struct Grid3 {
  const Real* f;
  int n0, n1, n2;
  __device__ Real at(int i, int j, int k) const { return f[wrap1(i, n0) + n0 * (wrap1(j, n1) + n1 * wrap1(k, n2))]; }
};

// Forward staggered difference along d of a component at node (i, j, k).
template <class Real, int DIM>
__device__ __forceinline__ Real dfwd(const Grid3<Real>& g, int d, int i, int j, int k, const Real* inv_dx) {
  if (d >= DIM) return Real(0);
  const Real a = g.at(i, j, k);
  const Real b = (d == 0) ? g.at(i + 1, j, k) : (d == 1 ? g.at(i, j + 1, k) : g.at(i, j, k + 1));
  return (b - a) * inv_dx[d];
}

// Faraday derivative along d: the Yee difference, times
// A_d = 1 + sum_e coef[d][e] delta_e^2 for M4 (Eq. Maxwell-A: the symbol
// -2[1 - cos(k_e dx_e)] of the second difference delta_e^2).
template <class Real, int DIM, bool M4>
__device__ __forceinline__ Real dfar(const Grid3<Real>& g, int d, int i, int j, int k, const RunDev<Real>& R) {
  const Real v = dfwd<Real, DIM>(g, d, i, j, k, R.inv_dx);
  if (!M4 || d >= DIM) return v;
  Real r = v;
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    const int oi = (e == 0), oj = (e == 1), ok = (e == 2);
    const Real vp = dfwd<Real, DIM>(g, d, i + oi, j + oj, k + ok, R.inv_dx);
    const Real vm = dfwd<Real, DIM>(g, d, i - oi, j - oj, k - ok, R.inv_dx);
    r += R.m4beta[d][e] * (vp - Real(2) * v + vm);
  }
  return r;
}

// Backward staggered difference along d (Ampere, unmodified Yee stencil).
template <class Real, int DIM>
__device__ __forceinline__ Real dbwd(const Grid3<Real>& g, int d, int i, int j, int k, const Real* inv_dx) {
  if (d >= DIM) return Real(0);
  const Real a = g.at(i, j, k);
  const Real b = (d == 0) ? g.at(i - 1, j, k) : (d == 1 ? g.at(i, j - 1, k) : g.at(i, j, k - 1));
  return (a - b) * inv_dx[d];
}

}  // namespace

// Cells per thread: a thread takes the same position in FR consecutive
// entries of the block table (256 cells of one run each) and computes every
// new value before it stores any, so that the loads of its FR cells are in
// flight together (the stores could alias the next cell's loads otherwise).
// For the Yee Faraday update four in FP32 and two in FP64; one for the wide
// M4 stencil, whose loads would otherwise take the registers of most of the
// waves, and one for the Ampere update, whose fifteen arrays per cell keep
// enough loads in flight (measured at 4096x2048: two or four cells per
// thread there cost 1-3%).
template <class Real, bool WIDE>
constexpr int cells_per_thread() {
  return WIDE ? 1 : (sizeof(Real) == 4 ? 4 : 2);
}

// B <- B - (c dt / 2) curl E.
template <class Real, int DIM, bool M4>
__global__ void __launch_bounds__(256) faraday_kernel(FieldArgs<Real> A) {
  constexpr int FR = cells_per_thread<Real, M4>();
  const long long NT = A.ncell_total;
  Real nb[FR][3];
  Real* out[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    // a thread past the end computes a valid cell again and stores nothing
    // (branch-free, so that the compiler issues every cell's loads together)
    const int bt = blockIdx.x * FR + r;
    const int b = min(bt, A.nblocks - 1);
    const RunDev<Real>& R = A.runs[A.blk_run[b]];
    const int nxy = R.n[0] * R.n[1];
    const int cr = A.blk_first[b] + threadIdx.x;
    const bool live = bt < A.nblocks && cr < nxy * R.n[2];
    const int ci = min(cr, nxy * R.n[2] - 1);
    const int q = ci / R.n[0];
    const int i = ci - q * R.n[0];
    const int j = (DIM == 2) ? q : q % R.n[1];
    const int k = (DIM == 2) ? 0 : q / R.n[1];
    Real* F = A.F + R.cell0;
    const Grid3<Real> E1{F, R.n[0], R.n[1], R.n[2]}, E2{F + NT, R.n[0], R.n[1], R.n[2]},
        E3{F + 2 * NT, R.n[0], R.n[1], R.n[2]};
    const Real c1 = dfar<Real, DIM, M4>(E3, 1, i, j, k, R) - dfar<Real, DIM, M4>(E2, 2, i, j, k, R);
    const Real c2 = dfar<Real, DIM, M4>(E1, 2, i, j, k, R) - dfar<Real, DIM, M4>(E3, 0, i, j, k, R);
    const Real c3 = dfar<Real, DIM, M4>(E2, 0, i, j, k, R) - dfar<Real, DIM, M4>(E1, 1, i, j, k, R);
    Real* o = F + 3 * NT + ci;
    nb[r][0] = o[0] - R.hcdt * c1;
    nb[r][1] = o[NT] - R.hcdt * c2;
    nb[r][2] = o[2 * NT] - R.hcdt * c3;
    out[r] = live ? o : nullptr;
  }
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    if (out[r] == nullptr) continue;
    out[r][0] = nb[r][0];
    out[r][NT] = nb[r][1];
    out[r][2 * NT] = nb[r][2];
  }
}

// E <- E + dt (c curl B - J); J <- 0 for the next deposit.
template <class Real, int DIM>
__global__ void __launch_bounds__(256) ampere_kernel(FieldArgs<Real> A) {
  constexpr int FR = cells_per_thread<Real, true>();
  const long long NT = A.ncell_total;
  Real ne[FR][3];
  Real* out[FR];
  double* jo[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    // a thread past the end computes a valid cell again and stores nothing
    // (branch-free, so that the compiler issues every cell's loads together)
    const int bt = blockIdx.x * FR + r;
    const int b = min(bt, A.nblocks - 1);
    const RunDev<Real>& R = A.runs[A.blk_run[b]];
    const int nxy = R.n[0] * R.n[1];
    const int cr = A.blk_first[b] + threadIdx.x;
    const bool live = bt < A.nblocks && cr < nxy * R.n[2];
    const int ci = min(cr, nxy * R.n[2] - 1);
    const int q = ci / R.n[0];
    const int i = ci - q * R.n[0];
    const int j = (DIM == 2) ? q : q % R.n[1];
    const int k = (DIM == 2) ? 0 : q / R.n[1];
    Real* F = A.F + R.cell0;
    double* J = A.J + R.cell0;
    const Grid3<Real> B1{F + 3 * NT, R.n[0], R.n[1], R.n[2]}, B2{F + 4 * NT, R.n[0], R.n[1], R.n[2]},
        B3{F + 5 * NT, R.n[0], R.n[1], R.n[2]};
    const Real d0 = dbwd<Real, DIM>(B3, 1, i, j, k, R.inv_dx) - dbwd<Real, DIM>(B2, 2, i, j, k, R.inv_dx);
    const Real d1 = dbwd<Real, DIM>(B1, 2, i, j, k, R.inv_dx) - dbwd<Real, DIM>(B3, 0, i, j, k, R.inv_dx);
    const Real d2 = dbwd<Real, DIM>(B2, 0, i, j, k, R.inv_dx) - dbwd<Real, DIM>(B1, 1, i, j, k, R.inv_dx);
    const Real j0 = Real(J[ci]), j1 = Real(J[NT + ci]), j2 = Real(J[2 * NT + ci]);
    Real* o = F + ci;
    ne[r][0] = o[0] + R.dt * (R.c * d0 - j0);
    ne[r][1] = o[NT] + R.dt * (R.c * d1 - j1);
    ne[r][2] = o[2 * NT] + R.dt * (R.c * d2 - j2);
    out[r] = live ? o : nullptr;
    jo[r] = live ? J + ci : nullptr;
  }
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    if (out[r] == nullptr) continue;
    out[r][0] = ne[r][0];
    out[r][NT] = ne[r][1];
    out[r][2 * NT] = ne[r][2];
    jo[r][0] = 0.0;
    jo[r][NT] = 0.0;
    jo[r][2 * NT] = 0.0;
  }
}

template <class Real>
__global__ void fill_kernel(Real* p, long long n, Real v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <class Real>
hipError_t launch_faraday_half(const FieldArgs<Real>& a, int ndim, bool m4, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  const int fr = m4 ? cells_per_thread<Real, true>() : cells_per_thread<Real, false>();
  const dim3 grid((a.nblocks + fr - 1) / fr), blk(256);
  if (ndim == 2) {
    if (m4)
      hipLaunchKernelGGL((faraday_kernel<Real, 2, true>), grid, blk, 0, s, a);
    else
      hipLaunchKernelGGL((faraday_kernel<Real, 2, false>), grid, blk, 0, s, a);
  } else {
    if (m4)
      hipLaunchKernelGGL((faraday_kernel<Real, 3, true>), grid, blk, 0, s, a);
    else
      hipLaunchKernelGGL((faraday_kernel<Real, 3, false>), grid, blk, 0, s, a);
  }
  return hipGetLastError();
}

template <class Real>
hipError_t launch_ampere(const FieldArgs<Real>& a, int ndim, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  const int fr = cells_per_thread<Real, true>();
  const dim3 grid((a.nblocks + fr - 1) / fr), blk(256);
  if (ndim == 2)
    hipLaunchKernelGGL((ampere_kernel<Real, 2>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((ampere_kernel<Real, 3>), grid, blk, 0, s, a);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_fill(Real* p, long long n, Real v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_kernel<Real>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template hipError_t launch_faraday_half<float>(const FieldArgs<float>&, int, bool, hipStream_t);
template hipError_t launch_faraday_half<double>(const FieldArgs<double>&, int, bool, hipStream_t);
template hipError_t launch_ampere<float>(const FieldArgs<float>&, int, hipStream_t);
template hipError_t launch_ampere<double>(const FieldArgs<double>&, int, hipStream_t);
template hipError_t launch_fill<float>(float*, long long, float, hipStream_t);
template hipError_t launch_fill<double>(double*, long long, double, hipStream_t);
template hipError_t launch_fill<int>(int*, long long, int, hipStream_t);

// ---------------------------------------------------------------------------
// Diagnostics (FP64).  acc: [0..2] sum E_d^2, [3..5] sum B_d^2, [6..7] sum
// M (gamma-1) c^2 per species, [8..10] sum M u c, [11] max |D.E - rho| (bits).
// The sums are taken per block into part[c][block] and then added block by
// block in a fixed order, so that repeated diagnostics of one state agree
// to the last bit.
// ---------------------------------------------------------------------------

namespace {

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

}  // namespace

template <class Real>
__global__ void __launch_bounds__(256) diag_fields_kernel(DiagArgs<Real> A, long long cells) {
  __shared__ double sh[16];
  const RunDev<Real>& R = A.runs[A.run];
  const Real* F = A.F + R.cell0;
  const long long NT = A.ncell_total;
  double s[6] = {0, 0, 0, 0, 0, 0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double v = (double)F[c * NT + i];
      s[c] += v * v;
    }
  }
  for (int c = 0; c < 6; ++c) {
    const double t = block_sum(s[c], sh);
    if (threadIdx.x == 0) A.part[c * kDiagBlocks + blockIdx.x] = t;
  }
}

template <class P, int DIM>
__global__ void __launch_bounds__(256) diag_particles_kernel(DiagArgs<typename P::Real> A, long long p0, long long np) {
  using Real = typename P::Real;
  __shared__ double sh[16];
  const RunDev<Real>& R = A.runs[A.run];
  const PBuf<Real> B = A.buf[A.st->parity];
  double s[5] = {0, 0, 0, 0, 0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const long long p = p0 + i;
    const int sp = (B.tag[p] >> kSpeciesShift) & 1;
    const double u0 = B.u[0][p], u1 = B.u[1][p], u2 = B.u[2][p];
    const double gam = sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2);
    const double M = R.M[sp];
    const double cc = (double)R.c;
    s[sp] += M * (gam - 1.0) * cc * cc;
    s[2] += M * u0 * cc;
    s[3] += M * u1 * cc;
    s[4] += M * u2 * cc;
  }
  for (int c = 0; c < 5; ++c) {
    const double t = block_sum(s[c], sh);
    if (threadIdx.x == 0) A.part[(6 + c) * kDiagBlocks + blockIdx.x] = t;
  }
}

// acc[c] = sum over blocks of part[c][block]: the field sums over nbf
// blocks, the particle sums over nbp blocks; one wave per accumulator, each
// lane a fixed stride of blocks, then a fixed butterfly.
__global__ void __launch_bounds__(704) diag_final_kernel(double* acc, const double* part, int nbf, int nbp) {
  const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nb = (c < 6) ? nbf : nbp;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[c * kDiagBlocks + b];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) acc[c] = s;
}

// Global-atomic variant for particles that are not in tile order (before the
// first step after particles were set); the tiled kernel is in gpd.hip.
// rho(m) += (Q/Vc) prod_d W_l(x_d - m_d) on integer nodes (Eq. shape-real).
template <class P, int L, int DIM>
__global__ void diag_rho_kernel(DiagArgs<typename P::Real> A, long long p0, long long np) {
  using Real = typename P::Real;
  const RunDev<Real>& R = A.runs[A.run];
  const PBuf<Real> B = A.buf[A.st->parity];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const long long p = p0 + i;
    const int sp = (B.tag[p] >> kSpeciesShift) & 1;
    int c[3] = {0, 0, 0};
    Real f[3] = {Real(0), Real(0), Real(0)};
    if (P::kAbs) {
      for (int d = 0; d < DIM; ++d) {
        const Real x = B.pos[d][p];
        const Real fl = floor(x);
        c[d] = (int)fl;
        f[d] = x - fl;
      }
    } else {
      unpack_cell<DIM>(B.cell[p], c[0], c[1], c[2]);
      for (int d = 0; d < DIM; ++d) f[d] = B.pos[d][p];
    }
    Real w[3][L + 1];
    int m0[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
      int base;
      Real g;
      tab_split(R.Wi[d], c[d], f[d], base, g);
      tab_eval<L, L + 1, false>(R.Wi[d], g, w[d]);
      m0[d] = base + R.Wi[d].first;
    }
    const double q = R.Q[sp] / R.Vc;
    const int nz = (DIM == 3) ? L + 1 : 1;
    for (int kz = 0; kz < nz; ++kz)
      for (int ky = 0; ky <= L; ++ky)
        for (int kx = 0; kx <= L; ++kx) {
          double wt = (double)w[0][kx] * (double)w[1][ky];
          int gz = 0;
          if (DIM == 3) {
            wt *= (double)w[2][kz];
            gz = wrapi(m0[2] + kz, R.n[2]);
          }
          const int gx = wrapi(m0[0] + kx, R.n[0]), gy = wrapi(m0[1] + ky, R.n[1]);
          unsafeAtomicAdd(A.rho + gx + (long long)R.n[0] * (gy + (long long)R.n[1] * gz), q * wt);
        }
  }
}

template <class Real, int DIM>
__global__ void __launch_bounds__(256) diag_gauss_kernel(DiagArgs<Real> A, long long cells) {
  const RunDev<Real>& R = A.runs[A.run];
  const Real* F = A.F + R.cell0;
  const long long NT = A.ncell_total;
  // a run has fewer than 2^30 cells (one particle per species per cell at
  // least, fewer than 2^31 particles)
  const int stride = gridDim.x * blockDim.x;
  const int nxy = R.n[0] * R.n[1];
  double mx = 0.0;
  for (int ci = blockIdx.x * blockDim.x + threadIdx.x; ci < (int)cells; ci += stride) {
    const int i = ci % R.n[0];
    const int j = (ci / R.n[0]) % R.n[1];
    const int k = ci / nxy;
    double div = 0.0;
    for (int d = 0; d < DIM; ++d) {
      const int pi = (d == 0) ? (i == 0 ? R.n[0] - 1 : i - 1) : i;
      const int pj = (d == 1) ? (j == 0 ? R.n[1] - 1 : j - 1) : j;
      const int pk = (d == 2) ? (k == 0 ? R.n[2] - 1 : k - 1) : k;
      const long long pc = pi + (long long)R.n[0] * (pj + (long long)R.n[1] * pk);
      div += ((double)F[d * NT + ci] - (double)F[d * NT + pc]) / R.dxd[d];
    }
    const double res = fabs(div - A.rho[ci]);
    mx = res > mx ? res : mx;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  // one atomic per block (a maximum is exact in any order)
  __shared__ double wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = wmax[w] > mx ? wmax[w] : mx;
    atomicMax(reinterpret_cast<unsigned long long*>(&A.acc[11]), __double_as_longlong(mx));
  }
}

template <class P>
hipError_t launch_diag(const DiagArgs<typename P::Real>& a, int ndim, int order, long long cells, long long p0,
                       long long np, bool rho_done, hipStream_t s) {
  using Real = typename P::Real;
  auto grid_for = [](long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > kDiagBlocks ? kDiagBlocks : b));
  };
  auto rho_grid = [](long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
  };
  const unsigned nbf = grid_for(cells), nbp = grid_for(np);
  hipLaunchKernelGGL(diag_fields_kernel<Real>, dim3(nbf), dim3(256), 0, s, a, cells);
  if (ndim == 2)
    hipLaunchKernelGGL((diag_particles_kernel<P, 2>), dim3(nbp), dim3(256), 0, s, a, p0, np);
  else
    hipLaunchKernelGGL((diag_particles_kernel<P, 3>), dim3(nbp), dim3(256), 0, s, a, p0, np);
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(11 * 64), 0, s, a.acc, a.part, (int)nbf, (int)nbp);
  if (!rho_done) {
    const dim3 rg(rho_grid(np)), rb(256);
    if (ndim == 2) {
      switch (order) {
        case 1: hipLaunchKernelGGL((diag_rho_kernel<P, 1, 2>), rg, rb, 0, s, a, p0, np); break;
        case 2: hipLaunchKernelGGL((diag_rho_kernel<P, 2, 2>), rg, rb, 0, s, a, p0, np); break;
        case 3: hipLaunchKernelGGL((diag_rho_kernel<P, 3, 2>), rg, rb, 0, s, a, p0, np); break;
        case 4: hipLaunchKernelGGL((diag_rho_kernel<P, 4, 2>), rg, rb, 0, s, a, p0, np); break;
      }
    } else {
      switch (order) {
        case 1: hipLaunchKernelGGL((diag_rho_kernel<P, 1, 3>), rg, rb, 0, s, a, p0, np); break;
        case 2: hipLaunchKernelGGL((diag_rho_kernel<P, 2, 3>), rg, rb, 0, s, a, p0, np); break;
        case 3: hipLaunchKernelGGL((diag_rho_kernel<P, 3, 3>), rg, rb, 0, s, a, p0, np); break;
        case 4: hipLaunchKernelGGL((diag_rho_kernel<P, 4, 3>), rg, rb, 0, s, a, p0, np); break;
      }
    }
  }
  if (ndim == 2)
    hipLaunchKernelGGL((diag_gauss_kernel<Real, 2>), dim3(grid_for(cells)), dim3(256), 0, s, a, cells);
  else
    hipLaunchKernelGGL((diag_gauss_kernel<Real, 3>), dim3(grid_for(cells)), dim3(256), 0, s, a, cells);
  return hipGetLastError();
}

template hipError_t launch_diag<F32>(const DiagArgs<float>&, int, int, long long, long long, long long, bool,
                                     hipStream_t);
template hipError_t launch_diag<F64>(const DiagArgs<double>&, int, int, long long, long long, long long, bool,
                                     hipStream_t);

}  // namespace wtpic
