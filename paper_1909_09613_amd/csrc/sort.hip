// Counting sort of the particles by (tile, species), run only when a tile's
// particles have outgrown the staging margin of the gather-push-deposit
// kernel (a device-side request flag; all kernels exit at once otherwise).
//
// prep    one block: latch the request, clear counters
// count   key = 2 * tile + species per particle; wave-aggregated counts
// scan    one block: exclusive scan of the counts into segment offsets;
//         reset every tile's box to its rectangle
// scatter ranks within a segment are read as a 16-row matrix and stored
//         transposed (rank r -> row r mod 16, column r div 16): ranks arrive in
//         the source order, where a cell's particles are consecutive, so
//         consecutive slots -- the lanes of a wave -- take particles from
//         different, neighbouring cells and their LDS accesses spread over
//         the banks instead of piling onto one stencil
// flip    swap the particle stores, clear the request
#include "common.hpp"
#include "launch.hpp"

namespace wtpic {

namespace {

constexpr int kInterleave = 16;  // rows of the rank transposition

template <class Real>
__device__ int find_run(const RunDev<Real>* runs, int nruns, long long p) {
  int lo = 0, hi = nruns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (runs[mid].p0 <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Adds the lanes' votes to ctr[key], one atomic per distinct key in the
// wave; returns each valid lane's rank among the lanes that shared its key,
// offset by the counter value the atomic returned.
__device__ int wave_add(int* ctr, int key, bool valid) {
  unsigned long long active = __ballot(valid);
  const int lane = __lane_id();
  int rank = 0;
  while (active) {
    const int leader = __ffsll((long long)active) - 1;
    const int lk = __shfl(key, leader);
    const unsigned long long match = __ballot(valid && key == lk) & active;
    int base = 0;
    if (lane == leader) base = atomicAdd(ctr + lk, __popcll(match));
    base = __shfl(base, leader);
    if ((match >> lane) & 1ull) rank = base + __popcll(match & ((1ull << lane) - 1ull));
    active &= ~match;
  }
  return rank;
}

}  // namespace

template <class Real>
__global__ void sort_prep(SortArgs<Real> A) {
  __shared__ int act;
  if (threadIdx.x == 0) {
    act = A.st->sort_request != 0;
    A.st->sort_active = act;
  }
  __syncthreads();
  if (!act) return;
  for (int i = threadIdx.x; i < A.nkeys; i += blockDim.x) {
    A.counts[i] = 0;
    A.cursor[i] = 0;
  }
}

template <class P, int DIM>
__global__ void sort_count(SortArgs<typename P::Real> A) {
  using Real = typename P::Real;
  if (!A.st->sort_active) return;
  const PBuf<Real> B = A.buf[A.st->parity];
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // every lane of a wave iterates the same number of times (wave_add)
  const long long nit = (A.np_total + stride - 1) / stride;
  for (long long it = 0; it < nit; ++it) {
    const long long p = start + it * stride;
    const bool valid = p < A.np_total;
    int key = 0;
    if (valid) {
      const int r = find_run(A.runs, A.nruns, p);
      const RunDev<Real>& R = A.runs[r];
      int c[3] = {0, 0, 0};
      if (P::kAbs) {
        for (int d = 0; d < DIM; ++d) c[d] = (int)floor(B.pos[d][p]);
      } else {
        unpack_cell<DIM>(B.cell[p], c[0], c[1], c[2]);
      }
      int t[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) {
        int m = c[d];
        if (m < 0 || m >= R.n[d]) {  // never for a valid store; keep the index in range
          atomicAdd(&A.st->n_out_of_range, 1ull);
          m = wrapi(m, R.n[d]);
        }
        t[d] = m / A.tile[d];
      }
      const int g = R.tile0 + t[0] + R.ntile[0] * (t[1] + R.ntile[1] * t[2]);
      const int s = (B.tag[p] >> kSpeciesShift) & 1;
      key = 2 * g + s;
      A.keys[p] = key;
    }
    wave_add(A.counts, key, valid);
  }
}

template <class Real>
__global__ void sort_scan(SortArgs<Real> A) {
  if (!A.st->sort_active) return;
  __shared__ long long part[1024];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int chunk = (A.nkeys + nth - 1) / nth;
  const int lo = tid * chunk;
  const int hi = min(lo + chunk, A.nkeys);
  long long s = 0;
  for (int i = lo; i < hi; ++i) s += A.counts[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < nth; off <<= 1) {
    const long long v = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  long long base = part[tid] - s;  // exclusive
  for (int i = lo; i < hi; ++i) {
    A.seg[i] = (int)base;
    base += A.counts[i];
  }
  if (tid == nth - 1) A.seg[A.nkeys] = (int)part[nth - 1];
  // every tile's particles now lie in its rectangle
  for (int g = tid; g < A.G; g += nth) {
    const RunDev<Real>& R = A.runs[A.tile_run[g]];
    const int lt = g - R.tile0;
    int tc[3];
    tc[0] = lt % R.ntile[0];
    tc[1] = (lt / R.ntile[0]) % R.ntile[1];
    tc[2] = lt / (R.ntile[0] * R.ntile[1]);
    for (int d = 0; d < 3; ++d) {
      const int org = tc[d] * A.tile[d];
      A.bbox[g * 6 + 2 * d] = 0;
      A.bbox[g * 6 + 2 * d + 1] = min(A.tile[d], R.n[d] - org) - 1;
    }
  }
}

template <class P, int DIM>
__global__ void sort_scatter(SortArgs<typename P::Real> A) {
  using Real = typename P::Real;
  if (!A.st->sort_active) return;
  const int par = A.st->parity;
  const PBuf<Real> S = A.buf[par];
  const PBuf<Real> D = A.buf[par ^ 1];
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nit = (A.np_total + stride - 1) / stride;
  for (long long it = 0; it < nit; ++it) {
    const long long p = start + it * stride;
    const bool valid = p < A.np_total;
    const int key = valid ? A.keys[p] : 0;
    const int rank = wave_add(A.cursor, key, valid);
    if (!valid) continue;
    const int s0 = A.seg[key];
    const int n = A.seg[key + 1] - s0;
    // transposed position: row ii holds ranks ii, ii + 16, ...; the first
    // n mod 16 rows have one entry more than the others
    const int nq = n / kInterleave, rem = n % kInterleave;
    const int ii = rank % kInterleave, mm = rank / kInterleave;
    const long long q = s0 + (long long)(ii * nq + min(ii, rem) + mm);
    if (!P::kAbs) D.cell[q] = S.cell[p];
    for (int d = 0; d < DIM; ++d) D.pos[d][q] = S.pos[d][p];
    D.u[0][q] = S.u[0][p];
    D.u[1][q] = S.u[1][p];
    D.u[2][q] = S.u[2][p];
    D.tag[q] = S.tag[p];
  }
}

template <class Real>
__global__ void sort_flip(SortArgs<Real> A) {
  if (!A.st->sort_active) return;
  A.st->parity ^= 1;
  A.st->sort_request = 0;
  A.st->sort_active = 0;
  A.st->n_sorts += 1;
}

template <class P>
hipError_t launch_sort(const SortArgs<typename P::Real>& a, int ndim, hipStream_t s) {
  using Real = typename P::Real;
  const long long blocks = (a.np_total + 255) / 256;
  const int grid = (int)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(sort_prep<Real>, dim3(1), dim3(1024), 0, s, a);
  if (ndim == 2)
    hipLaunchKernelGGL((sort_count<P, 2>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((sort_count<P, 3>), dim3(grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(sort_scan<Real>, dim3(1), dim3(1024), 0, s, a);
  if (ndim == 2)
    hipLaunchKernelGGL((sort_scatter<P, 2>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((sort_scatter<P, 3>), dim3(grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(sort_flip<Real>, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_sort<F32>(const SortArgs<float>&, int, hipStream_t);
template hipError_t launch_sort<F64>(const SortArgs<double>&, int, hipStream_t);

}  // namespace wtpic
