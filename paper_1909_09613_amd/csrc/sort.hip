// Counting sort of the particles by (tile, species), run only when a tile's
// particles have outgrown the staging margin of the gather-push-deposit
// kernel (a device-side request flag; all kernels exit at once otherwise).
//
// count    key = 2 * tile + species per particle; wave-aggregated counts;
//          the last block to finish scans the counts into segment offsets
//          (clearing the counts for the next sort) and resets every tile's
//          box to its rectangle
// scatter  each particle to its segment of the other store
// arrange  one block per segment: order the segment back into the current
//          store by (rank within its cell, cell): first every cell's first
//          particle, cells in tile order, then every cell's second particle,
//          and so on.  The lanes of a wave then hold particles of 64
//          nearby cells, one each, so that the gather reads and the current
//          atomics of a wave touch distinct, nearly consecutive LDS
//          addresses.  Ranks beyond `kcap` (dense cells) follow in cell order.
//          The last arrange block to finish clears the request and counts
//          the sort.  Between sorts the counts and cursors are zero, so a
//          sort needs no clearing pass, and each of the three kernels reads
//          the request flag itself (only the particle kernel sets it, and it
//          does not run during a sort).
#include "common.hpp"
#include "launch.hpp"

namespace wtpic {

namespace {

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

// Exclusive scan of the counts into segment offsets by one block (clearing
// the counts for the next sort), and every tile's box reset to its
// rectangle.  The counts were added with device-scope atomics; they are read
// the same way.
template <class Real>
__device__ void scan_counts(const SortArgs<Real>& A, long long* part) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int chunk = (A.nkeys + nth - 1) / nth;
  const int lo = tid * chunk;
  const int hi = min(lo + chunk, A.nkeys);
  long long s = 0;
  for (int i = lo; i < hi; ++i) s += __hip_atomic_load(&A.counts[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const int c = __hip_atomic_load(&A.counts[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    A.seg[i] = (int)base;
    base += c;
    A.counts[i] = 0;
  }
  if (tid == nth - 1) A.seg[A.nkeys] = (int)part[nth - 1];
  // every tile's particles now lie in its rectangle; its current bounds are
  // rebuilt by the arrange pass
  for (int i = tid; i < 4 * A.G; i += nth) A.jb[i] = 0.0f;
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
__global__ void sort_count(SortArgs<typename P::Real> A) {
  using Real = typename P::Real;
  if (!A.st->sort_request) return;
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
  // the last block to finish turns the counts into segment offsets
  __shared__ long long part[256];
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&A.st->count_done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  scan_counts(A, part);
  if (threadIdx.x == 0) A.st->count_done = 0;
}

template <class P, int DIM>
__global__ void sort_scatter(SortArgs<typename P::Real> A) {
  using Real = typename P::Real;
  if (!A.st->sort_request) return;
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
    const long long q = A.seg[key] + (long long)rank;
    if (!P::kAbs) D.cell[q] = S.cell[p];
    for (int d = 0; d < DIM; ++d) D.pos[d][q] = S.pos[d][p];
    D.u[0][q] = S.u[0][p];
    D.u[1][q] = S.u[1][p];
    D.u[2][q] = S.u[2][p];
    D.tag[q] = S.tag[p];
  }
}

// Index of a particle's cell in the order the arrange pass lays cells out.
// With an even tile width, in FP64 and for 2D tiles narrower than 32 cells:
// first the cells of even x, then those of odd x (each in x-then-y-then-z
// order), so that the lanes of a wave sit two cells apart along x and
// particles that drift at slightly different times still fall in different
// cells (same-address LDS atomics serialise).  Otherwise plain x-fastest
// order.  Measured in 2D: FP64 16x16 5% faster with the split; mixed
// precision 32x16 and 64x8 1-6% faster without it, 16x16 and 16x32 8-10%
// faster with it; 3D mixed precision 3% faster without it.
template <class P, int DIM>
__device__ __forceinline__ int cell_in_tile(const PBuf<typename P::Real>& S, long long q, const int org[3],
                                            const int tile[3]) {
  int c[3] = {0, 0, 0};
  if (P::kAbs) {
    for (int d = 0; d < DIM; ++d) c[d] = (int)floor(S.pos[d][q]);
  } else {
    unpack_cell<DIM>(S.cell[q], c[0], c[1], c[2]);
  }
  int m[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) m[d] = min(max(c[d] - org[d], 0), tile[d] - 1);
  if ((P::kAbs || (DIM == 2 && tile[0] < 32)) && (tile[0] & 1) == 0) {
    const int h = tile[0] >> 1;
    const int rest = m[1] + tile[1] * m[2];
    const int nrest = tile[1] * (DIM == 3 ? tile[2] : 1);
    return (m[0] & 1) * h * nrest + rest * h + (m[0] >> 1);
  }
  int cl = 0, stride = 1;
  for (int d = 0; d < DIM; ++d) {
    cl += m[d] * stride;
    stride *= tile[d];
  }
  return cl;
}

template <class P, int DIM>
__global__ void __launch_bounds__(kArrangeBlock) sort_arrange(SortArgs<typename P::Real> A) {
  using Real = typename P::Real;
  if (!A.st->sort_request) return;
  extern __shared__ __align__(16) int sm[];
  __shared__ int cmax_s;
  const int TC = A.tc, KC = A.kcap;
  int* cnt = sm;                                                // TC: particles per cell
  int* xpre = cnt + TC;                                         // TC + 1: prefix of ranks >= KC
  int* base = xpre + TC + 1;                                    // KC + 1: slots below level k
  unsigned short* pre = reinterpret_cast<unsigned short*>(base + KC + 1);  // KC x TC
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwave = kArrangeBlock / 64;
  const int par = A.st->parity;
  const PBuf<Real> S = A.buf[par ^ 1];
  const PBuf<Real> D = A.buf[par];
  const unsigned long long below = (1ull << lane) - 1ull;
  // the scatter is done with the cursors: clear them for the next sort
  for (int i = blockIdx.x * kArrangeBlock + tid; i < A.nkeys; i += gridDim.x * kArrangeBlock) A.cursor[i] = 0;
  for (int key = blockIdx.x; key < A.nkeys; key += gridDim.x) {
    const int s0 = A.seg[key];
    const int n = A.seg[key + 1] - s0;
    if (n == 0) continue;
    const int g = key >> 1;
    const RunDev<Real>& R = A.runs[A.tile_run[g]];
    const int lt = g - R.tile0;
    int org[3];
    org[0] = (lt % R.ntile[0]) * A.tile[0];
    org[1] = ((lt / R.ntile[0]) % R.ntile[1]) * A.tile[1];
    org[2] = (DIM == 3) ? (lt / (R.ntile[0] * R.ntile[1])) * A.tile[2] : 0;
    for (int i = tid; i < TC; i += kArrangeBlock) cnt[i] = 0;
    if (tid == 0) cmax_s = 0;
    __syncthreads();
    // rank of each particle within its cell
    for (int i = tid; i < n; i += kArrangeBlock) {
      const long long q = s0 + (long long)i;
      A.keys[q] = atomicAdd(&cnt[cell_in_tile<P, DIM>(S, q, org, A.tile)], 1);
    }
    __syncthreads();
    // level k < KC: cells holding more than k particles, numbered in cell order
    for (int k = wave; k < KC; k += nwave) {
      int run = 0;
      for (int c0 = 0; c0 < TC; c0 += 64) {
        const int c = c0 + lane;
        const bool f = c < TC && cnt[c] > k;
        const unsigned long long b = __ballot(f);
        if (c < TC) pre[k * TC + c] = (unsigned short)(run + __popcll(b & below));
        run += __popcll(b);
      }
      if (lane == 0) base[k + 1] = run;
    }
    // ranks >= KC: exclusive prefix over cells of max(0, count - KC)
    if (wave == 0) {
      int run = 0;
      for (int c0 = 0; c0 < TC; c0 += 64) {
        const int c = c0 + lane;
        const int v = c < TC ? max(0, cnt[c] - KC) : 0;
        int incl = v;
        for (int off = 1; off < 64; off <<= 1) {
          const int t = __shfl_up(incl, off);
          if (lane >= off) incl += t;
        }
        if (c < TC) xpre[c] = run + incl - v;
        run += __shfl(incl, 63);
      }
      if (lane == 0) xpre[TC] = run;
    }
    __syncthreads();
    if (tid == 0) {
      base[0] = 0;
      for (int k = 0; k < KC; ++k) base[k + 1] += base[k];
    }
    __syncthreads();
    float mb[3] = {0.0f, 0.0f, 0.0f};
    for (int i = tid; i < n; i += kArrangeBlock) {
      const long long q = s0 + (long long)i;
      const int cl = cell_in_tile<P, DIM>(S, q, org, A.tile);
      if (!P::kAbs) {
        // bounds of the next step's current contributions (see gpd.hip):
        // |step| per axis, and |v3| for the out-of-plane current in 2D
        const float u0 = (float)S.u[0][q], u1 = (float)S.u[1][q], u2 = (float)S.u[2][q];
        const float ig = 1.0f / sqrtf(1.0f + u0 * u0 + u1 * u1 + u2 * u2);
        mb[0] = fmaxf(mb[0], (float)R.a[0] * fabsf(u0) * ig);
        mb[1] = fmaxf(mb[1], (float)R.a[1] * fabsf(u1) * ig);
        mb[2] = fmaxf(mb[2], (DIM == 2 ? 1.0f : (float)R.a[2]) * fabsf(u2) * ig);
      }
      const int k = A.keys[q];
      const int slot = (k < KC) ? base[k] + (int)pre[k * TC + cl] : base[KC] + xpre[cl] + (k - KC);
      const long long o = s0 + (long long)slot;
      if (!P::kAbs) D.cell[o] = S.cell[q];
      for (int d = 0; d < DIM; ++d) D.pos[d][o] = S.pos[d][q];
      D.u[0][o] = S.u[0][q];
      D.u[1][o] = S.u[1][q];
      D.u[2][o] = S.u[2][q];
      D.tag[o] = S.tag[q];
    }
    if (!P::kAbs) {
      for (int c = 0; c < 3; ++c) {
        float m = mb[c];
        for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if (lane == 0) atomicMax(reinterpret_cast<int*>(A.jb) + 4 * g + c, __float_as_int(m));
      }
      // largest particle count of one cell; the two species' maxima add
      int cm = 0;
      for (int i = tid; i < TC; i += kArrangeBlock) cm = max(cm, cnt[i]);
      for (int off = 32; off >= 1; off >>= 1) cm = max(cm, __shfl_xor(cm, off));
      if (lane == 0) atomicMax(&cmax_s, cm);
      __syncthreads();
      if (tid == 0) atomicAdd(A.jb + 4 * g + 3, (float)cmax_s);
    }
    __syncthreads();
  }
  // the last group to finish ends the sort (every group has started and
  // read the request by then)
  if (tid == 0 && atomicAdd(&A.st->arrange_done, 1u) == gridDim.x - 1) {
    A.st->arrange_done = 0;
    A.st->n_sorts += 1;
    A.st->sort_request = 0;
  }
}

template <class P>
hipError_t launch_sort(const SortArgs<typename P::Real>& a, int ndim, hipStream_t s) {
  const long long blocks = (a.np_total + 255) / 256;
  // grid-stride kernels: enough groups to fill the chip when a sort runs,
  // few enough that the launches between sorts (all exit at once) are cheap
  const int grid = (int)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024);
  if (ndim == 2)
    hipLaunchKernelGGL((sort_count<P, 2>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((sort_count<P, 3>), dim3(grid), dim3(256), 0, s, a);
  if (ndim == 2)
    hipLaunchKernelGGL((sort_scatter<P, 2>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((sort_scatter<P, 3>), dim3(grid), dim3(256), 0, s, a);
  const int agrid = a.nkeys < 512 ? a.nkeys : 512;
  if (ndim == 2)
    hipLaunchKernelGGL((sort_arrange<P, 2>), dim3(agrid), dim3(kArrangeBlock), arrange_lds(a.tc, a.kcap), s, a);
  else
    hipLaunchKernelGGL((sort_arrange<P, 3>), dim3(agrid), dim3(kArrangeBlock), arrange_lds(a.tc, a.kcap), s, a);
  return hipGetLastError();
}

template hipError_t launch_sort<F32>(const SortArgs<float>&, int, hipStream_t);
template hipError_t launch_sort<F64>(const SortArgs<double>&, int, hipStream_t);

}  // namespace wtpic
