// Host-side launchers of the HIP kernels (defined in the .hip sources).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/wtpic.h"
#include "common.hpp"

namespace wtpic {

// Internal hooks of the allocation-free initialisation (static_scratch.hip):
// a function pic_destroy calls with arg once the context's stream has
// drained, and the text pic_last_error(NULL) returns.
void set_destroy_hook(pic_ctx* c, void (*hook)(int), int arg);
void set_global_error(const char* msg);

template <class Real>
struct SortArgs {
  const RunDev<Real>* runs;
  int nruns;
  DevState* st;
  PBuf<Real> buf[2];
  long long np_total;
  int G;
  int nkeys;          // 2 G
  int tile[3];
  int tc;             // cells of a full tile
  int kcap;           // ranks within a cell ordered level by level (arrange pass)
  int* counts;        // nkeys
  int* cursor;        // nkeys
  int* seg;           // nkeys + 1
  int* keys;          // np_total
  int* bbox;          // 6 G
  float* jb;          // 4 G: per-tile current bounds and cell counts, set from the sorted particles
  const int* tile_run;
};

// Block size and LDS bytes of the per-segment arrange pass of the sort.
constexpr int kArrangeBlock = 512;
inline size_t arrange_lds(int tc, int kcap) {
  return (size_t)4 * (2 * tc + kcap + 2) + (size_t)2 * kcap * tc + 16;
}
// Levels the arrange pass orders one by one for a tile of tc cells.
inline int arrange_kcap(int tc) {
  const int k = 8192 / (tc > 0 ? tc : 1);
  return k < 1 ? 1 : (k > 64 ? 64 : k);
}

template <class Real>
struct FieldArgs {
  const RunDev<Real>* runs;
  const int* blk_run;      // run of each block of a grid-wide cell launch
  const int* blk_first;    // first cell (within its run) of each block
  Real* F;                 // E1 E2 E3 B1 B2 B3, each ncell_total
  double* J;               // J1 J2 J3
  long long ncell_total;
  int nblocks;
};

template <class Real>
struct DiagArgs {
  const RunDev<Real>* runs;
  int run;
  DevState* st;
  PBuf<Real> buf[2];
  const Real* F;
  long long ncell_total;
  double* acc;             // 16 accumulators (see diag kernels)
  double* part;            // kDiagBlocks x 16 per-block partial sums
  double* rho;             // ncell of the run
};

// Blocks of the diagnostics sums (each leaves 16 partial sums).
constexpr int kDiagBlocks = 2048;

template <class P>
hipError_t launch_gpd(const GpdArgs<typename P::Real>& a, int order, int ndim, size_t lds, hipStream_t s);

// Particle-kernel groups one CU holds at once with lds bytes of dynamic LDS
// (plain or skip variant), at least 1.
template <class P>
int gpd_groups_per_cu(int order, int ndim, size_t lds, bool skip);

// Charge density of one run from the tile segments (diagnostics); lds bytes
// must hold 8 * (current window nodes).
template <class P>
hipError_t launch_rho_tiles(const GpdArgs<typename P::Real>& a, int run, int ntiles, double* rho, int order,
                            int ndim, size_t lds, hipStream_t s);

template <class P>
hipError_t launch_sort(const SortArgs<typename P::Real>& a, int ndim, hipStream_t s);

template <class Real>
hipError_t launch_faraday_half(const FieldArgs<Real>& a, int ndim, bool m4, hipStream_t s);
template <class Real>
hipError_t launch_ampere(const FieldArgs<Real>& a, int ndim, hipStream_t s);
template <class Real>
hipError_t launch_fill(Real* p, long long n, Real v, hipStream_t s);

template <class P>
hipError_t launch_diag(const DiagArgs<typename P::Real>& a, int ndim, int order, long long cells,
                       long long p0, long long np, bool rho_done, hipStream_t s);

}  // namespace wtpic
