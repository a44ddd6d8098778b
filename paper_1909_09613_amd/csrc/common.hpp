// Types shared by the host runtime and the HIP kernels of libwtpic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace wtpic {

// Precision policies.  F32: int32 cell + FP32 offsets, FP32 momenta, fields
// and weights; per-tile current in 32-bit fixed point (integer LDS atomics),
// global current FP64.  F64: absolute FP64 positions, FP64 everywhere.
struct F32 {
  using Real = float;
  using Acc = double;  // (unused: the fixed-point windows take the FP64 windows' place in LDS)
  static constexpr bool kAbs = false;
};
struct F64 {
  using Real = double;
  using Acc = double;
  static constexpr bool kAbs = true;
};

// Packed cell coordinates of the FP32 layout: 2D x | y << 16 (16 bits per
// axis), 3D x | y << 11 | z << 22 (11, 11 and 10 bits).  A coordinate must fit
// its field, so a run has at most max_cells_per_axis cells along an axis.
__host__ __device__ constexpr int max_cells_per_axis(int ndim, int axis) {
  return ndim == 2 ? 65535 : (axis == 2 ? 1 << 10 : 1 << 11);
}
template <int DIM>
__host__ __device__ inline int pack_cell(int x, int y, int z) {
  if (DIM == 2) return x | (y << 16);
  return x | (y << 11) | (z << 22);
}
template <int DIM>
__host__ __device__ inline void unpack_cell(int c, int& x, int& y, int& z) {
  if (DIM == 2) {
    x = c & 0xffff;
    y = (c >> 16) & 0xffff;
    z = 0;
  } else {
    x = c & 0x7ff;
    y = (c >> 11) & 0x7ff;
    z = (c >> 22) & 0x3ff;
  }
}

// Compile-time window pitches (elements; row, and plane in 3D) of the
// mixed-precision particle kernel's fixed-pitch variant, per dimension.  A
// window that fits them is laid out with them (padded if smaller), and the
// kernel then reads every row and plane of a stencil at an immediate LDS
// offset from one address (one vector add per row less).  They are the
// windows of the default tilings at the orders and Courant numbers of the
// benchmark workloads:
//  - 2D FP32 (32 x 16 tiles): field rows 64, current rows 48.  The LDS
//    serves a wave's 4-byte reads 32 lanes (one row of the wave's cells) at
//    a time over 32 banks; the lanes whose T_l or W_l stencil starts one row
//    lower read the row above, which with a pitch of 64 (a multiple of 32)
//    falls on other banks than the rest of the half-wave's reads.  Current
//    atomics showed no such dependence.
//  - 3D FP32 (16 x 4 x 4 tiles, l <= 2, c dt <= dx/2): fields 21 x 9 nodes
//    per plane at (21, 192), current 23 x 11 at (23, 256) (planes rounded up
//    to a multiple of 8).
// (The same for the FP64 kernel measured no faster at 4096x2048 and 4%
// slower at 256x128x128; it keeps its run-time pitches.)
template <int DIM>
struct FixedPitch;
template <>
struct FixedPitch<2> {
  static constexpr int f[2] = {64, 0}, j[2] = {48, 0};
};
template <>
struct FixedPitch<3> {
  static constexpr int f[2] = {21, 192}, j[2] = {23, 256};
};

// Per-run constants, one entry per run in device memory.
template <class Real>
struct RunDev {
  int n[3];           // cells per axis (n[2] = 1 in 2D)
  int ntile[3];       // tiles per axis
  int tile0;          // global index of the run's first tile
  int KT;             // nodes of the T table (max over axes)
  long long cell0;    // offset of the run's cells in the concatenated grids
  long long p0;       // offset of the run's particles in the particle stores
  long long np;       // particles of both species
  int glo[3], ghi[3]; // gather stencil reach (node offsets from the cell)
  int dlo[3], dhi[3]; // deposit stencil reach (old or new position)
  Real a[3];          // c dt / dx_d
  Real eps[2];        // (q/m) dt / (2 c) per species
  Real c;             // speed of light
  Real dt;            // time step
  Real hcdt;          // c dt / 2 (Faraday half step)
  Real inv_dx[3];     // 1 / dx_d
  Real m4beta[3][3];  // M4 Faraday coefficients (0 for Yee): [d][e]
  double js[2][3];    // current scale per species: -Q dx_d/(Vc dt); J3 in 2D: Q c/Vc
  double Vc;          // cell volume
  double dxd[3];      // cell sizes
  double Q[2];        // macro charge per species
  double M[2];        // macro mass per species
  // partially skipped calculation: box A0 in cell units, the time of A0 at
  // particle-kernel launch skip_l0, and c and dt in FP64 for t
  double skip_lo[3], skip_hi[3];
  double skip_t0, cd, dtd;
  long long skip_l0;
  int skip_on;
  Tab<Real> Wh[3];    // W_l on the half-integer lattice
  Tab<Real> Wi[3];    // W_l on the integer lattice (charge form factor)
  Tab<Real> T[3];     // T_l (WT) or W_l (MC) on the integer lattice
};

// One of the two particle stores.
template <class Real>
struct PBuf {
  int* cell;      // packed cell (F32 layout only)
  Real* pos[3];   // F32: in-cell offsets; F64: absolute positions (cell units)
  Real* u[3];     // momenta u = gamma v / c
  int* tag;       // species << 30 | index within (run, species)
};

constexpr int kSpeciesShift = 30;

// Device-side mutable state of a context.
struct DevState {
  int parity;                  // current particle store
  int sort_request;            // set when a tile's particles outgrew the staging margin
  int pad0;
  int tile_queue;              // next tile for the persistent particle kernel
  unsigned long long n_nonfinite;
  unsigned long long n_out_of_range;
  unsigned long long n_sorts;
  unsigned int groups_done;    // particle-kernel groups that found the queue empty
  unsigned int arrange_done;   // sort arrange groups finished
  long long gpd_launches;      // particle-kernel launches completed
  unsigned int count_done;     // sort count groups finished
  unsigned int pad1;
};

template <class Real>
struct GpdArgs {
  const RunDev<Real>* runs;
  const int* tile_run;   // run of each global tile
  const int* seg;        // 2G+1 segment offsets: key 2g+s covers [seg[key], seg[key+1])
  int* bbox;             // per tile: lo0, hi0, lo1, hi1, lo2, hi2 (cells, tile-relative)
  float* jb;             // per tile: bounds of the current contributions and cell counts (gpd.hip)
  DevState* st;
  PBuf<Real> buf[2];
  const Real* F;         // E1 E2 E3 B1 B2 B3, each ncell_total
  double* J;             // J1 J2 J3, each ncell_total
  long long ncell_total;
  int G;                 // tiles in all runs
  int tile[3];           // tile size (cells)
  int fw[3];             // field window capacity (nodes)
  int jw[3];             // current window capacity (nodes)
  int fp[2];             // field window row and plane pitch (elements; >= fw[0], >= fp[0] fw[1])
  int jp[2];             // current window row and plane pitch
  int guard[3];          // bbox extent above which a re-sort is requested
  int max_groups;        // workgroups launched (persistent, tile queue)
  int skip;              // some run uses the partially skipped calculation
  int* coarse;           // 3D mixed precision: per-group coarse current windows (zero between tiles)
  int coarse_cap;        // ints per group in coarse
};

// Position of a (possibly negative or >= n) lattice index on a periodic axis.
__host__ __device__ inline int wrapi(int m, int n) {
  m %= n;
  return m < 0 ? m + n : m;
}

}  // namespace wtpic
