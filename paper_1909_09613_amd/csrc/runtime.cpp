// Host runtime of libwtpic: validation, constant tables, buffer carving,
// step sequencing and graph capture behind the C-ABI of include/wtpic.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/wtpic.h"
#include "common.hpp"
#include "launch.hpp"

using namespace wtpic;

namespace {

thread_local std::string g_err = "no error";

// smallest tile edge; bounds the scratch layout
int min_tile(int ndim) { return ndim == 2 ? 4 : 2; }
constexpr int kMaxLds = 160 * 1024;     // LDS of a gfx950 CU: the most one workgroup can take
constexpr int kMaxGroups = 2048;        // persistent particle-kernel groups (8 per CU of 256)
constexpr int kCoarseCap = 3 * (kMaxLds / 12);  // ints of one group's coarse windows (3D mixed)
// budget of the default tile choice: half a CU's LDS, so that two groups
// share a CU (measured in 3D: 16x4x4 FP32 tiles at 74 KB and 4x4x4 FP64
// tiles at 67 KB beat the smaller tiles)
constexpr int kDefaultLds = 80 * 1024;
constexpr double kTuneMargin = 0.02;  // autotuner: relative gain needed to leave the default tiling
constexpr int kMaxTileCells = 4096; // the sort orders a tile's cells in LDS
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct RunHost {
  pic_run_desc d;
  int n[3];
  long long ncell;
  long long cell0;
  long long p0;
  long long nps;  // particles per species
  int ntile[3];
  int tile0;
  int ntiles;
  double dt;
  bool set[2];
  // partially skipped calculation (pic_set_skip_region)
  bool skip_on;
  double skip_lo[3], skip_hi[3], skip_t0;
  long long skip_l0;
};

// Offsets of every array inside the four caller buffers.
struct Layout {
  size_t bytes[4];
  // particles
  size_t p_cell[2], p_pos[2][3], p_u[2][3], p_tag[2];
  // fields / current: component-major
  // scratch
  size_t s_state, s_runs, s_tile_run, s_counts, s_cursor, s_seg, s_bbox, s_jb, s_keys, s_blk_run, s_blk_first, s_acc,
      s_part, s_rho, s_coarse;
  size_t coarse_bytes;
  long long gmax;
  long long nblocks;
};

bool validate(const pic_run_desc* runs, int n_runs, pic_status* st, std::string* msg) {
  auto fail = [&](pic_status s, const std::string& m) {
    *st = s;
    *msg = m;
    return false;
  };
  if (!runs || n_runs <= 0) return fail(PIC_ERR_ARG, "runs must be a non-empty array");
  const pic_run_desc& r0 = runs[0];
  long long np_total = 0;
  for (int r = 0; r < n_runs; ++r) {
    const pic_run_desc& d = runs[r];
    char buf[256];
    if (d.ndim != 2 && d.ndim != 3) return fail(PIC_ERR_UNSUPPORTED, "ndim must be 2 or 3");
    if (d.order < 1 || d.order > 4) return fail(PIC_ERR_UNSUPPORTED, "order must be 1..4");
    if (d.scheme != PIC_WT && d.scheme != PIC_MC) return fail(PIC_ERR_ARG, "unknown scheme");
    if (d.solver != PIC_YEE && d.solver != PIC_M4) return fail(PIC_ERR_ARG, "unknown solver");
    if (d.precision != PIC_FP64 && d.precision != PIC_MIXED32) return fail(PIC_ERR_ARG, "unknown precision");
    if (d.ndim != r0.ndim || d.order != r0.order || d.scheme != r0.scheme || d.solver != r0.solver ||
        d.precision != r0.precision)
      return fail(PIC_ERR_UNSUPPORTED, "runs of one context must share ndim, order, scheme, solver, precision");
    if (!(d.c > 0) || !std::isfinite(d.c)) return fail(PIC_ERR_ARG, "c must be positive");
    if (d.ppc_per_species < 1) return fail(PIC_ERR_ARG, "ppc_per_species must be >= 1");
    if (d.ndim == 2 && d.n[2] != 1) return fail(PIC_ERR_ARG, "2D runs need n[2] == 1");
    double inv2 = 0.0;
    long long ncell = 1;
    if (d.drift_axis < 0 || d.drift_axis >= d.ndim) return fail(PIC_ERR_ARG, "drift_axis must be in 0..ndim-1");
    for (int k = 0; k < d.ndim; ++k) {
      const int lim = max_cells_per_axis(d.ndim, k);
      if (d.n[k] < d.order + 3) {
        snprintf(buf, sizeof buf, "run %d: n[%d] = %d is smaller than order + 3", r, k, d.n[k]);
        return fail(PIC_ERR_ARG, buf);
      }
      if (d.n[k] > lim) {
        snprintf(buf, sizeof buf, "run %d: n[%d] = %d exceeds %d, the packed cell index's limit", r, k, d.n[k], lim);
        return fail(PIC_ERR_ARG, buf);
      }
      if (!(d.dx[k] > 0) || !std::isfinite(d.dx[k])) return fail(PIC_ERR_ARG, "dx must be positive");
      inv2 += 1.0 / (d.dx[k] * d.dx[k]);
      ncell *= d.n[k];
    }
    if (!(d.courant > 0) || !std::isfinite(d.courant)) return fail(PIC_ERR_ARG, "courant must be positive");
    const double cdt = d.courant * d.dx[0];
    if (cdt >= 1.0 / std::sqrt(inv2)) {
      snprintf(buf, sizeof buf, "run %d: c dt = %g violates the Yee Courant limit %g", r, cdt, 1.0 / std::sqrt(inv2));
      return fail(PIC_ERR_CFL, buf);
    }
    for (int k = 0; k < d.ndim; ++k)
      if (cdt / d.dx[k] >= 1.0) return fail(PIC_ERR_ARG, "c dt / dx must be < 1 on every axis");
    for (int s = 0; s < 2; ++s) {
      if (!std::isfinite(d.q_over_m[s]) || d.q_over_m[s] == 0.0) return fail(PIC_ERR_ARG, "q_over_m must be nonzero");
      if (!std::isfinite(d.macro_charge[s])) return fail(PIC_ERR_ARG, "macro_charge must be finite");
      if (d.macro_charge[s] != 0.0 && (d.macro_charge[s] > 0) != (d.q_over_m[s] > 0))
        return fail(PIC_ERR_ARG, "macro_charge and q_over_m must have the same sign");
    }
    np_total += 2LL * ncell * d.ppc_per_species;
    if (ncell * (long long)d.ppc_per_species >= (1LL << kSpeciesShift))
      return fail(PIC_ERR_ARG, "too many particles per species for the tag");
  }
  if (np_total >= (1LL << 31)) return fail(PIC_ERR_ARG, "too many particles (int32 segment offsets)");
  return true;
}

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

Layout make_layout(const pic_run_desc* runs, int n_runs) {
  Layout L{};
  const int ndim = runs[0].ndim;
  const bool f64 = runs[0].precision == PIC_FP64;
  const size_t rs = f64 ? 8 : 4;
  long long np = 0, nc = 0, maxc = 0, gmax = 0, nblocks = 0;
  for (int r = 0; r < n_runs; ++r) {
    long long c = 1, g = 1;
    for (int k = 0; k < ndim; ++k) {
      c *= runs[r].n[k];
      g *= ceil_div(runs[r].n[k], min_tile(ndim));
    }
    np += 2 * c * runs[r].ppc_per_species;
    nc += c;
    maxc = std::max(maxc, c);
    gmax += g;
    nblocks += ceil_div(c, 256);
  }
  L.gmax = gmax;
  L.nblocks = nblocks;
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    L.p_cell[b] = off;
    if (!f64) off += align_up(4 * np);
    for (int k = 0; k < 3; ++k) {
      L.p_pos[b][k] = off;
      if (k < ndim) off += align_up(rs * np);
    }
    for (int k = 0; k < 3; ++k) {
      L.p_u[b][k] = off;
      off += align_up(rs * np);
    }
    L.p_tag[b] = off;
    off += align_up(4 * np);
  }
  L.bytes[0] = off;
  L.bytes[1] = align_up(6 * rs * nc);
  L.bytes[2] = align_up(3 * 8 * nc);
  off = 0;
  L.s_state = off;
  off += align_up(sizeof(DevState));
  L.s_runs = off;
  off += align_up((f64 ? sizeof(RunDev<double>) : sizeof(RunDev<float>)) * n_runs);
  L.s_tile_run = off;
  off += align_up(4 * gmax);
  L.s_counts = off;
  off += align_up(4 * 2 * gmax);
  L.s_cursor = off;
  off += align_up(4 * 2 * gmax);
  L.s_seg = off;
  off += align_up(4 * (2 * gmax + 1));
  L.s_bbox = off;
  off += align_up(4 * 6 * gmax);
  L.s_jb = off;
  off += align_up(4 * 4 * gmax);
  L.s_keys = off;
  off += align_up(4 * np);
  L.s_blk_run = off;
  off += align_up(4 * nblocks);
  L.s_blk_first = off;
  off += align_up(4 * nblocks);
  L.s_acc = off;
  off += align_up(8 * 16);
  L.s_part = off;
  off += align_up(8 * 16 * (size_t)kDiagBlocks);
  L.s_rho = off;
  off += align_up(8 * maxc);
  // 3D mixed precision: each particle-kernel group's coarse current windows
  L.s_coarse = off;
  L.coarse_bytes = (ndim == 3 && !f64) ? (size_t)4 * kCoarseCap * kMaxGroups : 0;
  off += align_up(L.coarse_bytes);
  L.bytes[3] = off;
  return L;
}

}  // namespace

struct pic_ctx {
  std::vector<RunHost> runs;
  int nruns = 0, ndim = 2, order = 2, prec = PIC_MIXED32, scheme = PIC_WT, solver = PIC_YEE;
  hipStream_t stream = nullptr;
  long long ncell_total = 0, np_total = 0;
  int G = 0;
  int tile[3] = {32, 16, 1};
  int margin = 3, sort_every = 2;
  int fw[3] = {1, 1, 1}, jw[3] = {1, 1, 1}, guard[3] = {0, 0, 0};
  int fp[2] = {1, 1}, jp[2] = {1, 1};  // window row and plane pitches
  size_t lds = 0;
  size_t lds_budget = 64 * 1024;
  int cus = 256;
  // persistent particle-kernel groups: the ones a CU holds at once, times the
  // CUs (plain kernel and skip variant)
  int groups_plain = 2048, groups_skip = 2048;
  pic_buffers bufs{};
  Layout lay{};
  char* P = nullptr;
  char* S = nullptr;
  void* F = nullptr;
  double* J = nullptr;
  std::string err = "no error";
  long long step = 0;
  bool started = false;
  bool force_sort = true;
  bool sorted_once = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_steps = 0;
  bool timing = false;
  bool use_gpd_graph = false;  // set by pic_step while timing
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;   // eager launches since the last read
  // while timing: a graph of the particle kernel alone, replayed once per
  // step between two stream events
  hipGraphExec_t gexec_gpd = nullptr;
  hipGraph_t graph_gpd = nullptr;
  std::vector<int> tile_run_host;
  std::vector<int> blk_run_host, blk_first_host;
  // called by pic_destroy once the stream has drained (allocation-free
  // initialisation: releases the device's static scratch)
  void (*destroy_hook)(int) = nullptr;
  int destroy_hook_arg = -1;

  pic_status fail(pic_status s, const std::string& m) {
    err = m;
    return s;
  }
  pic_status hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return PIC_OK;
    err = std::string(where) + ": " + hipGetErrorString(e);
    return PIC_ERR_HIP;
  }
  bool f64() const { return prec == PIC_FP64; }
  size_t rsize() const { return f64() ? 8 : 4; }
  DevState* state() { return reinterpret_cast<DevState*>(S + lay.s_state); }

  template <class Real>
  PBuf<Real> pbuf(int b) {
    PBuf<Real> p{};
    p.cell = f64() ? nullptr : reinterpret_cast<int*>(P + lay.p_cell[b]);
    for (int k = 0; k < 3; ++k) {
      p.pos[k] = (k < ndim) ? reinterpret_cast<Real*>(P + lay.p_pos[b][k]) : nullptr;
      p.u[k] = reinterpret_cast<Real*>(P + lay.p_u[b][k]);
    }
    p.tag = reinterpret_cast<int*>(P + lay.p_tag[b]);
    return p;
  }
};

namespace {

// Host <-> device transfer of pageable host memory: drain the context stream,
// then a blocking copy that has completed when it returns.
hipError_t host_copy(pic_ctx* c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && bytes > 0) e = hipMemcpy(dst, src, bytes, kind);
  return e;
}

// Row and plane pitch of a staged window of w[0] x w[1] (x w[2]) nodes: in
// mixed precision the fixed pitches of FixedPitch (fixed[2]: row, plane)
// when the window fits them, so that the kernel's fixed-pitch variant runs;
// else the window's own
// row, and in 3D mixed precision a plane rounded up to a multiple of 8 (117
// -> 120 nodes: 2% faster at 256x128x128 with 8x4x4 tiles, the LDS bank
// conflicts of the wave's rows drop).  Measured on the benchmark workloads
// (mixed precision): 2D field rows at 64 and current rows at 48 were 2%
// faster at 4096x2048 than 48 for both, which was 1.8% faster than the bare
// 41.
void window_pitches(int ndim, bool f64, const int w[3], const int fixed[2], int p[2]) {
  p[0] = w[0];
  p[1] = p[0] * w[1];
  if (ndim == 3 && !f64) p[1] = (p[1] + 7) / 8 * 8;
  const bool fits = !f64 && w[0] <= fixed[0] && (ndim == 2 || fixed[0] * w[1] <= fixed[1]);
  if (fits) {
    p[0] = fixed[0];
    p[1] = (ndim == 2) ? p[0] * w[1] : fixed[1];
  }
}

// Reach of a table's nodes relative to the particle's cell: base - cell is 0
// or -1 (the latter only when sigma > 0).
void table_reach(const Tab<double>& t, int K, int& lo, int& hi) {
  lo = t.first - (t.sigma > 0.0 ? 1 : 0);
  hi = t.first + K - 1;
}

template <class Real>
pic_status build_runs(pic_ctx* c, std::vector<RunDev<Real>>& out) {
  out.resize(c->nruns);
  for (int r = 0; r < c->nruns; ++r) {
    const RunHost& H = c->runs[r];
    const pic_run_desc& d = H.d;
    RunDev<Real>& R = out[r];
    std::memset(&R, 0, sizeof R);
    const int l = d.order;
    for (int k = 0; k < 3; ++k) {
      R.n[k] = H.n[k];
      R.ntile[k] = H.ntile[k];
    }
    R.tile0 = H.tile0;
    R.cell0 = H.cell0;
    R.p0 = H.p0;
    R.np = 2 * H.nps;
    double Vc = 1.0;
    for (int k = 0; k < d.ndim; ++k) Vc *= d.dx[k];
    R.Vc = Vc;
    R.c = Real(d.c);
    R.dt = Real(H.dt);
    R.hcdt = Real(0.5 * H.dt * d.c);
    int KT = l + 1;
    for (int k = 0; k < 3; ++k) {
      const double a = (k < d.ndim) ? d.c * H.dt / d.dx[k] : 0.5;
      R.a[k] = Real(a);
      R.inv_dx[k] = Real(k < d.ndim ? 1.0 / d.dx[k] : 0.0);
      R.dxd[k] = k < d.ndim ? d.dx[k] : 1.0;
      if (k < d.ndim && d.scheme == PIC_WT && a > 0.5) KT = l + 2;
    }
    R.KT = KT;
    for (int k = 0; k < d.ndim; ++k) {
      Tab<double> wh, wi, tt;
      const char* e = nullptr;
      if (!build_table(l, 0, 0.5, wh, &e) || !build_table(l, 1, 0.5, wi, &e))
        return c->fail(PIC_ERR_ARG, std::string("table: ") + e);
      const double a = d.c * H.dt / d.dx[k];
      if (d.scheme == PIC_WT) {
        if (!build_table(l, 2, a, tt, &e)) return c->fail(PIC_ERR_ARG, std::string("table: ") + e);
      } else {
        if (!build_table(l, 2, 0.5, tt, &e)) return c->fail(PIC_ERR_ARG, std::string("table: ") + e);
      }
      convert_table(wh, R.Wh[k]);
      convert_table(wi, R.Wi[k]);
      convert_table(tt, R.T[k]);
      int lo1, hi1, lo2, hi2, lo3, hi3;
      table_reach(wh, l + 1, lo1, hi1);
      table_reach(tt, KT, lo2, hi2);
      table_reach(wi, l + 1, lo3, hi3);
      R.glo[k] = std::min(lo1, lo2);
      R.ghi[k] = std::max(hi1, hi2);
      R.dlo[k] = lo3 - 1;
      R.dhi[k] = hi3 + 1;
      for (int e2 = 0; e2 < d.ndim; ++e2) {
        const double ce = d.c * H.dt / d.dx[e2];
        double coef = 0.0;
        if (d.solver == PIC_M4) coef = (e2 == k) ? (ce * ce - 1.0) / 12.0 : ce * ce / 12.0;
        R.m4beta[k][e2] = Real(coef);
      }
    }
    R.skip_on = H.skip_on ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
      R.skip_lo[k] = H.skip_lo[k];
      R.skip_hi[k] = H.skip_hi[k];
    }
    R.skip_t0 = H.skip_t0;
    R.skip_l0 = H.skip_l0;
    R.cd = d.c;
    R.dtd = H.dt;
    for (int s = 0; s < 2; ++s) {
      const double Q = d.macro_charge[s], qm = d.q_over_m[s];
      R.eps[s] = Real(qm * H.dt / (2.0 * d.c));
      R.Q[s] = Q;
      R.M[s] = Q / qm;
      for (int k = 0; k < d.ndim; ++k) R.js[s][k] = -Q * d.dx[k] / (Vc * H.dt);
      if (d.ndim == 2) R.js[s][2] = Q * d.c / Vc;
    }
  }
  return PIC_OK;
}

// Rebuilds the per-run device table from the host state (tiling unchanged).
template <class Real>
pic_status upload_runs(pic_ctx* c) {
  std::vector<RunDev<Real>> rd;
  pic_status st = build_runs<Real>(c, rd);
  if (st != PIC_OK) return st;
  hipError_t e = host_copy(c, c->S + c->lay.s_runs, rd.data(), sizeof(RunDev<Real>) * rd.size(),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return c->hip(e, "run table upload");
}

// Tiling-dependent state: tiles per run, windows, guard, LDS size, and the
// device tables that depend on them.
template <class Real>
pic_status apply_tiling(pic_ctx* c) {
  const int nd = c->ndim;
  long long G = 0;
  for (auto& H : c->runs) {
    H.ntiles = 1;
    for (int k = 0; k < 3; ++k) {
      H.ntile[k] = (k < nd) ? (int)ceil_div(H.n[k], c->tile[k]) : 1;
      H.ntiles *= H.ntile[k];
    }
    H.tile0 = (int)G;
    G += H.ntiles;
  }
  if (G > c->lay.gmax) return c->fail(PIC_ERR_ARG, "tile too small for the scratch layout");
  if ((long long)c->tile[0] * c->tile[1] * c->tile[2] > kMaxTileCells)
    return c->fail(PIC_ERR_ARG, "tile has more cells than the sort's arrange pass supports");
  c->G = (int)G;
  std::vector<RunDev<Real>> rd;
  pic_status st = build_runs<Real>(c, rd);
  if (st != PIC_OK) return st;
  // windows: extent after a sort is tile - 1; it may reach guard + 2 * sort_every
  int span_g[3] = {0, 0, 0}, span_d[3] = {0, 0, 0};
  for (auto& R : rd)
    for (int k = 0; k < nd; ++k) {
      span_g[k] = std::max(span_g[k], R.ghi[k] - R.glo[k]);
      span_d[k] = std::max(span_d[k], R.dhi[k] - R.dlo[k]);
    }
  for (int k = 0; k < 3; ++k) {
    if (k >= nd) {
      c->fw[k] = c->jw[k] = 1;
      c->guard[k] = 0;
      continue;
    }
    // A step stages the box its particles had after the previous step.  A
    // box may exceed the guard by 2 cells per step until the next sort
    // opportunity (every sort_every steps), so a staged box spans at most
    // guard + 2 (sort_every - 1) cells plus the stencil reach.
    c->guard[k] = c->tile[k] + 2 * (c->margin - c->sort_every) - 1;
    c->fw[k] = c->guard[k] + 2 * (c->sort_every - 1) + span_g[k] + 1;
    c->jw[k] = c->guard[k] + 2 * (c->sort_every - 1) + span_d[k] + 1;
    if (c->guard[k] < c->tile[k]) return c->fail(PIC_ERR_ARG, "margin must exceed sort_every");
  }
  const int* ffix = nd == 2 ? FixedPitch<2>::f : FixedPitch<3>::f;
  const int* jfix = nd == 2 ? FixedPitch<2>::j : FixedPitch<3>::j;
  window_pitches(nd, c->f64(), c->fw, ffix, c->fp);
  window_pitches(nd, c->f64(), c->jw, jfix, c->jp);
  const size_t fcap = (size_t)(nd == 3 ? c->fp[1] * c->fw[2] : c->fp[0] * c->fw[1]);
  const size_t jcap = (size_t)(nd == 3 ? c->jp[1] * c->jw[2] : c->jp[0] * c->jw[1]);
  const size_t rs = sizeof(Real);
  // FP32: fine and coarse fixed-point current windows and a cell count in
  // 2D (7 ints per node), the fine windows in 3D (3 ints; its coarse ones
  // are in global memory); FP64: FP64 current windows
  c->lds = 6 * rs * fcap + (c->f64() ? 3 * sizeof(double) : (nd == 2 ? 7 : 3) * sizeof(int)) * jcap;
  if (nd == 3 && !c->f64() && 3 * jcap > (size_t)kCoarseCap)
    return c->fail(PIC_ERR_ARG, "tile too large for the coarse current windows");
  if (c->lds > (size_t)c->lds_budget) return c->fail(PIC_ERR_ARG, "tile and margin need more LDS than the workgroup budget");
  // one persistent group per slot the CUs hold at once (measured 1.5-2.5%
  // faster in 2D than launching more groups that find the queue empty)
  {
    using Pol = typename std::conditional<std::is_same<Real, double>::value, F64, F32>::type;
    c->groups_plain = std::min(kMaxGroups, c->cus * gpd_groups_per_cu<Pol>(c->order, nd, c->lds, false));
    c->groups_skip = std::min(kMaxGroups, c->cus * gpd_groups_per_cu<Pol>(c->order, nd, c->lds, true));
  }
  // device tables
  c->tile_run_host.assign(G, 0);
  for (int r = 0; r < c->nruns; ++r)
    for (int t = 0; t < c->runs[r].ntiles; ++t) c->tile_run_host[c->runs[r].tile0 + t] = r;
  hipError_t e = host_copy(c, c->S + c->lay.s_runs, rd.data(), sizeof(RunDev<Real>) * rd.size(),
                                hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = host_copy(c, c->S + c->lay.s_tile_run, c->tile_run_host.data(), 4 * G, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return c->hip(e, "apply_tiling");
}

template <class Real>
pic_status upload_static(pic_ctx* c) {
  c->blk_run_host.clear();
  c->blk_first_host.clear();
  for (int r = 0; r < c->nruns; ++r)
    for (long long f = 0; f < c->runs[r].ncell; f += 256) {
      c->blk_run_host.push_back(r);
      c->blk_first_host.push_back((int)f);
    }
  hipError_t e = host_copy(c, c->S + c->lay.s_blk_run, c->blk_run_host.data(), 4 * c->blk_run_host.size(),
                                hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = host_copy(c, c->S + c->lay.s_blk_first, c->blk_first_host.data(), 4 * c->blk_first_host.size(),
                       hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(c->F, 0, c->lay.bytes[1], c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->J, 0, c->lay.bytes[2], c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->P, 0, c->lay.bytes[0], c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->S + c->lay.s_state, 0, sizeof(DevState), c->stream);
  // the sort keeps its counts and cursors zero between sorts, the particle
  // kernel its global coarse windows
  if (e == hipSuccess) e = hipMemsetAsync(c->S + c->lay.s_counts, 0, c->lay.s_seg - c->lay.s_counts, c->stream);
  if (e == hipSuccess && c->lay.coarse_bytes)
    e = hipMemsetAsync(c->S + c->lay.s_coarse, 0, c->lay.coarse_bytes, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return c->hip(e, "init upload");
}

template <class Real>
GpdArgs<Real> gpd_args(pic_ctx* c) {
  GpdArgs<Real> a{};
  a.runs = reinterpret_cast<const RunDev<Real>*>(c->S + c->lay.s_runs);
  a.tile_run = reinterpret_cast<const int*>(c->S + c->lay.s_tile_run);
  a.seg = reinterpret_cast<const int*>(c->S + c->lay.s_seg);
  a.bbox = reinterpret_cast<int*>(c->S + c->lay.s_bbox);
  a.jb = reinterpret_cast<float*>(c->S + c->lay.s_jb);
  a.st = c->state();
  a.buf[0] = c->pbuf<Real>(0);
  a.buf[1] = c->pbuf<Real>(1);
  a.F = reinterpret_cast<const Real*>(c->F);
  a.J = c->J;
  a.ncell_total = c->ncell_total;
  a.G = c->G;
  a.skip = 0;
  for (const RunHost& H : c->runs) a.skip |= H.skip_on ? 1 : 0;
  a.max_groups = a.skip ? c->groups_skip : c->groups_plain;
  a.coarse = reinterpret_cast<int*>(c->S + c->lay.s_coarse);
  a.coarse_cap = kCoarseCap;
  for (int k = 0; k < 3; ++k) {
    a.tile[k] = c->tile[k];
    a.fw[k] = c->fw[k];
    a.jw[k] = c->jw[k];
    a.guard[k] = c->guard[k];
  }
  for (int k = 0; k < 2; ++k) {
    a.fp[k] = c->fp[k];
    a.jp[k] = c->jp[k];
  }
  return a;
}

template <class Real>
SortArgs<Real> sort_args(pic_ctx* c) {
  SortArgs<Real> a{};
  a.runs = reinterpret_cast<const RunDev<Real>*>(c->S + c->lay.s_runs);
  a.nruns = c->nruns;
  a.st = c->state();
  a.buf[0] = c->pbuf<Real>(0);
  a.buf[1] = c->pbuf<Real>(1);
  a.np_total = c->np_total;
  a.G = c->G;
  a.nkeys = 2 * c->G;
  for (int k = 0; k < 3; ++k) a.tile[k] = c->tile[k];
  a.tc = c->tile[0] * c->tile[1] * c->tile[2];
  a.kcap = arrange_kcap(a.tc);
  a.counts = reinterpret_cast<int*>(c->S + c->lay.s_counts);
  a.cursor = reinterpret_cast<int*>(c->S + c->lay.s_cursor);
  a.seg = reinterpret_cast<int*>(c->S + c->lay.s_seg);
  a.keys = reinterpret_cast<int*>(c->S + c->lay.s_keys);
  a.bbox = reinterpret_cast<int*>(c->S + c->lay.s_bbox);
  a.jb = reinterpret_cast<float*>(c->S + c->lay.s_jb);
  a.tile_run = reinterpret_cast<const int*>(c->S + c->lay.s_tile_run);
  return a;
}

template <class Real>
FieldArgs<Real> field_args(pic_ctx* c) {
  FieldArgs<Real> a{};
  a.runs = reinterpret_cast<const RunDev<Real>*>(c->S + c->lay.s_runs);
  a.blk_run = reinterpret_cast<const int*>(c->S + c->lay.s_blk_run);
  a.blk_first = reinterpret_cast<const int*>(c->S + c->lay.s_blk_first);
  a.F = reinterpret_cast<Real*>(c->F);
  a.J = c->J;
  a.ncell_total = c->ncell_total;
  a.nblocks = (int)c->blk_run_host.size();
  return a;
}

template <class P>
pic_status enqueue_gpd(pic_ctx* c, bool capture) {
  using Real = typename P::Real;
  hipError_t e = hipSuccess;
  if (c->force_sort || c->step % c->sort_every == 0) {
    e = launch_sort<P>(sort_args<Real>(c), c->ndim, c->stream);
    if (e != hipSuccess) return c->hip(e, "sort launch");
    c->force_sort = false;
  }
  // timing (never inside a capture): an event pair around the launch, which
  // in pic_step is a replay of a graph holding the particle kernel alone.
  // The events take no system-scope fence: recording one would otherwise
  // write back and invalidate the caches around every timed launch.
  const bool rec = c->timing && !capture;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rec) {
    e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (e != hipSuccess) return c->hip(e, "timing event");
    c->events.emplace_back(e0, e1);
    e = hipEventRecord(e0, c->stream);
    if (e != hipSuccess) return c->hip(e, "timing event record");
  }
  if (rec && c->use_gpd_graph) {
    if (!c->gexec_gpd) {
      e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return c->hip(e, "begin capture");
      const hipError_t el = launch_gpd<P>(gpd_args<Real>(c), c->order, c->ndim, c->lds, c->stream);
      hipGraph_t gg = nullptr;
      e = hipStreamEndCapture(c->stream, &gg);
      if (el != hipSuccess || e != hipSuccess) {
        if (gg) (void)hipGraphDestroy(gg);
        return c->hip(el != hipSuccess ? el : e, "particle-kernel graph capture");
      }
      c->graph_gpd = gg;
      e = hipGraphInstantiate(&c->gexec_gpd, gg, nullptr, nullptr, 0);
      if (e != hipSuccess) return c->hip(e, "particle-kernel graph instantiate");
    }
    e = hipGraphLaunch(c->gexec_gpd, c->stream);
  } else {
    e = launch_gpd<P>(gpd_args<Real>(c), c->order, c->ndim, c->lds, c->stream);
  }
  if (e != hipSuccess) return c->hip(e, "gather-push-deposit launch");
  if (rec) {
    e = hipEventRecord(e1, c->stream);
    if (e != hipSuccess) return c->hip(e, "timing event record");
  }
  c->step += 1;
  return PIC_OK;
}

template <class Real>
pic_status enqueue_fields(pic_ctx* c) {
  const FieldArgs<Real> a = field_args<Real>(c);
  const bool m4 = c->solver == PIC_M4;
  hipError_t e = launch_faraday_half<Real>(a, c->ndim, m4, c->stream);
  if (e == hipSuccess) e = launch_ampere<Real>(a, c->ndim, c->stream);
  if (e == hipSuccess) e = launch_faraday_half<Real>(a, c->ndim, m4, c->stream);
  return c->hip(e, "field update launch");
}

pic_status check_ready(pic_ctx* c) {
  for (int r = 0; r < c->nruns; ++r)
    for (int s = 0; s < 2; ++s)
      if (!c->runs[r].set[s]) return c->fail(PIC_ERR_STATE, "particles of every run and species must be set first");
  return PIC_OK;
}

pic_status do_gpd(pic_ctx* c, bool capture) {
  pic_status st = check_ready(c);
  if (st != PIC_OK) return st;
  c->started = true;
  c->sorted_once = true;
  return c->f64() ? enqueue_gpd<F64>(c, capture) : enqueue_gpd<F32>(c, capture);
}

pic_status do_fields(pic_ctx* c) { return c->f64() ? enqueue_fields<double>(c) : enqueue_fields<float>(c); }

int read_parity(pic_ctx* c, pic_status* st) {
  DevState ds{};
  hipError_t e = host_copy(c, &ds, c->state(), sizeof ds, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  *st = c->hip(e, "read state");
  return ds.parity;
}

// Autotuner candidates: tile (cells), staging margin, sort cadence; the first
// of each list is the default tiling of pic_init.
struct Cand {
  int t[3], margin, every;
};
int tuning_candidates(int ndim, bool f64, const Cand** out) {
  static const Cand c2s[] = {{{32, 16, 1}, 3, 2}, {{16, 16, 1}, 3, 2}, {{16, 32, 1}, 3, 2}, {{64, 8, 1}, 3, 2},
                             {{32, 8, 1}, 3, 2},  {{32, 16, 1}, 2, 1}, {{16, 16, 1}, 2, 1}};
  static const Cand c2d[] = {{{16, 16, 1}, 3, 2}, {{16, 8, 1}, 3, 2}, {{32, 8, 1}, 3, 2},
                             {{8, 16, 1}, 3, 2},  {{32, 16, 1}, 3, 2}, {{16, 16, 1}, 2, 1}};
  static const Cand c3s[] = {{{16, 4, 4}, 2, 1}, {{8, 8, 4}, 2, 1}, {{8, 4, 4}, 2, 1},
                             {{8, 8, 2}, 2, 1},  {{4, 4, 4}, 2, 1}, {{16, 4, 4}, 3, 2}};
  static const Cand c3d[] = {{{4, 4, 4}, 2, 1}, {{8, 4, 4}, 2, 1}, {{4, 4, 2}, 2, 1}, {{8, 8, 2}, 2, 1},
                             {{4, 4, 4}, 3, 2}};
  if (ndim == 2) {
    *out = f64 ? c2d : c2s;
    return f64 ? (int)(sizeof c2d / sizeof c2d[0]) : (int)(sizeof c2s / sizeof c2s[0]);
  }
  *out = f64 ? c3d : c3s;
  return f64 ? (int)(sizeof c3d / sizeof c3d[0]) : (int)(sizeof c3s / sizeof c3s[0]);
}

void drop_graph(pic_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_steps = 0;
  if (c->gexec_gpd) (void)hipGraphExecDestroy(c->gexec_gpd);
  if (c->graph_gpd) (void)hipGraphDestroy(c->graph_gpd);
  c->gexec_gpd = nullptr;
  c->graph_gpd = nullptr;
}

}  // namespace

namespace {

template <class Real>
pic_status set_particles_t(pic_ctx* c, int run, int species, const double* x, const double* u,
                                  int64_t n) {
  RunHost& H = c->runs[run];
  pic_status st;
  const int par = read_parity(c, &st);
  if (st != PIC_OK) return st;
  if (c->sorted_once) {
    // sorted stores interleave the species: the whole run must be re-set
    H.set[0] = H.set[1] = false;
  }
  const long long base = H.p0 + species * H.nps;
  std::vector<int> cell(c->f64() ? 0 : n), tag(n);
  std::vector<Real> pos[3], uu[3];
  for (int k = 0; k < 3; ++k) {
    if (k < c->ndim) pos[k].resize(n);
    uu[k].resize(n);
  }
  for (int64_t i = 0; i < n; ++i) {
    int cc[3] = {0, 0, 0};
    for (int k = 0; k < c->ndim; ++k) {
      double v = x[3 * i + k];
      const double nd = H.n[k];
      if (!std::isfinite(v)) return c->fail(PIC_ERR_ARG, "non-finite position");
      v = std::fmod(v, nd);
      while (v < 0.0) v += nd;
      while (v >= nd) v -= nd;
      if (c->f64()) {
        pos[k][i] = Real(v);
      } else {
        double fl = std::floor(v);
        float f = (float)(v - fl);
        if (f >= 1.0f) {
          f = 0.0f;
          fl += 1.0;
          if (fl >= nd) fl = 0.0;
        }
        cc[k] = (int)fl;
        pos[k][i] = Real(f);
      }
    }
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(u[3 * i + k])) return c->fail(PIC_ERR_ARG, "non-finite momentum");
      uu[k][i] = Real(u[3 * i + k]);
    }
    if (!c->f64()) cell[i] = (c->ndim == 2) ? pack_cell<2>(cc[0], cc[1], 0) : pack_cell<3>(cc[0], cc[1], cc[2]);
    tag[i] = (species << kSpeciesShift) | (int)i;
  }
  const size_t rs = sizeof(Real);
  hipError_t e = hipSuccess;
  if (!c->f64()) e = host_copy(c, c->P + c->lay.p_cell[par] + 4 * base, cell.data(), 4 * n, hipMemcpyHostToDevice);
  for (int k = 0; k < c->ndim && e == hipSuccess; ++k)
    e = host_copy(c, c->P + c->lay.p_pos[par][k] + rs * base, pos[k].data(), rs * n, hipMemcpyHostToDevice);
  for (int k = 0; k < 3 && e == hipSuccess; ++k)
    e = host_copy(c, c->P + c->lay.p_u[par][k] + rs * base, uu[k].data(), rs * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = host_copy(c, c->P + c->lay.p_tag[par] + 4 * base, tag.data(), 4 * n, hipMemcpyHostToDevice);
  const int one = 1;
  if (e == hipSuccess)
    e = host_copy(c, &c->state()->sort_request, &one, sizeof one, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip(e, "set_particles");
  H.set[species] = true;
  c->force_sort = true;
  if (!(H.set[0] && H.set[1])) c->sorted_once = false;
  return PIC_OK;
}

template <class Real>
pic_status get_particles_t(pic_ctx* c, int run, int species, double* x, double* u, int64_t n) {
  const RunHost& H = c->runs[run];
  pic_status st;
  const int par = read_parity(c, &st);
  if (st != PIC_OK) return st;
  const long long base = H.p0, cnt = 2 * H.nps;
  const size_t rs = sizeof(Real);
  std::vector<int> cell(c->f64() ? 0 : cnt), tag(cnt);
  std::vector<Real> pos[3], uu[3];
  hipError_t e = hipSuccess;
  if (!c->f64()) e = host_copy(c, cell.data(), c->P + c->lay.p_cell[par] + 4 * base, 4 * cnt, hipMemcpyDeviceToHost);
  for (int k = 0; k < 3; ++k) {
    uu[k].resize(cnt);
    if (e == hipSuccess)
      e = host_copy(c, uu[k].data(), c->P + c->lay.p_u[par][k] + rs * base, rs * cnt, hipMemcpyDeviceToHost);
    if (k < c->ndim) {
      pos[k].resize(cnt);
      if (e == hipSuccess)
        e = host_copy(c, pos[k].data(), c->P + c->lay.p_pos[par][k] + rs * base, rs * cnt, hipMemcpyDeviceToHost);
    }
  }
  if (e == hipSuccess) e = host_copy(c, tag.data(), c->P + c->lay.p_tag[par] + 4 * base, 4 * cnt, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip(e, "get_particles");
  long long found = 0;
  for (long long i = 0; i < cnt; ++i) {
    const int sp = (tag[i] >> kSpeciesShift) & 1;
    const long long id = tag[i] & ((1 << kSpeciesShift) - 1);
    if (sp != species || id >= n) continue;
    ++found;
    int cc[3] = {0, 0, 0};
    if (!c->f64()) {
      if (c->ndim == 2)
        unpack_cell<2>(cell[i], cc[0], cc[1], cc[2]);
      else
        unpack_cell<3>(cell[i], cc[0], cc[1], cc[2]);
    }
    for (int k = 0; k < 3; ++k) {
      if (k < c->ndim)
        x[3 * id + k] = c->f64() ? (double)pos[k][i] : (double)cc[k] + (double)pos[k][i];
      else
        x[3 * id + k] = 0.0;
      u[3 * id + k] = (double)uu[k][i];
    }
  }
  if (found != n) return c->fail(PIC_ERR_STATE, "particle identities are incomplete (were both species set?)");
  return PIC_OK;
}

template <class Real>
pic_status fields_io(pic_ctx* c, int run, const double* Ein, const double* Bin, double* Eout, double* Bout,
                            double* Jout) {
  const RunHost& H = c->runs[run];
  const long long nc = H.ncell, NT = c->ncell_total;
  Real* F = static_cast<Real*>(c->F);
  std::vector<Real> tmp(nc);
  hipError_t e = hipSuccess;
  for (int comp = 0; comp < 6 && e == hipSuccess; ++comp) {
    const double* src = (comp < 3) ? Ein : Bin;
    double* dst = (comp < 3) ? Eout : Bout;
    const int k = comp % 3;
    Real* dev = F + comp * NT + H.cell0;
    if (src) {
      for (long long i = 0; i < nc; ++i) tmp[i] = Real(src[k * nc + i]);
      e = host_copy(c, dev, tmp.data(), sizeof(Real) * nc, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (dst && e == hipSuccess) {
      e = host_copy(c, tmp.data(), dev, sizeof(Real) * nc, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      for (long long i = 0; i < nc; ++i) dst[k * nc + i] = (double)tmp[i];
    }
  }
  for (int k = 0; k < 3 && Jout && e == hipSuccess; ++k)
    e = host_copy(c, Jout + k * nc, c->J + k * NT + H.cell0, 8 * nc, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return c->hip(e, "field transfer");
}

template <class P>
pic_status diag_t(pic_ctx* c, int run, pic_diag* out) {
  using Real = typename P::Real;
  const RunHost& H = c->runs[run];
  DiagArgs<Real> a{};
  a.runs = reinterpret_cast<const RunDev<Real>*>(c->S + c->lay.s_runs);
  a.run = run;
  a.st = c->state();
  a.buf[0] = c->pbuf<Real>(0);
  a.buf[1] = c->pbuf<Real>(1);
  a.F = reinterpret_cast<const Real*>(c->F);
  a.ncell_total = c->ncell_total;
  a.acc = reinterpret_cast<double*>(c->S + c->lay.s_acc);
  a.part = reinterpret_cast<double*>(c->S + c->lay.s_part);
  a.rho = reinterpret_cast<double*>(c->S + c->lay.s_rho);
  // after a step the particles sit in their tiles' segments and the charge
  // density is accumulated tile by tile; right after particles were set it
  // takes the global-atomic kernel
  const bool tiled = c->sorted_once && !c->force_sort;
  hipError_t e = launch_fill<double>(a.acc, 16, 0.0, c->stream);
  if (e == hipSuccess) e = launch_fill<double>(a.rho, H.ncell, 0.0, c->stream);
  if (e == hipSuccess && tiled) {
    const size_t jcap = (size_t)c->jw[0] * c->jw[1] * c->jw[2];
    e = launch_rho_tiles<P>(gpd_args<Real>(c), run, H.ntiles, a.rho, c->order, c->ndim, 8 * jcap, c->stream);
  }
  if (e == hipSuccess) e = launch_diag<P>(a, c->ndim, c->order, H.ncell, H.p0, 2 * H.nps, tiled, c->stream);
  double acc[16];
  DevState ds{};
  if (e == hipSuccess) e = host_copy(c, acc, a.acc, sizeof acc, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = host_copy(c, &ds, c->state(), sizeof ds, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip(e, "diagnostics");
  double Vc = 1.0;
  for (int k = 0; k < c->ndim; ++k) Vc *= H.d.dx[k];
  std::memset(out, 0, sizeof *out);
  out->step = c->step;
  out->time = c->step * H.dt;
  for (int k = 0; k < 3; ++k) {
    out->UE[k] = 0.5 * acc[k] * Vc;
    out->UB[k] = 0.5 * acc[3 + k] * Vc;
    out->momentum[k] = acc[8 + k];
  }
  out->Ekin[0] = acc[6];
  out->Ekin[1] = acc[7];
  std::memcpy(&out->gauss_resid_max, &acc[11], sizeof(double));
  out->n_nonfinite = (int64_t)ds.n_nonfinite;
  out->n_out_of_range = (int64_t)ds.n_out_of_range;
  out->n_sorts = (int64_t)ds.n_sorts;
  if (ds.n_nonfinite || ds.n_out_of_range) return c->fail(PIC_ERR_NUMERIC, "device counted non-finite or out-of-window particles");
  return PIC_OK;
}

}  // namespace

namespace wtpic {

void set_destroy_hook(pic_ctx* c, void (*hook)(int), int arg) {
  c->destroy_hook = hook;
  c->destroy_hook_arg = arg;
}

void set_global_error(const char* msg) { g_err = msg; }

}  // namespace wtpic

extern "C" {

pic_status pic_query_layout(const pic_run_desc* runs, int32_t n_runs, size_t bytes_out[4]) {
  pic_status st;
  std::string msg;
  if (!bytes_out) {
    g_err = "bytes_out is NULL";
    return PIC_ERR_ARG;
  }
  if (!validate(runs, n_runs, &st, &msg)) {
    g_err = msg;
    return st;
  }
  Layout L = make_layout(runs, n_runs);
  for (int i = 0; i < 4; ++i) bytes_out[i] = L.bytes[i];
  return PIC_OK;
}

pic_status pic_init(const pic_run_desc* runs, int32_t n_runs, const pic_buffers* bufs, void* hip_stream,
                    pic_ctx** out) {
  pic_status st;
  std::string msg;
  if (!out || !bufs) {
    g_err = "out and bufs must not be NULL";
    return PIC_ERR_ARG;
  }
  if (!validate(runs, n_runs, &st, &msg)) {
    g_err = msg;
    return st;
  }
  Layout L = make_layout(runs, n_runs);
  for (int i = 0; i < 4; ++i) {
    void* p = (i == 0) ? bufs->particles : (i == 1) ? bufs->fields : (i == 2) ? bufs->current : bufs->scratch;
    if (!p || bufs->bytes[i] < L.bytes[i]) {
      char b[160];
      snprintf(b, sizeof b, "buffer %d: need %zu bytes, got %zu%s", i, L.bytes[i], bufs->bytes[i], p ? "" : " (NULL)");
      g_err = b;
      return PIC_ERR_ARG;
    }
  }
  pic_ctx* c = new pic_ctx();
  c->lay = L;
  c->bufs = *bufs;
  c->P = static_cast<char*>(bufs->particles);
  c->F = bufs->fields;
  c->J = static_cast<double*>(bufs->current);
  c->S = static_cast<char*>(bufs->scratch);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->nruns = n_runs;
  c->ndim = runs[0].ndim;
  c->order = runs[0].order;
  c->prec = runs[0].precision;
  c->scheme = runs[0].scheme;
  c->solver = runs[0].solver;
  long long cell0 = 0, p0 = 0;
  for (int r = 0; r < n_runs; ++r) {
    RunHost H{};
    H.d = runs[r];
    H.ncell = 1;
    for (int k = 0; k < 3; ++k) {
      H.n[k] = (k < c->ndim) ? runs[r].n[k] : 1;
      H.ncell *= H.n[k];
    }
    H.cell0 = cell0;
    H.p0 = p0;
    H.nps = H.ncell * runs[r].ppc_per_species;
    H.dt = runs[r].courant * runs[r].dx[0] / runs[r].c;
    H.set[0] = H.set[1] = false;
    cell0 += H.ncell;
    p0 += 2 * H.nps;
    c->runs.push_back(H);
  }
  c->ncell_total = cell0;
  c->np_total = p0;
  // default tiling: the first candidate whose LDS fits the budget.  2D
  // re-sorts are checked every 2 steps with a 3-cell margin; 3D windows are
  // costlier, so 3D checks every step with a 2-cell margin.
  {
    int dev = 0, lim = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lim > 0)
      c->lds_budget = std::min<size_t>((size_t)lim, (size_t)kMaxLds);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->cus = cus;
  }
  // measured in 2D (1024x512 cubic; 64 batched runs; 4096x2048): FP32 is
  // fastest with 32 x 16 tiles (7%, 13% and 2% ahead of 16 x 16; 32 x 32
  // and 64 x 16 need more than half the LDS), FP64 with 16 x 16
  static const int cand2s[][3] = {{32, 16, 1}, {16, 16, 1}, {16, 8, 1}, {8, 8, 1}, {8, 4, 1}, {4, 4, 1}};
  static const int cand2d[][3] = {{16, 16, 1}, {16, 8, 1}, {8, 8, 1}, {8, 4, 1}, {4, 4, 1}, {4, 4, 1}};
  // 3D: FP64 takes the largest tile within half a CU's LDS (4x4x4); mixed
  // precision keeps only its fine current windows in LDS, and with 512-thread
  // groups (two per CU, four waves per SIMD) 16x4x4 measured fastest at
  // 256x128x128 (2.90 ms; 8x8x4 2.96, 8x4x4 3.26)
  static const int cand3s[][3] = {{16, 4, 4}, {8, 4, 4}, {4, 4, 4}, {4, 4, 2}, {4, 2, 2}, {2, 2, 2}};
  static const int cand3d[][3] = {{8, 8, 4}, {8, 4, 4}, {4, 4, 4}, {4, 4, 2}, {4, 2, 2}, {2, 2, 2}};
  const int (*cand2)[3] = c->f64() ? cand2d : cand2s;
  const int (*cand3)[3] = c->f64() ? cand3d : cand3s;
  const int ncand = 6;
  c->margin = (c->ndim == 2) ? 3 : 2;
  c->sort_every = (c->ndim == 2) ? 2 : 1;
  // the largest candidate that fits the budget and gives every persistent
  // group a tile, down to tiles of 64 cells; a grid too small for that takes
  // the smallest of those (a 256 x 128 grid has only 64 tiles of 32 x 16
  // cells for 512 groups); smaller tiles only where the larger do not fit
  st = PIC_ERR_ARG;
  const size_t full = c->lds_budget;
  c->lds_budget = std::min(full, (size_t)kDefaultLds);
  int chosen = -1;
  for (int i = 0; i < ncand; ++i) {
    const int* t = (c->ndim == 2) ? cand2[i] : cand3[i];
    if (chosen >= 0 && t[0] * t[1] * t[2] < 64) break;
    for (int k = 0; k < 3; ++k) c->tile[k] = t[k];
    if ((c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c)) != PIC_OK) continue;
    chosen = i;
    if (c->G >= c->groups_plain) break;
  }
  if (chosen >= 0) {
    const int* t = (c->ndim == 2) ? cand2[chosen] : cand3[chosen];
    for (int k = 0; k < 3; ++k) c->tile[k] = t[k];
    st = c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c);
  }
  c->lds_budget = full;  // an explicit tiling may take up to the whole LDS
  if (st == PIC_OK) st = c->f64() ? upload_static<double>(c) : upload_static<float>(c);
  if (st != PIC_OK) {
    g_err = c->err;
    delete c;
    return st;
  }
  *out = c;
  return PIC_OK;
}

pic_status pic_set_skip_region(pic_ctx* c, int32_t run, const double* lo, const double* hi, double t0) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns) return c->fail(PIC_ERR_ARG, "run out of range");
  RunHost& H = c->runs[run];
  RunHost keep = H;
  if (!lo) {
    H.skip_on = false;
  } else {
    if (!hi) return c->fail(PIC_ERR_ARG, "hi is NULL");
    if (!(t0 >= 0.0) || !std::isfinite(t0)) return c->fail(PIC_ERR_ARG, "t0 must be finite and >= 0");
    for (int k = 0; k < c->ndim; ++k)
      if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(lo[k] >= 0.0) || !(lo[k] <= hi[k]) ||
          !(hi[k] <= (double)H.n[k]))
        return c->fail(PIC_ERR_ARG, "skip box needs 0 <= lo <= hi <= n on every axis");
    H.skip_on = true;
    for (int k = 0; k < 3; ++k) {
      H.skip_lo[k] = k < c->ndim ? lo[k] : 0.0;
      H.skip_hi[k] = k < c->ndim ? hi[k] : 0.0;
    }
    H.skip_t0 = t0;
    H.skip_l0 = c->step;  // launches enqueued so far: the next one is at t0
  }
  pic_status st = c->f64() ? upload_runs<double>(c) : upload_runs<float>(c);
  if (st != PIC_OK) {
    std::string e = c->err;
    H = keep;
    (void)(c->f64() ? upload_runs<double>(c) : upload_runs<float>(c));
    c->err = e;
  }
  drop_graph(c);  // the step graph holds the kernel variant
  return st;
}

pic_status pic_set_tiling(pic_ctx* c, const int32_t tile[3], int32_t margin, int32_t sort_every) {
  if (!c) return PIC_ERR_ARG;
  if (c->started) return c->fail(PIC_ERR_STATE, "tiling must be set before the first step");
  int old_tile[3] = {c->tile[0], c->tile[1], c->tile[2]};
  const int om = c->margin, os = c->sort_every;
  if (tile)
    for (int k = 0; k < c->ndim; ++k)
      if (tile[k] > 0) {
        if (tile[k] < min_tile(c->ndim)) return c->fail(PIC_ERR_ARG, "tile edges must be >= 4 (2D) or 2 (3D)");
        c->tile[k] = tile[k];
      }
  if (sort_every > 0) c->sort_every = sort_every;
  if (margin > 0) c->margin = margin;
  pic_status st = c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c);
  if (st != PIC_OK) {
    std::string keep = c->err;
    for (int k = 0; k < 3; ++k) c->tile[k] = old_tile[k];
    c->margin = om;
    c->sort_every = os;
    (void)(c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c));
    c->err = keep;
    return st;
  }
  drop_graph(c);
  c->force_sort = true;
  return PIC_OK;
}


pic_status pic_set_particles(pic_ctx* c, int32_t run, int32_t species, const double* x, const double* u, int64_t n) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns || species < 0 || species > 1) return c->fail(PIC_ERR_ARG, "bad run or species");
  if (!x || !u) return c->fail(PIC_ERR_ARG, "x and u must not be NULL");
  if (n != c->runs[run].nps) return c->fail(PIC_ERR_ARG, "n must equal ppc_per_species * ncell");
  return c->f64() ? set_particles_t<double>(c, run, species, x, u, n) : set_particles_t<float>(c, run, species, x, u, n);
}


pic_status pic_get_particles(pic_ctx* c, int32_t run, int32_t species, double* x, double* u, int64_t n) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns || species < 0 || species > 1) return c->fail(PIC_ERR_ARG, "bad run or species");
  if (!x || !u) return c->fail(PIC_ERR_ARG, "x and u must not be NULL");
  if (n != c->runs[run].nps) return c->fail(PIC_ERR_ARG, "n must equal ppc_per_species * ncell");
  return c->f64() ? get_particles_t<double>(c, run, species, x, u, n) : get_particles_t<float>(c, run, species, x, u, n);
}


pic_status pic_set_fields(pic_ctx* c, int32_t run, const double* E, const double* B) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns) return c->fail(PIC_ERR_ARG, "bad run");
  return c->f64() ? fields_io<double>(c, run, E, B, nullptr, nullptr, nullptr)
                  : fields_io<float>(c, run, E, B, nullptr, nullptr, nullptr);
}

pic_status pic_get_fields(pic_ctx* c, int32_t run, double* E, double* B, double* J) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns) return c->fail(PIC_ERR_ARG, "bad run");
  return c->f64() ? fields_io<double>(c, run, nullptr, nullptr, E, B, J)
                  : fields_io<float>(c, run, nullptr, nullptr, E, B, J);
}

pic_status pic_gather_push_deposit(pic_ctx* c) {
  if (!c) return PIC_ERR_ARG;
  return do_gpd(c, false);
}

pic_status pic_field_update(pic_ctx* c) {
  if (!c) return PIC_ERR_ARG;
  return do_fields(c);
}

pic_status pic_step(pic_ctx* c, int32_t n_steps) {
  if (!c) return PIC_ERR_ARG;
  if (n_steps < 0) return c->fail(PIC_ERR_ARG, "n_steps must be >= 0");
  pic_status st = check_ready(c);
  if (st != PIC_OK) return st;
  const int per_graph = c->sort_every * std::max(1, 8 / c->sort_every);
  if (c->timing && c->stream != nullptr) {
    // timed steps: the particle kernel replayed from its own graph between
    // two events, the sort checks and the field update launched around it
    c->use_gpd_graph = true;
    for (; n_steps > 0 && st == PIC_OK; --n_steps) {
      st = do_gpd(c, false);
      if (st == PIC_OK) st = do_fields(c);
    }
    c->use_gpd_graph = false;
    return st;
  }
  while (n_steps > 0) {
    const bool aligned = !c->force_sort && c->step % c->sort_every == 0 && c->stream != nullptr;
    if (aligned && n_steps >= per_graph) {
      if (!c->gexec) {
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return c->hip(e, "begin capture");
        const long long s0 = c->step;
        for (int i = 0; i < per_graph && st == PIC_OK; ++i) {
          st = do_gpd(c, true);
          if (st == PIC_OK) st = do_fields(c);
        }
        c->step = s0;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->stream, &g);
        if (st != PIC_OK) {
          if (g) hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return c->hip(e, "end capture");
        c->graph = g;
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          drop_graph(c);
          return c->hip(e, "graph instantiate");
        }
        c->graph_steps = per_graph;
      }
      hipError_t e = hipGraphLaunch(c->gexec, c->stream);
      if (e != hipSuccess) return c->hip(e, "graph launch");
      c->step += per_graph;
      n_steps -= per_graph;
      continue;
    }
    st = do_gpd(c, false);
    if (st == PIC_OK) st = do_fields(c);
    if (st != PIC_OK) return st;
    --n_steps;
  }
  return PIC_OK;
}


pic_status pic_step_diag(pic_ctx* c, int32_t n_steps, int32_t diag_every, int32_t run, pic_diag* history) {
  if (!c) return PIC_ERR_ARG;
  if (diag_every < 1 || n_steps < 0 || !history) return c->fail(PIC_ERR_ARG, "diag_every >= 1, n_steps >= 0, history != NULL");
  if (run < 0 || run >= c->nruns) return c->fail(PIC_ERR_ARG, "bad run");
  for (int32_t i = 0; i < n_steps / diag_every; ++i) {
    pic_status st = pic_step(c, diag_every);
    if (st == PIC_OK) st = pic_diagnostics(c, run, &history[i]);
    if (st != PIC_OK) return st;
  }
  return pic_step(c, n_steps % diag_every);
}

// Autotuner of the tiling.  Each candidate is timed over graph-replayed
// steps of the context's own workload, after untimed steps that take its first
// (full) sort and its graph capture.  The trial steps are undone afterwards
// from a host copy of the current particle store, the fields, the current and
// the device state, so the simulation resumes from where it was.
pic_status pic_autotune(pic_ctx* c, int32_t trial_steps, int32_t chosen[5], double* best_ms) {
  if (!c) return PIC_ERR_ARG;
  if (trial_steps < 1 || trial_steps > 4096) return c->fail(PIC_ERR_ARG, "trial_steps must be in 1..4096");
  if (c->started) return c->fail(PIC_ERR_STATE, "autotune must run before the first step");
  pic_status st = check_ready(c);
  if (st != PIC_OK) return st;
  const Cand* cand = nullptr;
  const int ncand = tuning_candidates(c->ndim, c->f64(), &cand);

  // snapshot: the current particle store (the other one is the sort's
  // destination and holds nothing yet), fields, current, device state
  const int par = read_parity(c, &st);
  if (st != PIC_OK) return st;
  const size_t p_lo = c->lay.p_cell[par];
  const size_t p_hi = par == 0 ? c->lay.p_cell[1] : c->lay.bytes[0];
  std::vector<char> hp(p_hi - p_lo), hf(c->lay.bytes[1]), hj(c->lay.bytes[2]);
  DevState ds{};
  hipError_t e = host_copy(c, hp.data(), c->P + p_lo, hp.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = host_copy(c, hf.data(), c->F, hf.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = host_copy(c, hj.data(), c->J, hj.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = host_copy(c, &ds, c->state(), sizeof ds, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return c->hip(e, "autotune snapshot");
  const Cand keep = {{c->tile[0], c->tile[1], c->tile[2]}, c->margin, c->sort_every};
  const bool keep_timing = c->timing, keep_sorted = c->sorted_once;
  const long long step0 = c->step;
  c->timing = false;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0.0, ms_first = 0.0;
  int bi = -1;
  for (int i = 0; i < ncand && e == hipSuccess && st == PIC_OK; ++i) {
    for (int k = 0; k < 3; ++k) c->tile[k] = k < c->ndim ? cand[i].t[k] : 1;
    c->margin = cand[i].margin;
    c->sort_every = cand[i].every;
    if ((c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c)) != PIC_OK) continue;  // LDS too small
    drop_graph(c);
    // the sort kernels run only on a device-side request: the particles are
    // still in the previous tiling's tile order
    c->force_sort = true;
    const int one = 1;
    e = host_copy(c, &c->state()->sort_request, &one, sizeof one, hipMemcpyHostToDevice);
    DevState d0{}, d1{};
    if (e == hipSuccess) e = host_copy(c, &d0, c->state(), sizeof d0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) break;
    const int per_graph = c->sort_every * std::max(1, 8 / c->sort_every);
    const int timed = (trial_steps + per_graph - 1) / per_graph * per_graph;
    st = pic_step(c, 2 * per_graph);
    if (st != PIC_OK) break;
    e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) st = pic_step(c, timed);
    if (e == hipSuccess && st == PIC_OK) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess && st == PIC_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && st == PIC_OK) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && st == PIC_OK) e = host_copy(c, &d1, c->state(), sizeof d1, hipMemcpyDeviceToHost);
    if (e != hipSuccess || st != PIC_OK) break;
    // a tile whose particles outgrew its windows is left unprocessed (and
    // counted): such a trial is not a measurement of the tiling
    if (d1.n_out_of_range != d0.n_out_of_range || d1.n_nonfinite != d0.n_nonfinite) {
      st = c->fail(PIC_ERR_NUMERIC, "autotune: a trial step left particles out of range or non-finite");
      break;
    }
    if (i == 0) ms_first = ms / timed;
    if (bi < 0 || ms / timed < best) {
      best = ms / timed;
      bi = i;
    }
  }
  // the default (first) candidate stays unless another is faster by more
  // than the spread of repeated timings
  if (bi > 0 && ms_first > 0.0 && best > (1.0 - kTuneMargin) * ms_first) {
    best = ms_first;
    bi = 0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  std::string trial_err;
  if (e != hipSuccess)
    trial_err = std::string("autotune trial: ") + hipGetErrorString(e);
  else if (st != PIC_OK)
    trial_err = c->err;

  // the chosen tiling (the previous one if no candidate ran), then the state
  const Cand& pick = (bi >= 0 && trial_err.empty()) ? cand[bi] : keep;
  for (int k = 0; k < 3; ++k) c->tile[k] = k < c->ndim ? pick.t[k] : 1;
  c->margin = pick.margin;
  c->sort_every = pick.every;
  pic_status rs = c->f64() ? apply_tiling<double>(c) : apply_tiling<float>(c);
  drop_graph(c);
  ds.sort_request = 1;  // the first step sorts into the chosen tiling
  hipError_t re = host_copy(c, c->P + p_lo, hp.data(), hp.size(), hipMemcpyHostToDevice);
  if (re == hipSuccess) re = host_copy(c, c->F, hf.data(), hf.size(), hipMemcpyHostToDevice);
  if (re == hipSuccess) re = host_copy(c, c->J, hj.data(), hj.size(), hipMemcpyHostToDevice);
  if (re == hipSuccess) re = host_copy(c, c->state(), &ds, sizeof ds, hipMemcpyHostToDevice);
  if (re == hipSuccess) re = hipStreamSynchronize(c->stream);
  c->step = step0;
  c->started = false;
  c->force_sort = true;
  c->sorted_once = keep_sorted;
  c->timing = keep_timing;
  if (re != hipSuccess) return c->hip(re, "autotune restore");
  if (rs != PIC_OK) return rs;
  if (!trial_err.empty()) return c->fail(e != hipSuccess ? PIC_ERR_HIP : st, trial_err);
  if (bi < 0) return c->fail(PIC_ERR_ARG, "no candidate tiling fits the LDS");
  if (chosen) {
    for (int k = 0; k < 3; ++k) chosen[k] = c->tile[k];
    chosen[3] = c->margin;
    chosen[4] = c->sort_every;
  }
  if (best_ms) *best_ms = best;
  return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx* c, int32_t run, pic_diag* out) {
  if (!c) return PIC_ERR_ARG;
  if (run < 0 || run >= c->nruns || !out) return c->fail(PIC_ERR_ARG, "bad run or NULL out");
  pic_status st = check_ready(c);
  if (st != PIC_OK) return st;
  // the diagnostic kernels take a particle's species from its tag, so they
  // read the stores in any order (also right after pic_set_particles)
  return c->f64() ? diag_t<F64>(c, run, out) : diag_t<F32>(c, run, out);
}

pic_status pic_kernel_timing(pic_ctx* c, int32_t enable, double* avg_ms, int64_t* launches) {
  if (!c) return PIC_ERR_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip(e, "timing sync");
  double tot = 0.0;
  for (auto& pr : c->events) {
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    tot += ms;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  const int64_t n = (int64_t)c->events.size();
  c->events.clear();
  if (e != hipSuccess) return c->hip(e, "kernel timing");
  if (avg_ms) *avg_ms = n ? tot / n : 0.0;
  if (launches) *launches = n;
  c->timing = enable != 0;
  return PIC_OK;
}

const char* pic_last_error(const pic_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

pic_status pic_destroy(pic_ctx* c) {
  if (!c) return PIC_ERR_ARG;
  hipStreamSynchronize(c->stream);
  drop_graph(c);
  for (auto& pr : c->events) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  if (c->destroy_hook) c->destroy_hook(c->destroy_hook_arg);
  delete c;
  return PIC_OK;
}

pic_status pic_table_weights(int32_t l, int32_t kind, double a, double f, int32_t* node_first, int32_t* count,
                             double* weights) {
  if (!node_first || !count || !weights) {
    g_err = "NULL output";
    return PIC_ERR_ARG;
  }
  if (!(f >= 0.0 && f < 1.0)) {
    g_err = "f must be in [0, 1)";
    return PIC_ERR_ARG;
  }
  Tab<double> t;
  const char* e = nullptr;
  if (!build_table(l, kind, kind == 2 ? a : 0.5, t, &e)) {
    g_err = e ? e : "bad table";
    return PIC_ERR_ARG;
  }
  int base;
  double g;
  tab_split(t, 0, f, base, g);
  double w[kMaxNodes] = {0};
  switch (l * 10 + t.K) {
    case 12: tab_eval<1, 2, true>(t, g, w); break;
    case 13: tab_eval<1, 3, true>(t, g, w); break;
    case 23: tab_eval<2, 3, true>(t, g, w); break;
    case 24: tab_eval<2, 4, true>(t, g, w); break;
    case 34: tab_eval<3, 4, true>(t, g, w); break;
    case 35: tab_eval<3, 5, true>(t, g, w); break;
    case 45: tab_eval<4, 5, true>(t, g, w); break;
    case 46: tab_eval<4, 6, true>(t, g, w); break;
    default: g_err = "internal: node count"; return PIC_ERR_ARG;
  }
  *node_first = base + t.first;
  *count = t.K;
  for (int k = 0; k < t.K; ++k) weights[k] = w[k];
  return PIC_OK;
}

pic_status pic_tiling_candidates(int32_t ndim, int32_t precision, int32_t* out, int32_t cap, int32_t* count) {
  if (!count || (cap > 0 && !out) || cap < 0) {
    g_err = "count must not be NULL, and out not NULL when cap > 0";
    return PIC_ERR_ARG;
  }
  if ((ndim != 2 && ndim != 3) || (precision != PIC_FP64 && precision != PIC_MIXED32)) {
    g_err = "ndim must be 2 or 3 and precision PIC_FP64 or PIC_MIXED32";
    return PIC_ERR_ARG;
  }
  const Cand* cand = nullptr;
  const int n = tuning_candidates(ndim, precision == PIC_FP64, &cand);
  *count = n;
  for (int i = 0; i < n && i < cap; ++i) {
    for (int k = 0; k < 3; ++k) out[5 * i + k] = k < ndim ? cand[i].t[k] : 1;
    out[5 * i + 3] = cand[i].margin;
    out[5 * i + 4] = cand[i].every;
  }
  return PIC_OK;
}

}  // extern "C"
