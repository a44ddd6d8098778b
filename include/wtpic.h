/*
 * wtpic.h -- C-ABI of the MI355X (gfx950) library for the per-particle hot
 * path of a relativistic electromagnetic PIC step with the time-step
 * dependent "WT" force interpolation of Lu, Kilian, Guo, Li and Liang,
 * "Time-step dependent force interpolation scheme for suppressing numerical
 * Cherenkov instability in relativistic particle-in-cell simulations"
 * (arXiv:1909.09613).
 *
 * One step of the path is
 *   gather   E, B from the staggered Yee grid to each particle with the WT
 *            tensor of Eq. interpolation-EB-real-mod (B-spline W_l along a
 *            component's staggered axes, the time-step dependent T_l of the
 *            equations following Eq. tau_l across them), or the MC tensor
 *            of Eq. interpolation-EB-real-org;
 *   push     relativistic Boris (Sec. 1);
 *   deposit  the exact charge-conserving current of Esirkepov (Sec. 1, 2),
 *            with the form factor of Eq. shape-real;
 *   fields   Yee leapfrog, or the Faraday stencil of Appendix C (M4).
 *
 * Conventions shared by every entry point
 *   - Units: positions in cell units along each axis, u = gamma v / c,
 *     Maxwell with 4 pi absorbed (dE/dt = c curl B - J, dB/dt = -c curl E),
 *     as in the dimensionless set of Appendix E.  Every axis is periodic.
 *   - Staggering (Sec. 2): E_i and J_i half a cell off along i, B_i half a
 *     cell off along the other axes, rho on integer nodes.  Host field arrays
 *     are double, component-major [3][ncell], cell index i + n0*(j + n1*k),
 *     and index m along a staggered axis holds the value at m + 1/2.
 *   - Time centring: x^n, u^{n-1/2}, E^n, B^n before a step; after
 *     pic_gather_push_deposit the device holds x^{n+1}, u^{n+1/2} and
 *     J^{n+1/2}; pic_field_update then advances E, B to n+1.
 *   - Memory: the caller allocates every device buffer (sizes from
 *     pic_query_layout) and keeps it alive until pic_destroy; the library
 *     never allocates or frees device memory.  It owns only its host-side
 *     context and graph objects.
 *   - Streams: all device work of a context is ordered on the HIP stream
 *     given to pic_init (NULL = the null stream).  Calls that return host
 *     data synchronise that stream.  A context is not thread-safe.
 *   - Errors: every call returns a pic_status; pic_last_error gives text.
 *     Nothing throws across the ABI.
 */
#ifndef WTPIC_H
#define WTPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_ERR_ARG = -1,          /* invalid argument (null pointer, size, range) */
  PIC_ERR_CFL = -2,          /* c dt exceeds the Yee Courant limit */
  PIC_ERR_UNSUPPORTED = -3,  /* order outside 1..4, mixed ndim/order/precision */
  PIC_ERR_HIP = -4,          /* a HIP runtime call failed */
  PIC_ERR_NUMERIC = -5,      /* device counted non-finite or out-of-window particles */
  PIC_ERR_STATE = -6         /* call out of order (e.g. stepping before particles are set) */
} pic_status;

typedef enum { PIC_WT = 0, PIC_MC = 1 } pic_scheme;           /* interpolation tensor */
typedef enum { PIC_YEE = 0, PIC_M4 = 1 } pic_solver;          /* Faraday stencil */
typedef enum { PIC_FP64 = 0, PIC_MIXED32 = 1 } pic_precision;
/* PIC_FP64:    absolute FP64 positions, FP64 u, fields, weights and current.
 * PIC_MIXED32: int32 cell + FP32 in-cell offset, FP32 u, fields, weights and
 *              per-tile current; FP64 global current and diagnostics. */

/* One independent periodic run.  Every run of a context must share ndim,
 * order, scheme, solver and precision; grids, Courant numbers and plasma
 * parameters may differ (the batched time-step sweep). */
typedef struct {
  int32_t ndim;             /* 2 or 3 */
  int32_t n[3];             /* cells per axis; n[2] = 1 in 2D.  Each n >= order + 3;
                               at most 65535 per axis in 2D, and 2048 (x1, x2) and
                               1024 (x3) in 3D (the packed cell index of the
                               mixed-precision layout) */
  double dx[3];             /* cell sizes */
  double c;                 /* speed of light */
  double courant;           /* c dt / dx[0]; the time step is dt = courant dx[0] / c.
                               Must satisfy c dt < 1/sqrt(sum 1/dx_d^2) and
                               c dt / dx_d < 1 on every axis */
  int32_t order;            /* B-spline order l, 1..4 (T_1..T_4 of Sec. 2) */
  int32_t scheme;           /* pic_scheme */
  int32_t solver;           /* pic_solver */
  int32_t drift_axis;       /* axis of the beam drift, 0..ndim-1; 0 is x1, the
                               beam direction of Sec. 2 and Appendix A.  The
                               particle path does not depend on it: the WT and
                               MC tensors treat every axis alike, and the
                               caller's particles carry the drift.  Recorded
                               for the caller and validated. */
  int32_t precision;        /* pic_precision */
  int32_t ppc_per_species;  /* particles per cell per species (electrons, positrons) */
  double q_over_m[2];       /* charge-to-mass ratio per species (e.g. -1, +1) */
  double macro_charge[2];   /* macro-particle charge Q per species (signed) */
} pic_run_desc;

/* Caller-owned device buffers, sized by pic_query_layout. */
typedef struct {
  void *particles;   /* two particle stores (the sort ping-pongs between them) */
  void *fields;      /* E and B of every run */
  void *current;     /* FP64 J of every run */
  void *scratch;     /* run tables, tile segments, sort keys, diagnostics */
  size_t bytes[4];   /* sizes actually provided, checked against the layout */
} pic_buffers;

typedef struct {
  int64_t step;          /* steps taken by this context */
  double time;           /* step * dt */
  double UE[3], UB[3];   /* 1/2 sum E_d^2 Vc, 1/2 sum B_d^2 Vc */
  double Ekin[2];        /* sum M (gamma - 1) c^2 per species, M = Q / (q/m) */
  double momentum[3];    /* sum M u c over both species */
  double gauss_resid_max;/* max |D.E - rho| on integer nodes (Appendix B, Eq. gauss) */
  int64_t n_nonfinite;   /* particles with a non-finite momentum or position */
  int64_t n_out_of_range;/* particles found outside their tile's staged window */
  int64_t n_sorts;       /* counting sorts performed so far (all runs) */
} pic_diag;

typedef struct pic_ctx pic_ctx;

/* Bytes the four caller buffers need for these runs.  Pure host call. */
pic_status pic_query_layout(const pic_run_desc *runs, int32_t n_runs, size_t bytes_out[4]);

/* Validates the runs, builds the per-run constant tables (the WT factors
 * T_l as polynomials in the in-cell coordinate), carves the caller buffers
 * and zeroes fields and current.  Errors: PIC_ERR_ARG, PIC_ERR_CFL,
 * PIC_ERR_UNSUPPORTED, PIC_ERR_HIP.  *out is set only on PIC_OK. */
pic_status pic_init(const pic_run_desc *runs, int32_t n_runs, const pic_buffers *bufs,
                    void *hip_stream, pic_ctx **out);

/* pic_init for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * context, but its scratch buffer is a file-scope device array of the
 * library, 64 MiB on each device that uses it (held until the process
 * ends), instead of bufs->scratch, which is ignored (bufs->bytes[3] too).
 * The caller still provides the particle, field and current buffers.  The
 * call allocates no device memory (no hipMalloc or hipFree, no allocating
 * library routine).  There is one such array per device, so at most one
 * context of this call may be alive per device: a second call on a device
 * whose array is in use returns PIC_ERR_STATE until the first context is
 * destroyed.  Runs whose scratch (pic_query_layout, bytes_out[3]) exceeds
 * 64 MiB are refused with PIC_ERR_ARG (e.g. 3D mixed precision, whose coarse
 * current windows alone take 335 MB; 2D runs of up to about 14M particles
 * fit).  Otherwise as pic_init. */
pic_status pic_init_static(const pic_run_desc *runs, int32_t n_runs, const pic_buffers *bufs,
                           void *hip_stream, pic_ctx **out);

/* Uploads one species of one run: x is host [n][3] positions in cell units
 * (entries past ndim ignored), u host [n][3] momenta u = gamma v / c; n must
 * equal ppc_per_species * ncell.  Positions are wrapped into [0, n_d).  The
 * particle's index in these arrays is its identity for pic_get_particles.
 * Synchronises the stream.  Errors: PIC_ERR_ARG, PIC_ERR_HIP. */
pic_status pic_set_particles(pic_ctx *ctx, int32_t run, int32_t species, const double *x,
                             const double *u, int64_t n);

/* Downloads one species of one run in identity order (same layout as
 * pic_set_particles).  Synchronises the stream. */
pic_status pic_get_particles(pic_ctx *ctx, int32_t run, int32_t species, double *x, double *u,
                             int64_t n);

/* Uploads E and B (host double [3][ncell] each) of one run; either may be
 * NULL to leave it unchanged.  Synchronises the stream. */
pic_status pic_set_fields(pic_ctx *ctx, int32_t run, const double *E, const double *B);

/* Downloads E, B (as stored, widened to double) and the FP64 J of one run;
 * any pointer may be NULL.  Synchronises the stream. */
pic_status pic_get_fields(pic_ctx *ctx, int32_t run, double *E, double *B, double *J);

/* One step of the particle hot path for every run: re-sorts particles by
 * tile when a tile's particles have spread beyond its staging margin, then
 * gathers E^n, B^n with the WT (or MC) tensor, Boris-pushes u^{n-1/2} ->
 * u^{n+1/2}, moves x^n -> x^{n+1} and deposits J^{n+1/2} (Esirkepov) into
 * the zeroed global current.  Asynchronous on the context stream. */
pic_status pic_gather_push_deposit(pic_ctx *ctx);

/* Field update for every run: B^n -> B^{n+1/2} (Faraday, E^n),
 * E^n -> E^{n+1} (Ampere, J^{n+1/2}), B^{n+1/2} -> B^{n+1} (Faraday, E^{n+1});
 * zeroes J for the next step.  Asynchronous. */
pic_status pic_field_update(pic_ctx *ctx);

/* n_steps full steps (pic_gather_push_deposit + pic_field_update), replayed
 * from a captured HIP graph of the step sequence.  Asynchronous. */
pic_status pic_step(pic_ctx *ctx, int32_t n_steps);

/* n_steps full steps with the diagnostics of one run recorded every
 * diag_every steps (Sec. 4 follows the field energy over time): history[i]
 * receives pic_diagnostics after step (i + 1) * diag_every, for
 * i < n_steps / diag_every; host array of that many pic_diag, owned by the
 * caller.  Synchronises the stream at each record.  PIC_ERR_ARG if
 * diag_every < 1 or history is NULL; PIC_ERR_NUMERIC as pic_diagnostics
 * (the history up to that record is filled). */
pic_status pic_step_diag(pic_ctx *ctx, int32_t n_steps, int32_t diag_every, int32_t run, pic_diag *history);

/* FP64 device reductions for one run (energies, momentum, Gauss residual,
 * error counters), copied to *out.  Synchronises the stream.  Returns
 * PIC_ERR_NUMERIC if the error counters are nonzero (out is still filled). */
pic_status pic_diagnostics(pic_ctx *ctx, int32_t run, pic_diag *out);

/* Partially skipped calculation (Sec. 3, "Partially skipping calculation"):
 * the region perturbed at time t is the set of points closer than c t to the
 * initially perturbed region A0 (A0 itself at t = 0); outside it a particle
 * follows pure drift, so its gather, momentum update and current deposit are
 * skipped and it only moves with its unchanged momentum.  A0 is the closed
 * box lo[d] <= x_d / dx_d <= hi[d] (cell units, host arrays of 3 doubles,
 * entries past ndim ignored) repeated periodically; the distance is
 * Euclidean in physical units, to the nearest periodic image.  t0 is the
 * time of the next step (t of x^n for the next pic_gather_push_deposit), and
 * t advances by dt per step.  lo == NULL switches the skip off for the run.
 * Membership is decided in FP64 from the particle's position at the start of
 * the step.  Synchronises the stream.  PIC_ERR_ARG unless
 * 0 <= lo[d] <= hi[d] <= n[d] and t0 >= 0 (all finite). */
pic_status pic_set_skip_region(pic_ctx *ctx, int32_t run, const double *lo, const double *hi, double t0);

/* Tuning knobs (tile shape in cells, staging margin in cells, sort check
 * cadence in steps).  Any value <= 0 keeps the current choice (by default
 * the first of a measured list of tile shapes whose LDS fits half a CU: 2D
 * 32x16 in mixed precision, 16x16 in FP64; 3D 16x4x4 and 4x4x4).  Must be
 * called before the first step; returns PIC_ERR_STATE afterwards, and
 * PIC_ERR_ARG if the windows need more LDS than a workgroup can have
 * (160 KB), if margin <= sort_every, or if a tile has more than 4096 cells. */
pic_status pic_set_tiling(pic_ctx *ctx, const int32_t tile[3], int32_t margin, int32_t sort_every);

/* Autotuner of the tiling (the library's own: the paper has no tiling).  For
 * each candidate of a fixed list for the context's dimension and precision
 * (tile shape, staging margin, sort cadence; the first is the default
 * tiling), skipping those whose windows exceed the LDS, it takes untimed steps
 * (the candidate's first full sort and graph capture) and then times
 * trial_steps full steps, rounded up to a whole graph, with HIP events around
 * graph replays on the context stream; the fastest candidate is applied as
 * pic_set_tiling would, except that the default stays unless another is more
 * than 2% faster.  A trial that leaves particles out of range or non-finite
 * fails the call with PIC_ERR_NUMERIC.  The trial steps are then undone: the current
 * particle store, the fields, the current and the device counters are copied
 * to pageable host memory before the trials (about the size of one particle
 * store plus the grids) and back afterwards, so the next step starts from the
 * state the call found.  chosen (host, 5 int32, may be NULL) receives tile[0],
 * tile[1], tile[2], margin and sort_every; *best_ms (may be NULL) the chosen
 * candidate's milliseconds per step.  Synchronises the stream.  PIC_ERR_ARG
 * unless 1 <= trial_steps <= 4096; PIC_ERR_STATE after the first step or
 * before the particles of every run and species are set; a trial's failure is
 * returned after the state and the previous tiling are restored. */
pic_status pic_autotune(pic_ctx *ctx, int32_t trial_steps, int32_t chosen[5], double *best_ms);

/* The autotuner's candidate list for a dimension and precision (host only,
 * no context): *count receives the number of candidates, and out (host,
 * cap x 5 int32, may be NULL when cap is 0) the first min(cap, *count) of
 * them as tile[0], tile[1], tile[2], margin, sort_every (tile[2] = 1 in 2D),
 * in the order pic_autotune tries them; the first is the default tiling.
 * PIC_ERR_ARG for a NULL count, cap < 0, or ndim/precision out of range. */
pic_status pic_tiling_candidates(int32_t ndim, int32_t precision, int32_t *out, int32_t cap, int32_t *count);

/* Device timing of the gather-push-deposit kernel.  enable != 0 starts
 * recording a HIP event pair on the context stream around every
 * gather-push-deposit kernel launch: eager launches of
 * pic_gather_push_deposit, and in pic_step (which then takes its steps one
 * by one instead of replaying the step graph) a graph holding the particle
 * kernel alone, replayed once per step between the two events, with the
 * sort checks and the field update launched around it.  enable == 0 stops.
 * The events are created without the system-scope fence, so recording them
 * flushes no cache.  On return *avg_ms holds the average kernel time in
 * milliseconds and *launches the number of launches recorded since the
 * previous call, which resets the record.  Synchronises the stream. */
pic_status pic_kernel_timing(pic_ctx *ctx, int32_t enable, double *avg_ms, int64_t *launches);

/* Text of the last error on this context (or of the last failed
 * pic_init/pic_query_layout when ctx is NULL).  Never NULL. */
const char *pic_last_error(const pic_ctx *ctx);

/* Releases the host context and its graphs (not the caller's buffers). */
pic_status pic_destroy(pic_ctx *ctx);

/* ---- host-only helpers (no device work) ---------------------------------
 * The per-axis interpolation tables the kernels evaluate: for kind 0 the
 * B-spline W_l on the half-integer lattice, 1 W_l on the integer lattice,
 * 2 the WT factor T_l(.; a) on the integer lattice (Sec. 2, equations after
 * Eq. tau_l; any 0 < a < 1).  Evaluates the weights of the table's nodes for
 * a particle at in-cell offset f in [0,1) of cell 0: node_first receives the
 * lattice index of the first node, weights[0..*count-1] the weights.
 * Returns PIC_ERR_ARG for bad l, kind or a. */
pic_status pic_table_weights(int32_t l, int32_t kind, double a, double f, int32_t *node_first,
                             int32_t *count, double *weights);

#ifdef __cplusplus
}
#endif
#endif
