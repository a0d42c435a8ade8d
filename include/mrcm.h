/*
 * mrcm.h -- C ABI of the MI355X (gfx950) library for GMRES with the
 * matrix-free MRCM-OS right preconditioner on 2-D Darcy pressure problems.
 *
 * Problem (Section 2, eqs. (1a)-(1d)): u = -K grad p, div u = f on a
 * rectangle covered by nx x ny square cells; each side is either no-flow or
 * Dirichlet.  The fine system A p = b (Section 3) is the lowest-order
 * Raviart-Thomas discretisation with vertex-quadrature mass lumping,
 * condensed to the cell-centred five-point stencil with harmonic-mean face
 * permeability.  T (Section 3, the modified MRCM-O with source r and
 * homogeneous boundary data) is the MRCM-OS operator of Section 2.1:
 * Robin local solves on the non-overlapping subdomains, informed multiplier
 * spaces from oversampled problems, weak flux / pressure continuity (eqs.
 * (13)-(14)) through a small interface system, then overlapping-Schwarz
 * smoothing sweeps.  gmres_solve is the right-preconditioned restarted GMRES
 * of Algorithm 1.
 *
 * Conventions shared by every entry point:
 *  - cell (ix, iy) has id iy * nx + ix (x fastest); cell (0,0) touches the
 *    corner x = 0, y = 0;
 *  - every vector argument is float64; a multi-RHS vector is nrhs
 *    consecutive vectors of length nx * ny ([nrhs][n]);
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller;
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream); all
 *    device work of a call is ordered on it;
 *  - a context is not thread-safe; distinct contexts may be used
 *    concurrently from different threads and streams;
 *  - every function returning int returns 0 on success or a negative MRCM_E*
 *    code; the message of the last failure of the calling thread is returned
 *    by mrcm_last_error().  No C++ exception crosses this interface.
 */
#ifndef MRCM_H
#define MRCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MRCM_OK = 0,
  MRCM_EINVAL = -1,    /* bad sizes or parameters, K not finite or not > 0 */
  MRCM_ENOMEM = -2,    /* host or device allocation failed */
  MRCM_ESINGULAR = -3, /* non-positive pivot in a local factorisation, or a
                          zero pivot in the interface system */
  MRCM_ENOCONV = -4,   /* gmres_solve reached maxit; p and stats are written */
  MRCM_EDEVICE = -5    /* a HIP runtime call failed */
};

/* Fine grid.  bc[side] for side W (x = 0), E, S (y = 0), N:
 * 0 = no-flow (u.n = 0), 1 = Dirichlet (p = g).  With no-flow on all four
 * sides A is singular (constants) and every result is projected to zero
 * mean. */
typedef struct {
  int32_t nx, ny;
  int32_t bc[4];
} mrcm_grid;

/* Method parameters (Section 2.1 and Section 4, Table 1).
 *  sx, sy          subdomain size in cells (last column/row narrower when it
 *                  does not divide the grid);
 *  oversample      l: hat-Omega_i = Omega_i grown by l cells, clipped; must not
 *                  reach the domain boundary across an interior side;
 *  alpha           Robin parameter, beta = alpha * L / K_H (Section 2.1);
 *  beta_len        0: L = H = max(sx, sy) cells; 1: L = h (one cell);
 *  smooth_sweeps   k smoothing sweeps (restricted additive Schwarz);
 *  smooth_overlap  delta: smoothing patch = Omega_i grown by delta, clipped;
 *  iface_degree    d >= 0: Legendre P_0..P_d per interface side;
 *  precision       0: FP64 preconditioner apply;
 *                  1: local and smoothing solves applied in FP32 (factors
 *                  computed in FP64, stored and applied in FP32, FP32
 *                  accumulation);
 *                  2: factors stored in FP32 (half the bytes), applied with
 *                  FP64 arithmetic and FP64 work vectors;
 *                  the interface solve and GMRES are FP64 in every mode. */
typedef struct {
  int32_t sx, sy;
  int32_t oversample;
  double alpha;
  int32_t beta_len;
  int32_t smooth_sweeps;
  int32_t smooth_overlap;
  int32_t iface_degree;
  int32_t precision;
} mrcm_params;

/* GMRES statistics, host memory owned by the caller.  est_hist / true_hist
 * may be NULL; otherwise they hold hist_cap doubles each. */
typedef struct {
  int32_t iterations;   /* inner steps = applications of T (all RHS summed) */
  int32_t cycles;       /* restart cycles started (all RHS summed) */
  int32_t converged;    /* 1 when every RHS met the tolerance */
  int32_t hist_cap;     /* in: capacity of the history arrays */
  int32_t hist_len;     /* out: entries written to est_hist (first RHS) */
  int32_t true_len;     /* out: entries written to true_hist (first RHS) */
  double final_relres;  /* max over RHS of the true ||b - A p|| / ||b|| */
  double* est_hist;     /* estimated relative residual after each inner step */
  double* true_hist;    /* true relative residual at the start and end of each cycle */
} mrcm_stats;

typedef struct mrcm_ctx mrcm_ctx;

/* Index-map sizes for (grid, params): m subdomains, E interior edges and nc
 * coarse dofs (= coarse rows).  Host only; no device is touched. */
int mrcm_map_sizes(const mrcm_grid* grid, const mrcm_params* params,
                   int64_t* m, int64_t* n_edges, int64_t* nc);

/* Decomposition maps (Section 2.1: Omega_i, Gamma_i, hat-Omega_i, and the
 * smoothing patches), written to caller-owned host arrays:
 *  owner[n]           subdomain id of every cell;
 *  boxes[4m]          (x0, x1, y0, y1) of Omega_i, half-open;
 *  oboxes[4m]         hat-Omega_i; pboxes[4m] smoothing patches;
 *  edges[5E]          (L, R, orientation 0 vertical / 1 horizontal, start, length);
 *  dof_table[3nc]     (subdomain, side W0 E1 S2 N3, q) of every coarse dof;
 *  dof_offset[m+1]    first coarse dof of every subdomain;
 *  row_table[3nc]     (edge, 0 flux / 1 pressure, q) of every coarse row.
 * Host only; any pointer may be NULL to skip that map. */
int mrcm_maps(const mrcm_grid* grid, const mrcm_params* params, int32_t* owner,
              int32_t* boxes, int32_t* oboxes, int32_t* pboxes, int32_t* edges,
              int32_t* dof_table, int32_t* dof_offset, int32_t* row_table);

/* Set up T for one permeability field (Section 2.1, steps one to three of
 * the MRCM-OS algorithm: decomposition, multiplier spaces from the
 * oversampled problems, multiscale basis functions and the interface system;
 * plus the smoothing-patch factorisations).  K_dev: device, n float64 cell
 * permeabilities (read once; the context keeps no reference).  Factorisations
 * are computed in FP64 and kept resident in device memory owned by the
 * context.  On success *out receives the new context. */
int mrcm_setup(const mrcm_grid* grid, const mrcm_params* params, const double* K_dev,
               void* stream, mrcm_ctx** out);

/* z = T r for nrhs vectors (Section 3: source r, homogeneous boundary data,
 * then the smoothing sweeps).  r, z: device [nrhs][n]; may not alias. */
int mrcm_apply(mrcm_ctx* ctx, const double* r, double* z, int32_t nrhs, void* stream);

/* z = T r for nrhs vectors, as mrcm_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  This call allocates nothing: its work
 * space (two cell vectors and the interface-solve vectors of one column) is
 * a static array of the library, 256 MiB per device, held from the first
 * call on a device until the process ends; a context whose work space does
 * not fit (more than about 16 M cells in FP64 work vectors) is rejected with
 * MRCM_EINVAL.  The columns run one after the other with the one-column
 * kernels, so z equals mrcm_apply's one-column result bit for bit.  Every
 * call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (other streams or threads) race
 * and must be ordered by the caller.  Per-phase timing is not recorded. */
int mrcm_apply_noalloc(mrcm_ctx* ctx, const double* r, double* z, int32_t nrhs, void* stream);

/* z_i = T_i r_i for n set-up contexts at once (Section 3, as mrcm_apply,
 * for several permeability fields or grids).  Every column of every context
 * is one work item, and each phase of T (local solves, every level of the
 * interface solve, reconstruction, each smoothing sweep, the projection) is
 * one launch over the (column, subdomain) items of all of them, for contexts
 * of one family (precision mode and box column widths; families run one
 * after the other).  ctx[i], r[i], z[i], nrhs[i]: host arrays of n entries;
 * r[i], z[i]: device [nrhs[i]][n_i] of context i; a context may appear once
 * per call (MRCM_EINVAL otherwise).  Runs on `stream`.  Column k of a
 * context uses that context's k-th column work space (allocated on first
 * use and kept until mrcm_destroy); the launch tables live with the first
 * context of the call, and a call waits on the host until the launches of
 * the previous call led by the same context have read them.  Calls that
 * share a context must not overlap.  Results are those of mrcm_apply, bit
 * for bit.  Per-phase timing is not recorded. */
int mrcm_apply_many(mrcm_ctx* const* ctx, int32_t n, const double* const* r, double* const* z,
                    const int32_t* nrhs, void* stream);

/* Device allocator for the contexts (2-D, and 3-D of mrcm3d.h) set up after
 * this call (not part of the
 * method: memory plumbing, so that a caller such as a framework's caching
 * allocator owns the device memory).  alloc(bytes, stream) returns device
 * memory of at least `bytes` bytes, 256-byte aligned, or NULL (mrcm_setup
 * then fails with MRCM_ENOMEM); release(ptr, stream) returns it.  `stream`
 * is the stream the context was set up on.  A context frees its memory in
 * mrcm_destroy with the pair it was created with, after draining its own
 * stream and its setup stream.  Passing NULL for either restores
 * hipMalloc / hipFree.  Process-wide; safe to call from any thread. */
typedef void* (*mrcm_alloc_fn)(size_t bytes, void* stream);
typedef void (*mrcm_free_fn)(void* ptr, void* stream);
void mrcm_set_allocator(mrcm_alloc_fn alloc, mrcm_free_fn release);

/* y = A x for nrhs vectors (Section 3, the condensed fine operator).
 * x, y: device [nrhs][n]; may not alias. */
int op_apply(mrcm_ctx* ctx, const double* x, double* y, int32_t nrhs, void* stream);

/* Solve A p = b with right-preconditioned restarted GMRES (Algorithm 1):
 * p_0 = 0, Krylov dimension `restart`, modified Gram-Schmidt, stored z_j.
 * Stops an inner cycle when the estimated residual is <= rtol * ||b|| (tested
 * after every step) and finishes when the true FP64 residual ||b - A p|| is
 * <= rtol * ||b||.  maxit bounds the number of applications of T per RHS.
 * b, p: device [nrhs][n]; st: host, may be NULL.  Returns MRCM_ENOCONV
 * (p and st written) when maxit is reached.
 * Up to lanes x width right-hand sides (mrcm_set_lanes, mrcm_set_batch) are
 * solved at once, each with its own Krylov space, ordered after the work
 * `stream` holds; the device work of all of them has finished when the call
 * returns.  Each right-hand side runs the same arithmetic in the same order
 * whatever the lanes and width, so p is identical bit for bit to the
 * one-at-a-time result.  st->iterations and st->cycles sum over the right-hand
 * sides, st->final_relres is the largest, the histories are those of the
 * first. */
int gmres_solve(mrcm_ctx* ctx, const double* b, double* p, int32_t nrhs, double rtol,
                int32_t restart, int32_t maxit, mrcm_stats* st, void* stream);

/* Batched GMRES over several contexts (Algorithm 1 for every right-hand
 * side of every member; continuous batching): right-hand sides of any
 * number of set-up contexts, added and removed at any time, advance together
 * in ticks.  A tick consumes the scalars fetched by the previous tick (norms
 * and Hessenberg columns), advances every right-hand side on the host as
 * gmres_solve does, runs the Arnoldi steps of all stepping right-hand sides
 * as one launch per phase of T and of the Arnoldi tail over all of them (as
 * mrcm_apply_many), and copies the scalars the host needs next in one
 * transfer.  Each right-hand side runs gmres_solve's kernels in the same
 * order, so its iterates equal gmres_solve's bit for bit (p_0 = 0, modified
 * Gram-Schmidt, the estimated residual tested after every step, the true
 * FP64 residual at every cycle end).  The batch has its own stream; calls
 * on one batch must come from one thread at a time. */
typedef struct mrcm_batch mrcm_batch;
/* A batch with Krylov dimension `restart` (1..200). */
int gmres_batch_create(int32_t restart, mrcm_batch** out);
/* Add the nrhs right-hand sides b of a context (device [nrhs][n]); their
 * solutions are written to p (device [nrhs][n]) as they progress.  b, the
 * context and p are used after the work `stream` holds when the call is
 * made.  Each right-hand side's Krylov space and work space come from the
 * context: buffers of the context's removed tags with the same restart
 * length are reused, others are allocated (all released by mrcm_destroy).
 * The context must outlive the tag.  *tag receives the handle of the group. */
int gmres_batch_add(mrcm_batch* batch, mrcm_ctx* ctx, const double* b, double* p,
                    int32_t nrhs, double rtol, int32_t maxit, void* stream, int32_t* tag);
/* One tick; *active receives the right-hand sides not yet finished. */
int gmres_batch_tick(mrcm_batch* batch, int32_t* active);
/* *done = 1 when every right-hand side of the tag has finished (converged
 * or maxit reached); p is then final.  st (host, may be NULL) receives the
 * sums of iterations and cycles over the tag, converged, and the largest
 * true relative residual; no histories. */
int gmres_batch_poll(mrcm_batch* batch, int32_t tag, int32_t* done, mrcm_stats* st);
/* Drop a tag's right-hand sides (finished or not) after the batch's device
 * work has ended; p keeps what was written. */
int gmres_batch_remove(mrcm_batch* batch, int32_t tag);
/* Drain and free the batch (its tags' contexts are not touched). */
void gmres_batch_destroy(mrcm_batch* batch);
/* Lanes (streams) gmres_solve may use at once on this context (1..64; 4
 * after mrcm_setup).  Lanes beyond the first are created, with their
 * streams and device work space, by the first solve that uses them and kept
 * until mrcm_destroy.  While mrcm_timing_enable is on, solves use one lane. */
int mrcm_set_lanes(mrcm_ctx* ctx, int32_t lanes);

/* Right-hand sides one lane of gmres_solve advances together (1..8; 4 after
 * mrcm_setup): each step applies T to all of them in one multi-column
 * application (as mrcm_apply with nrhs > 1), so up to lanes x width
 * right-hand sides are in flight.  Results do not depend on it. */
int mrcm_set_batch(mrcm_ctx* ctx, int32_t width);

/* Host threads the calling thread's later mrcm_setup calls use for the
 * host part of the set-up (0: OpenMP's default, all of them).  A server that
 * sets up several contexts at once on different threads gives each a share
 * of the cores instead of letting every set-up spread over all of them. */
int mrcm_set_host_threads(int32_t threads);

/* Right-hand side of the fine system (Section 3): b = f h^2 plus 2 K_c g on
 * every Dirichlet boundary face.  f_cell: device n values or NULL (zero
 * source); g_bc: device, the Dirichlet values of the W, E, S, N sides
 * concatenated (ny, ny, nx, nx values, each in increasing coordinate; entries
 * of no-flow sides are ignored) or NULL; h: cell size; b: device n. */
int mrcm_rhs(mrcm_ctx* ctx, const double* f_cell, const double* g_bc, double h, double* b,
             void* stream);

/* Device bytes a context for (grid, params) keeps resident, plus the work
 * space of nrhs right-hand sides in flight in gmres_solve with restart 10
 * (one lane each; admission control). */
size_t mrcm_footprint(const mrcm_grid* grid, const mrcm_params* params, int32_t nrhs);

/* Per-phase device timing of the preconditioner apply (Section 2.1, the
 * steps of one MRCM-OS application), measured with HIP events recorded on the
 * stream of each call.  on = 1 starts (and clears) the accumulation, 0 stops
 * it.  Phases: 0 local Robin solves with trace moments, 1 interface
 * right-hand side and interface solve, 2 multiscale reconstruction,
 * 3 smoothing residual, 4 smoothing patch solves, 5 output (and zero-mean
 * projection). */
int mrcm_timing_enable(mrcm_ctx* ctx, int32_t on);

/* Accumulated device milliseconds and event-pair counts of every phase since
 * mrcm_timing_enable(ctx, 1): ms[6], counts[6], host.  Waits for the recorded
 * events. */
int mrcm_timing_read(mrcm_ctx* ctx, double* ms, int64_t* counts);

/* Scalar facts about a set-up context, by `what`:
 *  MRCM_Q_SETUP_SECONDS   wall time of mrcm_setup;
 *  MRCM_Q_DEVICE_BYTES    device memory the context holds;
 *  MRCM_Q_COARSE_PIVOT    smallest |pivot| / max|row| met while factorising the
 *                         row-equilibrated interface system (its conditioning);
 *  MRCM_Q_COARSE_LEVELS   levels of the nested-dissection interface solve;
 *  MRCM_Q_COARSE_DOFS     interface unknowns nc;
 *  MRCM_Q_COARSE_BYTES    bytes one interface solve reads and writes: the
 *                         forward and backward matrices of every tree node
 *                         once per sweep (the first solve and every
 *                         refinement step), plus each refinement residual's
 *                         matrix rows and vectors;
 *  MRCM_Q_COARSE_LAUNCHES kernel launches of one interface solve (its levels,
 *                         forward and backward, per sweep, and two per
 *                         refinement step);
 *  MRCM_Q_TUNE_MS         milliseconds mrcm_setup spent timing workgroup shapes
 *                         of the one-column launches.  The timing runs only
 *                         with MRCM_TUNE=1 in the environment, once per shape
 *                         and process (0 otherwise: the defaults are kept);
 *                         with MRCM_TUNE=alt every choice takes its last
 *                         option, untimed and uncached;
 *  MRCM_Q_TUNE_CHANGES    workgroup shapes the set-up timing changed from the
 *                         defaults (interface levels, local and patch solves).
 *                         Every shape gives the same results bit for bit;
 *  MRCM_Q_COARSE_REFINE   refinement steps every interface solve runs after
 *                         the first (x += C^-1 (g - C x) with an FP64
 *                         residual): the set-up measures how far one solve
 *                         with the factor misses on a fixed right-hand side
 *                         and takes steps until a correction is below 1e-10
 *                         of the solution in precision mode 0, 1e-6 in modes
 *                         1 and 2 (at most four);
 *  MRCM_Q_MFMA_RECON      1 when the reconstruction of 8-column applications
 *                         runs on the matrix cores in the arithmetic type, 2
 *                         with BF16 inputs and FP32 accumulation, 0 with the
 *                         vector FMA kernel (the default).  Set at mrcm_setup
 *                         from MRCM_MFMA_RECON=mfma|bf16 in the environment
 *                         (interface degree <= 1; bf16 needs precision mode
 *                         1, else mfma is used); its sums round differently,
 *                         so 8-column results then differ from one-column
 *                         results in rounding;
 *  MRCM_Q_SETUP_HOST_S    seconds of mrcm_setup in the host preparation
 *                         (maps, transmissibilities, face weights, work
 *                         lists);
 *  MRCM_Q_SETUP_DEVICE_S  seconds in the device set-up (box factors,
 *                         oversampled solves, MBFs and their moments), until
 *                         its results are back on the host;
 *  MRCM_Q_SETUP_COARSE_S  seconds in the interface system's assembly,
 *                         factorisation and refinement count (host). */
enum {
  MRCM_Q_SETUP_SECONDS = 0,
  MRCM_Q_DEVICE_BYTES = 1,
  MRCM_Q_COARSE_PIVOT = 2,
  MRCM_Q_COARSE_LEVELS = 3,
  MRCM_Q_COARSE_DOFS = 4,
  MRCM_Q_COARSE_BYTES = 5,
  MRCM_Q_COARSE_LAUNCHES = 6,
  MRCM_Q_TUNE_MS = 7,
  MRCM_Q_TUNE_CHANGES = 8,
  MRCM_Q_COARSE_REFINE = 9,
  MRCM_Q_MFMA_RECON = 10,
  MRCM_Q_SETUP_HOST_S = 11,
  MRCM_Q_SETUP_DEVICE_S = 12,
  MRCM_Q_SETUP_COARSE_S = 13
};
int mrcm_query(mrcm_ctx* ctx, int32_t what, double* value);

/* Release a context and all device memory it owns (NULL is ignored). */
void mrcm_destroy(mrcm_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* mrcm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MRCM_H */
