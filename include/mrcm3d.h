/*
 * mrcm3d.h -- the MRCM-OS preconditioner and GMRES on 3-D Cartesian grids
 * (the paper's model problem with d = 3: Section 2, eqs. (1a)-(1d), posed on
 * d-dimensional Cartesian elements; Section 2.1 for the method; Section 3 and
 * Algorithm 1 for the preconditioned GMRES).
 *
 * Cubic cells, seven-point two-point-flux operator with harmonic-mean face
 * transmissibility (the system divided by h, so A does not depend on h);
 * box subdomains with six sides W, E (x), S, N (y), B, T (z); interfaces on
 * the faces shared by neighbouring subdomains; multiplier and test spaces of
 * tensor Legendre products P_a(xi) P_b(eta) per side, a and b below
 * min(degree + 1, faces in that direction); informed spaces from the
 * oversampled problems, multiscale basis functions as their restrictions,
 * the source-driven solution on the oversampled box; restricted additive
 * Schwarz smoothing; FP64 arithmetic throughout (the box factors optionally
 * stored in FP32: precision 2).  Vectors are FP64 device pointers of
 * nx ny nz values, cell (ix, iy, iz) at (iz ny + iy) nx + ix.
 *
 * Error codes and stats as in mrcm.h.  Limits: every oversampled box and
 * patch has at most 256 cells per z-plane (bx by <= 256) and 4096 cells, and
 * every separator of the interface solve (a plane of subdomains across the
 * longest axis of a region, halved recursively down to regions of at most
 * eight subdomains) and every border has at most 6144 interface rows;
 * larger configurations get MRCM_EINVAL.
 */
#ifndef MRCM3D_H
#define MRCM3D_H

#include <stddef.h>
#include <stdint.h>

#include "mrcm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[6]; /* W E S N B T: 1 Dirichlet, 0 no flow */
} mrcm3d_grid;

typedef struct {
  int32_t sx, sy, sz;     /* subdomain size in cells */
  int32_t oversample;     /* l: the oversampled box grows every side by l cells */
  double alpha;           /* beta = alpha L / K_H */
  int32_t beta_len;       /* 0: L = H = max(sx, sy, sz) cells, 1: L = h */
  int32_t smooth_sweeps;  /* k */
  int32_t smooth_overlap; /* delta */
  int32_t iface_degree;   /* d >= 0 */
  int32_t precision;      /* 0: FP64; 2: plane blocks of the box factors stored
                             in FP32 (rounded after the FP64 factorisation and
                             the set-up's own solves), FP64 arithmetic; 1 is not
                             offered in 3-D (MRCM_EINVAL) */
} mrcm3d_params;

typedef struct mrcm3d_ctx mrcm3d_ctx;

/* Set up T for the permeability K_dev (device, n values, finite and > 0):
 * the host computes the maps, the plane-block LDL^T factors of every
 * oversampled box and patch, the informed spaces, the multiscale basis
 * functions and the interface system, which it factors over a dissection of
 * the subdomain grid into planes (row-equilibrated block elimination with
 * partial pivoting in every separator, FP64, as the 2-D path), with the
 * number of FP64 refinement steps each interface solve runs set so that a
 * correction falls below 1e-10 of the solution in precision 0 and 1e-6 in
 * precision 2 (at most four), and uploads them.  The context owns all device
 * memory. */
int mrcm3d_setup(const mrcm3d_grid* grid, const mrcm3d_params* params, const double* K_dev,
                 void* stream, mrcm3d_ctx** out);

/* z = T r (Section 3: source r, homogeneous data, then the smoothing sweeps;
 * zero mean when no side has Dirichlet data).  r, z: device, may not alias. */
int mrcm3d_apply(mrcm3d_ctx* ctx, const double* r, double* z, void* stream);

/* y = A x (the seven-point operator).  x, y: device, may not alias. */
int mrcm3d_op_apply(mrcm3d_ctx* ctx, const double* x, double* y, void* stream);

/* Right-hand side of the fine system (Section 3, d = 3): b = f h^2 plus
 * 2 K_c g on every Dirichlet boundary face.  f_cell: device n values or NULL
 * (zero source); g_bc: device, the Dirichlet face values of the six sides
 * concatenated in the order W, E (ny nz values each, face (y, z) at
 * z ny + y), S, N (nx nz each, z nx + x), B, T (nx ny each, y nx + x), or
 * NULL; entries of no-flow sides are ignored; h: cell size (> 0); b: device
 * n values. */
int mrcm3d_rhs(mrcm3d_ctx* ctx, const double* f_cell, const double* g_bc, double h, double* b,
               void* stream);

/* Right-preconditioned restarted GMRES (Algorithm 1, as gmres_solve: p_0 = 0,
 * modified Gram-Schmidt, estimated residual tested after every step, true
 * FP64 residual at every cycle end).  One right-hand side b (device); p
 * (device) receives the solution.  st: host, may be NULL (no histories).
 * MRCM_ENOCONV when maxit is reached (p and st written). */
int mrcm3d_gmres_solve(mrcm3d_ctx* ctx, const double* b, double* p, double rtol,
                       int32_t restart, int32_t maxit, mrcm_stats* st, void* stream);

/* Per-phase device time of the applications since the last enable (HIP
 * events on the context's stream): ms[6] and counts[6] for local,
 * interface, reconstruct, residual, patch, finalize. */
int mrcm3d_timing_enable(mrcm3d_ctx* ctx, int32_t on);
int mrcm3d_timing_read(mrcm3d_ctx* ctx, double* ms, int64_t* counts);

/* Queries: 0 set-up seconds, 1 device bytes, 2 interface unknowns, 3 bytes
 * one application reads from the box factors (local and patch, each read
 * twice), 4 bytes one interface solve reads and writes (its factor matrices
 * once per sweep and the refinement residuals), 5 refinement steps of every
 * interface solve, 6 level launches of one sweep of the interface solve.
 * MRCM_EINVAL for another code. */
int mrcm3d_query(mrcm3d_ctx* ctx, int32_t what, double* value);

/* Release a context (NULL is ignored). */
void mrcm3d_destroy(mrcm3d_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MRCM3D_H */
