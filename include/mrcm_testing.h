/*
 * mrcm_testing.h -- test hooks of the host-side FP64 setup.
 *
 * For the test suite only (callers that check the setup arithmetic on a
 * machine without a GPU).  These functions are not a solver path: no entry
 * point of mrcm.h calls them, and they take and return host memory only.
 * Each call runs the whole FP64 setup again.  Error behaviour as in mrcm.h.
 */
#ifndef MRCM_TESTING_H
#define MRCM_TESTING_H

#include <stdint.h>

#include "mrcm.h"
#include "mrcm3d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Sizes of the interface system for (grid, params, K): nc and nnz of C. */
int mrcm_test_coarse_sizes(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                           int64_t* nc, int64_t* nnz);

/* The interface matrix C in CSR (rows x coarse dofs, row replacement for
 * all-no-flow grids applied): rp[nc+1], ci[nnz], cv[nnz], host. */
int mrcm_test_coarse_matrix(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                            int32_t* rp, int32_t* ci, double* cv);

/* z = T r evaluated on the host from the exact data layout that mrcm_setup
 * uploads (box factors, trace-moment weights, nested-dissection coarse
 * factor, multiscale basis functions, patch factors).  r, z: host, n values.
 * Also returns the smallest pivot ratio of the coarse factorisation. */
int mrcm_test_host_apply(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                         const double* r, double* z, double* min_pivot_ratio);

/* x = C^-1 g with the interface factorisation mrcm_setup uploads (row
 * equilibration and nested-dissection block LU) and the refinement steps the
 * apply runs after it, evaluated on the host.  g, x: host, nc values each (coarse
 * row order in, coarse dof order out). */
int mrcm_test_coarse_solve(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                           const double* g, double* x);

/* Failure injection for MRCM_ESINGULAR: validate K as
 * mrcm_setup does, then set K = 0 on one cell and factor every local and
 * patch box on the host (Section 2.1, the local problems).  A cell with
 * K = 0 has no conductance on any face, so its box matrix has a zero row and
 * the block LDL^T meets a zero pivot: MRCM_ESINGULAR.  Returns MRCM_OK when
 * every factorisation succeeds, MRCM_EINVAL for a bad cell index. */
int mrcm_test_zero_cell_setup(const mrcm_grid* grid, const mrcm_params* params,
                              const double* K, int64_t cell);

/* z = T r on a 3-D grid (include/mrcm3d.h) evaluated on the host from the
 * tables mrcm3d_setup uploads, in the order the device applies them (plane-
 * block local solves, trace moments, the interface solve through the
 * dissection factor with its refinement steps, reconstruction, smoothing,
 * projection).  K, r, z: host, n values; *nc (may be NULL) receives the
 * interface unknowns. */
int mrcm3d_test_host_apply(const mrcm3d_grid* grid, const mrcm3d_params* params,
                           const double* K, const double* r, double* z, int64_t* nc);

/* The dissection tree of the 3-D interface solve on an mx x my x mz grid of
 * subdomains (subdomain (I, J, L) at (L my + J) mx + I), nodes in post-order:
 * elim[s] the node that eliminates subdomain s (m values); parent[t] (-1 for
 * the root) and depth[t] per node; the border of node t in
 * border[border_ptr[t] .. border_ptr[t + 1]) (sorted).  Capacities: max_nodes
 * nodes (parent, depth: max_nodes; border_ptr: max_nodes + 1) and max_border
 * border entries; *nodes receives the node count.  MRCM_EINVAL when a
 * capacity is too small. */
int mrcm3d_test_dissection(int32_t mx, int32_t my, int32_t mz, int32_t* elim, int32_t* parent,
                           int32_t* depth, int32_t* border_ptr, int32_t* border,
                           int32_t max_nodes, int32_t max_border, int32_t* nodes);

#ifdef __cplusplus
}
#endif

#endif /* MRCM_TESTING_H */
