// Direct solver of the interface system C x = g (the weak flux and pressure
// continuity conditions (13)-(14) written in the multiscale basis).
//
// Every coarse row is owned by one subdomain (the flux rows of an edge by its
// left/lower subdomain, the pressure rows by its right/upper one), so every
// subdomain owns as many rows as it has dofs and C has the block five-point
// pattern of the subdomain grid.  A nested-dissection tree of cross (and line) separators
// on that grid gives a multifrontal block elimination: every node eliminates
// the dofs of its separator F against the dofs U of the subdomains bordering
// its region, storing
//   [W; E] = [C_FF^-1; C_UF C_FF^-1]  ((nf + nu) x nf)   forward
//   G      =  C_FF^-1 C_FU            (nf x nu)          backward
// (C_** are the Schur-updated front blocks, C_FF^-1 from LU with partial
// pivoting).  The solve is then GEMVs only:
//   forward, leaves to root:  v = g_F - (contributions of descendants),
//                             y_F = W v, c_n = E v;
//   backward, root to leaves: x_F = y_F - G x_U.
#pragma once

#include <memory>
#include <utility>
#include <vector>

#include "internal.h"

namespace mrcm {

struct CoarseNode {
  int depth = 0;
  std::vector<int> frow, fcol, urow, ucol;
  std::vector<double> fwd;  // (nf + nu) x nf row-major
  std::vector<double> bwd;  // nf x nu row-major
  int yoff = 0, coff = 0;   // offsets of y_F and c_n in the solve buffers
};

struct CoarseFactor {
  int nc = 0, depth = 0, ylen = 0, clen = 0;
  std::vector<CoarseNode> nodes;  // post-order
  // Tree order: position t = yoff_n + a holds the a-th separator row of node
  // n.  nd_row[t] is that row; slots[t * maxp + u] (u < maxp) are the
  // contribution slots (in cbuf) to subtract from it, in a fixed order,
  // padded with -1.
  std::vector<int> nd_row;
  // Row equilibration: the factor is of diag(rscale) C; g_nd[t] must be
  // multiplied by nd_scale[t] = rscale[nd_row[t]].
  std::vector<double> rscale, nd_scale;
  int maxp = 4;
  std::vector<int> slots;
  double min_pivot_ratio = 1.0;
  // The rows of diag(rscale) C in tree order (CSR over the tree positions,
  // columns = coarse dofs), for the residual r_nd = g_nd - diag(rscale) C x
  // of the refinement steps.
  std::vector<int> nd_rp, nd_ci;
  std::vector<double> nd_v;
  // Refinement steps x += solve(r_nd) after the first solve (set by
  // coarse_refine_steps).
  int refine = 0;
};

// A chunk of one level of the interface solve: rows [row0, row1) of one
// node's forward ([W; E], (nf + nu) x nf) or backward (G, nf x nu) matrix,
// with the node's sizes and offsets copied in so that a workgroup needs one
// descriptor load: mat, the matrix offset; yoff, the node's first tree
// position (its y_F rows); coff, its first contribution row; fcol, ucol,
// offsets of its separator and border dof lists in the index array.
struct CChunk {
  int row0, row1, nf, nu;
  int yoff, coff, fcol, ucol;
  long long mat;
};

// The tables of the level-scheduled GPU solve of a factor, built on the host
// and uploaded as they are:
//   idx            separator and border dof lists of every node, concatenated;
//   fwd, bwd       the node matrices, concatenated (fwd_len, bwd_len words);
//   chunks         forward: 64 rows each for a matrix of at most 128
//                  columns, else 16; backward: 16; forward levels leaves
//                  first (fwd_levels:
//                  first chunk and count per level), then backward levels
//                  root first (bwd_levels); a node without border rows has
//                  no backward chunk;
//   gsrc           per tree position t: the two dofs of its row, its kind
//                  (0 flux, 1 pressure, 2 pinned) and 0;
//   cdest          per contribution row q: the slot u * np + t it adds to;
//   max_nf, max_nu the largest separator and border of a node.
struct CoarseTables {
  std::vector<int> idx;
  std::unique_ptr<double[]> fwd, bwd;
  long long fwd_len = 0, bwd_len = 0;
  std::vector<CChunk> chunks;
  std::vector<std::pair<int, int>> fwd_levels, bwd_levels;
  std::vector<std::array<int, 4>> gsrc;
  std::vector<int> cdest;
  int max_nf = 1, max_nu = 1;
};
// rowL, rowR, rowKind: per interface row, the dofs whose trace moments it
// combines and its kind; pin_row (or -1) takes kind 2.  Separators or borders
// above kMaxCoarseFront rows are rejected (MRCM_EINVAL): the solve holds a
// node's vector in LDS.
constexpr int kMaxCoarseFront = 6144;
CoarseTables coarse_tables(const CoarseFactor& F, const int32_t* rowL, const int32_t* rowR,
                           const int32_t* rowKind, int pin_row, int nthreads);

// Factor C (CSR over rows x dofs) for the maps' subdomain grid.
CoarseFactor coarse_factor(const Maps& M, const std::vector<int>& rp, const std::vector<int>& ci,
                           const std::vector<double>& cv, int nthreads);

// A node of a dissection tree over the subdomains: the subdomains whose rows
// and dofs it eliminates (fsub), those bordering its region (usub, sorted),
// its depth (root 0) and children.  Rows of a subdomain couple only to dofs of
// itself and its face neighbours, so a region's interior and the rest of the
// grid meet only through its border.
struct DissectionNode {
  std::vector<int> fsub, usub;
  int depth = 0;
  std::vector<int> children;
};

// Factor C for a given tree (post-order: children before their parent).
// rows_of[i] lists the coarse rows owned by subdomain i, as many as its dofs
// dof_offset[i] .. dof_offset[i + 1] - 1.  Any grid of subdomains (2-D or
// 3-D) with such a tree; coarse_factor builds the 2-D one.
CoarseFactor coarse_factor_tree(const std::vector<DissectionNode>& tree,
                                const std::vector<std::vector<int>>& rows_of,
                                const std::vector<int32_t>& dof_offset,
                                const std::vector<int>& rp, const std::vector<int>& ci,
                                const std::vector<double>& cv, int nthreads);
// Host reference of the level-scheduled solve (used to check the factor).
// g_nd: the scaled right-hand side in tree order
// (g_nd[t] = nd_scale[t] * g[nd_row[t]]).
// nthreads: host threads of the level loops (the arithmetic of every row is
// the same for any count).
void coarse_solve_host(const CoarseFactor& F, const double* g_nd, double* x, int nthreads = 1);
// r_nd = g_nd - diag(rscale) C x in tree order (FP64, fixed order).
void coarse_residual_host(const CoarseFactor& F, const double* g_nd, const double* x,
                          double* r_nd, int nthreads = 1);
// The solve the apply runs: the level-scheduled solve, then F.refine steps of
// x += solve(g_nd - diag(rscale) C x).
void coarse_solve_refined_host(const CoarseFactor& F, const double* g_nd, double* x,
                               int nthreads = 1);
// Refinement steps the apply needs: the explicit front inverses of the factor
// are not backward stable, so on ill-conditioned interface systems one solve
// can be off by far more than the conditioning allows, and each refinement
// step with an FP64 residual shrinks that error by about the same factor.  The
// step count is measured on a fixed pseudo-random right-hand side: the
// number of corrections applied before a correction falls to tol times the
// solution (in max norm), at most max_steps.  Sets and returns F.refine.
int coarse_refine_steps(CoarseFactor& F, double tol, int max_steps, int nthreads = 1);
// The library's choice: corrections down to 1e-10 of the solution in the
// FP64 mode, at most four steps.  In the modes with FP32 box factors the
// interface solve needs only to stay below the effect of the factors' own
// FP32 rounding on T (1e-7 to 1e-5 on the workloads, bounded by the
// recurrence length times 2^-24): corrections down to 1e-6.
constexpr double kCoarseRefineTol = 1e-10;
constexpr double kCoarseRefineTolMixed = 1e-6;
constexpr int kCoarseRefineMax = 4;
inline double coarse_refine_tol(int precision) {
  return precision == 0 ? kCoarseRefineTol : kCoarseRefineTolMixed;
}

}  // namespace mrcm
