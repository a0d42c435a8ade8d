// Direct solver of the interface system C x = g (the weak flux and pressure
// continuity conditions (13)-(14) written in the multiscale basis).
//
// Every coarse row is owned by one subdomain (the flux rows of an edge by its
// left/lower subdomain, the pressure rows by its right/upper one), so every
// subdomain owns as many rows as it has dofs and C has the block five-point
// pattern of the subdomain grid.  A nested-dissection tree of line separators
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
};

// Factor C (CSR over rows x dofs) for the maps' subdomain grid.
CoarseFactor coarse_factor(const Maps& M, const std::vector<int>& rp, const std::vector<int>& ci,
                           const std::vector<double>& cv, int nthreads);
// Host reference of the level-scheduled solve (used to check the factor).
// g_nd: the scaled right-hand side in tree order
// (g_nd[t] = nd_scale[t] * g[nd_row[t]]).
void coarse_solve_host(const CoarseFactor& F, const double* g_nd, double* x);

}  // namespace mrcm
