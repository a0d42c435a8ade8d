// Host-side FP64 set-up of T on 3-D grids (include/mrcm3d.h): maps, face
// transmissibilities, plane-block LDL^T factors of the oversampled boxes and
// patches, multiscale basis functions, the interface system with its
// nested-dissection factor, and the tables the device apply reads.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "../../include/mrcm3d.h"
#include "coarse.h"
#include "internal.h"

namespace mrcm3d {

using mrcm::Error;

// A cell box, half-open per axis (x, y, z).
struct Box {
  int lo[3], hi[3];
  int n(int a) const { return hi[a] - lo[a]; }
  long long cells() const { return (long long)n(0) * n(1) * n(2); }
  int plane() const { return n(0) * n(1); }
};

// Block LDL^T of a box matrix by z-planes: D_j^-1 (P x P, symmetric, P =
// cells of a plane, x fastest) for every plane j, and the z-couplings T_j
// (P values: the transmissibility between plane j - 1 and plane j at each
// cell; plane 0's are unused).  pin: the box covers an all-no-flow domain and
// its first cell is fixed.  D_j^-1 is stored by its cyclic diagonals 0 ..
// H - 1 (H = P / 2 + 1): word d P + t holds D(t, (t + d) mod P), which holds
// every entry of a symmetric matrix once (twice on diagonal P / 2 when P is
// even); plane_dot reads it back.
struct PlaneFactor {
  int P = 0, bz = 0, pin = 0;
  std::vector<double> dinv;  // bz x H x P
  std::vector<double> coup;  // bz x P
  std::vector<double> full;  // bz x P x P, row-major: kept only while the set-up
                             // solves with the box (box_solve_full)
};
inline int half_rows(int P) { return P / 2 + 1; }
// sum_c D(t, c) v[c] of a block in cyclic-diagonal storage: diagonal 0, then
// for d = 1 .. H - 1 the term D(t, t + d) v[t + d] (read at d P + t) and,
// unless 2 d = P, D(t - d, t) v[t - d] (read at d P + t - d), indices mod P;
// the terms of odd and even d in separate sums, added last as
// (even up + odd up) + (even down + odd down).
double plane_dot(const double* D, const double* v, int P, int t);

// The faces of one side of Omega_i with the data of the trace moments: the
// inside and outside cell (global), and the four weights of U = w0 p_in +
// w1 p_out and pi = w2 p_in + w3 p_out of a solution with zero Robin data
// (interior faces of the oversampled box for l > 0, Robin faces for l = 0).
struct SideData {
  int side = 0, n0 = 0, n1 = 0;
  std::vector<long long> in, out;
  std::vector<double> t, rho, b, Kin, Kout;
  std::vector<std::array<double, 4>> w;
};

struct Setup {
  int nx = 0, ny = 0, nz = 0, bc[6] = {0, 0, 0, 0, 0, 0};
  int sx = 0, sy = 0, sz = 0, oversample = 0, sweeps = 0, overlap = 0, degree = 1;
  int precision = 0;  // 0 FP64, 2 FP32-stored plane blocks
  double alpha = 0.0, Lcells = 1.0;
  bool noflow = false;
  long long n = 0;
  std::vector<double> K, tx, ty, tz;  // tx (nz, ny, nx + 1), ty (nz, ny + 1, nx), tz (nz + 1, ny, nx)
  int m = 0, mdims[3] = {0, 0, 0};
  std::vector<Box> boxes, oboxes, pboxes;
  std::vector<int32_t> owner;
  std::vector<std::vector<int>> sides;     // interior sides per subdomain, W E S N B T order
  std::vector<std::vector<SideData>> gam;  // per subdomain, per interior side
  std::vector<std::array<int, 3>> faces;   // interfaces: lower subdomain, upper, axis
  std::vector<std::array<int, 5>> dofs;    // subdomain, side, q, a, b
  std::vector<int32_t> dof_off;            // m + 1
  std::vector<int32_t> row_off;            // interfaces + 1
  std::vector<int32_t> rowL, rowR, rowKind;  // per interface row: dofs combined, 0 flux / 1 pressure / 2 pinned
  int nc = 0, pin_row = -1;
  std::vector<PlaneFactor> over, patch;
  std::vector<std::vector<double>> mbf;    // per subdomain: Ni x cells of Omega_i, basis-major
  std::vector<int> Crp, Cci;               // the interface matrix C in CSR (columns ascending)
  std::vector<double> Cv;
  mrcm::CoarseFactor CF;                   // its factor over a dissection of the subdomain grid
};

// Dissection tree of an mx x my x mz subdomain grid (post-order): a region of
// more than eight subdomains is split across its longest axis by the plane of
// subdomains at its middle, which becomes the node's separator; smaller
// regions are eliminated whole.
std::vector<mrcm::DissectionNode> dissection3(int mx, int my, int mz);

long long cell_of(const Setup& S, int x, int y, int z);
void host_setup(Setup& S, const mrcm3d_grid& g, const mrcm3d_params& p, const double* K);
void box_solve(const PlaneFactor& F, double* x);
// The same solve from the full blocks (contiguous row products), for the
// set-up's own solves; needs F.full.
void box_solve_full(const PlaneFactor& F, double* x);
void host_op_apply(const Setup& S, const double* x, double* y);
void host_apply(const Setup& S, const double* r, double* z);
// Legendre P_q at the face-centre parameter of face j of n.
double legendre_face(int q, int j, int n);

}  // namespace mrcm3d
