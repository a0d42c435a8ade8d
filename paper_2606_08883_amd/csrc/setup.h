// Host-side FP64 setup of the MRCM-OS operator.
#pragma once

#include <vector>

#include "internal.h"
#include "setup_jobs.h"

namespace mrcm {

// Block LDL^T factor of the five-point matrix of one cell box, with cell rows
// (fixed y) as blocks: D_0 = A_0, D_j = A_j - T_j D_{j-1}^{-1} T_j, where A_j is
// the tridiagonal matrix of row j and T_j = diag(transmissibilities between
// rows j-1 and j).  Stored: D_j^{-1} (dense, symmetric, bx*bx per row) and the
// couplings T_j (bx per row, T_0 = 0).  A solve is
//   forward  u_j = D_j^{-1} (b_j + T_j u_{j-1}),
//   backward x_j = u_j + D_j^{-1} (T_{j+1} x_{j+1}).
// pin = 1 marks a singular box (no Robin and no Dirichlet face): its first cell
// is fixed to zero (row and column replaced by the unit row, rhs[0] = 0).
struct BoxFactor {
  Box box{};
  int pin = 0;
  std::vector<double> dinv;  // by * bx * bx
  std::vector<double> coup;  // by * bx
};

struct CoarseFactor;  // coarse.h

struct HostSetup {
  Maps maps;
  int nx = 0, ny = 0;
  int bc[4] = {0, 0, 0, 0};
  bool noflow = false;
  double alpha = 0.0, Lcells = 1.0;
  int sweeps = 0;
  std::vector<double> K, tx, ty;  // tx: ny*(nx+1) [row-major by y], ty: (ny+1)*nx
  std::vector<BoxFactor> local, patch;
  std::vector<std::vector<double>> mbf;  // per subdomain: N_i columns of bx*by
  // Coarse right-hand-side weights per coarse dof k = (i, side, q), over the
  // faces of that side: wU = rho_f P_q(xi_j), wP = b_f rho_f P_q(xi_j).
  std::vector<int> wOff;  // nc + 1
  std::vector<double> wU, wP;
  // Coarse rows: the two dofs (L side, R side) each row combines, and kind.
  std::vector<int> rowL, rowR, rowKind;
  int pin_row = -1, pin_dof = -1;
  // Coarse matrix in CSR (rows x dofs).
  std::vector<int> Crp, Cci;
  std::vector<double> Cv;
};

// Work lists of the set-up on the device (built on the host from the maps,
// transmissibilities and K; O(perimeter) per subdomain).  Offsets: FP64 work
// buffer `buf` (factors and couplings of subdomain and oversampled boxes,
// scratch vectors, phi), storage-type factor arrays (local: doffS/coffS of
// local_jobs; patch: of patch_jobs), MBF array and moment array.
struct DeviceTables {
  std::vector<FactorJob> local_jobs, patch_jobs, over_jobs;
  std::vector<SubJob> subs;
  std::vector<OverRhs> rhs;
  std::vector<GamFace> gam;
  std::vector<int> dof_side, dof_q;
  std::vector<long long> mbf_off, col_off;  // m + 1 entries
  long long buf_len = 0, ldinv_len = 0, lcoup_len = 0, pdinv_len = 0, pcoup_len = 0;
  int max_local = 0, max_patch = 0, max_over = 0;  // widest box of each kind
};
// epv: storage-type words per 16 bytes (4 for FP32, 2 for FP64).
void device_tables(const HostSetup& S, int epv, DeviceTables& T);

// Everything of the set-up but the box numerics: maps, transmissibilities,
// the right-hand-side weights and the row maps of the interface system.
void host_prepare(HostSetup& S, const mrcm_grid& g, const mrcm_params& p, const double* K);
// The interface system C from the moments of the MBFs: colU / colP of
// subdomain i, dof k, side index si, mode q at col_off[i] + (k * nsides_i +
// si) * (degree + 1) + q.
void assemble_coarse(HostSetup& S, const double* colU, const double* colP,
                     const std::vector<long long>& col_off);

void face_transmissibilities(HostSetup& S);
BoxFactor factor_box(const HostSetup& S, const Box& b, bool robin);
void box_solve(const BoxFactor& F, double* x);
void host_setup(HostSetup& S, const mrcm_grid& g, const mrcm_params& p, const double* K,
                int nthreads);
// y = A x on the host (FP64), used by setup checks and tests of the host logic.
void host_op_apply(const HostSetup& S, const double* x, double* y);

}  // namespace mrcm
