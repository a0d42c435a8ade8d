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
  // Factors of the oversampled boxes hat-Omega_i (Robin on their faces
  // inside the domain) and of the smoothing patches.
  std::vector<BoxFactor> over, patch;
  std::vector<std::vector<double>> mbf;  // per subdomain: N_i columns of bx*by (Omega_i)
  // Trace weights of the source-driven solutions, per face of Gamma_i
  // (subdomain i's faces from face_off[i], its interface sides in W E S N
  // order, faces in increasing coordinate): four values (cUi, cUo, cPi, cPo)
  // with U = cUi p_in + cUo p_out and pi = cPi p_in + cPo p_out, p_in the
  // value in the subdomain's cell and p_out in the cell across the face (both
  // in the oversampled box; without oversampling the face is a Robin face
  // and the out weights are zero).  Every coarse dof k = (i, side, q) reads
  // the faces of its side from dof_face0[k] with Legendre weight P_q.
  std::vector<int> face_off;  // m + 1
  std::vector<double> face_w;  // 4 per face
  std::vector<int> dof_face0, dof_q;  // nc
  // Coarse rows: the two dofs (L side, R side) each row combines, and kind.
  std::vector<int> rowL, rowR, rowKind;
  int pin_row = -1, pin_dof = -1;
  // Coarse matrix in CSR (rows x dofs).
  std::vector<int> Crp, Cci;
  std::vector<double> Cv;
};

// Work lists of the set-up on the device (built on the host from the maps,
// transmissibilities and K; O(perimeter) per subdomain).  local_jobs factor
// the oversampled boxes (the boxes of the particular solves of the apply and
// of the oversampled problems of the set-up): storage-type factors at
// doffS / coffS for the apply, FP64 factors in the work buffer `buf` for the
// set-up solves.  Offsets: `buf` (FP64 factors and couplings, scratch
// vectors), storage-type factor arrays (local: ldinv / lcoup; patch: pdinv /
// pcoup), MBF array and moment array.
struct DeviceTables {
  std::vector<FactorJob> local_jobs, patch_jobs;
  std::vector<SubJob> subs;
  std::vector<OverRhs> rhs;
  std::vector<GamFace> gam;
  std::vector<int> dof_side, dof_q;
  std::vector<long long> mbf_off, col_off;  // m + 1 entries
  long long buf_len = 0, ldinv_len = 0, lcoup_len = 0, pdinv_len = 0, pcoup_len = 0;
  int max_local = 0, max_patch = 0;  // widest box of each kind
};
// epv: storage-type words per 16 bytes (4 for FP32, 2 for FP64).
void device_tables(const HostSetup& S, int epv, DeviceTables& T);

// Everything of the set-up but the box numerics: maps, transmissibilities,
// the trace weights and the row maps of the interface system.
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
