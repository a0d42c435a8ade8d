// Work descriptors of the set-up kernels (plain structures shared by the
// host side, which builds them, and the device side).  Offsets are in
// elements of the buffer they index.
#pragma once

namespace mrcm {

// A cell box to factor (block LDL^T by cell rows in FP64, Section 2.1 local
// problems): Robin conductances on its faces inside the domain when robin,
// the principal submatrix of A otherwise; pin fixes the first cell (a box
// covering an all-no-flow domain).  Outputs: storage-type quad blocks at
// doffS (stride bs words) and couplings at coffS, FP64 row-major blocks at
// d64 and couplings at c64; -1 skips an output.
struct FactorJob {
  int x0, y0, bx, by;
  int robin, pin;
  int bs, unused;
  long long doffS, coffS;
  long long d64, c64;
};

// Robin data of an oversampled problem: value `val` at cell `cell` of the
// oversampled box, right-hand side of local dof k.
struct OverRhs {
  int k, cell;
  double val;
};

// A face of Gamma_i: its cells in the oversampled box (ocout = -1: the face
// is on the oversampled box's boundary) and in the subdomain box; the index
// si of its side among the subdomain's interface sides, the side code
// (W E S N), its position j among the nfs faces of the side; conductances.
struct GamFace {
  int ocin, ocout, lcin;
  int si, side, j, nfs;
  int unused;
  double rho, b, t, Kin, Kout;
};

// The set-up work of one subdomain: its box and oversampled box (origins are
// implied by the tables), ni local dofs (the first is dof0), nsides sides of
// Gamma_i, its entries of the OverRhs and GamFace tables, and offsets of
// its FP64 factors and couplings, scratch vectors (ni x cells), phi values
// (ni x faces), MBF output (ni x cells, storage type) and moments (ni x
// nsides x nb).
struct SubJob {
  int lbx, lby, lpin;
  int obx, oby, opin;
  int ni, nsides, dof0;
  int rhs0, rhs1, gam0, gam1;
  int unused;
  long long l64, lc64, o64, oc64;
  long long lscr, oscr, phi, mbf, col;
};

}  // namespace mrcm
