// Work descriptors of the set-up kernels and the storage layout of the box
// factors (plain structures and constexpr functions shared by the host side
// and the device side).  Offsets are in elements of the buffer they index.
#pragma once

namespace mrcm {

// Half-block layout of the symmetric row blocks D_j^-1 (n x n, n <= cols).
// Lane r of a box keeps the entries D(r, (r + k) mod n) for k = 0 .. cols / 2
// (the "rows" k of the half block); the entries D(r, r - k) it needs as well
// are entry k of lane r - k.  Row k holds zeros for k > n / 2, and for even n
// the row k = n / 2, which both ends of a pair hold, carries half the value
// (each end adds its half).  Rows k0 .. cols / 2 are stored in quads (word
// ((q * n + r) * 4 + i) holds row k0 + 4 q + i), the first k0 = (cols / 2 + 1)
// % 4 rows after them as single words (word 4 nh n + k n + r), so a lane reads
// its rows in 16-byte pieces (32 for FP64) and the group reads them
// contiguously.  cols is the launch's column width: box_cols(widest box).
constexpr int box_cols(int max_bx) {
  return max_bx <= 16 ? 16 : max_bx <= 20 ? 20 : max_bx <= 24 ? 24 : max_bx <= 32 ? 32
       : max_bx <= 36 ? 36 : max_bx <= 40 ? 40 : max_bx <= 48 ? 48 : 64;
}
constexpr int half_rows(int cols) { return cols / 2 + 1; }
constexpr int half_k0(int cols) { return half_rows(cols) % 4; }
constexpr int half_quads(int cols) { return half_rows(cols) / 4; }
// Words of one block of a box n cells wide, a multiple of 4 (16 bytes of FP32).
constexpr long long half_block_words(int n, int cols) {
  return ((long long)half_rows(cols) * n + 3) / 4 * 4;
}
// Word of row k, lane r in a block of a box n cells wide.
constexpr long long half_word(int k, int r, int n, int cols) {
  return k >= half_k0(cols)
             ? ((long long)((k - half_k0(cols)) / 4) * n + r) * 4 + (k - half_k0(cols)) % 4
             : (long long)4 * half_quads(cols) * n + (long long)k * n + r;
}

// A cell box to factor (block LDL^T by cell rows in FP64, Section 2.1 local
// problems): Robin conductances on its faces inside the domain when robin,
// the principal submatrix of A otherwise; pin fixes the first cell (a box
// covering an all-no-flow domain).  Outputs: storage-type half blocks of
// column width cols at doffS (stride bs words) and couplings at coffS, FP64
// row-major blocks at d64 and couplings at c64; -1 skips an output.
struct FactorJob {
  int x0, y0, bx, by;
  int robin, pin;
  int bs, cols;
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
// is on the oversampled box's boundary, which happens without oversampling),
// the index si of its side among the subdomain's interface sides, the side
// code (W E S N), its position j among the nfs faces of the side;
// conductances.
struct GamFace {
  int ocin, ocout;
  int si, side, j, nfs;
  int unused0, unused1;
  double rho, b, t, Kin, Kout;
};

// The set-up work of one subdomain: its oversampled box (obx x oby, pinned
// when opin) and the subdomain box inside it (lbx x lby at offset ox, oy);
// ni local dofs (the first is dof0), nsides sides of Gamma_i, its entries of
// the OverRhs and GamFace tables, and offsets of the oversampled factor and
// couplings (FP64), scratch vectors (ni x oversampled cells), MBF output
// (ni x subdomain cells, storage type) and moments (ni x nsides x nb).
struct SubJob {
  int obx, oby, opin;
  int lbx, lby, ox, oy;
  int ni, nsides, dof0;
  int rhs0, rhs1, gam0, gam1;
  int unused;
  long long o64, oc64, oscr, mbf, col;
};

}  // namespace mrcm
