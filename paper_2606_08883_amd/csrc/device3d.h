// Device-side descriptors and kernel launchers of the 3-D path
// (include/mrcm3d.h).
#pragma once

#include <hip/hip_runtime.h>

namespace mrcm3d {

constexpr int kBox3Threads = 256;  // cells of a box plane, at most (a thread per cell)
constexpr int kMaxBox3Cells = 4096;

// A cell box solved by one workgroup: origin lo and extents n (global),
// the owned subdomain inside it (olo relative to lo, extents on), the plane
// size P = n[0] n[1], and the offsets of its D_j^-1 blocks (bz P x P,
// symmetric) and z-couplings (bz x P) in the factor buffers.
struct Box3 {
  int lo[3], n[3];
  int olo[3], on[3];
  int P, pin;
  long long doff, coff;
};

// A coarse dof's trace table: its side's faces f0 .. f0 + nf (n0 x n1,
// lower tangential axis fastest) and its tensor Legendre indices (a, b).
struct Dof3 {
  int f0, nf, n0, n1;
  int a, b, pad0, pad1;
};

// Source-driven solves on the oversampled boxes (p on the owned cells, the
// trace moments mU, mP of every dof of the box's subdomain; face tables:
// box-local inside and outside cell, four weights per face).  max_cells and
// max_plane: the most cells and plane cells of a box of the launch (its LDS
// and threads, whole waves; at most kMaxBox3Cells and kBox3Threads).
// S: the storage type of the plane blocks (double or float), FP64 arithmetic.
template <typename S>
void launch_local3(const Box3* boxes, int m, int max_cells, int max_plane, const S* dinv,
                   const double* coup, const double* r, double* p, int nx, int ny,
                   const int* dof_off, const Dof3* dofs, const int* fin, const int* fout,
                   const double* fw, double* mU, double* mP, hipStream_t s);
// Patch solves of the smoothing sweep: p += A[S_i]^-1 rho[S_i] on the owned cells.
template <typename S>
void launch_patch3(const Box3* boxes, int m, int max_cells, int max_plane, const S* dinv,
                   const double* coup, const double* rho, double* p, int nx, int ny,
                   hipStream_t s);
// p[Omega_i] += P_i x_i (one workgroup per subdomain; mbf_off per subdomain).
void launch_reconstruct3(const Box3* boxes, int m, const double* mbf, const long long* mbf_off,
                         const int* dof_off, const double* x, double* p, int nx, int ny,
                         hipStream_t s);
// Seven-point operator: y = A x; rho = r - A p; w = A z with partial sums of
// w . v0; r = b - A p (b when p is NULL) with partial sums of r^2.
void launch_op3(const double* tx, const double* ty, const double* tz, int nx, int ny, int nz,
                const double* x, double* y, hipStream_t s);
void launch_residual3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                      int nz, const double* r, const double* p, double* rho, hipStream_t s);
// b = f h^2 (f may be NULL) plus 2 K_c g on the Dirichlet boundary faces
// (bcmask bit s for side s of W, E, S, N, B, T; g may be NULL).
void launch_rhs3(const double* tx, const double* ty, const double* tz, int nx, int ny, int nz,
                 int bcmask, const double* f, const double* g, double h, double* b,
                 hipStream_t s);
void launch_arnoldi_start3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                           int nz, const double* z, double* w, const double* v0,
                           double* partials, int nb, hipStream_t s);
void launch_resid_norm3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                        int nz, const double* b, const double* p, double* r, double* partials,
                        int nb, hipStream_t s);

}  // namespace mrcm3d
