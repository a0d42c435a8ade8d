// Device-side descriptors and kernel launchers of the MRCM-OS library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "coarse.h"
#include "setup_jobs.h"

namespace mrcm {

// One cell box solved by a workgroup (a subdomain or a smoothing patch).
// (x0, y0, bx, by): the box; (ox, oy, obx, oby): the owned subdomain, in
// coordinates relative to the box (patches add their solution there only).
struct BoxDesc {
  int x0, y0, bx, by;
  int pin;
  int ox, oy, obx, oby;
  int bs;          // stride between D_j^-1 blocks (words, a multiple of 16 bytes)
  long long doff;  // offset of the first D_j^-1 block (elements, 16-byte aligned)
  long long coff;  // offset of the couplings T_j (elements)
};

constexpr int kBoxThreads = 256;
constexpr int kVecThreads = 256;
constexpr int kMaxVecBlocks = 1024;
constexpr int kMaxRhs = 8;  // right-hand sides of one multi-RHS launch

inline int vec_blocks(long long n) {
  long long b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
  if (b < 1) b = 1;
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  return (int)b;
}

// ---- fine operator --------------------------------------------------------
void launch_op_apply(const double* tx, const double* ty, int nx, int ny, const double* x,
                     double* y, hipStream_t s);
void launch_rhs(const double* tx, const double* ty, int nx, int ny, const int* bc,
                const double* f, const double* g, double h, double* b, hipStream_t s);

// ---- preconditioner apply (arithmetic T, factor storage S) ------------------
// Boxes are solved by lane groups of 16, 32 or 64 lanes (>= the widest box,
// at most 64 cells wide); LDS per workgroup: box_lds_bytes() (all ones when a
// single group exceeds 64 KB).  t, w: bytes of the arithmetic type T and of
// the factor storage type S.
size_t box_lds_bytes(int max_bx, int max_cells, size_t t, size_t w);
// Lane groups per workgroup of the box kernels (the most that fit; a launch
// may take fewer, groups_cap > 0, which changes no result).
int box_groups(int max_bx, int max_cells, size_t t, size_t w);
// Source-driven solves on the oversampled boxes (boxes[i]: hat-Omega_i with
// Omega_i as its owned part): p = the solutions restricted to Omega_i, and
// the trace moments mU, mP of every coarse dof (dof_side, dof_q, first face
// dof_face0 of the four weights per face in face_w).
template <typename T, typename S>
void launch_local(const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                  const S* coup, const double* r, T* p, int nx, const int* dof_off,
                  const int* dof_side, const int* dof_q, const int* dof_face0,
                  const double* face_w, double* mU, double* mP, hipStream_t s,
                  int groups_cap = 0);
// Interface solve: the right-hand side g_nd in tree order (np positions;
// gsrc[t] = {L, R, kind, 0} names the trace moments of the row at tree
// position t and its kind, gscale[t] its equilibration scale), then one
// launch per tree level, forward levels leaves first, backward levels root
// first.  contrib (maxp slots per tree position, slot u of position t at
// u * np + t, zero where unused) receives the descendants' contributions at
// cdest; max_nf / max_nu bound the LDS vector.  A node without border rows
// (the root) writes its x_F in its forward level and has no backward level.
// threads: 64 or 256 per workgroup, 0 for the default (coarse_threads); the
// choice changes no result.  A forward chunk of at most 128 columns is taken
// whole, 16 rows per wave, when its rows fit the workgroup's waves; a
// backward one when a one-wave workgroup takes its (at most 16) rows; other
// chunks go four rows per wave at a time.
void launch_coarse_rhs(const int4* gsrc, const double* gscale, const double* mU,
                       const double* mP, double* g_nd, int np, hipStream_t s);
void launch_coarse_fwd(const CChunk* chunks, int nchunks, const double* fwd, const double* g_nd,
                       double* contrib, int maxp, int np, const int* cdest, double* ybuf,
                       const int* idx, double* x, int max_nf, hipStream_t s, int threads = 0);
void launch_coarse_bwd(const CChunk* chunks, int nchunks, const double* bwd, const int* idx,
                       const double* ybuf, double* x, int max_nu, hipStream_t s,
                       int threads = 0);
// Default threads of a level: 256 forward; backward 64 for levels of 2048
// chunks or more, else 256.
int coarse_threads(int nchunks, bool forward);
// Refinement of the interface solve, k columns: r_nd = g_nd - (scaled C in
// tree order, CSR rp / ci / v) x, and x += dx (n values).
void launch_coarse_resid(int k, const int* rp, const int* ci, const double* v,
                         const double* g_nd, const double* x, double* r_nd, int np, int nc,
                         hipStream_t s);
void launch_coarse_add(double* x, const double* dx, long long n, hipStream_t s);
template <typename T, typename S>
void launch_reconstruct(const BoxDesc* boxes, int m, const S* mbf, const long long* mbf_off,
                        const int* dof_off, const double* xc, T* p, int nx, hipStream_t s);
template <typename T>
void launch_residual(const T* tx, const T* ty, int nx, int ny, const double* r, const T* p,
                     T* rho, hipStream_t s);
template <typename T, typename S>
void launch_patch(const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                  const S* coup, const T* rho, T* p, int nx, hipStream_t s, int groups_cap = 0);
template <typename T>
void launch_finalize(const T* p, long long n, int noflow, double* z, double* partials,
                     hipStream_t s);
void launch_convert(const double* src, float* dst, long long n, hipStream_t s);

// ---- the same steps for K right-hand sides per launch (K = 2, 4 or 8) ------
// Per-RHS vectors are given by host arrays of K base pointers; the per-RHS
// work vectors of the interface solve are K consecutive blocks (mU, mP, xc:
// k * nc; g_nd, ybuf: k * np; contrib: k * maxp * np).  e: per-RHS scratch
// of the oversampled boxes and of the smoothing patches (box i at its
// coupling offset; as long as the larger of the two coupling arrays).
// Results equal K one-RHS launches bit for bit.
size_t box_lds_bytes_k(int k, int max_bx, int max_cells, size_t t, size_t w);
template <typename T, typename S>
void launch_local_k(int k, const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                    const S* coup, const double* const* r, T* const* p, T* const* e, int nx,
                    const int* dof_off, const int* dof_side, const int* dof_q,
                    const int* dof_face0, const double* face_w, double* mU, double* mP, int nc,
                    hipStream_t s);
void launch_coarse_rhs_k(int k, const int4* gsrc, const double* gscale, const double* mU,
                         const double* mP, double* g_nd, int np, int nc, hipStream_t s);
void launch_coarse_fwd_k(int k, const CChunk* chunks, int nchunks, const double* fwd,
                         const double* g_nd, double* contrib, int maxp, int np, const int* cdest,
                         double* ybuf, const int* idx, double* x, int nc, int max_nf,
                         hipStream_t s);
void launch_coarse_bwd_k(int k, const CChunk* chunks, int nchunks, const double* bwd,
                         const int* idx, const double* ybuf, double* x, int max_nu, int np, int nc,
                         hipStream_t s);
template <typename T, typename S>
void launch_reconstruct_k(int k, const BoxDesc* boxes, int m, const S* mbf,
                          const long long* mbf_off, const int* dof_off, const double* xc, int nc,
                          T* const* p, int nx, hipStream_t s);
// The reconstruction of 8 right-hand sides on the matrix cores (mode 1:
// the MFMA of the arithmetic type, FP32 or FP64; mode 2: BF16 inputs with
// FP32 accumulation, FP32 arithmetic only); rounding differs from
// launch_reconstruct_k.
template <typename T, typename S>
void launch_reconstruct_mfma(int mode, const BoxDesc* boxes, int m, const S* mbf,
                             const long long* mbf_off, const int* dof_off, const double* xc,
                             int nc, T* const* p, int nx, hipStream_t s);
template <typename T>
void launch_residual_k(int k, const T* tx, const T* ty, int nx, int ny, const double* const* r,
                       const T* const* p, T* const* rho, hipStream_t s);
template <typename T, typename S>
void launch_patch_k(int k, const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                    const S* coup, const T* const* rho, T* const* p, T* const* e, int nx,
                    hipStream_t s);
template <typename T>
void launch_finalize_k(int k, const T* const* p, long long n, int noflow, double* const* z,
                       double* partials, hipStream_t s);

// ---- launches over several contexts ----------------------------------------
// One column of a launch over several contexts: one right-hand side of one
// context, with the context's tables and factors and the column's own work
// vectors (the factor and work-vector pointers are typed by the launch's S
// and T).  A launch gives column c the workgroups [pre[c], pre[c + 1]) of its
// grid; workgroup pre[c] + b runs as block b of the column's own launch, so
// every column gets the results of its one-context launch bit for bit.
struct ManyCol {
  const BoxDesc *lbox, *pbox;
  const void *ldinv, *lcoup, *pdinv, *pcoup, *mbf;
  const long long* mbf_off;
  const int *dof_off, *dof_side, *dof_q, *dof_face0;
  const double* face_w;
  const int4* gsrc;
  const double* gscale;
  const double *cfwd, *cbwd;
  const int *cidx, *cdest;
  const CChunk* chunks;
  const int *crp, *cci;
  const double* cv;
  const void *txT, *tyT;
  const double *tx, *ty;
  int nx, ny, m, nc, np, maxp, noflow, nb;  // nb: blocks of the column's vector reductions
  long long n;
  const double* r;  // T is applied to r and written to z
  double* z;
  void *p, *rho;
  double *mU, *mP, *xc, *g_nd, *ybuf, *rnd, *dx, *contrib, *partials;
  // GMRES state of the column (batched solves): the Krylov basis V (restart
  // + 1 vectors), Z, the two halves of the reduction partials, the
  // Hessenberg column and the step j.
  double *V, *Z, *parts, *hcol;
  int j, pad;
};
// A copy of count doubles from src into a staging vector at dst.
struct GatherItem {
  const double* src;
  long long dst;
  int count, pad;
};
template <typename T, typename S>
void launch_local_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int max_cells,
                       int max_bx, hipStream_t s);
void launch_coarse_rhs_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s);
// Level of the interface solve: column c's chunks first[c] .. of its own
// chunk table; refine selects the refinement vectors (rnd, dx) instead of
// (g_nd, xc).
void launch_coarse_fwd_many(const ManyCol* cols, const int* pre, const int* first, int ncol,
                            int blocks, int refine, int max_nf, hipStream_t s);
void launch_coarse_bwd_many(const ManyCol* cols, const int* pre, const int* first, int ncol,
                            int blocks, int refine, int max_nu, hipStream_t s);
void launch_coarse_resid_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                              hipStream_t s);
void launch_coarse_add_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s);
template <typename T, typename S>
void launch_reconstruct_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                             hipStream_t s);
template <typename T>
void launch_residual_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                          hipStream_t s);
template <typename T, typename S>
void launch_patch_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int max_cells,
                       int max_bx, hipStream_t s);
template <typename T>
void launch_sum_many(const ManyCol* cols, const int* pre, int ncol, int blocks, hipStream_t s);
template <typename T>
void launch_finalize_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                          hipStream_t s);
// The Arnoldi tail of every column at its step j: w = A Z_j with w . v_0,
// modified Gram-Schmidt step i (columns with j >= i), normalisation.
void launch_arnoldi_start_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                               hipStream_t s);
void launch_mgs_step_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int i,
                          hipStream_t s);
void launch_norm_scale_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s);
void launch_gather(const GatherItem* items, int count, double* stage, hipStream_t s);

// ---- set-up on the device (FP64; one wave per box or subdomain) ------------
// Factor the boxes of `jobs` (LDS: two maxn x maxn blocks); status[0] = 1
// after a non-positive pivot.
template <typename S>
void launch_factor_boxes(const FactorJob* jobs, int njobs, int maxn, const double* K,
                         const double* tx, const double* ty, int nx, int ny, double aL, S* dS,
                         S* cS, double* d64, double* c64, int* status, hipStream_t s);
// Oversampled problems of every subdomain, their restrictions to Omega_i
// (the MBFs, storage type) and the moments of their traces on Gamma_i (buf:
// FP64 work buffer that the SubJob offsets index; over0: no oversampling).
template <typename S>
void launch_over_mbf(const SubJob* subs, int m, const OverRhs* rhs, const GamFace* gam,
                     const int* dof_side, const int* dof_q, int over0, int nb, double* buf,
                     S* mbf, double* colU, double* colP, hipStream_t s);

// ---- GMRES vector kernels (FP64) -------------------------------------------
// r = b - A p (p may be NULL for p = 0); partials[block] = sum r^2
void launch_resid_norm(const double* tx, const double* ty, int nx, int ny, const double* b,
                       const double* p, double* r, double* partials, int nb, hipStream_t s);
// v = alpha * v
void launch_scale(double* v, long long n, double alpha, hipStream_t s);
// v = 0 (a kernel, so that it can be captured in a graph)
void launch_zero(double* v, long long n, hipStream_t s);
// w = A z, partials = w . v0
void launch_arnoldi_start(const double* tx, const double* ty, int nx, int ny, const double* z,
                          double* w, const double* v0, double* partials, int nb, hipStream_t s);
// h = sum(part_in); hcol[i] = h; w -= h vi; part_out = w . vnext (or w . w when vnext NULL)
void launch_mgs_step(const double* part_in, double* part_out, int nb, double* hcol, int i,
                     double* w, const double* vi, const double* vnext, long long n,
                     hipStream_t s);
// hn = sqrt(sum(part_in)); hcol[j] = hn; w /= hn (if hn > 0)
void launch_norm_scale(const double* part_in, int nb, double* hcol, int j, double* w,
                       long long n, hipStream_t s);
// p += sum_i y[i] Z_i
void launch_update(double* p, const double* Z, const double* y, int k, long long n,
                   hipStream_t s);
// partials = sum of squares of x
void launch_sumsq(const double* x, long long n, double* partials, int nb, hipStream_t s);

}  // namespace mrcm
