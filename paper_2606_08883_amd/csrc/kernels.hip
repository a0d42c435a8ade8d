// HIP kernels for gfx950 (64-lane wavefronts): the fine five-point operator,
// the batched block-LDL^T box solves of the MRCM-OS apply, the level-scheduled
// coarse interface solve, multiscale reconstruction, Schwarz smoothing and the
// fused Arnoldi vector kernels of GMRES.  Every reduction has a fixed order,
// so results are bit-identical from run to run.
#include "device.h"

namespace mrcm {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of kVecThreads threads; result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) s += red[k];
  return s;
}

// Sum of nb partials, identical order in every block.
__device__ __forceinline__ double reduce_partials(const double* part, int nb, double* red) {
  double v = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) v += part[k];
  return block_sum(v, red);
}

// y_c = sum_f t_f (x_c - x_c') over the four faces; boundary faces carry the
// Dirichlet half-transmissibility (coupled to zero) or zero.
template <typename T>
__device__ __forceinline__ T stencil(const T* __restrict__ tx, const T* __restrict__ ty, int nx,
                                     int ny, int ix, int iy, const T* __restrict__ x) {
  const long long c = (long long)iy * nx + ix;
  const T tW = tx[(long long)iy * (nx + 1) + ix], tE = tx[(long long)iy * (nx + 1) + ix + 1];
  const T tS = ty[(long long)iy * nx + ix], tN = ty[(long long)(iy + 1) * nx + ix];
  const T xc = x[c];
  T v = (tW + tE + tS + tN) * xc;
  if (ix > 0) v -= tW * x[c - 1];
  if (ix + 1 < nx) v -= tE * x[c + 1];
  if (iy > 0) v -= tS * x[c - nx];
  if (iy + 1 < ny) v -= tN * x[c + nx];
  return v;
}

__global__ void __launch_bounds__(kVecThreads) k_op_apply(const double* __restrict__ tx,
                                                          const double* __restrict__ ty, int nx,
                                                          int ny, const double* __restrict__ x,
                                                          double* __restrict__ y) {
  const long long n = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    y[c] = stencil(tx, ty, nx, ny, ix, iy, x);
  }
}

__global__ void k_rhs(const double* __restrict__ tx, const double* __restrict__ ty, int nx,
                      int ny, int bcW, int bcE, int bcS, int bcN, const double* __restrict__ f,
                      const double* __restrict__ g, double h, double* __restrict__ b) {
  const long long n = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    double v = f ? f[c] * h * h : 0.0;
    if (g) {
      if (ix == 0 && bcW) v += tx[(long long)iy * (nx + 1)] * g[iy];
      if (ix == nx - 1 && bcE) v += tx[(long long)iy * (nx + 1) + nx] * g[ny + iy];
      if (iy == 0 && bcS) v += ty[ix] * g[2 * ny + ix];
      if (iy == ny - 1 && bcN) v += ty[(long long)ny * nx + ix] * g[2 * ny + nx + ix];
    }
    b[c] = v;
  }
}

// Block LDL^T solve of one cell box by one group of GS lanes of a wave
// (GS = 16, 32 or 64 >= bx; 64 / GS boxes per wave).  Lane r owns cell
// column r of every cell row j:
//   forward  u_j = D_j^-1 (b_j + T_j u_{j-1}),
//   backward x_j = u_j + D_j^-1 (T_{j+1} x_{j+1}).
// The elementwise coupling terms stay in the lane; the GEMV needs the whole
// vector, which the group broadcasts through its slot ys[0..bx) of LDS.  Lane
// r reads column r of the symmetric D_j^-1, i.e. D[c * bx + r] for every c, so
// each load instruction is contiguous across the group; the next block is
// prefetched into registers while the current one is used.  All exchange is
// wave-local (no workgroup barrier).  us holds b on entry, x on exit
// (by rows of bx, LDS).
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// 16-byte native vector type of a word type (clang vector extension, kept in
// registers by the optimiser).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; };
template <> struct Vec16<double> { using type = f64x2; };

// Staging of one D_j^-1 block (bstride words, 16-byte aligned, contiguous)
// through registers into an LDS buffer by all GS lanes of the group.  Indices
// past the block are clamped to its last vector (the load and the store then
// repeat that vector with identical data), which keeps the register array
// statically indexed.
template <typename V, int GS, int MAXV>
__device__ __forceinline__ void stage_load(V (&reg)[MAXV], const void* __restrict__ src, int nvec,
                                           int lane) {
  const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    const int q = k * GS + lane;
    reg[k] = s[q < nvec ? q : nvec - 1];
  }
}

template <typename V, int GS, int MAXV>
__device__ __forceinline__ void stage_store(const V (&reg)[MAXV], void* dst, int nvec, int lane) {
  V* d = reinterpret_cast<V*>(dst);
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    const int q = k * GS + lane;
    d[q < nvec ? q : nvec - 1] = reg[k];
  }
}

// acc = sum_c D[c * bx + r] ys[c]: lane r's column of the LDS block (symmetric,
// so it is row r) against the broadcast vector.
template <typename T, typename S, int NB>
__device__ __forceinline__ T lds_dot(const S* D, const T* ys, int bx, int r) {
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < bx) acc += (T)D[c * bx + r] * ys[c];
  return acc;
}

// Block LDL^T solve of one box by a group of GS lanes; lane r owns cell column
// r of every cell row j (see the comment above wave_sync):
//   forward  u_j = D_j^-1 (b_j + T_j u_{j-1}),
//   backward x_j = u_j + D_j^-1 (T_{j+1} x_{j+1}).
// Each D_j^-1 block is loaded one step ahead with 16-byte vector loads spread
// over the whole group and staged into one of two LDS buffers (Db), so the
// global loads of step j+1 are in flight while step j reads the other
// buffer.  us holds b on entry, x on exit (by rows of bx words, LDS).  S is
// the storage type of the factors, T the arithmetic and vector type (FP32
// factors may be applied in FP64 arithmetic).
template <typename T, typename S, int NB, int GS, int MAXV>
__device__ __forceinline__ void box_solve_rows(T* us, T* ys, S* Db, const S* __restrict__ Dinv,
                                               const S* __restrict__ coup, int bx, int by,
                                               int bstride, int r, bool act) {
  using V = typename Vec16<S>::type;
  constexpr int EPV = 16 / sizeof(S);
  const int nvec = bstride / EPV;
  V reg[MAXV];
  stage_load<V, GS, MAXV>(reg, Dinv, nvec, r);
  stage_store<V, GS, MAXV>(reg, Db, nvec, r);
  wave_sync();
  T u_prev = T(0);
  for (int j = 0; j < by; ++j) {
    if (j + 1 < by) stage_load<V, GS, MAXV>(reg, Dinv + (long long)(j + 1) * bstride, nvec, r);
    if (act) ys[r] = us[j * bx + r] + (j > 0 ? (T)coup[j * bx + r] * u_prev : T(0));
    wave_sync();
    const T acc = lds_dot<T, S, NB>(Db + (j & 1) * bstride, ys, bx, r);
    wave_sync();
    if (act) us[j * bx + r] = acc;
    u_prev = acc;
    if (j + 1 < by) stage_store<V, GS, MAXV>(reg, Db + ((j + 1) & 1) * bstride, nvec, r);
    wave_sync();
  }
  if (by < 2) return;
  T x_next = u_prev;
  stage_load<V, GS, MAXV>(reg, Dinv + (long long)(by - 2) * bstride, nvec, r);
  stage_store<V, GS, MAXV>(reg, Db, nvec, r);
  wave_sync();
  int buf = 0;
  for (int j = by - 2; j >= 0; --j) {
    if (j > 0) stage_load<V, GS, MAXV>(reg, Dinv + (long long)(j - 1) * bstride, nvec, r);
    if (act) ys[r] = (T)coup[(j + 1) * bx + r] * x_next;
    wave_sync();
    const T acc = lds_dot<T, S, NB>(Db + buf * bstride, ys, bx, r);
    wave_sync();
    T xj = T(0);
    if (act) {
      xj = us[j * bx + r] + acc;
      us[j * bx + r] = xj;
    }
    x_next = xj;
    if (j > 0) stage_store<V, GS, MAXV>(reg, Db + (buf ^ 1) * bstride, nvec, r);
    buf ^= 1;
    wave_sync();
  }
}

// Vectors per lane needed to stage the widest block of a launch.
template <typename T, int NB, int GS>
constexpr int stage_vectors() {
  return ((NB * NB + 16 / (int)sizeof(T) - 1) / (16 / (int)sizeof(T)) + GS - 1) / GS;
}

// Local Robin particular solves p_{i,r} = A_i^-1 r[Omega_i], one lane group
// per subdomain, fused with the trace moments of the coarse right-hand side:
// mU[k] = sum_j wU[k][j] p(face cell j), mP[k] likewise, for every coarse dof
// k = (i, side, q) of the subdomain (one lane per dof, FP64 sums).
template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_local(const BoxDesc* __restrict__ boxes, int m, int group_bytes, int blk_stride,
            const S* __restrict__ dinv, const S* __restrict__ coup,
            const double* __restrict__ r, T* __restrict__ p, int nx,
            const int* __restrict__ dof_off, const int* __restrict__ dof_side,
            const int* __restrict__ w_off, const double* __restrict__ wU,
            const double* __restrict__ wP, double* __restrict__ mU, double* __restrict__ mP) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i = blockIdx.x * (blockDim.x / GS) + grp;
  // per group: ys[GS] (T) | Db[2 * max block stride] (S) | us[max cells] (T),
  // every part 16-byte aligned
  char* base = smem_raw + (long long)grp * group_bytes;
  T* ys = reinterpret_cast<T*>(base);
  S* Db = reinterpret_cast<S*>(base + GS * sizeof(T));
  T* us = reinterpret_cast<T*>(base + GS * sizeof(T) + 2 * (long long)blk_stride * sizeof(S));
  if (i >= m) return;  // whole group leaves together
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const bool act = lane < bx;
  if (act)
    for (int j = 0; j < by; ++j) us[j * bx + lane] = (T)r[(long long)(d.y0 + j) * nx + d.x0 + lane];
  wave_sync();
  if (d.pin && lane == 0) us[0] = T(0);
  wave_sync();
  box_solve_rows<T, S, NB, GS, stage_vectors<S, NB, GS>()>(us, ys, Db, dinv + d.doff,
                                                          coup + d.coff, bx, by, d.bs, lane,
                                                          act);
  wave_sync();
  if (act)
    for (int j = 0; j < by; ++j) p[(long long)(d.y0 + j) * nx + d.x0 + lane] = us[j * bx + lane];
  for (int k = dof_off[i] + lane; k < dof_off[i + 1]; k += GS) {
    const int side = dof_side[k];
    const int len = (side <= 1) ? by : bx;
    const double* wu = wU + w_off[k];
    const double* wp = wP + w_off[k];
    double su = 0.0, sp = 0.0;
    for (int jf = 0; jf < len; ++jf) {
      const int cell = side == 0 ? jf * bx
                     : side == 1 ? jf * bx + bx - 1
                     : side == 2 ? jf
                                 : (by - 1) * bx + jf;
      const double v = (double)us[cell];
      su += wu[jf] * v;
      sp += wp[jf] * v;
    }
    mU[k] = su;
    mP[k] = sp;
  }
}

// Interface right-hand side in tree order: g_nd[t] for the coarse row
// nd_row[t] is minus the row functional of the particular traces (a flux row
// adds the two sides' moments, a pressure row subtracts them), times the
// row's equilibration scale; the replaced row of an all-no-flow grid gets zero.
__global__ void k_coarse_rhs(const int* __restrict__ nd_row, const double* __restrict__ nd_scale,
                             const int* __restrict__ rowL, const int* __restrict__ rowR,
                             const int* __restrict__ rowKind, int pin_row,
                             const double* __restrict__ mU, const double* __restrict__ mP,
                             double* __restrict__ g_nd, int nc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const int row = nd_row[t];
  const int L = rowL[row], R = rowR[row];
  const double v = rowKind[row] == 0 ? -(mU[L] + mU[R]) : -(mP[L] - mP[R]);
  g_nd[t] = row == pin_row ? 0.0 : nd_scale[t] * v;
}

// Rows [row0, row1) of an (rows x ncol) row-major matrix times the LDS vector
// vec, one wave per group of four rows; lane 0 hands each result to
// emit(row, value).  The column loop is unrolled eight deep, so a wave has up
// to 32 loads in flight before it waits.
template <typename Emit>
__device__ __forceinline__ void gemv_rows(const double* __restrict__ M, int ncol, int row0,
                                          int row1, const double* vec, Emit emit) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = row0 + 4 * wid; r < row1; r += 4 * nw) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const int nrow = row1 - r < 4 ? row1 - r : 4;
    for (int b0 = lane; b0 < ncol; b0 += 64 * 8) {
      double m[4][8], x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = b0 + 64 * q;
        const bool in = b < ncol;
        x[q] = in ? vec[b] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          m[u][q] = (in && u < nrow) ? M[(long long)(r + u) * ncol + b] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += m[u][q] * x[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double t = wave_sum(s[u]);
      if (lane == 0 && u < nrow) emit(r + u, t);
    }
  }
}

// Forward level of the coarse solve: v = g_F - contributions of descendants
// (fixed order, slots read four at a time), then rows [row0, row1) of
// [W; E] v: y_F for the separator rows, c_n for the bordering rows.
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_fwd(const CChunk* __restrict__ chunks, const CNodeDesc* __restrict__ nodes,
                 const double* __restrict__ fwd, const double* __restrict__ g_nd,
                 const int* __restrict__ slots, int maxp, double* __restrict__ ybuf,
                 double* __restrict__ cbuf) {
  extern __shared__ double v[];
  const CChunk ch = chunks[blockIdx.x];
  const CNodeDesc nd = nodes[ch.node];
  const int nf = nd.nf;
  for (int a = threadIdx.x; a < nf; a += blockDim.x) {
    const long long t = (long long)nd.yoff + a;
    double s = g_nd[t];
    const int4* sl = reinterpret_cast<const int4*>(slots + t * maxp);
    for (int u = 0; u < maxp / 4; ++u) {
      const int4 q = sl[u];
      const double c0 = q.x >= 0 ? cbuf[q.x] : 0.0, c1 = q.y >= 0 ? cbuf[q.y] : 0.0;
      const double c2 = q.z >= 0 ? cbuf[q.z] : 0.0, c3 = q.w >= 0 ? cbuf[q.w] : 0.0;
      s -= c0;
      s -= c1;
      s -= c2;
      s -= c3;
    }
    v[a] = s;
  }
  __syncthreads();
  const int yoff = nd.yoff, coff = nd.coff;
  gemv_rows(fwd + nd.fwd, nf, ch.row0, ch.row1, v, [&](int row, double val) {
    if (row < nf)
      ybuf[yoff + row] = val;
    else
      cbuf[coff + row - nf] = val;
  });
}

// Backward level: x_F = y_F - G x_U for rows [row0, row1).
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_bwd(const CChunk* __restrict__ chunks, const CNodeDesc* __restrict__ nodes,
                 const double* __restrict__ bwd, const int* __restrict__ idx,
                 const double* __restrict__ ybuf, double* __restrict__ x) {
  extern __shared__ double xu[];
  const CChunk ch = chunks[blockIdx.x];
  const CNodeDesc nd = nodes[ch.node];
  const int nu = nd.nu;
  for (int b = threadIdx.x; b < nu; b += blockDim.x) xu[b] = x[idx[nd.ucol + b]];
  __syncthreads();
  const int yoff = nd.yoff, fcol = nd.fcol;
  if (nu == 0) {
    for (int row = ch.row0 + threadIdx.x; row < ch.row1; row += blockDim.x)
      x[idx[fcol + row]] = ybuf[yoff + row];
    return;
  }
  gemv_rows(bwd + nd.bwd, nu, ch.row0, ch.row1, xu, [&](int row, double val) {
    x[idx[fcol + row]] = ybuf[yoff + row] - val;
  });
}

// p[Omega_i] += P_i x_i (multiscale reconstruction), one workgroup per subdomain.
template <typename T, typename S>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct(const BoxDesc* __restrict__ boxes, const S* __restrict__ mbf,
                  const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                  const double* __restrict__ xc, T* __restrict__ p, int nx) {
  __shared__ T xs[64];
  const int i = blockIdx.x;
  const BoxDesc d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0, ncell = d.bx * d.by;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) xs[k] = (T)xc[k0 + k];
  __syncthreads();
  const S* P = mbf + mbf_off[i];
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % d.bx, j = q / d.bx;
    const long long c = (long long)(d.y0 + j) * nx + d.x0 + a;
    T s = p[c];
    for (int k = 0; k < nk; ++k) s += (T)P[(long long)k * ncell + q] * xs[k];
    p[c] = s;
  }
}

// Smoothing residual rho = r - A p.
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_residual(const T* __restrict__ tx, const T* __restrict__ ty, int nx, int ny,
               const double* __restrict__ r, const T* __restrict__ p, T* __restrict__ rho) {
  const long long n = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    rho[c] = (T)r[c] - stencil(tx, ty, nx, ny, ix, iy, p);
  }
}

// Restricted additive Schwarz: solve A[S_i] e = rho[S_i] on patch i (one
// lane group per patch) and add e on the owned subdomain Omega_i (each cell
// is written by one patch only).
template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_patch(const BoxDesc* __restrict__ boxes, int m, int group_bytes, int blk_stride,
            const S* __restrict__ dinv, const S* __restrict__ coup, const T* __restrict__ rho,
            T* __restrict__ p, int nx) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i = blockIdx.x * (blockDim.x / GS) + grp;
  // per group: ys[GS] (T) | Db[2 * max block stride] (S) | us[max cells] (T),
  // every part 16-byte aligned
  char* base = smem_raw + (long long)grp * group_bytes;
  T* ys = reinterpret_cast<T*>(base);
  S* Db = reinterpret_cast<S*>(base + GS * sizeof(T));
  T* us = reinterpret_cast<T*>(base + GS * sizeof(T) + 2 * (long long)blk_stride * sizeof(S));
  if (i >= m) return;
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const bool act = lane < bx;
  if (act)
    for (int j = 0; j < by; ++j) us[j * bx + lane] = rho[(long long)(d.y0 + j) * nx + d.x0 + lane];
  wave_sync();
  if (d.pin && lane == 0) us[0] = T(0);
  wave_sync();
  box_solve_rows<T, S, NB, GS, stage_vectors<S, NB, GS>()>(us, ys, Db, dinv + d.doff,
                                                          coup + d.coff, bx, by, d.bs, lane,
                                                          act);
  wave_sync();
  if (lane >= d.ox && lane < d.ox + d.obx)
    for (int j = 0; j < d.oby; ++j) {
      const long long c = (long long)(d.y0 + d.oy + j) * nx + d.x0 + lane;
      p[c] += us[(d.oy + j) * bx + lane];
    }
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_sum(const T* __restrict__ p, long long n, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    s += (double)p[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// z = p - mean(p) (no-flow) or z = p, in FP64.
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_finalize(const T* __restrict__ p, long long n, const double* __restrict__ partials, int nb,
               double* __restrict__ z) {
  __shared__ double red[kVecThreads / 64];
  const double mean = partials ? reduce_partials(partials, nb, red) / (double)n : 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    z[c] = (double)p[c] - mean;
}

__global__ void k_convert(const double* __restrict__ s, float* __restrict__ d, long long n) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    d[c] = (float)s[c];
}

// ---- GMRES -----------------------------------------------------------------
__global__ void __launch_bounds__(kVecThreads)
    k_resid_norm(const double* __restrict__ tx, const double* __restrict__ ty, int nx, int ny,
                 const double* __restrict__ b, const double* __restrict__ p,
                 double* __restrict__ r, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long n = (long long)nx * ny;
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    const double v = p ? b[c] - stencil(tx, ty, nx, ny, ix, iy, p) : b[c];
    r[c] = v;
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_scale(double* __restrict__ v, long long n, double alpha) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    v[c] *= alpha;
}

__global__ void __launch_bounds__(kVecThreads)
    k_arnoldi_start(const double* __restrict__ tx, const double* __restrict__ ty, int nx, int ny,
                    const double* __restrict__ z, double* __restrict__ w,
                    const double* __restrict__ v0, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long n = (long long)nx * ny;
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    const double v = stencil(tx, ty, nx, ny, ix, iy, z);
    w[c] = v;
    s += v * v0[c];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kVecThreads)
    k_mgs_step(const double* __restrict__ part_in, double* __restrict__ part_out, int nb,
               double* __restrict__ hcol, int i, double* __restrict__ w,
               const double* __restrict__ vi, const double* __restrict__ vnext, long long n) {
  __shared__ double red[kVecThreads / 64];
  const double h = reduce_partials(part_in, nb, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) hcol[i] = h;
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const double v = w[c] - h * vi[c];
    w[c] = v;
    s += v * (vnext ? vnext[c] : v);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kVecThreads)
    k_norm_scale(const double* __restrict__ part_in, int nb, double* __restrict__ hcol, int j,
                 double* __restrict__ w, long long n) {
  __shared__ double red[kVecThreads / 64];
  const double hn = sqrt(reduce_partials(part_in, nb, red));
  if (blockIdx.x == 0 && threadIdx.x == 0) hcol[j] = hn;
  if (hn > 0.0) {
    const double inv = 1.0 / hn;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x)
      w[c] *= inv;
  }
}

__global__ void k_update(double* __restrict__ p, const double* __restrict__ Z,
                         const double* __restrict__ y, int k, long long n) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    double s = p[c];
    for (int i = 0; i < k; ++i) s += y[i] * Z[(long long)i * n + c];
    p[c] = s;
  }
}

__global__ void __launch_bounds__(kVecThreads)
    k_sumsq(const double* __restrict__ x, long long n, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    s += x[c] * x[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

inline int grid_for(long long n) {
  long long b = (n + kVecThreads - 1) / kVecThreads;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void launch_op_apply(const double* tx, const double* ty, int nx, int ny, const double* x,
                     double* y, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_op_apply, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny, x,
                     y);
}

void launch_rhs(const double* tx, const double* ty, int nx, int ny, const int* bc,
                const double* f, const double* g, double h, double* b, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny, bc[0],
                     bc[1], bc[2], bc[3], f, g, h, b);
}

// Column-buffer width (registers) and lane-group size for boxes up to max_bx
// cells wide.
inline int col_width(int max_bx) {
  return max_bx <= 16 ? 16 : max_bx <= 24 ? 24 : max_bx <= 32 ? 32 : max_bx <= 40 ? 40
       : max_bx <= 48 ? 48 : 64;
}
inline int group_size(int max_bx) { return max_bx <= 16 ? 16 : max_bx <= 32 ? 32 : 64; }

// LDS bytes of one lane group: broadcast slot and box (arithmetic words t),
// two staged blocks (storage words w), rounded to 16 bytes.
inline size_t group_bytes(int max_bx, int max_cells, int max_bs, size_t t, size_t w) {
  const size_t b = (size_t)group_size(max_bx) * t + 2 * (size_t)max_bs * w + (size_t)max_cells * t;
  return (b + 15) / 16 * 16;
}

// Lane groups per workgroup: up to 256 threads, fewer when the boxes' LDS
// would exceed 64 KB (0 when even one group does not fit).
int box_groups(int max_bx, int max_cells, int max_bs, size_t t, size_t w) {
  const int gs = group_size(max_bx);
  for (int groups = kBoxThreads / gs; groups >= 1; groups /= 2)
    if (groups * group_bytes(max_bx, max_cells, max_bs, t, w) <= 64 * 1024) return groups;
  return 0;
}

size_t box_lds_bytes(int max_bx, int max_cells, int max_bs, size_t t, size_t w) {
  const int groups = box_groups(max_bx, max_cells, max_bs, t, w);
  return groups ? groups * group_bytes(max_bx, max_cells, max_bs, t, w) : ~(size_t)0;
}

#define MRCM_BOX_DISPATCH(KERNEL, T, S, max_bx, ...)                                      \
  do {                                                                                   \
    switch (col_width(max_bx)) {                                                         \
      case 16: hipLaunchKernelGGL((KERNEL<T, S, 16>), __VA_ARGS__); break;               \
      case 24: hipLaunchKernelGGL((KERNEL<T, S, 24>), __VA_ARGS__); break;               \
      case 32: hipLaunchKernelGGL((KERNEL<T, S, 32>), __VA_ARGS__); break;               \
      case 40: hipLaunchKernelGGL((KERNEL<T, S, 40>), __VA_ARGS__); break;               \
      case 48: hipLaunchKernelGGL((KERNEL<T, S, 48>), __VA_ARGS__); break;               \
      default: hipLaunchKernelGGL((KERNEL<T, S, 64>), __VA_ARGS__); break;               \
    }                                                                                    \
  } while (0)

template <typename T, typename S>
void launch_local(const BoxDesc* boxes, int m, int max_cells, int max_bx, int max_bs,
                  const S* dinv, const S* coup, const double* r, T* p, int nx,
                  const int* dof_off, const int* dof_side, const int* w_off, const double* wU,
                  const double* wP, double* mU, double* mP, hipStream_t s) {
  const int groups = box_groups(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const size_t shm = box_lds_bytes(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const int gb = (int)group_bytes(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
  MRCM_BOX_DISPATCH(k_local, T, S, max_bx, grid, block, shm, s, boxes, m, gb, max_bs,
                    dinv, coup, r, p, nx, dof_off, dof_side, w_off, wU, wP, mU, mP);
}

void launch_coarse_rhs(const int* nd_row, const double* nd_scale, const int* rowL,
                       const int* rowR, const int* rowKind, int pin_row, const double* mU,
                       const double* mP, double* g_nd, int nc, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_coarse_rhs, dim3((nc + 255) / 256), dim3(256), 0, s, nd_row, nd_scale,
                     rowL, rowR, rowKind, pin_row, mU, mP, g_nd, nc);
}

void launch_coarse_fwd(const CChunk* chunks, int nchunks, const CNodeDesc* nodes,
                       const double* fwd, const double* g_nd, const int* slots, int maxp,
                       double* ybuf, double* cbuf, int max_nf, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_coarse_fwd, dim3(nchunks), dim3(kVecThreads),
                     sizeof(double) * (size_t)max_nf, s, chunks, nodes, fwd, g_nd, slots, maxp,
                     ybuf, cbuf);
}

void launch_coarse_bwd(const CChunk* chunks, int nchunks, const CNodeDesc* nodes,
                       const double* bwd, const int* idx, const double* ybuf, double* x,
                       int max_nu, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_coarse_bwd, dim3(nchunks), dim3(kVecThreads),
                     sizeof(double) * (size_t)(max_nu > 0 ? max_nu : 1), s, chunks, nodes, bwd,
                     idx, ybuf, x);
}

template <typename T, typename S>
void launch_reconstruct(const BoxDesc* boxes, int m, const S* mbf, const long long* mbf_off,
                        const int* dof_off, const double* xc, T* p, int nx, hipStream_t s) {
  hipLaunchKernelGGL((k_reconstruct<T, S>), dim3(m), dim3(kBoxThreads), 0, s, boxes, mbf,
                     mbf_off, dof_off, xc, p, nx);
}

template <typename T>
void launch_residual(const T* tx, const T* ty, int nx, int ny, const double* r, const T* p,
                     T* rho, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_residual<T>, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny,
                     r, p, rho);
}

template <typename T, typename S>
void launch_patch(const BoxDesc* boxes, int m, int max_cells, int max_bx, int max_bs,
                  const S* dinv, const S* coup, const T* rho, T* p, int nx, hipStream_t s) {
  const int groups = box_groups(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const size_t shm = box_lds_bytes(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const int gb = (int)group_bytes(max_bx, max_cells, max_bs, sizeof(T), sizeof(S));
  const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
  MRCM_BOX_DISPATCH(k_patch, T, S, max_bx, grid, block, shm, s, boxes, m, gb, max_bs,
                    dinv, coup, rho, p, nx);
}

template <typename T>
void launch_finalize(const T* p, long long n, int noflow, double* z, double* partials,
                     hipStream_t s) {
  const int nb = vec_blocks(n);
  if (noflow) hipLaunchKernelGGL(k_sum<T>, dim3(nb), dim3(kVecThreads), 0, s, p, n, partials);
  hipLaunchKernelGGL(k_finalize<T>, dim3(nb), dim3(kVecThreads), 0, s, p, n,
                     noflow ? partials : (const double*)nullptr, nb, z);
}

void launch_convert(const double* src, float* dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(n)), dim3(kVecThreads), 0, s, src, dst, n);
}

void launch_resid_norm(const double* tx, const double* ty, int nx, int ny, const double* b,
                       const double* p, double* r, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_norm, dim3(nb), dim3(kVecThreads), 0, s, tx, ty, nx, ny, b, p, r,
                     partials);
}

void launch_scale(double* v, long long n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kVecThreads), 0, s, v, n, alpha);
}

void launch_arnoldi_start(const double* tx, const double* ty, int nx, int ny, const double* z,
                          double* w, const double* v0, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_start, dim3(nb), dim3(kVecThreads), 0, s, tx, ty, nx, ny, z, w, v0,
                     partials);
}

void launch_mgs_step(const double* part_in, double* part_out, int nb, double* hcol, int i,
                     double* w, const double* vi, const double* vnext, long long n,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_step, dim3(nb), dim3(kVecThreads), 0, s, part_in, part_out, nb, hcol, i,
                     w, vi, vnext, n);
}

void launch_norm_scale(const double* part_in, int nb, double* hcol, int j, double* w,
                       long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_scale, dim3(nb), dim3(kVecThreads), 0, s, part_in, nb, hcol, j, w, n);
}

void launch_update(double* p, const double* Z, const double* y, int k, long long n,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(grid_for(n)), dim3(kVecThreads), 0, s, p, Z, y, k, n);
}

void launch_sumsq(const double* x, long long n, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(kVecThreads), 0, s, x, n, partials);
}

#define MRCM_INSTANTIATE_TS(T, S)                                                              \
  template void launch_local<T, S>(const BoxDesc*, int, int, int, int, const S*, const S*,     \
                                   const double*, T*, int, const int*, const int*, const int*,   \
                                   const double*, const double*, double*, double*, hipStream_t); \
  template void launch_reconstruct<T, S>(const BoxDesc*, int, const S*, const long long*,       \
                                         const int*, const double*, T*, int, hipStream_t);      \
  template void launch_patch<T, S>(const BoxDesc*, int, int, int, int, const S*, const S*,     \
                                   const T*, T*, int, hipStream_t);
#define MRCM_INSTANTIATE_T(T)                                                                  \
  template void launch_residual<T>(const T*, const T*, int, int, const double*, const T*, T*,   \
                                   hipStream_t);                                                \
  template void launch_finalize<T>(const T*, long long, int, double*, double*, hipStream_t);

MRCM_INSTANTIATE_TS(double, double)
MRCM_INSTANTIATE_TS(float, float)
MRCM_INSTANTIATE_TS(double, float)
MRCM_INSTANTIATE_T(double)
MRCM_INSTANTIATE_T(float)

}  // namespace mrcm
