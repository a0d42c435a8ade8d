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

// Block LDL^T solve of one box held in LDS (x: by rows of bx values).
//   forward  u_j = D_j^-1 (x_j + T_j u_{j-1})
//   backward x_j = u_j + D_j^-1 (T_{j+1} x_{j+1})
// GEMV mapping: thread t handles row r = t % bx of D_j^-1 over the columns
// c = g, g + G, ... with g = t / bx and G = blockDim / bx groups; D_j^-1 is
// symmetric, so D[c * bx + r] is read with consecutive r in consecutive
// lanes (coalesced).  The G partial sums are reduced through LDS.
template <typename T>
__device__ void ldl_box_solve(T* x, T* part, const T* __restrict__ Dinv,
                              const T* __restrict__ coup, int bx, int by) {
  const int t = threadIdx.x;
  const int G = blockDim.x / bx;
  const int r = t % bx, g = t / bx;
  const bool act = g < G;
  for (int j = 0; j < by; ++j) {
    if (j > 0 && t < bx) x[j * bx + t] += coup[j * bx + t] * x[(j - 1) * bx + t];
    __syncthreads();
    T acc = T(0);
    if (act) {
      const T* D = Dinv + (long long)j * bx * bx;
      for (int c = g; c < bx; c += G) acc += D[c * bx + r] * x[j * bx + c];
      part[g * bx + r] = acc;
    }
    __syncthreads();
    if (t < bx) {
      T s = T(0);
      for (int q = 0; q < G; ++q) s += part[q * bx + t];
      x[j * bx + t] = s;
    }
    __syncthreads();
  }
  for (int j = by - 2; j >= 0; --j) {
    T acc = T(0);
    if (act) {
      const T* D = Dinv + (long long)j * bx * bx;
      const T* cp = coup + (j + 1) * bx;
      const T* xn = x + (j + 1) * bx;
      for (int c = g; c < bx; c += G) acc += D[c * bx + r] * (cp[c] * xn[c]);
      part[g * bx + r] = acc;
    }
    __syncthreads();
    if (t < bx) {
      T s = T(0);
      for (int q = 0; q < G; ++q) s += part[q * bx + t];
      x[j * bx + t] += s;
    }
    __syncthreads();
  }
}

// Local Robin particular solves p_{i,r} = A_i^-1 r[Omega_i] (one workgroup per
// subdomain) fused with the trace moments of the coarse right-hand side:
// mU[k] = sum_j wU[k][j] p(face cell j), mP[k] likewise, for every coarse dof k
// = (i, side, q) of the subdomain.
template <typename T>
__global__ void __launch_bounds__(kBoxThreads)
    k_local(const BoxDesc* __restrict__ boxes, const T* __restrict__ dinv,
            const T* __restrict__ coup, const double* __restrict__ r, T* __restrict__ p, int nx,
            const int* __restrict__ dof_off, const int* __restrict__ dof_side,
            const int* __restrict__ w_off, const double* __restrict__ wU,
            const double* __restrict__ wP, double* __restrict__ mU, double* __restrict__ mP) {
  extern __shared__ __align__(16) char smem_raw[];
  const BoxDesc d = boxes[blockIdx.x];
  const int bx = d.bx, by = d.by, ncell = bx * by;
  T* part = reinterpret_cast<T*>(smem_raw);
  T* x = part + kBoxThreads;
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % bx, j = q / bx;
    x[q] = (T)r[(long long)(d.y0 + j) * nx + d.x0 + a];
  }
  __syncthreads();
  if (d.pin && threadIdx.x == 0) x[0] = T(0);
  __syncthreads();
  ldl_box_solve<T>(x, part, dinv + d.doff, coup + d.coff, bx, by);
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % bx, j = q / bx;
    p[(long long)(d.y0 + j) * nx + d.x0 + a] = x[q];
  }
  const int i = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = dof_off[i] + wid; k < dof_off[i + 1]; k += nw) {
    const int side = dof_side[k];
    const int len = (side <= 1) ? by : bx;
    double su = 0.0, sp = 0.0;
    for (int jf = lane; jf < len; jf += 64) {
      int cell;
      if (side == 0) cell = jf * bx;
      else if (side == 1) cell = jf * bx + bx - 1;
      else if (side == 2) cell = jf;
      else cell = (by - 1) * bx + jf;
      const double v = (double)x[cell];
      su += wU[w_off[k] + jf] * v;
      sp += wP[w_off[k] + jf] * v;
    }
    su = wave_sum(su);
    sp = wave_sum(sp);
    if (lane == 0) {
      mU[k] = su;
      mP[k] = sp;
    }
  }
}

// Coarse right-hand side: minus the flux and pressure row functionals of the
// particular traces (flux rows add the two sides, pressure rows subtract).
__global__ void k_coarse_rhs(const double* __restrict__ mU, const double* __restrict__ mP,
                             const int* __restrict__ rowL, const int* __restrict__ rowR,
                             const int* __restrict__ rowKind, int nc, int pin_row,
                             double* __restrict__ g) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nc) return;
  const int L = rowL[r], R = rowR[r];
  double v = rowKind[r] == 0 ? -(mU[L] + mU[R]) : -(mP[L] - mP[R]);
  g[r] = (r == pin_row) ? 0.0 : v;
}

// Forward level of the coarse solve: gather v = g_F - contributions of
// descendants (fixed order), then rows [row0, row1) of [W; E] v.
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_fwd(const CChunk* __restrict__ chunks, const CNodeDesc* __restrict__ nodes,
                 const double* __restrict__ fwd, const int* __restrict__ idx,
                 const int* __restrict__ pull_ptr, const int* __restrict__ pull_idx,
                 const double* __restrict__ g, double* __restrict__ ybuf,
                 double* __restrict__ cbuf) {
  extern __shared__ double v[];
  const CChunk ch = chunks[blockIdx.x];
  const CNodeDesc nd = nodes[ch.node];
  const int nf = nd.nf;
  for (int a = threadIdx.x; a < nf; a += blockDim.x) {
    const int row = idx[nd.frow + a];
    double s = g[row];
    for (int q = pull_ptr[row]; q < pull_ptr[row + 1]; ++q) s -= cbuf[pull_idx[q]];
    v[a] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int row = ch.row0 + wid; row < ch.row1; row += nw) {
    const double* M = fwd + nd.fwd + (long long)row * nf;
    double s = 0.0;
    for (int b = lane; b < nf; b += 64) s += M[b] * v[b];
    s = wave_sum(s);
    if (lane == 0) {
      if (row < nf)
        ybuf[nd.yoff + row] = s;
      else
        cbuf[nd.coff + row - nf] = s;
    }
  }
}

// Backward level: x_F = y_F - G x_U for rows [row0, row1).
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_bwd(const CChunk* __restrict__ chunks, const CNodeDesc* __restrict__ nodes,
                 const double* __restrict__ bwd, const int* __restrict__ idx,
                 const double* __restrict__ ybuf, double* __restrict__ x) {
  extern __shared__ double xu[];
  const CChunk ch = chunks[blockIdx.x];
  const CNodeDesc nd = nodes[ch.node];
  const int nf = nd.nf, nu = nd.nu;
  for (int b = threadIdx.x; b < nu; b += blockDim.x) xu[b] = x[idx[nd.ucol + b]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int row = ch.row0 + wid; row < ch.row1; row += nw) {
    double s = 0.0;
    if (nu > 0) {
      const double* M = bwd + nd.bwd + (long long)row * nu;
      for (int b = lane; b < nu; b += 64) s += M[b] * xu[b];
      s = wave_sum(s);
    }
    if (lane == 0) x[idx[nd.fcol + row]] = ybuf[nd.yoff + row] - s;
  }
  (void)nf;
}

// p[Omega_i] += P_i x_i (multiscale reconstruction), one workgroup per subdomain.
template <typename T>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct(const BoxDesc* __restrict__ boxes, const T* __restrict__ mbf,
                  const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                  const double* __restrict__ xc, T* __restrict__ p, int nx) {
  __shared__ T xs[64];
  const int i = blockIdx.x;
  const BoxDesc d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0, ncell = d.bx * d.by;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) xs[k] = (T)xc[k0 + k];
  __syncthreads();
  const T* P = mbf + mbf_off[i];
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % d.bx, j = q / d.bx;
    const long long c = (long long)(d.y0 + j) * nx + d.x0 + a;
    T s = p[c];
    for (int k = 0; k < nk; ++k) s += P[(long long)k * ncell + q] * xs[k];
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

// Restricted additive Schwarz: solve A[S_i] e = rho[S_i] on patch i and add
// e on the owned subdomain Omega_i (each cell is written by one patch only).
template <typename T>
__global__ void __launch_bounds__(kBoxThreads)
    k_patch(const BoxDesc* __restrict__ boxes, const T* __restrict__ dinv,
            const T* __restrict__ coup, const T* __restrict__ rho, T* __restrict__ p, int nx) {
  extern __shared__ __align__(16) char smem_raw[];
  const BoxDesc d = boxes[blockIdx.x];
  const int bx = d.bx, by = d.by, ncell = bx * by;
  T* part = reinterpret_cast<T*>(smem_raw);
  T* x = part + kBoxThreads;
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % bx, j = q / bx;
    x[q] = rho[(long long)(d.y0 + j) * nx + d.x0 + a];
  }
  __syncthreads();
  if (d.pin && threadIdx.x == 0) x[0] = T(0);
  __syncthreads();
  ldl_box_solve<T>(x, part, dinv + d.doff, coup + d.coff, bx, by);
  const int oc = d.obx * d.oby;
  for (int q = threadIdx.x; q < oc; q += blockDim.x) {
    const int a = q % d.obx, j = q / d.obx;
    const long long c = (long long)(d.y0 + d.oy + j) * nx + d.x0 + d.ox + a;
    p[c] += x[(d.oy + j) * bx + d.ox + a];
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

template <typename T>
void launch_local(const BoxDesc* boxes, int m, int max_cells, const T* dinv, const T* coup,
                  const double* r, T* p, int nx, const int* dof_off, const int* dof_side,
                  const int* w_off, const double* wU, const double* wP, double* mU, double* mP,
                  hipStream_t s) {
  const size_t shm = sizeof(T) * (size_t)(kBoxThreads + max_cells);
  hipLaunchKernelGGL(k_local<T>, dim3(m), dim3(kBoxThreads), shm, s, boxes, dinv, coup, r, p, nx,
                     dof_off, dof_side, w_off, wU, wP, mU, mP);
}

void launch_coarse_rhs(const double* mU, const double* mP, const int* rowL, const int* rowR,
                       const int* rowKind, int nc, int pin_row, double* g, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_coarse_rhs, dim3((nc + 255) / 256), dim3(256), 0, s, mU, mP, rowL, rowR,
                     rowKind, nc, pin_row, g);
}

void launch_coarse_fwd(const CChunk* chunks, int nchunks, const CNodeDesc* nodes,
                       const double* fwd, const int* idx, const int* pull_ptr,
                       const int* pull_idx, const double* g, double* ybuf, double* cbuf,
                       int max_nf, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_coarse_fwd, dim3(nchunks), dim3(kVecThreads),
                     sizeof(double) * (size_t)max_nf, s, chunks, nodes, fwd, idx, pull_ptr,
                     pull_idx, g, ybuf, cbuf);
}

void launch_coarse_bwd(const CChunk* chunks, int nchunks, const CNodeDesc* nodes,
                       const double* bwd, const int* idx, const double* ybuf, double* x,
                       int max_nu, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_coarse_bwd, dim3(nchunks), dim3(kVecThreads),
                     sizeof(double) * (size_t)(max_nu > 0 ? max_nu : 1), s, chunks, nodes, bwd,
                     idx, ybuf, x);
}

template <typename T>
void launch_reconstruct(const BoxDesc* boxes, int m, const T* mbf, const long long* mbf_off,
                        const int* dof_off, const double* xc, T* p, int nx, hipStream_t s) {
  hipLaunchKernelGGL(k_reconstruct<T>, dim3(m), dim3(kBoxThreads), 0, s, boxes, mbf, mbf_off,
                     dof_off, xc, p, nx);
}

template <typename T>
void launch_residual(const T* tx, const T* ty, int nx, int ny, const double* r, const T* p,
                     T* rho, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_residual<T>, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny,
                     r, p, rho);
}

template <typename T>
void launch_patch(const BoxDesc* boxes, int m, int max_cells, const T* dinv, const T* coup,
                  const T* rho, T* p, int nx, hipStream_t s) {
  const size_t shm = sizeof(T) * (size_t)(kBoxThreads + max_cells);
  hipLaunchKernelGGL(k_patch<T>, dim3(m), dim3(kBoxThreads), shm, s, boxes, dinv, coup, rho, p,
                     nx);
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

#define MRCM_INSTANTIATE(T)                                                                    \
  template void launch_local<T>(const BoxDesc*, int, int, const T*, const T*, const double*, T*, \
                                int, const int*, const int*, const int*, const double*,          \
                                const double*, double*, double*, hipStream_t);                   \
  template void launch_reconstruct<T>(const BoxDesc*, int, const T*, const long long*,          \
                                      const int*, const double*, T*, int, hipStream_t);         \
  template void launch_residual<T>(const T*, const T*, int, int, const double*, const T*, T*,   \
                                   hipStream_t);                                                \
  template void launch_patch<T>(const BoxDesc*, int, int, const T*, const T*, const T*, T*, int, \
                                hipStream_t);                                                   \
  template void launch_finalize<T>(const T*, long long, int, double*, double*, hipStream_t);

MRCM_INSTANTIATE(double)
MRCM_INSTANTIATE(float)

}  // namespace mrcm
