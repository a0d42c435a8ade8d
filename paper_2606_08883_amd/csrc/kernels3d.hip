// HIP kernels of the 3-D path (include/mrcm3d.h), FP64: plane-block LDL^T
// box solves (one workgroup per box, one thread per cell of a plane), trace
// moments with tensor Legendre test functions, reconstruction, and the
// seven-point operator in its forms for smoothing and GMRES (the interface
// solve runs the level kernels of the 2-D path on the 3-D factor).  Every
// reduction has a fixed order.
#include "device3d.h"

namespace mrcm3d {

namespace {

constexpr int kVec3Threads = 256;

__device__ __forceinline__ double legendre_face3(int q, int j, int n) {
  const double xi = (2.0 * j + 1.0) / n - 1.0;
  if (q == 0) return 1.0;
  double pm = 1.0, pq = xi;
  for (int k = 1; k < q; ++k) {
    const double pn = ((2.0 * k + 1.0) * xi * pq - k * pm) / (k + 1.0);
    pm = pq;
    pq = pn;
  }
  return pq;
}

// Global cell of box-local cell q (x fastest, then y, then z).
__device__ __forceinline__ long long global_cell(const Box3& d, int q, int nx, int ny) {
  const int x = q % d.n[0], y = (q / d.n[0]) % d.n[1], z = q / (d.n[0] * d.n[1]);
  return ((long long)(d.lo[2] + z) * ny + (d.lo[1] + y)) * nx + (d.lo[0] + x);
}

// sum_c D(t, c) v[c] for a block in cyclic-diagonal storage (word d P + t
// holds D(t, (t + d) mod P), d < P / 2 + 1): diagonal d gives D(t, t + d)
// v[t + d] from word d P + t and, unless 2 d = P, D(t - d, t) v[t - d] from
// word d P + t - d, indices mod P.  Consecutive threads read consecutive
// words of one diagonal in both terms, so each stored word comes from HBM
// once.  Odd and even d in separate sums, added as (even up + odd up) +
// (even down + odd down): the host solve's order.
template <typename S>
__device__ __forceinline__ double plane_dot(const S* __restrict__ D, const double* v, int P,
                                            int t) {
  const int H = P / 2 + 1;
  double u0 = (double)D[t] * v[t], u1 = 0.0, w0 = 0.0, w1 = 0.0;
  // kU diagonals per pass, every load of the pass issued before its
  // multiply-adds (eight for FP32 blocks, which leave the loop latency-bound;
  // two for FP64, where four and eight measured slower); d starts odd, so
  // diagonal d + q is odd for even q.  Only the diagonal d = P / 2 of an
  // even P has no second term, and it is the last: the passes stop before
  // it, so their loop holds no branch (a branch there made every pass wait
  // for all of its loads).
  constexpr int kU = sizeof(S) == 4 ? 8 : 2;
  const int Hd = P % 2 == 0 ? P / 2 : H;  // diagonals 1 .. Hd - 1 have both terms
  int d = 1;
  for (; d + kU <= Hd; d += kU) {
    double a[kU], b[kU], x[kU], y[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      int up = t + d + q, dn = t - d - q;
      if (up >= P) up -= P;
      if (dn < 0) dn += P;
      const S* row = D + (long long)(d + q) * P;
      a[q] = row[t];
      b[q] = row[dn];
      x[q] = v[up];
      y[q] = v[dn];
    }
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      double& u = q & 1 ? u0 : u1;
      double& w = q & 1 ? w0 : w1;
      u = fma(a[q], x[q], u);
      w = fma(b[q], y[q], w);
    }
  }
  for (; d < H; ++d) {
    int up = t + d, dn = t - d;
    if (up >= P) up -= P;
    if (dn < 0) dn += P;
    const S* row = D + (long long)d * P;
    double& u = d & 1 ? u1 : u0;
    double& w = d & 1 ? w1 : w0;
    u = fma((double)row[t], v[up], u);
    if (2 * d != P) w = fma((double)row[dn], v[dn], w);
  }
  return (u0 + u1) + (w0 + w1);
}

// Block LDL^T solve of the box in LDS: us holds b on entry and x on exit in
// planes stop .. bz - 1 (planes below keep their forward values).
template <typename S>
__device__ __forceinline__ void plane_solve(double* us, double* v, const Box3& d,
                                            const S* __restrict__ dinv,
                                            const double* __restrict__ coup, int stop) {
  const int P = d.P, bz = d.n[2], t = threadIdx.x;
  const long long HP = (long long)(P / 2 + 1) * P;  // words of one stored block
  const S* D = dinv + d.doff;
  const double* T = coup + d.coff;
  for (int j = 0; j < bz; ++j) {
    if (t < P) v[t] = j > 0 ? fma(T[(long long)j * P + t], us[(j - 1) * P + t], us[j * P + t])
                            : us[j * P + t];
    __syncthreads();
    if (t < P) us[j * P + t] = plane_dot(D + j * HP, v, P, t);
    __syncthreads();
  }
  for (int j = bz - 2; j >= stop; --j) {
    if (t < P) v[t] = T[(long long)(j + 1) * P + t] * us[(j + 1) * P + t];
    __syncthreads();
    if (t < P) us[j * P + t] += plane_dot(D + j * HP, v, P, t);
    __syncthreads();
  }
}

// LDS: us[cells] | v[P].  S: the storage type of the plane blocks (FP64 or
// FP32); the arithmetic is FP64.
template <typename S>
__global__ void __launch_bounds__(kBox3Threads)
    k_local3(const Box3* __restrict__ boxes, const S* __restrict__ dinv,
             const double* __restrict__ coup, const double* __restrict__ r,
             double* __restrict__ p, int nx, int ny, const int* __restrict__ dof_off,
             const Dof3* __restrict__ dofs, const int* __restrict__ fin,
             const int* __restrict__ fout, const double* __restrict__ fw,
             double* __restrict__ mU, double* __restrict__ mP) {
  extern __shared__ double sm3[];
  const int i = blockIdx.x;
  const Box3 d = boxes[i];
  const int cells = d.P * d.n[2];
  double* us = sm3;
  double* v = sm3 + cells;
  for (int q = threadIdx.x; q < cells; q += blockDim.x) us[q] = r[global_cell(d, q, nx, ny)];
  __syncthreads();
  if (d.pin && threadIdx.x == 0) us[0] = 0.0;
  __syncthreads();
  plane_solve(us, v, d, dinv, coup, d.olo[2] > 0 ? d.olo[2] - 1 : 0);
  // p on the owned cells
  const int oc = d.on[0] * d.on[1] * d.on[2];
  for (int q = threadIdx.x; q < oc; q += blockDim.x) {
    const int x = q % d.on[0], y = (q / d.on[0]) % d.on[1], z = q / (d.on[0] * d.on[1]);
    const int lq = ((d.olo[2] + z) * d.n[1] + d.olo[1] + y) * d.n[0] + d.olo[0] + x;
    p[global_cell(d, lq, nx, ny)] = us[lq];
  }
  // trace moments of every dof of the subdomain
  for (int k = dof_off[i] + threadIdx.x; k < dof_off[i + 1]; k += blockDim.x) {
    const Dof3 q = dofs[k];
    double su = 0.0, sp = 0.0;
    for (int f = 0; f < q.nf; ++f) {
      const int ff = q.f0 + f;
      const double pin = us[fin[ff]], pout = us[fout[ff]];
      const double bv = legendre_face3(q.a, f % q.n0, q.n0) * legendre_face3(q.b, f / q.n0, q.n1);
      const double U = fma(fw[4LL * ff + 1], pout, fw[4LL * ff] * pin);
      const double Pi = fma(fw[4LL * ff + 3], pout, fw[4LL * ff + 2] * pin);
      su = fma(bv, U, su);
      sp = fma(bv, Pi, sp);
    }
    mU[k] = su;
    mP[k] = sp;
  }
}

template <typename S>
__global__ void __launch_bounds__(kBox3Threads)
    k_patch3(const Box3* __restrict__ boxes, const S* __restrict__ dinv,
             const double* __restrict__ coup, const double* __restrict__ rho,
             double* __restrict__ p, int nx, int ny) {
  extern __shared__ double sm3[];
  const Box3 d = boxes[blockIdx.x];
  const int cells = d.P * d.n[2];
  double* us = sm3;
  double* v = sm3 + cells;
  for (int q = threadIdx.x; q < cells; q += blockDim.x) us[q] = rho[global_cell(d, q, nx, ny)];
  __syncthreads();
  if (d.pin && threadIdx.x == 0) us[0] = 0.0;
  __syncthreads();
  plane_solve(us, v, d, dinv, coup, d.olo[2]);
  const int oc = d.on[0] * d.on[1] * d.on[2];
  for (int q = threadIdx.x; q < oc; q += blockDim.x) {
    const int x = q % d.on[0], y = (q / d.on[0]) % d.on[1], z = q / (d.on[0] * d.on[1]);
    const int lq = ((d.olo[2] + z) * d.n[1] + d.olo[1] + y) * d.n[0] + d.olo[0] + x;
    const long long c = global_cell(d, lq, nx, ny);
    p[c] += us[lq];
  }
}

__device__ __forceinline__ double wave_sum3(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kBox3Threads)
    k_reconstruct3(const Box3* __restrict__ boxes, const double* __restrict__ mbf,
                   const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                   const double* __restrict__ x, double* __restrict__ p, int nx, int ny) {
  const int i = blockIdx.x;
  const Box3 d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0;
  const int oc = d.on[0] * d.on[1] * d.on[2];
  const double* Pm = mbf + mbf_off[i];
  for (int q = threadIdx.x; q < oc; q += blockDim.x) {
    const int xx = q % d.on[0], y = (q / d.on[0]) % d.on[1], z = q / (d.on[0] * d.on[1]);
    const int lq = ((d.olo[2] + z) * d.n[1] + d.olo[1] + y) * d.n[0] + d.olo[0] + xx;
    const long long c = global_cell(d, lq, nx, ny);
    double s = p[c];
    for (int k = 0; k < nk; ++k) s = fma(Pm[(long long)k * oc + q], x[k0 + k], s);
    p[c] = s;
  }
}

// The seven-point stencil at cell c: sum over the faces of t_f (x_c - x_c'),
// boundary faces coupled to zero.
__device__ __forceinline__ double stencil3(const double* __restrict__ tx,
                                           const double* __restrict__ ty,
                                           const double* __restrict__ tz, int nx, int ny, int nz,
                                           long long c, const double* __restrict__ x) {
  const int ix = (int)(c % nx), iy = (int)((c / nx) % ny), iz = (int)(c / ((long long)nx * ny));
  const long long fx = ((long long)iz * ny + iy) * (nx + 1) + ix;
  const long long fy = ((long long)iz * (ny + 1) + iy) * nx + ix;
  const long long fz = ((long long)iz * ny + iy) * nx + ix;
  const double tW = tx[fx], tE = tx[fx + 1], tS = ty[fy], tN = ty[fy + nx], tB = tz[fz],
               tT = tz[fz + (long long)nx * ny];
  const double xc = x[c];
  double v = (tW + tE + tS + tN + tB + tT) * xc;
  if (ix > 0) v -= tW * x[c - 1];
  if (ix + 1 < nx) v -= tE * x[c + 1];
  if (iy > 0) v -= tS * x[c - nx];
  if (iy + 1 < ny) v -= tN * x[c + nx];
  if (iz > 0) v -= tB * x[c - (long long)nx * ny];
  if (iz + 1 < nz) v -= tT * x[c + (long long)nx * ny];
  return v;
}

__global__ void __launch_bounds__(kVec3Threads)
    k_op3(const double* __restrict__ tx, const double* __restrict__ ty,
          const double* __restrict__ tz, int nx, int ny, int nz, const double* __restrict__ x,
          double* __restrict__ y, const double* __restrict__ r, int mode) {
  const long long n = (long long)nx * ny * nz;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const double a = stencil3(tx, ty, tz, nx, ny, nz, c, x);
    y[c] = mode == 0 ? a : r[c] - a;
  }
}

__device__ __forceinline__ double block_sum3(double v, double* red) {
  v = wave_sum3(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// mode 0: w = A z, partials of w . v0 (v0 = aux); mode 1: r = b - A p (b when
// p is NULL; b = aux), partials of r^2.
__global__ void __launch_bounds__(kVec3Threads)
    k_op_reduce3(const double* __restrict__ tx, const double* __restrict__ ty,
                 const double* __restrict__ tz, int nx, int ny, int nz,
                 const double* __restrict__ x, double* __restrict__ out,
                 const double* __restrict__ aux, double* __restrict__ partials, int mode) {
  __shared__ double red[kVec3Threads / 64];
  const long long n = (long long)nx * ny * nz;
  double s = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    if (mode == 0) {
      const double w = stencil3(tx, ty, tz, nx, ny, nz, c, x);
      out[c] = w;
      s = fma(w, aux[c], s);
    } else {
      const double rr = x ? aux[c] - stencil3(tx, ty, tz, nx, ny, nz, c, x) : aux[c];
      out[c] = rr;
      s = fma(rr, rr, s);
    }
  }
  s = block_sum3(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// b = f h^2 plus t_f g_f on every Dirichlet boundary face (t_f = 2 K_c
// there), sides in the order W, E, S, N, B, T; g: the six sides' face values
// concatenated (W, E: z ny + y; S, N: z nx + x; B, T: y nx + x).
__global__ void __launch_bounds__(kVec3Threads)
    k_rhs3(const double* __restrict__ tx, const double* __restrict__ ty,
           const double* __restrict__ tz, int nx, int ny, int nz, int bcmask,
           const double* __restrict__ f, const double* __restrict__ g, double h,
           double* __restrict__ b) {
  const long long n = (long long)nx * ny * nz;
  const long long oW = 0, oE = (long long)ny * nz, oS = 2LL * ny * nz,
                  oN = oS + (long long)nx * nz, oB = oN + (long long)nx * nz,
                  oT = oB + (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(c % nx), iy = (int)((c / nx) % ny), iz = (int)(c / ((long long)nx * ny));
    double v = f ? f[c] * h * h : 0.0;
    if (g) {
      const long long fx = ((long long)iz * ny + iy) * (nx + 1) + ix;
      const long long fy = ((long long)iz * (ny + 1) + iy) * nx + ix;
      const long long fz = ((long long)iz * ny + iy) * nx + ix;
      if (ix == 0 && (bcmask & 1)) v += tx[fx] * g[oW + (long long)iz * ny + iy];
      if (ix == nx - 1 && (bcmask & 2)) v += tx[fx + 1] * g[oE + (long long)iz * ny + iy];
      if (iy == 0 && (bcmask & 4)) v += ty[fy] * g[oS + (long long)iz * nx + ix];
      if (iy == ny - 1 && (bcmask & 8)) v += ty[fy + nx] * g[oN + (long long)iz * nx + ix];
      if (iz == 0 && (bcmask & 16)) v += tz[fz] * g[oB + (long long)iy * nx + ix];
      if (iz == nz - 1 && (bcmask & 32))
        v += tz[fz + (long long)nx * ny] * g[oT + (long long)iy * nx + ix];
    }
    b[c] = v;
  }
}

inline int grid3(long long n) {
  long long b = (n + kVec3Threads - 1) / kVec3Threads;
  return (int)(b < 1 ? 1 : b > 4096 ? 4096 : b);
}

}  // namespace

// Threads of a box launch: one per cell of the widest plane, whole waves.
inline int box3_threads(int max_plane) { return (max_plane + 63) / 64 * 64; }

template <typename S>
void launch_local3(const Box3* boxes, int m, int max_cells, int max_plane, const S* dinv,
                   const double* coup, const double* r, double* p, int nx, int ny,
                   const int* dof_off, const Dof3* dofs, const int* fin, const int* fout,
                   const double* fw, double* mU, double* mP, hipStream_t s) {
  if (m <= 0) return;
  const size_t shm = sizeof(double) * (max_cells + max_plane);
  hipLaunchKernelGGL(k_local3<S>, dim3(m), dim3(box3_threads(max_plane)), shm, s, boxes, dinv,
                     coup, r, p, nx, ny, dof_off, dofs, fin, fout, fw, mU, mP);
}
template <typename S>
void launch_patch3(const Box3* boxes, int m, int max_cells, int max_plane, const S* dinv,
                   const double* coup, const double* rho, double* p, int nx, int ny,
                   hipStream_t s) {
  if (m <= 0) return;
  const size_t shm = sizeof(double) * (max_cells + max_plane);
  hipLaunchKernelGGL(k_patch3<S>, dim3(m), dim3(box3_threads(max_plane)), shm, s, boxes, dinv,
                     coup, rho, p, nx, ny);
}
#define MRCM3D_INSTANTIATE(S)                                                                  \
  template void launch_local3<S>(const Box3*, int, int, int, const S*, const double*,          \
                                 const double*, double*, int, int, const int*, const Dof3*,    \
                                 const int*, const int*, const double*, double*, double*,      \
                                 hipStream_t);                                                 \
  template void launch_patch3<S>(const Box3*, int, int, int, const S*, const double*,          \
                                 const double*, double*, int, int, hipStream_t);
MRCM3D_INSTANTIATE(double)
MRCM3D_INSTANTIATE(float)
#undef MRCM3D_INSTANTIATE
void launch_reconstruct3(const Box3* boxes, int m, const double* mbf, const long long* mbf_off,
                         const int* dof_off, const double* x, double* p, int nx, int ny,
                         hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_reconstruct3, dim3(m), dim3(kBox3Threads), 0, s, boxes, mbf, mbf_off,
                     dof_off, x, p, nx, ny);
}
void launch_op3(const double* tx, const double* ty, const double* tz, int nx, int ny, int nz,
                const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_op3, dim3(grid3((long long)nx * ny * nz)), dim3(kVec3Threads), 0, s, tx,
                     ty, tz, nx, ny, nz, x, y, (const double*)nullptr, 0);
}
void launch_residual3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                      int nz, const double* r, const double* p, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_op3, dim3(grid3((long long)nx * ny * nz)), dim3(kVec3Threads), 0, s, tx,
                     ty, tz, nx, ny, nz, p, rho, r, 1);
}
void launch_rhs3(const double* tx, const double* ty, const double* tz, int nx, int ny, int nz,
                 int bcmask, const double* f, const double* g, double h, double* b,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_rhs3, dim3(grid3((long long)nx * ny * nz)), dim3(kVec3Threads), 0, s, tx,
                     ty, tz, nx, ny, nz, bcmask, f, g, h, b);
}
void launch_arnoldi_start3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                           int nz, const double* z, double* w, const double* v0,
                           double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_op_reduce3, dim3(nb), dim3(kVec3Threads), 0, s, tx, ty, tz, nx, ny, nz, z,
                     w, v0, partials, 0);
}
void launch_resid_norm3(const double* tx, const double* ty, const double* tz, int nx, int ny,
                        int nz, const double* b, const double* p, double* r, double* partials,
                        int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_op_reduce3, dim3(nb), dim3(kVec3Threads), 0, s, tx, ty, tz, nx, ny, nz, p,
                     r, b, partials, 1);
}

}  // namespace mrcm3d
