// HIP kernels of the set-up of T (Section 2.1), FP64, one wave per box or
// subdomain:
//  - k_factor_boxes: block LDL^T factorisation of a cell box by cell rows
//    with explicit inverses of the row blocks (Gauss-Jordan in LDS);
//  - k_over_mbf: the oversampled Robin problems with Legendre data on each
//    side of the oversampled box; their restrictions to Omega_i are the
//    multiscale basis functions (the local Robin problem on Omega_i with the
//    informed multiplier phi as data has exactly this solution), and their
//    flux and pressure moments on Gamma_i are the columns of the interface
//    system.
#include "device.h"
#include "setup_jobs.h"

namespace mrcm {

namespace {

__device__ __forceinline__ void wsync() { __builtin_amdgcn_wave_barrier(); }

// Stores of this work-item complete before its later loads, and the wave's
// stores are visible to the wave (workgroup scope: waits only).
__device__ __forceinline__ void wfence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Row i and column b of the flat index e = lane + 64 t of an array with n
// columns, stepped from one t to the next without a division (64 = dq n + dr).
struct FlatIndex {
  int i, b, dq, dr, n;
  __device__ FlatIndex(int lane, int n_) : n(n_) {
    i = lane / n;
    b = lane - i * n;
    dq = 64 / n;
    dr = 64 - dq * n;
  }
  __device__ void next() {
    i += dq;
    b += dr;
    if (b >= n) {
      b -= n;
      ++i;
    }
  }
};

// Robin conductance of a face leaving a cell box: 1 / (1 / (2 K_c) + b_f),
// b_f = alpha L / t_f.
__device__ __forceinline__ double robin(double Kc, double t, double aL) {
  return 1.0 / (1.0 / (2.0 * Kc) + aL / t);
}

// Legendre polynomial P_q at xi (three-term recurrence) and the face
// parameter xi_j = (2 j + 1) / n - 1.
__device__ __forceinline__ double legendre_d(int q, double xi) {
  double pm = 1.0, p = xi;
  if (q == 0) return 1.0;
  for (int k = 1; k < q; ++k) {
    const double pn = ((2.0 * k + 1.0) * xi * p - k * pm) / (k + 1.0);
    pm = p;
    p = pn;
  }
  return p;
}
__device__ __forceinline__ double xi_d(int j, int n) { return (2.0 * j + 1.0) / n - 1.0; }

// Block LDL^T factor of a box with cell rows as blocks (the form the apply
// kernels use): D_0 = A_0, D_j = A_j - T_j D_{j-1}^-1 T_j, stored as D_j^-1.
// A_j is the tridiagonal matrix of row j (Robin conductances on the box's
// faces inside the domain when robin, else the principal submatrix of A),
// T_j the vertical transmissibilities between rows j - 1 and j.  The inverse
// of each row block is taken in place by Gauss-Jordan elimination (the
// blocks are symmetric positive definite, so no pivoting); a non-positive
// pivot sets status[0] = 1.  LDS: two blocks and two vectors of maxn.
template <typename S>
__global__ void __launch_bounds__(64)
    k_factor_boxes(const FactorJob* __restrict__ jobs, int maxn, const double* __restrict__ K,
                   const double* __restrict__ tx, const double* __restrict__ ty, int nx, int ny,
                   double aL, S* __restrict__ dS, S* __restrict__ cS, double* __restrict__ d64,
                   double* __restrict__ c64, int* __restrict__ status) {
  extern __shared__ double sm[];
  const FactorJob J = jobs[blockIdx.x];
  const int n = J.bx, lane = threadIdx.x;
  const FlatIndex at0(lane, n);
  double* D = sm;
  double* P = sm + (long long)maxn * maxn;
  double* C = sm + 2LL * maxn * maxn;
  double* T = C + maxn;
  for (int j = 0; j < J.by; ++j) {
    const int y = J.y0 + j;
    for (int e = lane; e < n * n; e += 64) D[e] = 0.0;
    wsync();
    for (int a = lane; a < n; a += 64) {
      const int x = J.x0 + a;
      const long long c = (long long)y * nx + x;
      const long long fx = (long long)y * (nx + 1) + x;
      const double Kc = K[c];
      double tW = tx[fx], tE = tx[fx + 1], tS = ty[c], tN = ty[c + nx];
      if (J.robin) {
        if (a == 0 && x > 0) tW = robin(Kc, tW, aL);
        if (a == n - 1 && x + 1 < nx) tE = robin(Kc, tE, aL);
        if (j == 0 && y > 0) tS = robin(Kc, tS, aL);
        if (j == J.by - 1 && y + 1 < ny) tN = robin(Kc, tN, aL);
      }
      D[a * n + a] = tW + tE + tS + tN;
      if (a > 0) {
        D[a * n + a - 1] = -tx[fx];
        D[(a - 1) * n + a] = -tx[fx];
      }
      double tc = j > 0 ? ty[c] : 0.0;
      if (J.pin && j == 1 && a == 0) tc = 0.0;
      T[a] = tc;
      if (J.coffS >= 0) cS[J.coffS + (long long)j * n + a] = (S)tc;
      if (J.c64 >= 0) c64[J.c64 + (long long)j * n + a] = tc;
    }
    wsync();
    if (J.pin && j == 0) {
      for (int a = lane; a < n; a += 64) {
        D[a] = 0.0;
        D[a * n] = 0.0;
      }
      wsync();
      if (lane == 0) D[0] = 1.0;
      wsync();
    }
    if (j > 0) {
      FlatIndex f = at0;
      for (int e = lane; e < n * n; e += 64, f.next()) D[e] -= T[f.i] * P[e] * T[f.b];
      wsync();
    }
    for (int k = 0; k < n; ++k) {
      const double p = D[k * n + k];
      if (!(p > 0.0) || !isfinite(p)) {  // the same value in every lane
        if (lane == 0) status[0] = 1;
        return;
      }
      for (int i = lane; i < n; i += 64) C[i] = D[i * n + k];
      wsync();
      const double inv = 1.0 / p;
      for (int b = lane; b < n; b += 64) D[k * n + b] = b == k ? inv : D[k * n + b] * inv;
      wsync();
      FlatIndex f = at0;
      for (int e = lane; e < n * n; e += 64, f.next())
        if (f.i != k) D[e] = f.b == k ? -C[f.i] * inv : D[e] - C[f.i] * D[k * n + f.b];
      wsync();
    }
    if (J.d64 >= 0)
      for (int e = lane; e < n * n; e += 64) d64[J.d64 + (long long)j * n * n + e] = D[e];
    if (J.doffS >= 0) {
      // half-block layout (setup_jobs.h): row k of lane r is D(r, (r + k) mod
      // n) for k <= n / 2, halved for k = n / 2 when n is even, zero beyond
      const int rows = half_rows(J.cols), h = n / 2;
      FlatIndex f = at0;
      for (int w = lane; w < rows * n; w += 64, f.next()) {
        const int k = f.i, r = f.b;
        double v = 0.0;
        if (k <= h) {
          v = D[r * n + (r + k >= n ? r + k - n : r + k)];
          if (2 * k == n) v *= 0.5;
        }
        dS[J.doffS + (long long)j * J.bs + half_word(k, r, n, J.cols)] = (S)v;
      }
    }
    double* t = P;
    P = D;
    D = t;
  }
}

// x_k = A_box^-1 x_k for the vectors x_k = X + k * ncell, k < nrhs <= kSolveRhs,
// of one box (FP64 factor, lane r owning column r): the rows of each block
// are read once for all the vectors, and every vector sums its terms in
// column order.  ys: LDS, kSolveRhs x 64.
constexpr int kSolveRhs = 8;
__device__ void box_solve64_multi(double* X, int nrhs, long long ncell, int bx, int by,
                                  const double* __restrict__ Dinv,
                                  const double* __restrict__ coup, int pin, int lane,
                                  double (*ys)[64]) {
  const bool act = lane < bx;
  if (pin && lane == 0)
    for (int k = 0; k < nrhs; ++k) X[k * ncell] = 0.0;
  wfence();
  for (int j = 0; j < by; ++j) {
    if (act) {
      const double cj = j > 0 ? coup[(long long)j * bx + lane] : 0.0;
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k)
        if (k < nrhs) {
          const double* x = X + k * ncell;
          ys[k][lane] = x[(long long)j * bx + lane] +
                        (j > 0 ? cj * x[(long long)(j - 1) * bx + lane] : 0.0);
        }
    }
    wsync();
    if (act) {
      const double* Di = Dinv + (long long)j * bx * bx + (long long)lane * bx;
      double acc[kSolveRhs];
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k) acc[k] = 0.0;
      for (int c = 0; c < bx; ++c) {
        const double d = Di[c];
#pragma unroll
        for (int k = 0; k < kSolveRhs; ++k)
          if (k < nrhs) acc[k] += d * ys[k][c];
      }
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k)
        if (k < nrhs) X[k * ncell + (long long)j * bx + lane] = acc[k];
    }
    wsync();
  }
  for (int j = by - 2; j >= 0; --j) {
    if (act) {
      const double cn = coup[(long long)(j + 1) * bx + lane];
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k)
        if (k < nrhs) ys[k][lane] = cn * X[k * ncell + (long long)(j + 1) * bx + lane];
    }
    wsync();
    if (act) {
      const double* Di = Dinv + (long long)j * bx * bx + (long long)lane * bx;
      double acc[kSolveRhs];
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k) acc[k] = 0.0;
      for (int c = 0; c < bx; ++c) {
        const double d = Di[c];
#pragma unroll
        for (int k = 0; k < kSolveRhs; ++k)
          if (k < nrhs) acc[k] += d * ys[k][c];
      }
#pragma unroll
      for (int k = 0; k < kSolveRhs; ++k)
        if (k < nrhs) X[k * ncell + (long long)j * bx + lane] += acc[k];
    }
    wsync();
  }
  wfence();
}

// Oversampled problems of one subdomain (one right-hand side per local dof:
// its Legendre function as Robin data on its side of the oversampled box),
// solved in the scratch vectors; then
//   mbf = the solutions restricted to Omega_i (storage type), and
//   colU = sum_j P_q(xi_j) U_j,  colP = sum_j P_q(xi_j) pi_j
// over the faces of every side si of Gamma_i and mode q, with U, pi the flux
// and pressure of the oversampled solution across the face (from the cells
// on both sides, or, when the oversampled box is the subdomain box, from the
// Robin data lambda of the face: U = rho (p - lambda), pi = lambda + b U).
template <typename S>
__global__ void __launch_bounds__(64)
    k_over_mbf(const SubJob* __restrict__ subs, const OverRhs* __restrict__ rhs,
               const GamFace* __restrict__ gam, const int* __restrict__ dof_side,
               const int* __restrict__ dof_q, int over0, int nb, double* __restrict__ buf,
               S* __restrict__ mbf, double* __restrict__ colU, double* __restrict__ colP) {
  __shared__ double ys[kSolveRhs][64];
  const SubJob J = subs[blockIdx.x];
  const int lane = threadIdx.x;
  const int ncell = J.obx * J.oby;
  double* X = buf + J.oscr;
  for (long long e = lane; e < (long long)J.ni * ncell; e += 64) X[e] = 0.0;
  wfence();
  for (int e = J.rhs0 + lane; e < J.rhs1; e += 64) {
    const OverRhs R = rhs[e];
    X[(long long)R.k * ncell + R.cell] += R.val;
  }
  wfence();
  for (int k0 = 0; k0 < J.ni; k0 += kSolveRhs)
    box_solve64_multi(X + (long long)k0 * ncell, J.ni - k0 < kSolveRhs ? J.ni - k0 : kSolveRhs,
                      ncell, J.obx, J.oby, buf + J.o64, buf + J.oc64, J.opin, lane, ys);
  const int lc = J.lbx * J.lby;
  for (long long e = lane; e < (long long)J.ni * lc; e += 64) {
    const int k = (int)(e / lc), q = (int)(e - (long long)k * lc);
    const int j = q / J.lbx, a = q - j * J.lbx;
    mbf[J.mbf + e] = (S)X[(long long)k * ncell + (long long)(J.oy + j) * J.obx + J.ox + a];
  }
  const int ng = J.gam1 - J.gam0;
  const int nt = J.ni * J.nsides * nb;
  for (int e = lane; e < nt; e += 64) {
    const int k = e / (J.nsides * nb), rem = e - k * (J.nsides * nb);
    const int si = rem / nb, q = rem - si * nb;
    const int dk = J.dof0 + k;
    double su = 0.0, sp = 0.0;
    for (int f = 0; f < ng; ++f) {
      const GamFace G = gam[J.gam0 + f];
      if (G.si != si || q >= (nb < G.nfs ? nb : G.nfs)) continue;
      const double pc = X[(long long)k * ncell + G.ocin];
      double U, pi;
      if (over0) {
        const double lam =
            G.side == dof_side[dk] ? legendre_d(dof_q[dk], xi_d(G.j, G.nfs)) : 0.0;
        U = G.rho * (pc - lam);
        pi = lam + G.b * U;
      } else {
        const double pn = X[(long long)k * ncell + G.ocout];
        U = G.t * (pc - pn);
        pi = (G.Kin * pc + G.Kout * pn) / (G.Kin + G.Kout);
      }
      const double w = legendre_d(q, xi_d(G.j, G.nfs));
      su += w * U;
      sp += w * pi;
    }
    colU[J.col + e] = su;
    colP[J.col + e] = sp;
  }
}

}  // namespace

template <typename S>
void launch_factor_boxes(const FactorJob* jobs, int njobs, int maxn, const double* K,
                         const double* tx, const double* ty, int nx, int ny, double aL, S* dS,
                         S* cS, double* d64, double* c64, int* status, hipStream_t s) {
  if (njobs <= 0) return;
  const size_t shm = sizeof(double) * (2 * (size_t)maxn * maxn + 2 * (size_t)maxn);
  if (shm > 64 * 1024)  // boxes wider than 62 cells: ask for the larger LDS of gfx950
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_boxes<S>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_factor_boxes<S>, dim3(njobs), dim3(64), shm, s, jobs, maxn, K, tx, ty, nx,
                     ny, aL, dS, cS, d64, c64, status);
}

template <typename S>
void launch_over_mbf(const SubJob* subs, int m, const OverRhs* rhs, const GamFace* gam,
                     const int* dof_side, const int* dof_q, int over0, int nb, double* buf,
                     S* mbf, double* colU, double* colP, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_over_mbf<S>, dim3(m), dim3(64), 0, s, subs, rhs, gam, dof_side, dof_q,
                     over0, nb, buf, mbf, colU, colP);
}

template void launch_factor_boxes<float>(const FactorJob*, int, int, const double*, const double*,
                                         const double*, int, int, double, float*, float*, double*,
                                         double*, int*, hipStream_t);
template void launch_factor_boxes<double>(const FactorJob*, int, int, const double*,
                                          const double*, const double*, int, int, double,
                                          double*, double*, double*, double*, int*, hipStream_t);
template void launch_over_mbf<float>(const SubJob*, int, const OverRhs*, const GamFace*,
                                     const int*, const int*, int, int, double*, float*, double*,
                                     double*, hipStream_t);
template void launch_over_mbf<double>(const SubJob*, int, const OverRhs*, const GamFace*,
                                      const int*, const int*, int, int, double*, double*,
                                      double*, double*, hipStream_t);

}  // namespace mrcm
