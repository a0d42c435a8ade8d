// Nested-dissection multifrontal factorisation of the interface system and a
// host reference of its level-scheduled solve (the GPU solve is in
// kernels.hip).  See coarse.h for the structure.  The dissection is four-way:
// a region of the subdomain grid is split by a cross of subdomains into four
// quadrants (by a line into two halves when it is thinner than three
// subdomains), so the tree has about half the levels of a two-way dissection
// and the solve half the dependent launches, at the price of larger fronts
// near the root (bytes, which cost less than launch latency there).
#include "coarse.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <functional>

namespace mrcm {

namespace {

constexpr int kLeafArea = 16;  // boxes of at most this many subdomains are eliminated whole


// C rows [i0, i1) = alpha * A * B + beta * C (row-major, k inner terms).  A 4 x 16
// tile of C is held in registers across the whole sum; every element adds its
// terms in p order, one fused multiply-add each, as the plain triple loop
// would.  Built for AVX-512, AVX2 and baseline x86-64, picked at run time.
__attribute__((target_clones("avx512f", "avx2", "default")))
void gemm_rows(int i0, int i1, int n, int k, double alpha, const double* __restrict__ A, int lda,
               const double* __restrict__ B, int ldb, double beta, double* __restrict__ C,
               int ldc) {
  constexpr int TR = 4, TC = 16;
  for (int i = i0; i < i1; i += TR) {
    const int nr = std::min(TR, i1 - i);
    for (int j = 0; j < n; j += TC) {
      const int nc = std::min(TC, n - j);
      if (nr == TR && nc == TC) {
        double acc[TR][TC];
        for (int r = 0; r < TR; ++r)
          for (int c = 0; c < TC; ++c) {
            const double v = C[(size_t)(i + r) * ldc + j + c];
            acc[r][c] = beta == 0.0 ? 0.0 : beta == 1.0 ? v : v * beta;
          }
        for (int q = 0; q < k; ++q) {
          const double* b = B + (size_t)q * ldb + j;
          double av[TR];
          for (int r = 0; r < TR; ++r) av[r] = alpha * A[(size_t)(i + r) * lda + q];
          if (av[0] == 0.0 && av[1] == 0.0 && av[2] == 0.0 && av[3] == 0.0) continue;
          for (int r = 0; r < TR; ++r)
            for (int c = 0; c < TC; ++c) acc[r][c] = std::fma(av[r], b[c], acc[r][c]);
        }
        for (int r = 0; r < TR; ++r)
          for (int c = 0; c < TC; ++c) C[(size_t)(i + r) * ldc + j + c] = acc[r][c];
      } else {
        for (int r = 0; r < nr; ++r) {
          double* cr = C + (size_t)(i + r) * ldc + j;
          for (int c = 0; c < nc; ++c)
            cr[c] = beta == 0.0 ? 0.0 : beta == 1.0 ? cr[c] : cr[c] * beta;
          for (int q = 0; q < k; ++q) {
            const double av = alpha * A[(size_t)(i + r) * lda + q];
            if (av == 0.0) continue;
            const double* b = B + (size_t)q * ldb + j;
            for (int c = 0; c < nc; ++c) cr[c] = std::fma(av, b[c], cr[c]);
          }
        }
      }
    }
  }
}

// C (m x n) = alpha * A (m x k) * B (k x n) + beta * C, row-major; nth OpenMP
// threads over blocks of rows when the product is large and no parallel
// region is active.
void gemm(int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
          double beta, double* C, int ldc, int nth) {
  const bool par = !omp_in_parallel() && (double)m * n * k > 2e6;
  const int nblk = (m + 15) / 16;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth) if (par)
  for (int bi = 0; bi < nblk; ++bi)
    gemm_rows(16 * bi, std::min(m, 16 * bi + 16), n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

// X := U^-1 L^-1 X for the columns [c0, c1) of X (n x n, row-major), with L
// the unit lower and U the upper triangle of A (the LU factor), blocked by 64
// rows: each row block first takes the product of the rows already solved
// through gemm_rows (columns before the block in the forward substitution,
// after it in the backward one), then substitutes within the block.
__attribute__((target_clones("avx512f", "avx2", "default")))
void lu_solve_cols(const double* __restrict__ A, int n, double* __restrict__ X, int c0, int c1) {
  constexpr int RB = 64;
  const int w = c1 - c0;
  for (int b0 = 0; b0 < n; b0 += RB) {
    const int b1 = std::min(n, b0 + RB);
    if (b0 > 0)
      gemm_rows(0, b1 - b0, w, b0, -1.0, A + (size_t)b0 * n, n, X + c0, n, 1.0,
                X + (size_t)b0 * n + c0, n);
    for (int i = b0 + 1; i < b1; ++i) {
      double* xi = X + (size_t)i * n + c0;
      for (int j = b0; j < i; ++j) {
        const double l = A[(size_t)i * n + j];
        if (l == 0.0) continue;
        const double* xj = X + (size_t)j * n + c0;
        for (int c = 0; c < w; ++c) xi[c] = std::fma(-l, xj[c], xi[c]);
      }
    }
  }
  for (int b1 = n; b1 > 0; b1 -= RB) {
    const int b0 = std::max(0, b1 - RB);
    if (b1 < n)
      gemm_rows(0, b1 - b0, w, n - b1, -1.0, A + (size_t)b0 * n + b1, n, X + (size_t)b1 * n + c0,
                n, 1.0, X + (size_t)b0 * n + c0, n);
    for (int i = b1 - 1; i >= b0; --i) {
      double* xi = X + (size_t)i * n + c0;
      for (int j = i + 1; j < b1; ++j) {
        const double u = A[(size_t)i * n + j];
        if (u == 0.0) continue;
        const double* xj = X + (size_t)j * n + c0;
        for (int c = 0; c < w; ++c) xi[c] = std::fma(-u, xj[c], xi[c]);
      }
      const double d = A[(size_t)i * n + i];
      for (int c = 0; c < w; ++c) xi[c] /= d;
    }
  }
}

// Inverse of a dense n x n row-major matrix by LU with partial pivoting, nth
// OpenMP threads in its loops.  Returns the smallest |pivot| / max|A| ratio
// (0 when singular).  The factorisation is blocked by panels of kPanel
// columns: each panel is factored with row pivoting over the whole column
// (full rows swapped), the panel's rows of U to its right are formed by the
// unit-lower panel, and the trailing matrix takes the panel's rank-kPanel
// update through gemm.  The pivots are those of the unblocked elimination;
// every trailing entry receives its updates in the same order of k.
double lu_inverse(std::vector<double>& A, int n, std::vector<double>& inv, int nth) {
  constexpr int kPanel = 64;
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  double ratio = 1.0;
  for (int k0 = 0; k0 < n; k0 += kPanel) {
    const int k1 = std::min(n, k0 + kPanel);
    for (int k = k0; k < k1; ++k) {
      int p = k;
      double best = std::fabs(A[(size_t)k * n + k]);
      for (int i = k + 1; i < n; ++i)
        if (std::fabs(A[(size_t)i * n + k]) > best) {
          best = std::fabs(A[(size_t)i * n + k]);
          p = i;
        }
      if (!(best > 0.0) || !std::isfinite(best)) return 0.0;
      ratio = std::min(ratio, best / amax);
      if (p != k) {
        for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        std::swap(perm[k], perm[p]);
      }
      const double piv = A[(size_t)k * n + k];
      // the multipliers of column k and the update of the panel's columns
      const bool par = !omp_in_parallel() && (double)(n - k) * (k1 - k) > 2e5;
#pragma omp parallel for schedule(static) num_threads(nth) if (par)
      for (int i = k + 1; i < n; ++i) {
        double l = A[(size_t)i * n + k] / piv;
        A[(size_t)i * n + k] = l;
        if (l == 0.0) continue;
        for (int j = k + 1; j < k1; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
      }
    }
    if (k1 == n) break;
    // the panel's rows of U right of the panel: unit-lower panel solve
    const int nt = n - k1;
    const bool par = !omp_in_parallel() && (double)nt * (k1 - k0) * (k1 - k0) > 2e5;
#pragma omp parallel for schedule(static) num_threads(nth) if (par)
    for (int jb = 0; jb < nt; jb += 64) {
      const int j0 = k1 + jb, j1 = std::min(n, j0 + 64);
      for (int k = k0; k < k1; ++k)
        for (int i = k + 1; i < k1; ++i) {
          const double l = A[(size_t)i * n + k];
          if (l == 0.0) continue;
          for (int j = j0; j < j1; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    // trailing update A22 -= L21 U12
    gemm(nt, nt, k1 - k0, -1.0, &A[(size_t)k1 * n + k0], n, &A[(size_t)k0 * n + k1], n, 1.0,
         &A[(size_t)k1 * n + k1], n, nth);
  }
  // inv = U^-1 L^-1 P: the permuted identity, solved a block of columns at a
  // time
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + perm[i]] = 1.0;
  const int nblk = (n + 63) / 64;
  const bool par = !omp_in_parallel() && n > 64;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth) if (par)
  for (int bi = 0; bi < nblk; ++bi)
    lu_solve_cols(A.data(), n, inv.data(), 64 * bi, std::min(n, 64 * bi + 64));
  return ratio;
}

}  // namespace

CoarseFactor coarse_factor(const Maps& M, const std::vector<int>& rp, const std::vector<int>& ci,
                           const std::vector<double>& cv, int nthreads) {
  const int nc = M.nc();
  if (nc == 0) {
    CoarseFactor F;
    return F;
  }
  // rows owned by each subdomain: flux rows -> L, pressure rows -> R
  std::vector<std::vector<int>> rows_of(M.m);
  for (int r = 0; r < nc; ++r) {
    const auto& e = M.edges[M.rows[r][0]];
    rows_of[M.rows[r][1] == 0 ? e[0] : e[1]].push_back(r);
  }
  // nested dissection on the mx x my subdomain grid
  std::vector<DissectionNode> tree;
  std::function<int(int, int, int, int, int)> build = [&](int x0, int x1, int y0, int y1,
                                                          int depth) -> int {
    if (x0 >= x1 || y0 >= y1) return -1;
    DissectionNode nd;
    nd.depth = depth;
    if ((x1 - x0) * (y1 - y0) <= kLeafArea) {
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) nd.fsub.push_back(y * M.mx + x);
    } else if (x1 - x0 >= 3 && y1 - y0 >= 3) {
      // a cross of subdomains (one column and one row) splits the region
      // into four quadrants, which couple only through it (the interface
      // system has the five-point pattern of the subdomain grid)
      const int xm = (x0 + x1) / 2, ym = (y0 + y1) / 2;
      for (int k = 0; k < 4; ++k) {
        const int c = build(k & 1 ? xm + 1 : x0, k & 1 ? x1 : xm, k & 2 ? ym + 1 : y0,
                            k & 2 ? y1 : ym, depth + 1);
        if (c >= 0) nd.children.push_back(c);
      }
      for (int y = y0; y < y1; ++y) nd.fsub.push_back(y * M.mx + xm);
      for (int x = x0; x < x1; ++x)
        if (x != xm) nd.fsub.push_back(ym * M.mx + x);
    } else if (x1 - x0 >= y1 - y0) {
      const int xm = (x0 + x1) / 2;
      int a = build(x0, xm, y0, y1, depth + 1), b = build(xm + 1, x1, y0, y1, depth + 1);
      if (a >= 0) nd.children.push_back(a);
      if (b >= 0) nd.children.push_back(b);
      for (int y = y0; y < y1; ++y) nd.fsub.push_back(y * M.mx + xm);
    } else {
      const int ym = (y0 + y1) / 2;
      int a = build(x0, x1, y0, ym, depth + 1), b = build(x0, x1, ym + 1, y1, depth + 1);
      if (a >= 0) nd.children.push_back(a);
      if (b >= 0) nd.children.push_back(b);
      for (int x = x0; x < x1; ++x) nd.fsub.push_back(ym * M.mx + x);
    }
    for (int y = y0; y < y1; ++y) {
      if (x0 > 0) nd.usub.push_back(y * M.mx + x0 - 1);
      if (x1 < M.mx) nd.usub.push_back(y * M.mx + x1);
    }
    for (int x = x0; x < x1; ++x) {
      if (y0 > 0) nd.usub.push_back((y0 - 1) * M.mx + x);
      if (y1 < M.my) nd.usub.push_back(y1 * M.mx + x);
    }
    std::sort(nd.usub.begin(), nd.usub.end());
    tree.push_back(nd);
    return (int)tree.size() - 1;
  };
  build(0, M.mx, 0, M.my, 0);
  return coarse_factor_tree(tree, rows_of, M.dof_offset, rp, ci, cv, nthreads);
}

CoarseFactor coarse_factor_tree(const std::vector<DissectionNode>& tree,
                                const std::vector<std::vector<int>>& rows_of,
                                const std::vector<int32_t>& dof_offset,
                                const std::vector<int>& rp, const std::vector<int>& ci,
                                const std::vector<double>& cv, int nthreads) {
  CoarseFactor F;
  const int nc = dof_offset.empty() ? 0 : dof_offset.back();
  F.nc = nc;
  if (nc == 0) return F;
  for (size_t i = 0; i + 1 < dof_offset.size(); ++i)
    if ((int)rows_of[i].size() != dof_offset[i + 1] - dof_offset[i])
      throw Error(MRCM_EINVAL, "coarse row ownership is not square");
  const int nn = (int)tree.size();
  F.nodes.resize(nn);
  int maxdepth = 0;
  for (int t = 0; t < nn; ++t) {
    CoarseNode& cn = F.nodes[t];
    cn.depth = tree[t].depth;
    maxdepth = std::max(maxdepth, cn.depth);
    for (int s : tree[t].fsub) {
      cn.frow.insert(cn.frow.end(), rows_of[s].begin(), rows_of[s].end());
      for (int k = dof_offset[s]; k < dof_offset[s + 1]; ++k) cn.fcol.push_back(k);
    }
    for (int s : tree[t].usub) {
      cn.urow.insert(cn.urow.end(), rows_of[s].begin(), rows_of[s].end());
      for (int k = dof_offset[s]; k < dof_offset[s + 1]; ++k) cn.ucol.push_back(k);
    }
  }
  F.depth = maxdepth;
  // row equilibration: every row of C scaled to unit max-norm (the solve scales
  // g the same way), so pivot tests do not depend on the units of flux and
  // pressure rows, which differ by the permeability contrast
  F.rscale.assign(nc, 1.0);
  std::vector<double> cvs(cv);
  for (int r = 0; r < nc; ++r) {
    double mx = 0.0;
    for (int q = rp[r]; q < rp[r + 1]; ++q) mx = std::max(mx, std::fabs(cv[q]));
    if (!(mx > 0.0)) throw Error(MRCM_ESINGULAR, "zero row in the interface system");
    F.rscale[r] = 1.0 / mx;
    for (int q = rp[r]; q < rp[r + 1]; ++q) cvs[q] = cv[q] * F.rscale[r];
  }
  // factor level by level, deepest first; update matrices are passed to parents
  std::vector<std::vector<double>> update(nn);
  std::vector<std::vector<int>> by_depth(maxdepth + 1);
  for (int t = 0; t < nn; ++t) by_depth[F.nodes[t].depth].push_back(t);
  double min_ratio = 1.0;
  int failed = 0;
  for (int d = maxdepth; d >= 0; --d) {
    const auto& lvl = by_depth[d];
    // a level with fewer nodes than threads runs its nodes one at a time,
    // each with parallel dense kernels
    const bool par_nodes = (int)lvl.size() >= std::max(2, nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) if (par_nodes)
    for (int li = 0; li < (int)lvl.size(); ++li) {
      const int t = lvl[li];
      CoarseNode& cn = F.nodes[t];
      const int nf = (int)cn.frow.size(), nu = (int)cn.urow.size(), nt = nf + nu;
      // local positions of the front's rows and columns (-1: not in the front)
      static thread_local std::vector<int> rpos, cpos;
      if ((int)rpos.size() < nc) {
        rpos.assign(nc, -1);
        cpos.assign(nc, -1);
      }
      for (int a = 0; a < nf; ++a) {
        rpos[cn.frow[a]] = a;
        cpos[cn.fcol[a]] = a;
      }
      for (int a = 0; a < nu; ++a) {
        rpos[cn.urow[a]] = nf + a;
        cpos[cn.ucol[a]] = nf + a;
      }
      std::vector<double> Fm((size_t)nt * nt, 0.0);
      for (int a = 0; a < nt; ++a) {
        const int r = a < nf ? cn.frow[a] : cn.urow[a - nf];
        for (int q = rp[r]; q < rp[r + 1]; ++q) {
          const int b = cpos[ci[q]];
          if (b < 0) continue;
          if (a >= nf && b >= nf) continue;  // both later: assembled at an ancestor
          Fm[(size_t)a * nt + b] += cvs[q];
        }
      }
      for (int ch : tree[t].children) {
        const CoarseNode& cc = F.nodes[ch];
        const int cu = (int)cc.urow.size();
        std::vector<int> ra(cu), cb(cu);
        for (int u = 0; u < cu; ++u) {
          ra[u] = rpos[cc.urow[u]];
          cb[u] = cpos[cc.ucol[u]];
        }
        const std::vector<double>& S = update[ch];
        for (int u = 0; u < cu; ++u)
          for (int v = 0; v < cu; ++v) Fm[(size_t)ra[u] * nt + cb[v]] += S[(size_t)u * cu + v];
        update[ch].clear();
        update[ch].shrink_to_fit();
      }
      for (int a = 0; a < nf; ++a) rpos[cn.frow[a]] = cpos[cn.fcol[a]] = -1;
      for (int a = 0; a < nu; ++a) rpos[cn.urow[a]] = cpos[cn.ucol[a]] = -1;
      std::vector<double> Aff((size_t)nf * nf), Winv;
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) Aff[(size_t)a * nf + b] = Fm[(size_t)a * nt + b];
      const double ratio = lu_inverse(Aff, nf, Winv, nthreads);
      if (!(ratio > 0.0)) {  // exact zero or non-finite pivot
#pragma omp atomic write
        failed = 1;
        continue;
      }
#pragma omp critical
      min_ratio = std::min(min_ratio, ratio);
      cn.fwd.assign((size_t)nt * nf, 0.0);
      std::copy(Winv.begin(), Winv.end(), cn.fwd.begin());
      if (nu > 0) {
        // E = A_UF Winv
        gemm(nu, nf, nf, 1.0, &Fm[(size_t)nf * nt], nt, Winv.data(), nf, 0.0,
             &cn.fwd[(size_t)nf * nf], nf, nthreads);
        // G = Winv A_FU
        cn.bwd.assign((size_t)nf * nu, 0.0);
        gemm(nf, nu, nf, 1.0, Winv.data(), nf, &Fm[nf], nt, 0.0, cn.bwd.data(), nu, nthreads);
        // S = A_UU - A_UF G
        std::vector<double> S((size_t)nu * nu);
        for (int a = 0; a < nu; ++a)
          for (int b = 0; b < nu; ++b) S[(size_t)a * nu + b] = Fm[(size_t)(nf + a) * nt + nf + b];
        gemm(nu, nu, nf, -1.0, &Fm[(size_t)nf * nt], nt, cn.bwd.data(), nu, 1.0, S.data(), nu,
             nthreads);
        update[t] = std::move(S);
      }
    }
    if (failed) throw Error(MRCM_ESINGULAR, "singular block in the interface system");
  }
  F.min_pivot_ratio = min_ratio;
  // buffer offsets and pull lists
  int yo = 0, co = 0;
  for (auto& cn : F.nodes) {
    cn.yoff = yo;
    cn.coff = co;
    yo += (int)cn.frow.size();
    co += (int)cn.urow.size();
  }
  F.ylen = yo;
  F.clen = co;
  std::vector<std::vector<int>> pulls(nc);
  for (const auto& cn : F.nodes)
    for (size_t u = 0; u < cn.urow.size(); ++u) pulls[cn.urow[u]].push_back(cn.coff + (int)u);
  size_t mp = 1;
  for (const auto& pl : pulls) mp = std::max(mp, pl.size());
  F.maxp = (int)((mp + 3) / 4 * 4);
  F.nd_row.assign(nc, -1);
  F.nd_scale.assign(nc, 1.0);
  F.slots.assign((size_t)nc * F.maxp, -1);
  for (const auto& cn : F.nodes)
    for (size_t a = 0; a < cn.frow.size(); ++a) {
      const int t = cn.yoff + (int)a, r = cn.frow[a];
      F.nd_row[t] = r;
      F.nd_scale[t] = F.rscale[r];
      for (size_t u = 0; u < pulls[r].size(); ++u) F.slots[(size_t)t * F.maxp + u] = pulls[r][u];
    }
  // the scaled rows in tree order, for the refinement residual
  F.nd_rp.assign(nc + 1, 0);
  for (int t = 0; t < nc; ++t) F.nd_rp[t + 1] = F.nd_rp[t] + (rp[F.nd_row[t] + 1] - rp[F.nd_row[t]]);
  F.nd_ci.resize(F.nd_rp[nc]);
  F.nd_v.resize(F.nd_rp[nc]);
  for (int t = 0; t < nc; ++t) {
    const int r = F.nd_row[t];
    for (int q = rp[r], o = F.nd_rp[t]; q < rp[r + 1]; ++q, ++o) {
      F.nd_ci[o] = ci[q];
      F.nd_v[o] = cvs[q];
    }
  }
  return F;
}

CoarseTables coarse_tables(const CoarseFactor& F, const int32_t* rowL, const int32_t* rowR,
                           const int32_t* rowKind, int pin_row, int nthreads) {
  CoarseTables T;
  const int nn = (int)F.nodes.size();
  std::vector<long long> fwd_off(nn), bwd_off(nn);
  std::vector<int> fcol_off(nn), ucol_off(nn);
  for (int t = 0; t < nn; ++t) {
    const auto& cn = F.nodes[t];
    fcol_off[t] = (int)T.idx.size();
    T.idx.insert(T.idx.end(), cn.fcol.begin(), cn.fcol.end());
    ucol_off[t] = (int)T.idx.size();
    T.idx.insert(T.idx.end(), cn.ucol.begin(), cn.ucol.end());
    fwd_off[t] = T.fwd_len;
    T.fwd_len += (long long)cn.fwd.size();
    bwd_off[t] = T.bwd_len;
    T.bwd_len += (long long)cn.bwd.size();
    T.max_nf = std::max(T.max_nf, (int)cn.frow.size());
    T.max_nu = std::max(T.max_nu, (int)cn.urow.size());
  }
  if (T.max_nf > kMaxCoarseFront || T.max_nu > kMaxCoarseFront)
    throw Error(MRCM_EINVAL, "interface separator too large for one workgroup");
  // the node matrices, concatenated by the host threads (uninitialised
  // storage: every element is written)
  T.fwd.reset(new double[std::max(T.fwd_len, 1LL)]);
  T.bwd.reset(new double[std::max(T.bwd_len, 1LL)]);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int t = 0; t < nn; ++t) {
    const auto& cn = F.nodes[t];
    std::copy(cn.fwd.begin(), cn.fwd.end(), T.fwd.get() + fwd_off[t]);
    std::copy(cn.bwd.begin(), cn.bwd.end(), T.bwd.get() + bwd_off[t]);
  }
  // Rows per forward chunk: 64 when the node's separator has at most 128
  // rows (a 256-thread workgroup takes the chunk whole, 16 rows per wave,
  // with one gather of the vector for all 64 rows), else 16 (four rows per
  // wave at a time).  Backward chunks have 16 rows (a one-wave workgroup
  // takes a chunk of at most 128 columns whole): wider backward chunks
  // measured slower.
  auto rows_per_chunk = [](int ncol) { return ncol <= 128 ? 64 : 16; };
  for (int d = F.depth; d >= 0; --d) {
    const int first = (int)T.chunks.size();
    for (int t = 0; t < nn; ++t) {
      const auto& cn = F.nodes[t];
      if (cn.depth != d) continue;
      const int nf = (int)cn.frow.size(), nu = (int)cn.urow.size(), rows = nf + nu;
      const int step = rows_per_chunk(nf);
      for (int r0 = 0; r0 < rows; r0 += step)
        T.chunks.push_back(CChunk{r0, std::min(rows, r0 + step), nf, nu, cn.yoff, cn.coff,
                                  fcol_off[t], ucol_off[t], fwd_off[t]});
    }
    T.fwd_levels.push_back({first, (int)T.chunks.size() - first});
  }
  for (int d = 0; d <= F.depth; ++d) {
    const int first = (int)T.chunks.size();
    for (int t = 0; t < nn; ++t) {
      const auto& cn = F.nodes[t];
      if (cn.depth != d) continue;
      const int nf = (int)cn.frow.size(), nu = (int)cn.urow.size();
      if (nu == 0) continue;  // x_F = y_F, written by the forward level
      const int step = 16;
      for (int r0 = 0; r0 < nf; r0 += step)
        T.chunks.push_back(CChunk{r0, std::min(nf, r0 + step), nf, nu, cn.yoff, cn.coff,
                                  fcol_off[t], ucol_off[t], bwd_off[t]});
    }
    if ((int)T.chunks.size() > first) T.bwd_levels.push_back({first, (int)T.chunks.size() - first});
  }
  // right-hand-side sources and contribution destinations by tree position
  const int np = F.ylen;
  T.gsrc.resize(np);
  for (int t = 0; t < np; ++t) {
    const int row = F.nd_row[t];
    const int kind = row == pin_row ? 2 : rowKind[row];
    T.gsrc[t] = {rowL[row], rowR[row], kind, 0};
  }
  T.cdest.assign(std::max(F.clen, 1), 0);
  for (int t = 0; t < np; ++t)
    for (int u = 0; u < F.maxp; ++u) {
      const int q = F.slots[(size_t)t * F.maxp + u];
      if (q >= 0) T.cdest[q] = u * np + t;
    }
  return T;
}

void coarse_residual_host(const CoarseFactor& F, const double* g_nd, const double* x,
                          double* r_nd, int nthreads) {
#pragma omp parallel for schedule(static) num_threads(std::max(1, nthreads)) if (nthreads > 1)
  for (int t = 0; t < F.nc; ++t) {
    double s = g_nd[t];
    for (int q = F.nd_rp[t]; q < F.nd_rp[t + 1]; ++q) s = std::fma(-F.nd_v[q], x[F.nd_ci[q]], s);
    r_nd[t] = s;
  }
}

void coarse_solve_refined_host(const CoarseFactor& F, const double* g_nd, double* x,
                               int nthreads) {
  coarse_solve_host(F, g_nd, x, nthreads);
  std::vector<double> r(F.nc), dx(F.nc);
  for (int s = 0; s < F.refine; ++s) {
    coarse_residual_host(F, g_nd, x, r.data(), nthreads);
    coarse_solve_host(F, r.data(), dx.data(), nthreads);
    for (int q = 0; q < F.nc; ++q) x[q] += dx[q];
  }
}

int coarse_refine_steps(CoarseFactor& F, double tol, int max_steps, int nthreads) {
  F.refine = 0;
  const int nc = F.nc;
  if (nc == 0) return 0;
  // right-hand side: a fixed sequence of values in [-1, 1) (64-bit linear
  // congruential generator), in tree order
  std::vector<double> g(nc), x(nc), r(nc), dx(nc);
  unsigned long long st = 0x9E3779B97F4A7C15ULL;
  for (int t = 0; t < nc; ++t) {
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    g[t] = (double)(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  coarse_solve_host(F, g.data(), x.data(), nthreads);
  int steps = 0;
  while (steps < max_steps) {
    coarse_residual_host(F, g.data(), x.data(), r.data(), nthreads);
    coarse_solve_host(F, r.data(), dx.data(), nthreads);
    double dmax = 0.0, xmax = 0.0;
    for (int q = 0; q < nc; ++q) {
      dmax = std::max(dmax, std::fabs(dx[q]));
      xmax = std::max(xmax, std::fabs(x[q]));
    }
    if (!(dmax > tol * xmax)) break;
    for (int q = 0; q < nc; ++q) x[q] += dx[q];
    ++steps;
  }
  F.refine = steps;
  return steps;
}

void coarse_solve_host(const CoarseFactor& F, const double* g_nd, double* x, int nthreads) {
  constexpr int kRows = 32;  // rows of a work item
  std::vector<double> ybuf(F.ylen), cbuf(F.clen), v(F.ylen);
  std::vector<std::vector<int>> level(F.depth + 1);
  for (int t = 0; t < (int)F.nodes.size(); ++t) level[F.nodes[t].depth].push_back(t);
  const int nth = std::max(1, nthreads);
  std::vector<std::pair<int, int>> items;  // (node, first row)
  for (int d = F.depth; d >= 0; --d) {
    const auto& lv = level[d];
    // the vectors of the level's nodes (descendants' contributions in slot
    // order), then their rows of [W; E]
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth) if (nth > 1)
    for (int li = 0; li < (int)lv.size(); ++li) {
      const CoarseNode& cn = F.nodes[lv[li]];
      for (int a = 0; a < (int)cn.frow.size(); ++a) {
        const size_t t = (size_t)cn.yoff + a;
        double s = g_nd[t];
        for (int u = 0; u < F.maxp; ++u) {
          const int q = F.slots[t * F.maxp + u];
          if (q >= 0) s -= cbuf[q];
        }
        v[t] = s;
      }
    }
    items.clear();
    for (int t : lv) {
      const CoarseNode& cn = F.nodes[t];
      for (int r0 = 0; r0 < (int)(cn.frow.size() + cn.urow.size()); r0 += kRows) items.push_back({t, r0});
    }
#pragma omp parallel for schedule(dynamic, 4) num_threads(nth) if (nth > 1)
    for (int it = 0; it < (int)items.size(); ++it) {
      const CoarseNode& cn = F.nodes[items[it].first];
      const int nf = (int)cn.frow.size(), nu = (int)cn.urow.size();
      const double* vn = &v[cn.yoff];
      const int r1 = std::min(nf + nu, items[it].second + kRows);
      for (int a = items[it].second; a < r1; ++a) {
        double s = 0.0;
        for (int b = 0; b < nf; ++b) s += cn.fwd[(size_t)a * nf + b] * vn[b];
        if (a < nf)
          ybuf[cn.yoff + a] = s;
        else
          cbuf[cn.coff + a - nf] = s;
      }
    }
  }
  for (int d = 0; d <= F.depth; ++d) {
    items.clear();
    for (int t : level[d]) {
      const CoarseNode& cn = F.nodes[t];
      for (int r0 = 0; r0 < (int)cn.frow.size(); r0 += kRows) items.push_back({t, r0});
    }
#pragma omp parallel for schedule(dynamic, 4) num_threads(nth) if (nth > 1)
    for (int it = 0; it < (int)items.size(); ++it) {
      const CoarseNode& cn = F.nodes[items[it].first];
      const int nf = (int)cn.frow.size(), nu = (int)cn.urow.size();
      const int r1 = std::min(nf, items[it].second + kRows);
      for (int a = items[it].second; a < r1; ++a) {
        double s = ybuf[cn.yoff + a];
        for (int b = 0; b < nu; ++b) s -= cn.bwd[(size_t)a * nu + b] * x[cn.ucol[b]];
        x[cn.fcol[a]] = s;
      }
    }
  }
}

}  // namespace mrcm
