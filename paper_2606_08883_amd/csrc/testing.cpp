// Test hooks (include/mrcm_testing.h): the host FP64 setup exposed for the
// test suite, and a host evaluation of T from the uploaded data layout.
#include "../../include/mrcm_testing.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "coarse.h"
#include "setup.h"
#include "setup3d.h"

namespace {

int fail(const mrcm::Error& e) {
  mrcm::set_last_error(e.what());
  return e.code;
}

mrcm::HostSetup make_setup(const mrcm_grid* g, const mrcm_params* p, const double* K) {
  if (!g || !p || !K) throw mrcm::Error(MRCM_EINVAL, "null argument");
  mrcm::HostSetup S;
  mrcm::host_setup(S, *g, *p, K, std::max(1, omp_get_max_threads()));
  return S;
}

}  // namespace

extern "C" {

int mrcm3d_test_host_apply(const mrcm3d_grid* grid, const mrcm3d_params* params,
                           const double* K, const double* r, double* z, int64_t* nc) {
  try {
    if (!grid || !params || !K || !r || !z) throw mrcm::Error(MRCM_EINVAL, "null argument");
    mrcm3d::Setup S;
    mrcm3d::host_setup(S, *grid, *params, K);
    mrcm3d::host_apply(S, r, z);
    if (nc) *nc = S.nc;
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm3d_test_dissection(int32_t mx, int32_t my, int32_t mz, int32_t* elim, int32_t* parent,
                           int32_t* depth, int32_t* border_ptr, int32_t* border,
                           int32_t max_nodes, int32_t max_border, int32_t* nodes) {
  try {
    if (mx < 1 || my < 1 || mz < 1 || !elim || !parent || !depth || !border_ptr || !border ||
        !nodes)
      throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    const std::vector<mrcm::DissectionNode> tree = mrcm3d::dissection3(mx, my, mz);
    const int nn = (int)tree.size();
    size_t nb = 0;
    for (const auto& nd : tree) nb += nd.usub.size();
    if (nn > max_nodes || (long long)nb > max_border)
      throw mrcm::Error(MRCM_EINVAL, "capacity too small");
    for (int t = 0; t < nn; ++t) parent[t] = -1;
    border_ptr[0] = 0;
    for (int t = 0; t < nn; ++t) {
      depth[t] = tree[t].depth;
      for (int c : tree[t].children) parent[c] = t;
      for (int s : tree[t].fsub) elim[s] = t;
      std::copy(tree[t].usub.begin(), tree[t].usub.end(), border + border_ptr[t]);
      border_ptr[t + 1] = border_ptr[t] + (int32_t)tree[t].usub.size();
    }
    *nodes = nn;
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm_test_zero_cell_setup(const mrcm_grid* grid, const mrcm_params* params,
                              const double* K, int64_t cell) {
  try {
    if (!grid || !params || !K) throw mrcm::Error(MRCM_EINVAL, "null argument");
    if (cell < 0 || cell >= (int64_t)grid->nx * grid->ny)
      throw mrcm::Error(MRCM_EINVAL, "cell out of range");
    mrcm::HostSetup S;
    mrcm::host_prepare(S, *grid, *params, K);  // validates K
    S.K[(size_t)cell] = 0.0;                    // the degenerate cell, after validation
    mrcm::face_transmissibilities(S);
    const mrcm::Maps& M = S.maps;
    for (int i = 0; i < M.m; ++i) {
      if (S.sweeps > 0) (void)mrcm::factor_box(S, M.pboxes[i], false);
      (void)mrcm::factor_box(S, M.oboxes[i], true);
    }
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm_test_coarse_sizes(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                           int64_t* nc, int64_t* nnz) {
  try {
    mrcm::HostSetup S = make_setup(grid, params, K);
    if (nc) *nc = S.maps.nc();
    if (nnz) *nnz = (int64_t)S.Cv.size();
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm_test_coarse_matrix(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                            int32_t* rp, int32_t* ci, double* cv) {
  try {
    mrcm::HostSetup S = make_setup(grid, params, K);
    std::copy(S.Crp.begin(), S.Crp.end(), rp);
    std::copy(S.Cci.begin(), S.Cci.end(), ci);
    std::copy(S.Cv.begin(), S.Cv.end(), cv);
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm_test_host_apply(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                         const double* r, double* z, double* min_pivot_ratio) {
  try {
    mrcm::HostSetup S = make_setup(grid, params, K);
    const mrcm::Maps& M = S.maps;
    mrcm::CoarseFactor CF =
        mrcm::coarse_factor(M, S.Crp, S.Cci, S.Cv, std::max(1, omp_get_max_threads()));
    mrcm::coarse_refine_steps(CF, mrcm::coarse_refine_tol(params->precision),
                              mrcm::kCoarseRefineMax);
    if (min_pivot_ratio) *min_pivot_ratio = CF.min_pivot_ratio;
    const int nx = S.nx;
    const size_t n = (size_t)S.nx * S.ny;
    const int nc = M.nc();
    std::vector<double> p(n, 0.0), mU(nc), mP(nc), g(nc), xc(nc);
    auto gather = [&](const mrcm::Box& b, const double* v, std::vector<double>& x) {
      x.assign((size_t)b.bx() * b.by(), 0.0);
      for (int j = 0; j < b.by(); ++j)
        for (int a = 0; a < b.bx(); ++a)
          x[(size_t)j * b.bx() + a] = v[(size_t)(b.y0 + j) * nx + b.x0 + a];
    };
    std::vector<double> x;
    for (int i = 0; i < M.m; ++i) {
      // source-driven solve on hat-Omega_i, kept on Omega_i
      const mrcm::Box& b = M.boxes[i];
      const mrcm::Box& ob = M.oboxes[i];
      gather(ob, r, x);
      mrcm::box_solve(S.over[i], x.data());
      const int ox = b.x0 - ob.x0, oy = b.y0 - ob.y0, obx = ob.bx(), oby = ob.by();
      for (int j = 0; j < b.by(); ++j)
        for (int a = 0; a < b.bx(); ++a)
          p[(size_t)(b.y0 + j) * nx + b.x0 + a] = x[(size_t)(oy + j) * obx + ox + a];
      // trace moments: U = cUi p_in + cUo p_out, pi = cPi p_in + cPo p_out
      for (int k = M.dof_offset[i]; k < M.dof_offset[i + 1]; ++k) {
        const int side = M.dofs[k][1], q = M.dofs[k][2];
        const int len = mrcm::side_len(b, side);
        double su = 0.0, sp = 0.0;
        for (int jf = 0; jf < len; ++jf) {
          int row, col, dr = 0, dc = 0;
          if (side == 0) {
            row = oy + jf; col = ox; dc = -1;
          } else if (side == 1) {
            row = oy + jf; col = ox + b.bx() - 1; dc = 1;
          } else if (side == 2) {
            row = oy; col = ox + jf; dr = -1;
          } else {
            row = oy + b.by() - 1; col = ox + jf; dr = 1;
          }
          const int r2 = row + dr, c2 = col + dc;
          const bool across = r2 >= 0 && r2 < oby && c2 >= 0 && c2 < obx;
          const double pin = x[(size_t)row * obx + col];
          const double pout = across ? x[(size_t)r2 * obx + c2] : pin;
          const double* w = &S.face_w[(size_t)4 * (S.dof_face0[k] + jf)];
          const double lw = mrcm::legendre(q, (2.0 * jf + 1.0) / len - 1.0);
          su += lw * (w[0] * pin + w[1] * pout);
          sp += lw * (w[2] * pin + w[3] * pout);
        }
        mU[k] = su;
        mP[k] = sp;
      }
    }
    if (nc > 0) {
      for (int rr = 0; rr < nc; ++rr) {
        const int L = S.rowL[rr], R = S.rowR[rr];
        g[rr] = S.rowKind[rr] == 0 ? -(mU[L] + mU[R]) : -(mP[L] - mP[R]);
        if (rr == S.pin_row) g[rr] = 0.0;
      }
      std::vector<double> gnd(nc);
      for (int q = 0; q < nc; ++q) gnd[q] = CF.nd_scale[q] * g[CF.nd_row[q]];
      mrcm::coarse_solve_refined_host(CF, gnd.data(), xc.data());
      for (int i = 0; i < M.m; ++i) {
        const mrcm::Box& b = M.boxes[i];
        const int ncell = b.bx() * b.by();
        for (int q = 0; q < ncell; ++q) {
          double s = 0.0;
          for (int k = 0; k < M.dof_offset[i + 1] - M.dof_offset[i]; ++k)
            s += S.mbf[i][(size_t)k * ncell + q] * xc[M.dof_offset[i] + k];
          p[(size_t)(b.y0 + q / b.bx()) * nx + b.x0 + q % b.bx()] += s;
        }
      }
    }
    std::vector<double> rho(n);
    for (int sweep = 0; sweep < S.sweeps; ++sweep) {
      mrcm::host_op_apply(S, p.data(), rho.data());
      for (size_t c = 0; c < n; ++c) rho[c] = r[c] - rho[c];
      for (int i = 0; i < M.m; ++i) {
        const mrcm::Box& pb = M.pboxes[i];
        const mrcm::Box& b = M.boxes[i];
        gather(pb, rho.data(), x);
        mrcm::box_solve(S.patch[i], x.data());
        for (int y = b.y0; y < b.y1; ++y)
          for (int xx = b.x0; xx < b.x1; ++xx)
            p[(size_t)y * nx + xx] += x[(size_t)(y - pb.y0) * pb.bx() + xx - pb.x0];
      }
    }
    double mean = 0.0;
    if (S.noflow) {
      for (size_t c = 0; c < n; ++c) mean += p[c];
      mean /= (double)n;
    }
    for (size_t c = 0; c < n; ++c) z[c] = p[c] - mean;
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm_test_coarse_solve(const mrcm_grid* grid, const mrcm_params* params, const double* K,
                           const double* g, double* x) {
  try {
    if (!g || !x) throw mrcm::Error(MRCM_EINVAL, "null argument");
    mrcm::HostSetup S = make_setup(grid, params, K);
    const int nc = S.maps.nc();
    if (nc == 0) return MRCM_OK;
    mrcm::CoarseFactor CF =
        mrcm::coarse_factor(S.maps, S.Crp, S.Cci, S.Cv, std::max(1, omp_get_max_threads()));
    mrcm::coarse_refine_steps(CF, mrcm::coarse_refine_tol(params->precision),
                              mrcm::kCoarseRefineMax);
    std::vector<double> gnd(nc);
    for (int q = 0; q < nc; ++q) gnd[q] = CF.nd_scale[q] * g[CF.nd_row[q]];
    mrcm::coarse_solve_refined_host(CF, gnd.data(), x);
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    return fail(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    return fail(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

}  // extern "C"
