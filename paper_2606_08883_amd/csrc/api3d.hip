// C ABI of the 3-D path (include/mrcm3d.h): set-up (host FP64 tables
// uploaded to HBM), the preconditioner apply, the fine operator, and the
// host-driven GMRES loop of Algorithm 1 with device-resident Krylov vectors
// (the vector kernels of the 2-D path: Gram-Schmidt, normalisation, update,
// norms, projection).
#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "device3d.h"
#include "setup3d.h"

namespace {

void check3(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw mrcm::Error(e == hipErrorOutOfMemory ? MRCM_ENOMEM : MRCM_EDEVICE,
                      std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct mrcm3d_ctx {
  int nx = 0, ny = 0, nz = 0, m = 0, nc = 0, sweeps = 0, noflow = 0;
  int bcmask = 0;  // bit s: side s (W E S N B T) has Dirichlet data
  long long n = 0;
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  double setup_seconds = 0.0, factor_bytes = 0.0, coarse_bytes = 0.0, resid_bytes = 0.0;
  double *tx = nullptr, *ty = nullptr, *tz = nullptr;
  mrcm3d::Box3 *lbox = nullptr, *pbox = nullptr;
  int lmax_cells = 1, pmax_cells = 1;  // the most cells of a box of each list
  int lmax_plane = 1, pmax_plane = 1;  // and the most cells of a plane
  // plane blocks: double, or float with precision 2
  void *ldinv = nullptr, *pdinv = nullptr;
  double *lcoup = nullptr, *pcoup = nullptr;
  int precision = 0;
  double* mbf = nullptr;
  long long* mbf_off = nullptr;
  int* dof_off = nullptr;
  mrcm3d::Dof3* dofs = nullptr;
  int *fin = nullptr, *fout = nullptr;
  double* fw = nullptr;
  // the interface solve: the nested-dissection factor and its level lists,
  // right-hand-side sources and scales by tree position, the scaled rows of C
  // in tree order for the refinement residual
  int4* gsrc = nullptr;
  double* gscale = nullptr;
  mrcm::CChunk* chunks = nullptr;
  double *cfwd = nullptr, *cbwd = nullptr;
  int *cidx = nullptr, *cdest = nullptr;
  std::vector<std::pair<int, int>> fwd_levels, bwd_levels;
  int maxp = 4, np = 0, max_nf = 1, max_nu = 1, refine = 0;
  int *crp = nullptr, *cci = nullptr;
  double* cv = nullptr;
  // work space of one application and of GMRES (contrib: zero where unused)
  double *p = nullptr, *rho = nullptr, *mU = nullptr, *mP = nullptr, *g_nd = nullptr;
  double *x = nullptr, *rnd = nullptr, *dx = nullptr, *ybuf = nullptr, *contrib = nullptr;
  double* partials = nullptr;
  int krylov_cap = 0;
  double *V = nullptr, *Z = nullptr, *hcol = nullptr, *parts = nullptr, *yd = nullptr;
  double *h_fetch = nullptr, *h_y = nullptr;  // pinned
  hipStream_t st = nullptr;
  hipEvent_t ev_in = nullptr;
  // per-phase timing: (phase, start, end)
  bool timing = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  double phase_ms[6] = {0, 0, 0, 0, 0, 0};
  long long phase_n[6] = {0, 0, 0, 0, 0, 0};

  // allocator of this context (null: hipMalloc / hipFree; mrcm_set_allocator)
  // and the stream its callbacks are given (the set-up stream)
  mrcm_alloc_fn alloc_fn = nullptr;
  mrcm_free_fn free_fn = nullptr;
  hipStream_t alloc_stream = nullptr;

  template <typename X>
  X* alloc(size_t count) {
    void* q = nullptr;
    const size_t bytes = ((count ? count : 1) * sizeof(X) + 255) / 256 * 256;
    if (alloc_fn) {
      q = alloc_fn(bytes, alloc_stream);
      if (!q) throw mrcm::Error(MRCM_ENOMEM, "allocator callback returned NULL");
    } else {
      check3(hipMalloc(&q, bytes), "hipMalloc");
    }
    allocs.push_back(q);
    device_bytes += bytes;
    return static_cast<X*>(q);
  }
  // A set-up upload; it returns once the host data has been read, so the
  // caller may release it.
  template <typename X>
  X* upload(const X* v, size_t count) {
    X* d = alloc<X>(count);
    if (count) {
      check3(hipMemcpyAsync(d, v, count * sizeof(X), hipMemcpyHostToDevice, st),
             "hipMemcpyAsync");
      check3(hipStreamSynchronize(st), "hipStreamSynchronize");
    }
    return d;
  }
  template <typename X>
  X* upload(const std::vector<X>& v) {
    return upload(v.data(), v.size());
  }
  void fold() {
    for (auto& mk : marks) {
      float ms = 0.0f;
      check3(hipEventSynchronize(mk.second.second), "hipEventSynchronize");
      check3(hipEventElapsedTime(&ms, mk.second.first, mk.second.second), "hipEventElapsedTime");
      phase_ms[mk.first] += ms;
      phase_n[mk.first] += 1;
      (void)hipEventDestroy(mk.second.first);
      (void)hipEventDestroy(mk.second.second);
    }
    marks.clear();
  }
  ~mrcm3d_ctx() {
    if (st) (void)hipStreamSynchronize(st);
    for (auto& mk : marks) {
      (void)hipEventDestroy(mk.second.first);
      (void)hipEventDestroy(mk.second.second);
    }
    if (alloc_stream) (void)hipStreamSynchronize(alloc_stream);
    for (void* q : allocs) {
      if (free_fn)
        free_fn(q, alloc_stream);
      else
        (void)hipFree(q);
    }
    if (h_fetch) (void)hipHostFree(h_fetch);
    if (h_y) (void)hipHostFree(h_y);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (st) (void)hipStreamDestroy(st);
  }
};

namespace {

thread_local std::string g_err3;

int fail3(const mrcm::Error& e) {
  g_err3 = e.what();
  mrcm::set_last_error(g_err3);
  return e.code;
}

// The return code of an entry point that stopped on an exception other than
// mrcm::Error: MRCM_ENOMEM for a failed host allocation, else MRCM_EINVAL
// (no C++ exception leaves the C ABI).
int fail3_std(const std::exception& e) {
  if (dynamic_cast<const std::bad_alloc*>(&e))
    return fail3(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  return fail3(mrcm::Error(MRCM_EINVAL, e.what()));
}

// Box descriptors and the concatenated factors of a list of boxes.
void upload_boxes(mrcm3d_ctx* c, const mrcm3d::Setup& S, const std::vector<mrcm3d::Box>& boxes,
                  const std::vector<mrcm3d::PlaneFactor>& F, mrcm3d::Box3*& dbox, void*& ddinv,
                  double*& dcoup, int& max_cells, int& max_plane) {
  std::vector<mrcm3d::Box3> desc(boxes.size());
  std::vector<double> dinv, coup;
  for (size_t i = 0; i < boxes.size(); ++i) {
    const mrcm3d::Box& b = boxes[i];
    const mrcm3d::Box& own = S.boxes[i];
    mrcm3d::Box3& d = desc[i];
    for (int a = 0; a < 3; ++a) {
      d.lo[a] = b.lo[a];
      d.n[a] = b.n(a);
      d.olo[a] = own.lo[a] - b.lo[a];
      d.on[a] = own.n(a);
    }
    d.P = b.plane();
    d.pin = F[i].pin;
    if (d.P > mrcm3d::kBox3Threads || b.cells() > mrcm3d::kMaxBox3Cells)
      throw mrcm::Error(MRCM_EINVAL, "3-D box too large (at most 256 cells per z-plane and 4096 cells)");
    max_cells = std::max(max_cells, (int)b.cells());
    max_plane = std::max(max_plane, d.P);
    d.doff = (long long)dinv.size();
    d.coff = (long long)coup.size();
    dinv.insert(dinv.end(), F[i].dinv.begin(), F[i].dinv.end());
    coup.insert(coup.end(), F[i].coup.begin(), F[i].coup.end());
  }
  const double word = S.precision == 2 ? 4.0 : 8.0;
  c->factor_bytes += 2.0 * word * (double)dinv.size();
  dbox = c->upload(desc);
  if (S.precision == 2) {
    const std::vector<float> f(dinv.begin(), dinv.end());
    ddinv = c->upload(f);
  } else {
    ddinv = c->upload(dinv);
  }
  dcoup = c->upload(coup);
}

void mark(mrcm3d_ctx* c, int phase, hipEvent_t a) {
  hipEvent_t b;
  check3(hipEventCreate(&b), "hipEventCreate");
  check3(hipEventRecord(b, c->st), "hipEventRecord");
  c->marks.push_back({phase, {a, b}});
}
hipEvent_t start_mark(mrcm3d_ctx* c) {
  if (!c->timing) return nullptr;
  hipEvent_t a;
  check3(hipEventCreate(&a), "hipEventCreate");
  check3(hipEventRecord(a, c->st), "hipEventRecord");
  return a;
}

// x = C^-1 g by the level-scheduled solve of the factor (g in tree order,
// x by dof): forward levels leaves first, backward levels root first.
void coarse_sweep(mrcm3d_ctx* c, const double* g, double* x, hipStream_t s) {
  for (const auto& lv : c->fwd_levels)
    mrcm::launch_coarse_fwd(c->chunks + lv.first, lv.second, c->cfwd, g, c->contrib, c->maxp,
                            c->np, c->cdest, c->ybuf, c->cidx, x, c->max_nf, s);
  for (const auto& lv : c->bwd_levels)
    mrcm::launch_coarse_bwd(c->chunks + lv.first, lv.second, c->cbwd, c->cidx, c->ybuf, x,
                            c->max_nu, s);
}

// z = T r on the context stream.
void apply3(mrcm3d_ctx* c, const double* r, double* z) {
  hipStream_t s = c->st;
  hipEvent_t e = start_mark(c);
  if (c->precision == 2)
    mrcm3d::launch_local3(c->lbox, c->m, c->lmax_cells, c->lmax_plane,
                          static_cast<const float*>(c->ldinv), c->lcoup, r, c->p, c->nx, c->ny,
                          c->dof_off, c->dofs, c->fin, c->fout, c->fw, c->mU, c->mP, s);
  else
    mrcm3d::launch_local3(c->lbox, c->m, c->lmax_cells, c->lmax_plane,
                          static_cast<const double*>(c->ldinv), c->lcoup, r, c->p, c->nx, c->ny,
                          c->dof_off, c->dofs, c->fin, c->fout, c->fw, c->mU, c->mP, s);
  if (e) mark(c, 0, e);
  if (c->nc > 0) {
    e = start_mark(c);
    mrcm::launch_coarse_rhs(c->gsrc, c->gscale, c->mU, c->mP, c->g_nd, c->np, s);
    coarse_sweep(c, c->g_nd, c->x, s);
    for (int k = 0; k < c->refine; ++k) {
      mrcm::launch_coarse_resid(1, c->crp, c->cci, c->cv, c->g_nd, c->x, c->rnd, c->np, c->nc, s);
      coarse_sweep(c, c->rnd, c->dx, s);
      mrcm::launch_coarse_add(c->x, c->dx, c->nc, s);
    }
    if (e) mark(c, 1, e);
    e = start_mark(c);
    mrcm3d::launch_reconstruct3(c->lbox, c->m, c->mbf, c->mbf_off, c->dof_off, c->x, c->p, c->nx,
                                c->ny, s);
    if (e) mark(c, 2, e);
  }
  for (int k = 0; k < c->sweeps; ++k) {
    e = start_mark(c);
    mrcm3d::launch_residual3(c->tx, c->ty, c->tz, c->nx, c->ny, c->nz, r, c->p, c->rho, s);
    if (e) mark(c, 3, e);
    e = start_mark(c);
    if (c->precision == 2)
      mrcm3d::launch_patch3(c->pbox, c->m, c->pmax_cells, c->pmax_plane,
                            static_cast<const float*>(c->pdinv), c->pcoup, c->rho, c->p, c->nx,
                            c->ny, s);
    else
      mrcm3d::launch_patch3(c->pbox, c->m, c->pmax_cells, c->pmax_plane,
                            static_cast<const double*>(c->pdinv), c->pcoup, c->rho, c->p, c->nx,
                            c->ny, s);
    if (e) mark(c, 4, e);
  }
  e = start_mark(c);
  mrcm::launch_finalize<double>(c->p, c->n, c->noflow, z, c->partials, s);
  if (e) mark(c, 5, e);
}

double host_sum3(const double* v, int nb) {
  double s = 0.0;
  for (int k = 0; k < nb; ++k) s += v[k];
  return s;
}

}  // namespace

extern "C" {

int mrcm3d_setup(const mrcm3d_grid* grid, const mrcm3d_params* params, const double* K_dev,
                 void* stream, mrcm3d_ctx** out) {
  mrcm3d_ctx* c = nullptr;
  try {
    if (!grid || !params || !K_dev || !out) throw mrcm::Error(MRCM_EINVAL, "null argument");
    const auto t0 = std::chrono::steady_clock::now();
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1)
      throw mrcm::Error(MRCM_EINVAL, "invalid grid");
    c = new mrcm3d_ctx();
    mrcm::current_allocator(&c->alloc_fn, &c->free_fn);
    c->alloc_stream = static_cast<hipStream_t>(stream);
    check3(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking), "hipStreamCreate");
    check3(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming), "hipEventCreate");
    std::vector<double> K((size_t)n);
    hipStream_t cs = static_cast<hipStream_t>(stream);
    check3(hipMemcpyAsync(K.data(), K_dev, sizeof(double) * n, hipMemcpyDeviceToHost, cs),
           "hipMemcpyAsync");
    check3(hipStreamSynchronize(cs), "hipStreamSynchronize");
    mrcm3d::Setup S;
    mrcm3d::host_setup(S, *grid, *params, K.data());
    c->nx = S.nx;
    c->ny = S.ny;
    c->nz = S.nz;
    c->n = S.n;
    c->m = S.m;
    c->nc = S.nc;
    c->sweeps = S.sweeps;
    c->precision = S.precision;
    c->noflow = S.noflow ? 1 : 0;
    for (int sd = 0; sd < 6; ++sd) c->bcmask |= S.bc[sd] ? 1 << sd : 0;
    c->tx = c->upload(S.tx);
    c->ty = c->upload(S.ty);
    c->tz = c->upload(S.tz);
    upload_boxes(c, S, S.oboxes, S.over, c->lbox, c->ldinv, c->lcoup, c->lmax_cells,
                 c->lmax_plane);
    if (S.sweeps > 0)
      upload_boxes(c, S, S.pboxes, S.patch, c->pbox, c->pdinv, c->pcoup, c->pmax_cells,
                   c->pmax_plane);
    // multiscale basis functions
    std::vector<double> mbf;
    std::vector<long long> mbf_off(S.m);
    for (int i = 0; i < S.m; ++i) {
      mbf_off[i] = (long long)mbf.size();
      mbf.insert(mbf.end(), S.mbf[i].begin(), S.mbf[i].end());
    }
    c->mbf = c->upload(mbf);
    c->mbf_off = c->upload(mbf_off);
    c->dof_off = c->upload(S.dof_off);
    // trace tables: the faces of every side of Gamma_i, box-local in hat-Omega_i
    std::vector<mrcm3d::Dof3> dofs(S.nc);
    std::vector<int> fin, fout;
    std::vector<double> fw;
    for (int i = 0; i < S.m; ++i) {
      const mrcm3d::Box& oi = S.oboxes[i];
      auto local = [&](long long cell) {
        const int x = (int)(cell % S.nx), y = (int)((cell / S.nx) % S.ny),
                  z = (int)(cell / ((long long)S.nx * S.ny));
        return ((z - oi.lo[2]) * oi.n(1) + (y - oi.lo[1])) * oi.n(0) + (x - oi.lo[0]);
      };
      for (const mrcm3d::SideData& d : S.gam[i]) {
        const int f0 = (int)fin.size();
        for (size_t f = 0; f < d.in.size(); ++f) {
          fin.push_back(local(d.in[f]));
          fout.push_back(S.oversample > 0 ? local(d.out[f]) : local(d.in[f]));
          for (int w = 0; w < 4; ++w) fw.push_back(d.w[f][w]);
        }
        for (int k = S.dof_off[i]; k < S.dof_off[i + 1]; ++k)
          if (S.dofs[k][1] == d.side)
            dofs[k] = mrcm3d::Dof3{f0, (int)d.in.size(), d.n0, d.n1, S.dofs[k][3], S.dofs[k][4], 0, 0};
      }
    }
    c->dofs = c->upload(dofs);
    c->fin = c->upload(fin);
    c->fout = c->upload(fout);
    c->fw = c->upload(fw);
    if (S.nc > 0) {
      const mrcm::CoarseFactor& F = S.CF;
      mrcm::CoarseTables T = mrcm::coarse_tables(F, S.rowL.data(), S.rowR.data(),
                                                 S.rowKind.data(), S.pin_row,
                                                 std::max(1, omp_get_max_threads()));
      static_assert(sizeof(int4) == sizeof(std::array<int, 4>), "gsrc layout");
      c->gsrc = reinterpret_cast<int4*>(c->upload(&T.gsrc[0][0], 4 * T.gsrc.size()));
      c->gscale = c->upload(F.nd_scale);
      c->chunks = c->upload(T.chunks);
      c->cfwd = c->upload(T.fwd.get(), (size_t)T.fwd_len);
      c->cbwd = c->upload(T.bwd.get(), (size_t)T.bwd_len);
      c->cidx = c->upload(T.idx);
      c->cdest = c->upload(T.cdest);
      c->fwd_levels = T.fwd_levels;
      c->bwd_levels = T.bwd_levels;
      c->maxp = F.maxp;
      c->np = F.ylen;
      c->max_nf = T.max_nf;
      c->max_nu = T.max_nu;
      c->refine = F.refine;
      c->crp = c->upload(F.nd_rp);
      c->cci = c->upload(F.nd_ci);
      c->cv = c->upload(F.nd_v);
      c->coarse_bytes = 8.0 * ((double)T.fwd_len + (double)T.bwd_len);
      c->resid_bytes = 12.0 * (double)F.nd_v.size() + 4.0 * (c->np + 1) + 24.0 * c->np;
    }
    const size_t nc = std::max(S.nc, 1);
    c->p = c->alloc<double>(S.n);
    c->rho = c->alloc<double>(S.n);
    c->mU = c->alloc<double>(nc);
    c->mP = c->alloc<double>(nc);
    c->g_nd = c->alloc<double>(nc);
    c->x = c->alloc<double>(nc);
    c->rnd = c->alloc<double>(nc);
    c->dx = c->alloc<double>(nc);
    c->ybuf = c->alloc<double>(nc);
    c->contrib = c->alloc<double>(nc * (size_t)c->maxp);
    check3(hipMemsetAsync(c->contrib, 0, sizeof(double) * nc * (size_t)c->maxp, c->st),
           "hipMemsetAsync");
    c->partials = c->alloc<double>(2 * mrcm::kMaxVecBlocks);
    c->parts = c->alloc<double>(2 * mrcm::kMaxVecBlocks);
    check3(hipHostMalloc((void**)&c->h_fetch, sizeof(double) * (mrcm::kMaxVecBlocks + 256),
                         hipHostMallocDefault),
           "hipHostMalloc");
    check3(hipHostMalloc((void**)&c->h_y, sizeof(double) * 256, hipHostMallocDefault),
           "hipHostMalloc");
    check3(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    c->setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = c;
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    delete c;
    return fail3(e);
  } catch (const std::bad_alloc&) {
    delete c;
    return fail3(mrcm::Error(MRCM_ENOMEM, "host allocation failed"));
  } catch (const std::exception& e) {
    delete c;
    return fail3(mrcm::Error(MRCM_EINVAL, e.what()));
  }
}

int mrcm3d_apply(mrcm3d_ctx* c, const double* r, double* z, void* stream) {
  try {
    if (!c || !r || !z) throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    check3(hipEventRecord(c->ev_in, s), "hipEventRecord");
    check3(hipStreamWaitEvent(c->st, c->ev_in, 0), "hipStreamWaitEvent");
    apply3(c, r, z);
    check3(hipEventRecord(c->ev_in, c->st), "hipEventRecord");
    check3(hipStreamWaitEvent(s, c->ev_in, 0), "hipStreamWaitEvent");
    check3(hipGetLastError(), "kernel launch");
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_op_apply(mrcm3d_ctx* c, const double* x, double* y, void* stream) {
  try {
    if (!c || !x || !y) throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    mrcm3d::launch_op3(c->tx, c->ty, c->tz, c->nx, c->ny, c->nz, x, y,
                       static_cast<hipStream_t>(stream));
    check3(hipGetLastError(), "kernel launch");
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_rhs(mrcm3d_ctx* c, const double* f_cell, const double* g_bc, double h, double* b,
               void* stream) {
  try {
    if (!c || !b || !(h > 0.0) || !std::isfinite(h))
      throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    mrcm3d::launch_rhs3(c->tx, c->ty, c->tz, c->nx, c->ny, c->nz, c->bcmask, f_cell, g_bc, h, b,
                        static_cast<hipStream_t>(stream));
    check3(hipGetLastError(), "kernel launch");
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_gmres_solve(mrcm3d_ctx* c, const double* b, double* p, double rtol, int32_t restart,
                       int32_t maxit, mrcm_stats* st, void* stream) {
  try {
    if (!c || !b || !p || restart < 1 || restart > 200 || maxit < 0 || !(rtol >= 0.0))
      throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    hipStream_t s = c->st;
    check3(hipEventRecord(c->ev_in, static_cast<hipStream_t>(stream)), "hipEventRecord");
    check3(hipStreamWaitEvent(s, c->ev_in, 0), "hipStreamWaitEvent");
    const long long n = c->n;
    if (restart > c->krylov_cap) {
      c->V = c->alloc<double>((size_t)(restart + 1) * n);
      c->Z = c->alloc<double>((size_t)restart * n);
      c->hcol = c->alloc<double>(restart + 2);
      c->yd = c->alloc<double>(restart + 1);
      c->krylov_cap = restart;
    }
    const int nb = mrcm::vec_blocks(n);
    auto fetch = [&](const double* src, int cnt) {
      check3(hipMemcpyAsync(c->h_fetch, src, sizeof(double) * cnt, hipMemcpyDeviceToHost, s),
             "hipMemcpyAsync");
      check3(hipStreamSynchronize(s), "hipStreamSynchronize");
      if (c->timing) c->fold();
    };
    std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart),
        gv(restart + 1), y(restart);
    int it = 0, cycles = 0;
    bool conv = false;
    double relres = 1.0;
    mrcm::launch_zero(p, n, s);
    mrcm::launch_sumsq(b, n, c->parts, nb, s);
    fetch(c->parts, nb);
    const double bnorm = std::sqrt(host_sum3(c->h_fetch, nb));
    if (bnorm == 0.0) {
      conv = true;
      relres = 0.0;
    } else {
      const double tol = rtol * bnorm;
      bool first = true;
      for (;;) {
        mrcm3d::launch_resid_norm3(c->tx, c->ty, c->tz, c->nx, c->ny, c->nz, b,
                                   first ? nullptr : p, c->V, c->parts, nb, s);
        first = false;
        fetch(c->parts, nb);
        const double beta = std::sqrt(host_sum3(c->h_fetch, nb));
        relres = beta / bnorm;
        if (beta <= tol) {
          conv = true;
          break;
        }
        if (it >= maxit) break;
        ++cycles;
        mrcm::launch_scale(c->V, n, 1.0 / beta, s);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int j = 0;
        for (;;) {
          double* vj = c->V + (size_t)j * n;
          double* zj = c->Z + (size_t)j * n;
          double* w = c->V + (size_t)(j + 1) * n;
          apply3(c, vj, zj);
          mrcm3d::launch_arnoldi_start3(c->tx, c->ty, c->tz, c->nx, c->ny, c->nz, zj, w, c->V,
                                        c->parts, nb, s);
          for (int i = 0; i <= j; ++i)
            mrcm::launch_mgs_step(c->parts + (i % 2) * mrcm::kMaxVecBlocks,
                                  c->parts + ((i + 1) % 2) * mrcm::kMaxVecBlocks, nb, c->hcol, i,
                                  w, c->V + (size_t)i * n,
                                  i < j ? c->V + (size_t)(i + 1) * n : nullptr, n, s);
          mrcm::launch_norm_scale(c->parts + ((j + 1) % 2) * mrcm::kMaxVecBlocks, nb, c->hcol,
                                  j + 1, w, n, s);
          fetch(c->hcol, j + 2);
          const double* hh = c->h_fetch;
          ++it;
          for (int i = 0; i <= j + 1; ++i) H[(size_t)i * restart + j] = hh[i];
          const double hnext = hh[j + 1];
          for (int i = 0; i < j; ++i) {
            const double a = H[(size_t)i * restart + j], bb = H[(size_t)(i + 1) * restart + j];
            H[(size_t)i * restart + j] = cs[i] * a + sn[i] * bb;
            H[(size_t)(i + 1) * restart + j] = -sn[i] * a + cs[i] * bb;
          }
          const double a = H[(size_t)j * restart + j], bb = H[(size_t)(j + 1) * restart + j];
          const double rr = std::hypot(a, bb);
          cs[j] = a / rr;
          sn[j] = bb / rr;
          H[(size_t)j * restart + j] = rr;
          H[(size_t)(j + 1) * restart + j] = 0.0;
          gv[j + 1] = -sn[j] * gv[j];
          gv[j] = cs[j] * gv[j];
          const int jj = j + 1;
          if (!(hnext == 0.0 || std::fabs(gv[j + 1]) <= tol || it >= maxit || jj == restart)) {
            j = jj;
            continue;
          }
          for (int i = jj - 1; i >= 0; --i) {
            double sum = gv[i];
            for (int q = i + 1; q < jj; ++q) sum -= H[(size_t)i * restart + q] * y[q];
            y[i] = sum / H[(size_t)i * restart + i];
          }
          std::memcpy(c->h_y, y.data(), sizeof(double) * jj);
          check3(hipMemcpyAsync(c->yd, c->h_y, sizeof(double) * jj, hipMemcpyHostToDevice, s),
                 "hipMemcpyAsync");
          mrcm::launch_update(p, c->Z, c->yd, jj, n, s);
          break;
        }
      }
    }
    check3(hipEventRecord(c->ev_in, s), "hipEventRecord");
    check3(hipStreamWaitEvent(static_cast<hipStream_t>(stream), c->ev_in, 0), "hipStreamWaitEvent");
    check3(hipGetLastError(), "kernel launch");
    if (st) {
      st->iterations = it;
      st->cycles = cycles;
      st->converged = conv ? 1 : 0;
      st->hist_len = st->true_len = 0;
      st->final_relres = relres;
    }
    if (!conv) throw mrcm::Error(MRCM_ENOCONV, "GMRES reached maxit");
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_timing_enable(mrcm3d_ctx* c, int32_t on) {
  try {
    if (!c) throw mrcm::Error(MRCM_EINVAL, "null context");
    check3(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    c->fold();
    for (int k = 0; k < 6; ++k) {
      c->phase_ms[k] = 0.0;
      c->phase_n[k] = 0;
    }
    c->timing = on != 0;
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_timing_read(mrcm3d_ctx* c, double* ms, int64_t* counts) {
  try {
    if (!c || !ms || !counts) throw mrcm::Error(MRCM_EINVAL, "invalid argument");
    check3(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    c->fold();
    for (int k = 0; k < 6; ++k) {
      ms[k] = c->phase_ms[k];
      counts[k] = c->phase_n[k];
    }
    return MRCM_OK;
  } catch (const mrcm::Error& e) {
    return fail3(e);
  } catch (const std::exception& e) {
    return fail3_std(e);
  }
}

int mrcm3d_query(mrcm3d_ctx* c, int32_t what, double* value) {
  if (!c || !value) return MRCM_EINVAL;
  switch (what) {
    case 0: *value = c->setup_seconds; break;
    case 1: *value = (double)c->device_bytes; break;
    case 2: *value = c->nc; break;
    case 3: *value = c->factor_bytes; break;
    case 4: *value = (1.0 + c->refine) * c->coarse_bytes + c->refine * c->resid_bytes; break;
    case 5: *value = c->refine; break;
    case 6: *value = (double)(c->fwd_levels.size() + c->bwd_levels.size()); break;
    default: return MRCM_EINVAL;
  }
  return MRCM_OK;
}

void mrcm3d_destroy(mrcm3d_ctx* c) { delete c; }

}  // extern "C"
