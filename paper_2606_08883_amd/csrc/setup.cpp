// Host-side FP64 setup of T (Section 2.1): face transmissibilities, Robin
// coefficients (beta = alpha L / K_H), block LDL^T factors of the oversampled
// Robin problems (which inform the multiplier spaces and on which every
// multiscale basis function is built, the source-driven one of the apply
// included), the multiscale basis functions as restrictions of the
// oversampled solutions, the interface system, and the factors of the
// smoothing patches.
#include "setup.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <utility>

namespace mrcm {

void face_transmissibilities(HostSetup& S) {
  const int nx = S.nx, ny = S.ny;
  const double* K = S.K.data();
  S.tx.assign((size_t)ny * (nx + 1), 0.0);
  S.ty.assign((size_t)(ny + 1) * nx, 0.0);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 1; x < nx; ++x) {
      double a = K[(size_t)y * nx + x - 1], b = K[(size_t)y * nx + x];
      S.tx[(size_t)y * (nx + 1) + x] = 2.0 * a * b / (a + b);
    }
    if (S.bc[SW]) S.tx[(size_t)y * (nx + 1)] = 2.0 * K[(size_t)y * nx];
    if (S.bc[SE]) S.tx[(size_t)y * (nx + 1) + nx] = 2.0 * K[(size_t)y * nx + nx - 1];
  }
#pragma omp parallel for schedule(static)
  for (int y = 1; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double a = K[(size_t)(y - 1) * nx + x], b = K[(size_t)y * nx + x];
      S.ty[(size_t)y * nx + x] = 2.0 * a * b / (a + b);
    }
  for (int x = 0; x < nx; ++x) {
    if (S.bc[SS]) S.ty[x] = 2.0 * K[x];
    if (S.bc[SN]) S.ty[(size_t)ny * nx + x] = 2.0 * K[(size_t)(ny - 1) * nx + x];
  }
}

static inline double txv(const HostSetup& S, int y, int x) {
  return S.tx[(size_t)y * (S.nx + 1) + x];
}
static inline double tyv(const HostSetup& S, int y, int x) { return S.ty[(size_t)y * S.nx + x]; }

// Robin conductance of a face leaving a cell set: 1 / (1 / (2 K_c) + b_f),
// b_f = alpha L_cells / K_H(f), K_H(f) = t_f for square cells.
static inline double robin_rho(const HostSetup& S, double Kc, double t) {
  return 1.0 / (1.0 / (2.0 * Kc) + S.alpha * S.Lcells / t);
}

// In-place SPD inverse of an n x n row-major matrix through Cholesky.
static bool spd_inverse(double* A, int n, std::vector<double>& L, std::vector<double>& Li) {
  L.assign((size_t)n * n, 0.0);
  Li.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    double ljj = std::sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = s / ljj;
    }
  }
  for (int j = 0; j < n; ++j) {
    Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = -s / L[(size_t)i * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
      A[(size_t)i * n + j] = s;
      A[(size_t)j * n + i] = s;
    }
  return true;
}

BoxFactor factor_box(const HostSetup& S, const Box& b, bool robin) {
  BoxFactor F;
  F.box = b;
  const int bx = b.bx(), by = b.by(), nx = S.nx, ny = S.ny;
  F.pin = (S.noflow && b.x0 == 0 && b.y0 == 0 && b.x1 == nx && b.y1 == ny) ? 1 : 0;
  F.dinv.assign((size_t)by * bx * bx, 0.0);
  F.coup.assign((size_t)by * bx, 0.0);
  std::vector<double> D((size_t)bx * bx), L, Li;
  for (int j = 0; j < by; ++j) {
    const int y = b.y0 + j;
    std::fill(D.begin(), D.end(), 0.0);
    for (int a = 0; a < bx; ++a) {
      const int x = b.x0 + a;
      const double Kc = S.K[(size_t)y * nx + x];
      double tW = txv(S, y, x), tE = txv(S, y, x + 1), tS = tyv(S, y, x), tN = tyv(S, y + 1, x);
      // faces leaving the box inside the domain: Robin conductance or the
      // principal-submatrix transmissibility (unchanged)
      if (robin) {
        if (a == 0 && x > 0) tW = robin_rho(S, Kc, tW);
        if (a == bx - 1 && x + 1 < nx) tE = robin_rho(S, Kc, tE);
        if (j == 0 && y > 0) tS = robin_rho(S, Kc, tS);
        if (j == by - 1 && y + 1 < ny) tN = robin_rho(S, Kc, tN);
      }
      D[(size_t)a * bx + a] = tW + tE + tS + tN;
      if (a > 0) {
        D[(size_t)a * bx + a - 1] = -txv(S, y, x);
        D[(size_t)(a - 1) * bx + a] = -txv(S, y, x);
      }
      if (j > 0) F.coup[(size_t)j * bx + a] = tyv(S, y, x);
    }
    if (F.pin && j == 0) {
      for (int a = 0; a < bx; ++a) {
        D[a] = 0.0;
        D[(size_t)a * bx] = 0.0;
      }
      D[0] = 1.0;
    }
    if (F.pin && j == 1) F.coup[(size_t)bx] = 0.0;
    if (j > 0) {
      const double* Dp = &F.dinv[(size_t)(j - 1) * bx * bx];
      const double* T = &F.coup[(size_t)j * bx];
      for (int a = 0; a < bx; ++a)
        for (int c = 0; c < bx; ++c) D[(size_t)a * bx + c] -= T[a] * Dp[(size_t)a * bx + c] * T[c];
    }
    if (!spd_inverse(D.data(), bx, L, Li))
      throw Error(MRCM_ESINGULAR, "non-positive pivot in a local factorisation");
    std::copy(D.begin(), D.end(), F.dinv.begin() + (size_t)j * bx * bx);
  }
  return F;
}

void box_solve(const BoxFactor& F, double* x) {
  const int bx = F.box.bx(), by = F.box.by();
  std::vector<double> y(bx);
  if (F.pin) x[0] = 0.0;
  for (int j = 0; j < by; ++j) {
    const double* T = &F.coup[(size_t)j * bx];
    for (int a = 0; a < bx; ++a)
      y[a] = x[(size_t)j * bx + a] + (j > 0 ? T[a] * x[(size_t)(j - 1) * bx + a] : 0.0);
    const double* Di = &F.dinv[(size_t)j * bx * bx];
    for (int a = 0; a < bx; ++a) {
      double s = 0.0;
      for (int c = 0; c < bx; ++c) s += Di[(size_t)a * bx + c] * y[c];
      x[(size_t)j * bx + a] = s;
    }
  }
  for (int j = by - 2; j >= 0; --j) {
    const double* T = &F.coup[(size_t)(j + 1) * bx];
    for (int a = 0; a < bx; ++a) y[a] = T[a] * x[(size_t)(j + 1) * bx + a];
    const double* Di = &F.dinv[(size_t)j * bx * bx];
    for (int a = 0; a < bx; ++a) {
      double s = 0.0;
      for (int c = 0; c < bx; ++c) s += Di[(size_t)a * bx + c] * y[c];
      x[(size_t)j * bx + a] += s;
    }
  }
}

void host_op_apply(const HostSetup& S, const double* x, double* y) {
  const int nx = S.nx, ny = S.ny;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      size_t c = (size_t)iy * nx + ix;
      double tW = txv(S, iy, ix), tE = txv(S, iy, ix + 1), tS = tyv(S, iy, ix),
             tN = tyv(S, iy + 1, ix);
      double v = (tW + tE + tS + tN) * x[c];
      if (ix > 0) v -= tW * x[c - 1];
      if (ix + 1 < nx) v -= tE * x[c + 1];
      if (iy > 0) v -= tS * x[c - nx];
      if (iy + 1 < ny) v -= tN * x[c + nx];
      y[c] = v;
    }
}

namespace {

// Data of one side of Gamma_i (faces in increasing coordinate).
struct GammaSide {
  int side;
  std::vector<Face> faces;
  std::vector<double> t, b, rho, Kin, Kout;
};

inline int loc_of(const Box& b, int cell, int nx) {
  return (cell / nx - b.y0) * b.bx() + (cell % nx - b.x0);
}

GammaSide make_side(const HostSetup& S, const Box& b, int side) {
  GammaSide g;
  g.side = side;
  g.faces = side_faces(b, side, S.nx);
  for (const Face& f : g.faces) {
    double t = f.kind == 0 ? txv(S, f.row, f.col) : tyv(S, f.row, f.col);
    double Kin = S.K[f.inside], Kout = S.K[f.outside];
    double bf = S.alpha * S.Lcells / t;
    g.t.push_back(t);
    g.b.push_back(bf);
    g.rho.push_back(1.0 / (1.0 / (2.0 * Kin) + bf));
    g.Kin.push_back(Kin);
    g.Kout.push_back(Kout);
  }
  return g;
}

inline double xi_of(int j, int n) { return (2.0 * j + 1.0) / n - 1.0; }

// Edge index across `side` of subdomain i, and whether i is its L subdomain.
int edge_across(const Maps& M, int i, int side, bool& isL) {
  const int I = i % M.mx, J = i / M.mx, nV = M.my * (M.mx - 1);
  switch (side) {
    case SE: isL = true; return J * (M.mx - 1) + I;
    case SW: isL = false; return J * (M.mx - 1) + I - 1;
    case SN: isL = true; return nV + J * M.mx + I;
    default: isL = false; return nV + (J - 1) * M.mx + I;
  }
}

struct SubResult {
  // column contributions: for dof k of i, for each side s' of i and q': flux and pressure moments
  std::vector<std::vector<std::vector<double>>> colU, colP;  // [k][side index][q']
};

}  // namespace

void host_prepare(HostSetup& S, const mrcm_grid& g, const mrcm_params& p, const double* K) {
  S.maps = build_maps(g, p);
  const Maps& M = S.maps;
  S.nx = g.nx;
  S.ny = g.ny;
  for (int s = 0; s < 4; ++s) S.bc[s] = g.bc[s];
  S.noflow = !(g.bc[0] || g.bc[1] || g.bc[2] || g.bc[3]);
  S.alpha = p.alpha;
  S.Lcells = p.beta_len == 0 ? (double)std::max(p.sx, p.sy) : 1.0;
  S.sweeps = p.smooth_sweeps;
  const size_t n = (size_t)g.nx * g.ny;
  S.K.assign(K, K + n);
  long long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (long long c = 0; c < (long long)n; ++c)
    if (!(S.K[c] > 0.0) || !std::isfinite(S.K[c])) ++bad;
  if (bad) throw Error(MRCM_EINVAL, "K must be finite and positive on every cell");
  face_transmissibilities(S);
  const int m = M.m, nc = M.nc();
  // trace weights of the source-driven solutions, per face of Gamma_i:
  // inside the oversampled box U = t (p_in - p_out) and the flux-continuous
  // pi = (K_in p_in + K_out p_out) / (K_in + K_out); without oversampling the
  // face is a Robin face with zero data: U = rho p_in, pi = b U
  S.face_off.assign(m + 1, 0);
  for (int i = 0; i < m; ++i) {
    int nf = 0;
    for (int s : M.sides[i]) nf += side_len(M.boxes[i], s);
    S.face_off[i + 1] = S.face_off[i] + nf;
  }
  S.face_w.assign((size_t)4 * S.face_off[m], 0.0);
  S.dof_face0.assign(nc, 0);
  S.dof_q.assign(nc, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < m; ++i) {
    int f = S.face_off[i];
    for (int s : M.sides[i]) {
      const GammaSide gs = make_side(S, M.boxes[i], s);
      for (int dof = M.dof_offset[i]; dof < M.dof_offset[i + 1]; ++dof)
        if (M.dofs[dof][1] == s) {
          S.dof_face0[dof] = f;
          S.dof_q[dof] = M.dofs[dof][2];
        }
      for (size_t j = 0; j < gs.faces.size(); ++j, ++f) {
        double* w = &S.face_w[(size_t)4 * f];
        if (M.oversample == 0) {
          w[0] = gs.rho[j];
          w[1] = 0.0;
          w[2] = gs.b[j] * gs.rho[j];
          w[3] = 0.0;
        } else {
          w[0] = gs.t[j];
          w[1] = -gs.t[j];
          w[2] = gs.Kin[j] / (gs.Kin[j] + gs.Kout[j]);
          w[3] = gs.Kout[j] / (gs.Kin[j] + gs.Kout[j]);
        }
      }
    }
  }
  // coarse rows: the dofs of the L and R sides each row combines
  const int E = (int)M.edges.size();
  S.rowL.assign(nc, -1);
  S.rowR.assign(nc, -1);
  S.rowKind.assign(nc, 0);
  for (int e = 0; e < E; ++e) {
    const int L = M.edges[e][0], R = M.edges[e][1], o = M.edges[e][2];
    const int sL = o == 0 ? SE : SN, sR = o == 0 ? SW : SS;
    const int nb = M.nbasis(M.edges[e][4]);
    for (int kind = 0; kind < 2; ++kind)
      for (int q = 0; q < nb; ++q) {
        int r = M.row_offset[e] + kind * nb + q;
        S.rowL[r] = M.dof_of(L, sL, q);
        S.rowR[r] = M.dof_of(R, sR, q);
        S.rowKind[r] = kind;
      }
  }
}

void device_tables(const HostSetup& S, int epv, DeviceTables& T) {
  const Maps& M = S.maps;
  const int m = M.m, nb = M.degree + 1, nx = S.nx, ny = S.ny;
  auto whole = [&](const Box& b) {
    return S.noflow && b.x0 == 0 && b.y0 == 0 && b.x1 == nx && b.y1 == ny;
  };
  // column widths of the local (oversampled) and patch launches, which fix
  // the half-block layout of their factors
  int lmax = 1, pmax = 1;
  for (int i = 0; i < m; ++i) {
    lmax = std::max(lmax, M.oboxes[i].bx());
    if (S.sweeps > 0) pmax = std::max(pmax, M.pboxes[i].bx());
  }
  const int lcols = box_cols(lmax), pcols = box_cols(pmax);
  auto hstride = [&](const Box& b, int cols) {
    const long long w = half_block_words(b.bx(), cols);
    return (int)((w + epv - 1) / epv * epv);
  };
  // per subdomain (in parallel): the jobs with sizes only, the Robin data of
  // its oversampled problems and its faces of Gamma_i
  struct Part {
    FactorJob lj, pj;
    SubJob sj;
    std::vector<OverRhs> rhs;
    std::vector<GamFace> gam;
  };
  std::vector<Part> part(m);
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < m; ++i) {
    Part& P = part[i];
    const Box& bi = M.boxes[i];
    const Box& oi = M.oboxes[i];
    const int ni = M.dof_offset[i + 1] - M.dof_offset[i];
    const int ns = (int)M.sides[i].size();
    P.lj = FactorJob{oi.x0, oi.y0, oi.bx(), oi.by(), 1, whole(oi) ? 1 : 0, hstride(oi, lcols),
                     lcols, 0, 0, 0, 0};
    if (S.sweeps > 0) {
      const Box& pb = M.pboxes[i];
      P.pj = FactorJob{pb.x0, pb.y0, pb.bx(), pb.by(), 0, whole(pb) ? 1 : 0,
                       hstride(pb, pcols), pcols, 0, 0, -1, -1};
    }
    SubJob& sj = P.sj;
    sj = SubJob{};
    sj.obx = oi.bx();
    sj.oby = oi.by();
    sj.opin = P.lj.pin;
    sj.lbx = bi.bx();
    sj.lby = bi.by();
    sj.ox = bi.x0 - oi.x0;
    sj.oy = bi.y0 - oi.y0;
    sj.ni = ni;
    sj.nsides = ns;
    sj.dof0 = M.dof_offset[i];
    // Robin data of the oversampled problems: P_q on side ks of the
    // oversampled box, times the face conductance
    for (int k = 0; k < ni; ++k) {
      const int dof = M.dof_offset[i] + k;
      const int ks = M.dofs[dof][1], kq = M.dofs[dof][2];
      const std::vector<Face> fs = side_faces(oi, ks, nx);
      const int nf = (int)fs.size();
      for (int j = 0; j < nf; ++j) {
        const Face& f = fs[j];
        const double t = f.kind == 0 ? txv(S, f.row, f.col) : tyv(S, f.row, f.col);
        const double rho = robin_rho(S, S.K[f.inside], t);
        P.rhs.push_back(OverRhs{k, loc_of(oi, f.inside, nx), rho * legendre(kq, xi_of(j, nf))});
      }
    }
    // faces of Gamma_i, side by side in the order of M.sides[i]
    for (int si = 0; si < ns; ++si) {
      const GammaSide gs = make_side(S, bi, M.sides[i][si]);
      const int nfs = (int)gs.faces.size();
      for (int j = 0; j < nfs; ++j) {
        const Face& f = gs.faces[j];
        GamFace g{};
        g.ocin = loc_of(oi, f.inside, nx);
        g.ocout = M.oversample == 0 ? -1 : loc_of(oi, f.outside, nx);
        g.si = si;
        g.side = gs.side;
        g.j = j;
        g.nfs = nfs;
        g.rho = gs.rho[j];
        g.b = gs.b[j];
        g.t = gs.t[j];
        g.Kin = gs.Kin[j];
        g.Kout = gs.Kout[j];
        P.gam.push_back(g);
      }
    }
  }
  // offsets, in subdomain order
  T = DeviceTables();
  T.mbf_off.assign(m + 1, 0);
  T.col_off.assign(m + 1, 0);
  size_t nrhs = 0, ngam = 0;
  for (const Part& P : part) {
    nrhs += P.rhs.size();
    ngam += P.gam.size();
  }
  T.rhs.reserve(nrhs);
  T.gam.reserve(ngam);
  long long buf = 0;
  for (int i = 0; i < m; ++i) {
    Part& P = part[i];
    SubJob& sj = P.sj;
    const long long lc = (long long)sj.lbx * sj.lby, oc = (long long)sj.obx * sj.oby;
    T.max_local = std::max(T.max_local, sj.obx);
    P.lj.doffS = T.ldinv_len;
    P.lj.coffS = T.lcoup_len;
    P.lj.d64 = buf;
    P.lj.c64 = buf + oc * sj.obx;
    T.ldinv_len += (long long)P.lj.bs * sj.oby;
    T.lcoup_len += oc;
    sj.o64 = P.lj.d64;
    sj.oc64 = P.lj.c64;
    buf += oc * sj.obx + oc;
    T.local_jobs.push_back(P.lj);
    if (S.sweeps > 0) {
      T.max_patch = std::max(T.max_patch, P.pj.bx);
      P.pj.doffS = T.pdinv_len;
      P.pj.coffS = T.pcoup_len;
      T.pdinv_len += (long long)P.pj.bs * P.pj.by;
      T.pcoup_len += (long long)P.pj.bx * P.pj.by;
      T.patch_jobs.push_back(P.pj);
    }
    sj.oscr = buf;
    buf += sj.ni * oc;
    sj.rhs0 = (int)T.rhs.size();
    T.rhs.insert(T.rhs.end(), P.rhs.begin(), P.rhs.end());
    sj.rhs1 = (int)T.rhs.size();
    sj.gam0 = (int)T.gam.size();
    T.gam.insert(T.gam.end(), P.gam.begin(), P.gam.end());
    sj.gam1 = (int)T.gam.size();
    T.mbf_off[i + 1] = T.mbf_off[i] + sj.ni * lc;
    T.col_off[i + 1] = T.col_off[i] + (long long)sj.ni * sj.nsides * nb;
    sj.mbf = T.mbf_off[i];
    sj.col = T.col_off[i];
    T.subs.push_back(sj);
  }
  T.buf_len = buf;
  for (const auto& d : M.dofs) {
    T.dof_side.push_back(d[1]);
    T.dof_q.push_back(d[2]);
  }
}

void assemble_coarse(HostSetup& S, const double* colU, const double* colP,
                     const std::vector<long long>& col_off) {
  // Row (e, kind, q) of C couples the dofs of the two subdomains of edge e,
  // L (left / lower) before R: C[r][(L, k)] = colU_L[k][side of L facing
  // e][q] (flux rows) or colP_L[...] (pressure rows); R's entries likewise,
  // with a minus sign on its pressure moments.
  const Maps& M = S.maps;
  const int nc = M.nc(), nbm = M.degree + 1;
  const int E = (int)M.edges.size();
  auto side_index = [&](int i, int side) {
    const auto& sd = M.sides[i];
    return (int)(std::find(sd.begin(), sd.end(), side) - sd.begin());
  };
  S.Crp.assign(nc + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int L = M.edges[e][0], R = M.edges[e][1];
    const int w = (M.dof_offset[L + 1] - M.dof_offset[L]) + (M.dof_offset[R + 1] - M.dof_offset[R]);
    for (int r = M.row_offset[e]; r < M.row_offset[e + 1]; ++r) S.Crp[r + 1] = w;
  }
  S.pin_row = -1;
  S.pin_dof = -1;
  if (S.noflow && E > 0) {
    const int L0 = M.edges[0][0], o0 = M.edges[0][2];
    S.pin_row = M.row_offset[0];
    S.pin_dof = M.dof_of(L0, o0 == 0 ? SE : SN, 0);
    S.Crp[S.pin_row + 1] = 1;
  }
  for (int r = 0; r < nc; ++r) S.Crp[r + 1] += S.Crp[r];
  S.Cci.assign(S.Crp[nc], 0);
  S.Cv.assign(S.Crp[nc], 0.0);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e) {
    const int L = M.edges[e][0], R = M.edges[e][1], o = M.edges[e][2];
    const int sl = side_index(L, o == 0 ? SE : SN), sr = side_index(R, o == 0 ? SW : SS);
    const int nsl = (int)M.sides[L].size(), nsr = (int)M.sides[R].size();
    const int nb = M.nbasis(M.edges[e][4]);
    for (int kind = 0; kind < 2; ++kind)
      for (int q = 0; q < nb; ++q) {
        const int r = M.row_offset[e] + kind * nb + q;
        int at = S.Crp[r];
        if (r == S.pin_row) {
          S.Cci[at] = S.pin_dof;
          S.Cv[at] = 1.0;
          continue;
        }
        const double* src = kind == 0 ? colU : colP;
        for (int k = 0; k < M.dof_offset[L + 1] - M.dof_offset[L]; ++k, ++at) {
          S.Cci[at] = M.dof_offset[L] + k;
          S.Cv[at] = src[col_off[L] + ((long long)k * nsl + sl) * nbm + q];
        }
        const double sign = kind == 0 ? 1.0 : -1.0;
        for (int k = 0; k < M.dof_offset[R + 1] - M.dof_offset[R]; ++k, ++at) {
          S.Cci[at] = M.dof_offset[R] + k;
          S.Cv[at] = sign * src[col_off[R] + ((long long)k * nsr + sr) * nbm + q];
        }
      }
  }
}

void host_setup(HostSetup& S, const mrcm_grid& g, const mrcm_params& p, const double* K,
                int nthreads) {
  host_prepare(S, g, p, K);
  const Maps& M = S.maps;
  const int m = M.m, nb = M.degree + 1;
  S.over.resize(m);
  S.patch.resize(S.sweeps > 0 ? m : 0);
  S.mbf.resize(m);
  std::vector<SubResult> sub(m);

  int err_code = 0;
  std::string err_msg;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int i = 0; i < m; ++i) {
    try {
      const Box& bi = M.boxes[i];
      const Box& oi = M.oboxes[i];
      if (S.sweeps > 0) S.patch[i] = factor_box(S, M.pboxes[i], false);
      S.over[i] = factor_box(S, oi, true);
      std::vector<GammaSide> gam;
      for (int s : M.sides[i]) gam.push_back(make_side(S, bi, s));
      const int Ni = M.dof_offset[i + 1] - M.dof_offset[i];
      const size_t nloc = (size_t)bi.bx() * bi.by();
      S.mbf[i].assign((size_t)Ni * nloc, 0.0);
      sub[i].colU.assign(Ni, std::vector<std::vector<double>>(gam.size(), std::vector<double>(nb)));
      sub[i].colP = sub[i].colU;
      std::vector<double> ph((size_t)oi.bx() * oi.by());
      for (int k = 0; k < Ni; ++k) {
        // oversampled problem k: P_q Robin data on side ks of hat-Omega_i
        const int ks = M.dofs[M.dof_offset[i] + k][1], kq = M.dofs[M.dof_offset[i] + k][2];
        GammaSide os = make_side(S, oi, ks);
        std::fill(ph.begin(), ph.end(), 0.0);
        const int nf = (int)os.faces.size();
        for (int j = 0; j < nf; ++j)
          ph[loc_of(oi, os.faces[j].inside, S.nx)] += os.rho[j] * legendre(kq, xi_of(j, nf));
        box_solve(S.over[i], ph.data());
        // the multiscale basis function is its restriction to Omega_i
        double* pk = &S.mbf[i][(size_t)k * nloc];
        for (int y = bi.y0; y < bi.y1; ++y)
          for (int x = bi.x0; x < bi.x1; ++x)
            pk[(size_t)(y - bi.y0) * bi.bx() + (x - bi.x0)] =
                ph[(size_t)(y - oi.y0) * oi.bx() + (x - oi.x0)];
        // and its flux and pressure moments on Gamma_i (columns of C)
        for (size_t si = 0; si < gam.size(); ++si) {
          const GammaSide& gs = gam[si];
          const int nfs = (int)gs.faces.size();
          for (int j = 0; j < nfs; ++j) {
            const double pc = ph[loc_of(oi, gs.faces[j].inside, S.nx)];
            double U, pi;
            if (M.oversample == 0) {
              const double lam = gs.side == ks ? legendre(kq, xi_of(j, nfs)) : 0.0;
              U = gs.rho[j] * (pc - lam);
              pi = lam + gs.b[j] * U;
            } else {
              const double pn = ph[loc_of(oi, gs.faces[j].outside, S.nx)];
              U = gs.t[j] * (pc - pn);
              pi = (gs.Kin[j] * pc + gs.Kout[j] * pn) / (gs.Kin[j] + gs.Kout[j]);
            }
            for (int q = 0; q < M.nbasis(nfs); ++q) {
              const double w = legendre(q, xi_of(j, nfs));
              sub[i].colU[k][si][q] += w * U;
              sub[i].colP[k][si][q] += w * pi;
            }
          }
        }
      }
    } catch (const Error& e) {
#pragma omp critical
      {
        if (!err_code) {
          err_code = e.code;
          err_msg = e.what();
        }
      }
    }
  }
  if (err_code) throw Error(err_code, err_msg);
  std::vector<long long> col_off(m + 1, 0);
  for (int i = 0; i < m; ++i)
    col_off[i + 1] = col_off[i] + (long long)(M.dof_offset[i + 1] - M.dof_offset[i]) *
                                      (long long)M.sides[i].size() * nb;
  std::vector<double> cu((size_t)col_off[m]), cp((size_t)col_off[m]);
  for (int i = 0; i < m; ++i) {
    const int ns = (int)M.sides[i].size();
    for (size_t k = 0; k < sub[i].colU.size(); ++k)
      for (int si = 0; si < ns; ++si)
        for (int q = 0; q < nb; ++q) {
          const size_t at = (size_t)col_off[i] + ((size_t)k * ns + si) * nb + q;
          cu[at] = sub[i].colU[k][si][q];
          cp[at] = sub[i].colP[k][si][q];
        }
  }
  assemble_coarse(S, cu.data(), cp.data(), col_off);
}

}  // namespace mrcm
