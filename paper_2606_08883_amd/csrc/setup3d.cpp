// Host-side FP64 set-up of T on 3-D grids (Section 2 with d = 3; Section
// 2.1): the decomposition into box subdomains with six sides, face
// transmissibilities, Robin coefficients beta = alpha L / K_H, plane-block
// LDL^T factors of the oversampled Robin problems and of the smoothing
// patches, the multiscale basis functions as restrictions of the oversampled
// solutions with tensor Legendre data, the interface system (weak flux and
// pressure continuity per interface and test function) and its dense
// inverse.  host_apply evaluates T from these tables in the order the device
// runs it.
#include "setup3d.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <tuple>

namespace mrcm3d {

namespace {

enum { SW = 0, SE = 1, SS = 2, SN = 3, SB = 4, ST = 5 };

inline int axis_of(int side) { return side / 2; }
// The two tangential axes of a side, lower first.
inline void tangential(int side, int& t0, int& t1) {
  const int a = axis_of(side);
  t0 = a == 0 ? 1 : 0;
  t1 = a == 2 ? 1 : 2;
}

inline double& tx_at(Setup& S, int z, int y, int x) {
  return S.tx[((size_t)z * S.ny + y) * (S.nx + 1) + x];
}
inline double& ty_at(Setup& S, int z, int y, int x) {
  return S.ty[((size_t)z * (S.ny + 1) + y) * S.nx + x];
}
inline double& tz_at(Setup& S, int z, int y, int x) {
  return S.tz[((size_t)z * S.ny + y) * S.nx + x];
}
inline double txc(const Setup& S, int z, int y, int x) {
  return S.tx[((size_t)z * S.ny + y) * (S.nx + 1) + x];
}
inline double tyc(const Setup& S, int z, int y, int x) {
  return S.ty[((size_t)z * (S.ny + 1) + y) * S.nx + x];
}
inline double tzc(const Setup& S, int z, int y, int x) {
  return S.tz[((size_t)z * S.ny + y) * S.nx + x];
}

// Transmissibility of the face on side `side` of cell (x, y, z).
double face_t(const Setup& S, int x, int y, int z, int side) {
  switch (side) {
    case SW: return txc(S, z, y, x);
    case SE: return txc(S, z, y, x + 1);
    case SS: return tyc(S, z, y, x);
    case SN: return tyc(S, z, y + 1, x);
    case SB: return tzc(S, z, y, x);
    default: return tzc(S, z + 1, y, x);
  }
}

double robin_rho(const Setup& S, double Kc, double t) {
  return 1.0 / (1.0 / (2.0 * Kc) + S.alpha * S.Lcells / t);
}

void face_transmissibilities(Setup& S) {
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  S.tx.assign((size_t)nz * ny * (nx + 1), 0.0);
  S.ty.assign((size_t)nz * (ny + 1) * nx, 0.0);
  S.tz.assign((size_t)(nz + 1) * ny * nx, 0.0);
  auto K = [&](int x, int y, int z) { return S.K[((size_t)z * ny + y) * nx + x]; };
  auto hm = [](double a, double b) { return 2.0 * a * b / (a + b); };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      for (int x = 1; x < nx; ++x) tx_at(S, z, y, x) = hm(K(x - 1, y, z), K(x, y, z));
      if (S.bc[SW]) tx_at(S, z, y, 0) = 2.0 * K(0, y, z);
      if (S.bc[SE]) tx_at(S, z, y, nx) = 2.0 * K(nx - 1, y, z);
    }
  for (int z = 0; z < nz; ++z)
    for (int x = 0; x < nx; ++x) {
      for (int y = 1; y < ny; ++y) ty_at(S, z, y, x) = hm(K(x, y - 1, z), K(x, y, z));
      if (S.bc[SS]) ty_at(S, z, 0, x) = 2.0 * K(x, 0, z);
      if (S.bc[SN]) ty_at(S, z, ny, x) = 2.0 * K(x, ny - 1, z);
    }
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      for (int z = 1; z < nz; ++z) tz_at(S, z, y, x) = hm(K(x, y, z - 1), K(x, y, z));
      if (S.bc[SB]) tz_at(S, 0, y, x) = 2.0 * K(x, y, 0);
      if (S.bc[ST]) tz_at(S, nz, y, x) = 2.0 * K(x, y, nz - 1);
    }
}

Box grown(const Box& b, int g, const int dims[3]) {
  Box o = b;
  for (int a = 0; a < 3; ++a) {
    o.lo[a] = std::max(0, b.lo[a] - g);
    o.hi[a] = std::min(dims[a], b.hi[a] + g);
  }
  return o;
}

std::vector<int> interior_sides(const Box& b, const int dims[3]) {
  std::vector<int> s;
  for (int a = 0; a < 3; ++a) {
    if (b.lo[a] > 0) s.push_back(2 * a);
    if (b.hi[a] < dims[a]) s.push_back(2 * a + 1);
  }
  return s;
}

// Face counts of a side along its two tangential axes.
void side_extent(const Box& b, int side, int& n0, int& n1) {
  int t0, t1;
  tangential(side, t0, t1);
  n0 = b.n(t0);
  n1 = b.n(t1);
}

int nbasis_1d(int degree, int len) { return std::min(degree + 1, len); }

// Faces of one side of a box, lower tangential axis fastest.
SideData side_data(const Setup& S, const Box& b, int side) {
  SideData d;
  d.side = side;
  int t0, t1;
  tangential(side, t0, t1);
  const int a = axis_of(side);
  const bool hi = side % 2 == 1;
  d.n0 = b.n(t0);
  d.n1 = b.n(t1);
  const int pos = hi ? b.hi[a] - 1 : b.lo[a];
  const int out = hi ? pos + 1 : pos - 1;
  for (int c1 = b.lo[t1]; c1 < b.hi[t1]; ++c1)
    for (int c0 = b.lo[t0]; c0 < b.hi[t0]; ++c0) {
      int ci[3], co[3];
      ci[t0] = co[t0] = c0;
      ci[t1] = co[t1] = c1;
      ci[a] = pos;
      co[a] = out;
      const long long cin = cell_of(S, ci[0], ci[1], ci[2]);
      const long long cout = cell_of(S, co[0], co[1], co[2]);
      const double t = face_t(S, ci[0], ci[1], ci[2], side);
      const double Kin = S.K[(size_t)cin];
      const double Kout = cout >= 0 ? S.K[(size_t)cout] : 1.0;
      const double bb = S.alpha * S.Lcells / t;
      const double rho = 1.0 / (1.0 / (2.0 * Kin) + bb);
      d.in.push_back(cin);
      d.out.push_back(cout);
      d.t.push_back(t);
      d.rho.push_back(rho);
      d.b.push_back(bb);
      d.Kin.push_back(Kin);
      d.Kout.push_back(Kout);
    }
  return d;
}

// In-place SPD inverse of an n x n row-major matrix (Cholesky).
bool spd_inverse(double* A, int n) {
  std::vector<double> L((size_t)n * n, 0.0), Li((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
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
      for (int k = j; k < i; ++k) s -= L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = s / L[(size_t)i * n + i];
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

// Plane-block LDL^T of the box matrix: faces inside the box couple as in A,
// domain-boundary faces keep the global condition, faces leaving the box
// inside the domain carry rho_f (robin) or t_f with zero data beyond (the
// principal submatrix of A).
PlaneFactor factor_box(const Setup& S, const Box& b, bool robin, bool keep_full) {
  PlaneFactor F;
  const int bx = b.n(0), by = b.n(1), bz = b.n(2), P = bx * by;
  F.P = P;
  F.bz = bz;
  bool whole = true;
  const int dims[3] = {S.nx, S.ny, S.nz};
  for (int a = 0; a < 3; ++a) whole = whole && b.lo[a] == 0 && b.hi[a] == dims[a];
  F.pin = S.noflow && whole ? 1 : 0;
  const int H = half_rows(P);
  F.dinv.assign((size_t)bz * H * P, 0.0);
  F.coup.assign((size_t)bz * P, 0.0);
  std::vector<double> D((size_t)P * P), Dp((size_t)P * P);
  for (int j = 0; j < bz; ++j) {
    const int z = b.lo[2] + j;
    std::fill(D.begin(), D.end(), 0.0);
    for (int yy = 0; yy < by; ++yy)
      for (int xx = 0; xx < bx; ++xx) {
        const int x = b.lo[0] + xx, y = b.lo[1] + yy, c = yy * bx + xx;
        const double Kc = S.K[(size_t)cell_of(S, x, y, z)];
        double diag = 0.0;
        for (int side = 0; side < 6; ++side) {
          double t = face_t(S, x, y, z, side);
          const int a = axis_of(side);
          const int coord = a == 0 ? x : a == 1 ? y : z;
          const bool at_box = side % 2 == 0 ? coord == b.lo[a] : coord == b.hi[a] - 1;
          const bool in_domain = side % 2 == 0 ? coord > 0 : coord < dims[a] - 1;
          if (at_box && in_domain && robin) t = robin_rho(S, Kc, t);
          diag += t;
        }
        D[(size_t)c * P + c] = diag;
        if (xx > 0) {
          const double t = txc(S, z, y, x);
          D[(size_t)c * P + c - 1] = -t;
          D[(size_t)(c - 1) * P + c] = -t;
        }
        if (yy > 0) {
          const double t = tyc(S, z, y, x);
          D[(size_t)c * P + c - bx] = -t;
          D[(size_t)(c - bx) * P + c] = -t;
        }
        if (j > 0) F.coup[(size_t)j * P + c] = tzc(S, z, y, x);
      }
    if (F.pin && j == 0) {
      for (int c = 0; c < P; ++c) {
        D[c] = 0.0;
        D[(size_t)c * P] = 0.0;
      }
      D[0] = 1.0;
    }
    if (F.pin && j == 1) F.coup[(size_t)P] = 0.0;
    if (j > 0) {
      const double* Tj = &F.coup[(size_t)j * P];
      for (int a = 0; a < P; ++a)
        for (int c = 0; c < P; ++c) D[(size_t)a * P + c] -= Tj[a] * Dp[(size_t)a * P + c] * Tj[c];
    }
    if (!spd_inverse(D.data(), P))
      throw Error(MRCM_ESINGULAR, "non-positive pivot in a local factorisation");
    double* Dh = &F.dinv[(size_t)j * H * P];
    for (int d = 0; d < H; ++d)
      for (int t = 0; t < P; ++t) Dh[(size_t)d * P + t] = D[(size_t)t * P + (t + d) % P];
    if (keep_full) F.full.insert(F.full.end(), D.begin(), D.end());
    std::swap(D, Dp);
  }
  return F;
}

// Values of a box-local solution at a global cell.
inline double at(const Box& b, const double* v, long long cell, const Setup& S) {
  const int x = (int)(cell % S.nx), y = (int)((cell / S.nx) % S.ny), z = (int)(cell / ((long long)S.nx * S.ny));
  return v[((size_t)(z - b.lo[2]) * b.n(1) + (y - b.lo[1])) * b.n(0) + (x - b.lo[0])];
}

// Tensor Legendre value of basis function (a, b) at face f of a side n0 x n1.
inline double basis_value(int a, int bq, int f, int n0, int n1) {
  return legendre_face(a, f % n0, n0) * legendre_face(bq, f / n0, n1);
}

}  // namespace

double legendre_face(int q, int j, int n) {
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

long long cell_of(const Setup& S, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= S.nx || y >= S.ny || z >= S.nz) return -1;
  return ((long long)z * S.ny + y) * S.nx + x;
}

double plane_dot(const double* D, const double* v, int P, int t) {
  const int H = half_rows(P);
  double u0 = D[t] * v[t], u1 = 0.0, w0 = 0.0, w1 = 0.0;
  int up = t, dn = t;
  for (int d = 1; d < H; ++d) {
    up = up + 1 == P ? 0 : up + 1;
    dn = dn == 0 ? P - 1 : dn - 1;
    const double* row = D + (size_t)d * P;
    double& u = d & 1 ? u1 : u0;
    double& w = d & 1 ? w1 : w0;
    u = std::fma(row[t], v[up], u);
    if (2 * d != P) w = std::fma(row[dn], v[dn], w);
  }
  return (u0 + u1) + (w0 + w1);
}

void box_solve_full(const PlaneFactor& F, double* x) {
  const int P = F.P, bz = F.bz;
  if (F.pin) x[0] = 0.0;
  std::vector<double> v(P);
  auto product = [&](const double* D, double* out, bool add) {
    for (int a = 0; a < P; ++a) {
      const double* row = D + (size_t)a * P;
      double s = 0.0;
      for (int c = 0; c < P; ++c) s += row[c] * v[c];
      out[a] = add ? out[a] + s : s;
    }
  };
  for (int j = 0; j < bz; ++j) {
    double* xj = x + (size_t)j * P;
    for (int c = 0; c < P; ++c)
      v[c] = j > 0 ? xj[c] + F.coup[(size_t)j * P + c] * x[(size_t)(j - 1) * P + c] : xj[c];
    product(&F.full[(size_t)j * P * P], xj, false);
  }
  for (int j = bz - 2; j >= 0; --j) {
    for (int c = 0; c < P; ++c) v[c] = F.coup[(size_t)(j + 1) * P + c] * x[(size_t)(j + 1) * P + c];
    product(&F.full[(size_t)j * P * P], x + (size_t)j * P, true);
  }
}

void box_solve(const PlaneFactor& F, double* x) {
  const int P = F.P, bz = F.bz, H = half_rows(P);
  if (F.pin) x[0] = 0.0;
  std::vector<double> v(P);
  for (int j = 0; j < bz; ++j) {
    double* xj = x + (size_t)j * P;
    for (int c = 0; c < P; ++c)
      v[c] = j > 0 ? std::fma(F.coup[(size_t)j * P + c], x[(size_t)(j - 1) * P + c], xj[c]) : xj[c];
    const double* D = &F.dinv[(size_t)j * H * P];
    for (int a = 0; a < P; ++a) xj[a] = plane_dot(D, v.data(), P, a);
  }
  for (int j = bz - 2; j >= 0; --j) {
    double* xj = x + (size_t)j * P;
    const double* xn = x + (size_t)(j + 1) * P;
    for (int c = 0; c < P; ++c) v[c] = F.coup[(size_t)(j + 1) * P + c] * xn[c];
    const double* D = &F.dinv[(size_t)j * H * P];
    for (int a = 0; a < P; ++a) xj[a] += plane_dot(D, v.data(), P, a);
  }
}

void host_setup(Setup& S, const mrcm3d_grid& g, const mrcm3d_params& p, const double* Kin) {
  if (g.nx < 1 || g.ny < 1 || g.nz < 1 || p.sx < 1 || p.sy < 1 || p.sz < 1 || p.oversample < 0 ||
      p.smooth_sweeps < 0 || p.smooth_overlap < 0 || p.iface_degree < 0 || !(p.alpha > 0.0) ||
      (p.precision != 0 && p.precision != 2))
    throw Error(MRCM_EINVAL, "invalid grid or parameters");
  S.nx = g.nx;
  S.ny = g.ny;
  S.nz = g.nz;
  for (int s = 0; s < 6; ++s) S.bc[s] = g.bc[s] ? 1 : 0;
  S.noflow = !(S.bc[0] || S.bc[1] || S.bc[2] || S.bc[3] || S.bc[4] || S.bc[5]);
  S.sx = p.sx;
  S.sy = p.sy;
  S.sz = p.sz;
  S.oversample = p.oversample;
  S.sweeps = p.smooth_sweeps;
  S.overlap = p.smooth_overlap;
  S.degree = p.iface_degree;
  S.precision = p.precision;
  S.alpha = p.alpha;
  S.Lcells = p.beta_len == 0 ? (double)std::max(p.sx, std::max(p.sy, p.sz)) : 1.0;
  S.n = (long long)g.nx * g.ny * g.nz;
  S.K.assign(Kin, Kin + S.n);
  for (long long c = 0; c < S.n; ++c)
    if (!(S.K[(size_t)c] > 0.0) || !std::isfinite(S.K[(size_t)c]))
      throw Error(MRCM_EINVAL, "K must be finite and positive on every cell");
  face_transmissibilities(S);
  const int dims[3] = {S.nx, S.ny, S.nz}, sizes[3] = {p.sx, p.sy, p.sz};
  for (int a = 0; a < 3; ++a) S.mdims[a] = (dims[a] + sizes[a] - 1) / sizes[a];
  S.m = S.mdims[0] * S.mdims[1] * S.mdims[2];
  for (int L = 0; L < S.mdims[2]; ++L)
    for (int J = 0; J < S.mdims[1]; ++J)
      for (int I = 0; I < S.mdims[0]; ++I) {
        const int idx[3] = {I, J, L};
        Box b;
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = idx[a] * sizes[a];
          b.hi[a] = std::min(dims[a], (idx[a] + 1) * sizes[a]);
        }
        S.boxes.push_back(b);
        S.oboxes.push_back(grown(b, p.oversample, dims));
        S.pboxes.push_back(grown(b, p.smooth_overlap, dims));
      }
  S.owner.assign((size_t)S.n, 0);
  for (int i = 0; i < S.m; ++i) {
    const Box& b = S.boxes[i];
    for (int z = b.lo[2]; z < b.hi[2]; ++z)
      for (int y = b.lo[1]; y < b.hi[1]; ++y)
        for (int x = b.lo[0]; x < b.hi[0]; ++x) S.owner[(size_t)cell_of(S, x, y, z)] = i;
  }
  S.sides.resize(S.m);
  for (int i = 0; i < S.m; ++i) {
    S.sides[i] = interior_sides(S.boxes[i], dims);
    if (interior_sides(S.oboxes[i], dims) != S.sides[i])
      throw Error(MRCM_EINVAL, "oversampling reaches the domain boundary across an interior side");
  }
  // interfaces: x first, then y, then z, each by (L, J, I) of the lower subdomain
  const int mx = S.mdims[0], my = S.mdims[1], mz = S.mdims[2];
  const int stride[3] = {1, mx, mx * my};
  for (int a = 0; a < 3; ++a)
    for (int L = 0; L < mz; ++L)
      for (int J = 0; J < my; ++J)
        for (int I = 0; I < mx; ++I) {
          const int c[3] = {I, J, L};
          if (c[a] + 1 < S.mdims[a]) {
            const int lo = (L * my + J) * mx + I;
            S.faces.push_back({lo, lo + stride[a], a});
          }
        }
  // coarse dofs: per subdomain, per interior side, tensor functions a fastest
  S.dof_off.assign(S.m + 1, 0);
  for (int i = 0; i < S.m; ++i) {
    for (int s : S.sides[i]) {
      int n0, n1;
      side_extent(S.boxes[i], s, n0, n1);
      const int b0 = nbasis_1d(S.degree, n0), b1 = nbasis_1d(S.degree, n1);
      for (int bq = 0; bq < b1; ++bq)
        for (int a = 0; a < b0; ++a)
          S.dofs.push_back({i, s, bq * b0 + a, a, bq});
    }
    S.dof_off[i + 1] = (int32_t)S.dofs.size();
  }
  S.nc = (int)S.dofs.size();
  auto dof_of = [&](int i, int side, int q) {
    for (int k = S.dof_off[i]; k < S.dof_off[i + 1]; ++k)
      if (S.dofs[k][1] == side && S.dofs[k][2] == q) return k;
    return -1;
  };
  // interface rows
  S.row_off.assign(S.faces.size() + 1, 0);
  for (size_t f = 0; f < S.faces.size(); ++f) {
    const int L = S.faces[f][0], R = S.faces[f][1], a = S.faces[f][2];
    const int sL = 2 * a + 1, sR = 2 * a;
    int n0, n1;
    side_extent(S.boxes[L], sL, n0, n1);
    const int nb = nbasis_1d(S.degree, n0) * nbasis_1d(S.degree, n1);
    for (int kind = 0; kind < 2; ++kind)
      for (int q = 0; q < nb; ++q) {
        S.rowL.push_back(dof_of(L, sL, q));
        S.rowR.push_back(dof_of(R, sR, q));
        S.rowKind.push_back(kind);
      }
    S.row_off[f + 1] = (int32_t)S.rowL.size();
  }
  if ((int)S.rowL.size() != S.nc) throw Error(MRCM_EINVAL, "interface system is not square");
  // the interface on each side of each subdomain
  std::vector<int> face_at((size_t)S.m * 6, -1);
  for (size_t f = 0; f < S.faces.size(); ++f) {
    const int L = S.faces[f][0], R = S.faces[f][1], a = S.faces[f][2];
    face_at[(size_t)L * 6 + 2 * a + 1] = (int)f;
    face_at[(size_t)R * 6 + 2 * a] = (int)f;
  }
  // face data of every side of Gamma_i: weights of the traces of a solution
  // with zero Robin data
  S.gam.resize(S.m);
  for (int i = 0; i < S.m; ++i)
    for (int s : S.sides[i]) {
      SideData d = side_data(S, S.boxes[i], s);
      d.w.resize(d.in.size());
      for (size_t f = 0; f < d.in.size(); ++f) {
        if (S.oversample == 0)
          d.w[f] = {d.rho[f], 0.0, d.b[f] * d.rho[f], 0.0};
        else
          d.w[f] = {d.t[f], -d.t[f], d.Kin[f] / (d.Kin[f] + d.Kout[f]),
                    d.Kout[f] / (d.Kin[f] + d.Kout[f])};
      }
      S.gam[i].push_back(d);
    }
  // factors, multiscale basis functions, and the columns of C
  S.over.resize(S.m);
  S.patch.resize(S.sweeps > 0 ? S.m : 0);
  S.mbf.resize(S.m);
  // entries of C by column owner: (row, column, value), each written once
  std::vector<std::vector<std::tuple<int, int, double>>> centries(S.m);
  int err = 0;
  std::string msg;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < S.m; ++i) {
    try {
      const Box& bi = S.boxes[i];
      const Box& oi = S.oboxes[i];
      if (S.sweeps > 0) S.patch[i] = factor_box(S, S.pboxes[i], false, false);
      S.over[i] = factor_box(S, oi, true, true);
      const int Ni = S.dof_off[i + 1] - S.dof_off[i];
      S.mbf[i].assign((size_t)Ni * bi.cells(), 0.0);
      std::vector<double> ph((size_t)oi.cells());
      for (int k = 0; k < Ni; ++k) {
        const auto& dk = S.dofs[S.dof_off[i] + k];
        const int ks = dk[1], ka = dk[3], kb = dk[4];
        // Legendre data on side ks of the oversampled box
        SideData os = side_data(S, oi, ks);
        std::fill(ph.begin(), ph.end(), 0.0);
        for (size_t f = 0; f < os.in.size(); ++f) {
          const long long c = os.in[f];
          const int x = (int)(c % S.nx), y = (int)((c / S.nx) % S.ny), z = (int)(c / ((long long)S.nx * S.ny));
          ph[((size_t)(z - oi.lo[2]) * oi.n(1) + (y - oi.lo[1])) * oi.n(0) + (x - oi.lo[0])] +=
              os.rho[f] * basis_value(ka, kb, (int)f, os.n0, os.n1);
        }
        box_solve_full(S.over[i], ph.data());
        double* pk = &S.mbf[i][(size_t)k * bi.cells()];
        for (int z = bi.lo[2]; z < bi.hi[2]; ++z)
          for (int y = bi.lo[1]; y < bi.hi[1]; ++y)
            for (int x = bi.lo[0]; x < bi.hi[0]; ++x)
              pk[((size_t)(z - bi.lo[2]) * bi.n(1) + (y - bi.lo[1])) * bi.n(0) + (x - bi.lo[0])] =
                  ph[((size_t)(z - oi.lo[2]) * oi.n(1) + (y - oi.lo[1])) * oi.n(0) + (x - oi.lo[0])];
        // moments of its traces on every side of Gamma_i: the column of C
        const int col = S.dof_off[i] + k;
        for (const SideData& d : S.gam[i]) {
          const int b0 = nbasis_1d(S.degree, d.n0), b1 = nbasis_1d(S.degree, d.n1);
          for (int bq = 0; bq < b1; ++bq)
            for (int a = 0; a < b0; ++a) {
              double su = 0.0, sp = 0.0;
              for (size_t f = 0; f < d.in.size(); ++f) {
                const double pin = at(oi, ph.data(), d.in[f], S);
                double U, Pi;
                if (S.oversample == 0) {
                  const double lam = d.side == ks ? basis_value(ka, kb, (int)f, d.n0, d.n1) : 0.0;
                  U = d.rho[f] * (pin - lam);
                  Pi = lam + d.b[f] * U;
                } else {
                  const double pout = at(oi, ph.data(), d.out[f], S);
                  U = d.w[f][0] * pin + d.w[f][1] * pout;
                  Pi = d.w[f][2] * pin + d.w[f][3] * pout;
                }
                const double bv = basis_value(a, bq, (int)f, d.n0, d.n1);
                su += bv * U;
                sp += bv * Pi;
              }
              // rows of the interface on this side: flux rows F_q, then
              // pressure rows with + for the lower subdomain (its E, N, T
              // sides) and - for the upper one
              const int q = bq * b0 + a;
              const int fidx = face_at[(size_t)i * 6 + d.side];
              const int r0 = S.row_off[fidx];
              const int nbf = (S.row_off[fidx + 1] - r0) / 2;
              const double sign = d.side % 2 == 1 ? 1.0 : -1.0;
              centries[i].emplace_back(r0 + q, col, su);
              centries[i].emplace_back(r0 + nbf + q, col, sign * sp);
            }
        }
      }
      std::vector<double>().swap(S.over[i].full);  // the full blocks are done with
    } catch (const Error& e) {
#pragma omp critical
      {
        err = e.code;
        msg = e.what();
      }
    }
  }
  if (err) throw Error(err, msg);
  // C in CSR; with no flow on every side the first flux row of the first
  // interface is replaced by the pin of its lower subdomain's first dof
  int pin_col = -1;
  if (S.noflow && !S.faces.empty()) {
    const int L0 = S.faces[0][0], a0 = S.faces[0][2];
    pin_col = dof_of(L0, 2 * a0 + 1, 0);
    S.pin_row = 0;
    S.rowKind[0] = 2;
  }
  std::vector<std::vector<std::pair<int, double>>> rows(S.nc);
  for (int i = 0; i < S.m; ++i)
    for (const auto& e : centries[i])
      if (std::get<0>(e) != S.pin_row) rows[std::get<0>(e)].push_back({std::get<1>(e), std::get<2>(e)});
  if (S.pin_row >= 0) rows[S.pin_row].push_back({pin_col, 1.0});
  S.Crp.assign(S.nc + 1, 0);
  for (int r = 0; r < S.nc; ++r) {
    std::sort(rows[r].begin(), rows[r].end());
    for (const auto& e : rows[r]) {
      S.Cci.push_back(e.first);
      S.Cv.push_back(e.second);
    }
    S.Crp[r + 1] = (int)S.Cci.size();
  }
  if (S.nc > 0) {
    // rows owned by each subdomain: flux rows by the lower one, pressure rows
    // by the upper one (as many as its dofs)
    std::vector<std::vector<int>> rows_of(S.m);
    for (int r = 0; r < S.nc; ++r) {
      const int f = (int)(std::upper_bound(S.row_off.begin(), S.row_off.end(), r) -
                          S.row_off.begin()) - 1;
      const int nbf = (S.row_off[f + 1] - S.row_off[f]) / 2;
      rows_of[r - S.row_off[f] < nbf ? S.faces[f][0] : S.faces[f][1]].push_back(r);
    }
    S.CF = mrcm::coarse_factor_tree(dissection3(S.mdims[0], S.mdims[1], S.mdims[2]), rows_of,
                                    S.dof_off, S.Crp, S.Cci, S.Cv,
                                    std::max(1, omp_get_max_threads()));
    // refinement to 1e-10 of the solution in FP64, to 1e-6 with FP32-stored
    // blocks (below their own effect on T), as in 2-D
    mrcm::coarse_refine_steps(S.CF, mrcm::coarse_refine_tol(S.precision),
                              mrcm::kCoarseRefineMax, std::max(1, omp_get_max_threads()));
  }
  // precision 2: the apply reads the plane blocks rounded to FP32 (the MBFs,
  // C and its factor above came from the FP64 blocks)
  if (S.precision == 2)
    for (auto* list : {&S.over, &S.patch})
      for (PlaneFactor& F : *list)
        for (double& x : F.dinv) x = (double)(float)x;
}

std::vector<mrcm::DissectionNode> dissection3(int mx, int my, int mz) {
  std::vector<mrcm::DissectionNode> tree;
  const int dims[3] = {mx, my, mz};
  auto id = [&](int x, int y, int z) { return (z * my + y) * mx + x; };
  std::function<int(std::array<int, 3>, std::array<int, 3>, int)> build =
      [&](std::array<int, 3> lo, std::array<int, 3> hi, int depth) -> int {
    for (int a = 0; a < 3; ++a)
      if (lo[a] >= hi[a]) return -1;
    mrcm::DissectionNode nd;
    nd.depth = depth;
    const int ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    auto add_region = [&](std::array<int, 3> l, std::array<int, 3> h, std::vector<int>& out) {
      for (int z = l[2]; z < h[2]; ++z)
        for (int y = l[1]; y < h[1]; ++y)
          for (int x = l[0]; x < h[0]; ++x) out.push_back(id(x, y, z));
    };
    if (ext[0] * ext[1] * ext[2] <= 8) {
      add_region(lo, hi, nd.fsub);
    } else {
      int ax = 0;
      for (int a = 1; a < 3; ++a)
        if (ext[a] > ext[ax]) ax = a;
      const int mid = (lo[ax] + hi[ax]) / 2;
      std::array<int, 3> h1 = hi, l2 = lo, pl = lo, ph = hi;
      h1[ax] = mid;
      l2[ax] = mid + 1;
      pl[ax] = mid;
      ph[ax] = mid + 1;
      const int c1 = build(lo, h1, depth + 1), c2 = build(l2, hi, depth + 1);
      if (c1 >= 0) nd.children.push_back(c1);
      if (c2 >= 0) nd.children.push_back(c2);
      add_region(pl, ph, nd.fsub);
    }
    // the border: the face neighbours of the region outside it
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        const int at = side == 0 ? lo[a] - 1 : hi[a];
        if (at < 0 || at >= dims[a]) continue;
        std::array<int, 3> l = lo, h = hi;
        l[a] = at;
        h[a] = at + 1;
        add_region(l, h, nd.usub);
      }
    std::sort(nd.usub.begin(), nd.usub.end());
    tree.push_back(nd);
    return (int)tree.size() - 1;
  };
  build({0, 0, 0}, {mx, my, mz}, 0);
  return tree;
}

void host_op_apply(const Setup& S, const double* x, double* y) {
  for (int z = 0; z < S.nz; ++z)
    for (int yy = 0; yy < S.ny; ++yy)
      for (int xx = 0; xx < S.nx; ++xx) {
        const long long c = cell_of(S, xx, yy, z);
        double v = 0.0;
        for (int side = 0; side < 6; ++side) {
          const double t = face_t(S, xx, yy, z, side);
          const int dx = side == 0 ? -1 : side == 1 ? 1 : 0;
          const int dy = side == 2 ? -1 : side == 3 ? 1 : 0;
          const int dz = side == 4 ? -1 : side == 5 ? 1 : 0;
          const long long o = cell_of(S, xx + dx, yy + dy, z + dz);
          v += t * (x[c] - (o >= 0 ? x[o] : 0.0));
        }
        y[c] = v;
      }
}

void host_apply(const Setup& S, const double* r, double* z) {
  std::vector<double> p((size_t)S.n, 0.0), mU(S.nc, 0.0), mP(S.nc, 0.0);
  auto box_vals = [&](const Box& b, const double* v, std::vector<double>& out) {
    out.resize((size_t)b.cells());
    size_t k = 0;
    for (int zz = b.lo[2]; zz < b.hi[2]; ++zz)
      for (int y = b.lo[1]; y < b.hi[1]; ++y)
        for (int x = b.lo[0]; x < b.hi[0]; ++x) out[k++] = v[(size_t)cell_of(S, x, y, zz)];
  };
  std::vector<double> ph;
  for (int i = 0; i < S.m; ++i) {
    const Box& bi = S.boxes[i];
    const Box& oi = S.oboxes[i];
    box_vals(oi, r, ph);
    box_solve(S.over[i], ph.data());
    for (int zz = bi.lo[2]; zz < bi.hi[2]; ++zz)
      for (int y = bi.lo[1]; y < bi.hi[1]; ++y)
        for (int x = bi.lo[0]; x < bi.hi[0]; ++x) {
          const long long c = cell_of(S, x, y, zz);
          p[(size_t)c] = at(oi, ph.data(), c, S);
        }
    for (int k = S.dof_off[i]; k < S.dof_off[i + 1]; ++k) {
      const int s = S.dofs[k][1], a = S.dofs[k][3], bq = S.dofs[k][4];
      const SideData* d = nullptr;
      for (const SideData& dd : S.gam[i])
        if (dd.side == s) d = &dd;
      double su = 0.0, sp = 0.0;
      for (size_t f = 0; f < d->in.size(); ++f) {
        const double pin = at(oi, ph.data(), d->in[f], S);
        const double pout = S.oversample == 0 ? pin : at(oi, ph.data(), d->out[f], S);
        const double bv = basis_value(a, bq, (int)f, d->n0, d->n1);
        su += bv * (d->w[f][0] * pin + d->w[f][1] * pout);
        sp += bv * (d->w[f][2] * pin + d->w[f][3] * pout);
      }
      mU[k] = su;
      mP[k] = sp;
    }
  }
  std::vector<double> g(S.nc), x(S.nc, 0.0);
  for (int t = 0; t < S.nc; ++t) {
    const int L = S.rowL[t], R = S.rowR[t];
    g[t] = S.rowKind[t] == 2 ? 0.0
           : S.rowKind[t] == 0 ? -(mU[L] + mU[R]) : -(mP[L] - mP[R]);
  }
  if (S.nc > 0) {
    std::vector<double> gnd(S.nc);
    for (int t = 0; t < S.nc; ++t) gnd[t] = S.CF.nd_scale[t] * g[S.CF.nd_row[t]];
    mrcm::coarse_solve_refined_host(S.CF, gnd.data(), x.data(), std::max(1, omp_get_max_threads()));
  }
  for (int i = 0; i < S.m; ++i) {
    const Box& bi = S.boxes[i];
    const int Ni = S.dof_off[i + 1] - S.dof_off[i];
    size_t q = 0;
    for (int zz = bi.lo[2]; zz < bi.hi[2]; ++zz)
      for (int y = bi.lo[1]; y < bi.hi[1]; ++y)
        for (int xx = bi.lo[0]; xx < bi.hi[0]; ++xx, ++q) {
          const long long c = cell_of(S, xx, y, zz);
          double s = p[(size_t)c];
          for (int k = 0; k < Ni; ++k) s += S.mbf[i][(size_t)k * bi.cells() + q] * x[S.dof_off[i] + k];
          p[(size_t)c] = s;
        }
  }
  std::vector<double> Ap((size_t)S.n), rho((size_t)S.n), e;
  for (int sw = 0; sw < S.sweeps; ++sw) {
    host_op_apply(S, p.data(), Ap.data());
    for (long long c = 0; c < S.n; ++c) rho[(size_t)c] = r[c] - Ap[(size_t)c];
    std::vector<double> corr((size_t)S.n, 0.0);
    for (int i = 0; i < S.m; ++i) {
      const Box& pb = S.pboxes[i];
      box_vals(pb, rho.data(), e);
      box_solve(S.patch[i], e.data());
      size_t k = 0;
      for (int zz = pb.lo[2]; zz < pb.hi[2]; ++zz)
        for (int y = pb.lo[1]; y < pb.hi[1]; ++y)
          for (int xx = pb.lo[0]; xx < pb.hi[0]; ++xx, ++k) {
            const long long c = cell_of(S, xx, y, zz);
            if (S.owner[(size_t)c] == i) corr[(size_t)c] = e[k];
          }
    }
    for (long long c = 0; c < S.n; ++c) p[(size_t)c] += corr[(size_t)c];
  }
  double mean = 0.0;
  if (S.noflow) {
    for (long long c = 0; c < S.n; ++c) mean += p[(size_t)c];
    mean /= (double)S.n;
  }
  for (long long c = 0; c < S.n; ++c) z[c] = p[(size_t)c] - mean;
}

}  // namespace mrcm3d
