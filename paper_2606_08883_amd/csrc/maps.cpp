// Decomposition geometry and index maps (Section 2.1: Omega_i, Gamma_i,
// hat-Omega_i; smoothing patches for the overlapping Schwarz sweeps).
// Integer-only host code; the orderings are documented in include/mrcm.h.
#include <algorithm>

#include "internal.h"

namespace mrcm {

std::vector<int> interior_sides(const Box& b, int nx, int ny) {
  std::vector<int> s;
  if (b.x0 > 0) s.push_back(SW);
  if (b.x1 < nx) s.push_back(SE);
  if (b.y0 > 0) s.push_back(SS);
  if (b.y1 < ny) s.push_back(SN);
  return s;
}

int side_len(const Box& b, int side) { return (side == SW || side == SE) ? b.by() : b.bx(); }

static Box grow(const Box& b, int g, int nx, int ny) {
  return Box{std::max(0, b.x0 - g), std::min(nx, b.x1 + g), std::max(0, b.y0 - g),
             std::min(ny, b.y1 + g)};
}

int Maps::dof_of(int i, int side, int q) const {
  for (int k = dof_offset[i]; k < dof_offset[i + 1]; ++k)
    if (dofs[k][1] == side && dofs[k][2] == q) return k;
  return -1;
}

Maps build_maps(const mrcm_grid& g, const mrcm_params& p) {
  if (g.nx < 1 || g.ny < 1 || p.sx < 1 || p.sy < 1 || p.oversample < 0 ||
      p.smooth_overlap < 0 || p.smooth_sweeps < 0 || p.iface_degree < 0 ||
      p.iface_degree > 8 || !(p.alpha > 0.0) || (p.beta_len != 0 && p.beta_len != 1) ||
      p.precision < 0 || p.precision > 2)
    throw Error(MRCM_EINVAL, "invalid grid or method parameters");
  for (int s = 0; s < 4; ++s)
    if (g.bc[s] != 0 && g.bc[s] != 1) throw Error(MRCM_EINVAL, "bc must be 0 or 1");
  if ((int64_t)g.nx * g.ny > (int64_t)1 << 30) throw Error(MRCM_EINVAL, "grid too large");
  Maps M;
  M.nx = g.nx;
  M.ny = g.ny;
  M.sx = p.sx;
  M.sy = p.sy;
  M.oversample = p.oversample;
  M.overlap = p.smooth_overlap;
  M.degree = p.iface_degree;
  M.mx = (g.nx + p.sx - 1) / p.sx;
  M.my = (g.ny + p.sy - 1) / p.sy;
  M.m = M.mx * M.my;
  M.boxes.resize(M.m);
  for (int J = 0; J < M.my; ++J)
    for (int I = 0; I < M.mx; ++I)
      M.boxes[J * M.mx + I] = Box{I * p.sx, std::min(g.nx, (I + 1) * p.sx), J * p.sy,
                                  std::min(g.ny, (J + 1) * p.sy)};
  M.oboxes.resize(M.m);
  M.pboxes.resize(M.m);
  M.sides.resize(M.m);
  M.owner.assign((size_t)g.nx * g.ny, 0);
  for (int i = 0; i < M.m; ++i) {
    const Box& b = M.boxes[i];
    M.oboxes[i] = grow(b, p.oversample, g.nx, g.ny);
    M.pboxes[i] = grow(b, p.smooth_overlap, g.nx, g.ny);
    M.sides[i] = interior_sides(b, g.nx, g.ny);
    if (interior_sides(M.oboxes[i], g.nx, g.ny) != M.sides[i])
      throw Error(MRCM_EINVAL,
                  "oversampling reaches the domain boundary across an interior side");
    for (int y = b.y0; y < b.y1; ++y)
      for (int x = b.x0; x < b.x1; ++x) M.owner[(size_t)y * g.nx + x] = i;
  }
  for (int J = 0; J < M.my; ++J)
    for (int I = 0; I + 1 < M.mx; ++I) {
      int L = J * M.mx + I;
      M.edges.push_back({L, L + 1, 0, M.boxes[L].y0, M.boxes[L].by()});
    }
  for (int J = 0; J + 1 < M.my; ++J)
    for (int I = 0; I < M.mx; ++I) {
      int L = J * M.mx + I;
      M.edges.push_back({L, L + M.mx, 1, M.boxes[L].x0, M.boxes[L].bx()});
    }
  M.dof_offset.push_back(0);
  for (int i = 0; i < M.m; ++i) {
    for (int s : M.sides[i])
      for (int q = 0; q < M.nbasis(side_len(M.boxes[i], s)); ++q) M.dofs.push_back({i, s, q});
    M.dof_offset.push_back((int32_t)M.dofs.size());
  }
  M.row_offset.push_back(0);
  for (size_t e = 0; e < M.edges.size(); ++e) {
    const int nb = M.nbasis(M.edges[e][4]);
    for (int kind = 0; kind < 2; ++kind)
      for (int q = 0; q < nb; ++q) M.rows.push_back({(int)e, kind, q});
    M.row_offset.push_back((int32_t)M.rows.size());
  }
  if (M.rows.size() != M.dofs.size()) throw Error(MRCM_EINVAL, "coarse system is not square");
  return M;
}

std::vector<Face> side_faces(const Box& b, int side, int nx) {
  std::vector<Face> f;
  if (side == SW) {
    for (int y = b.y0; y < b.y1; ++y) f.push_back({y * nx + b.x0, y * nx + b.x0 - 1, 0, y, b.x0});
  } else if (side == SE) {
    for (int y = b.y0; y < b.y1; ++y)
      f.push_back({y * nx + b.x1 - 1, y * nx + b.x1, 0, y, b.x1});
  } else if (side == SS) {
    for (int x = b.x0; x < b.x1; ++x)
      f.push_back({b.y0 * nx + x, (b.y0 - 1) * nx + x, 1, b.y0, x});
  } else {
    for (int x = b.x0; x < b.x1; ++x)
      f.push_back({(b.y1 - 1) * nx + x, b.y1 * nx + x, 1, b.y1, x});
  }
  return f;
}

double legendre(int q, double xi) {
  double pm = 1.0, p = xi;
  if (q == 0) return 1.0;
  for (int k = 1; k < q; ++k) {
    double pn = ((2.0 * k + 1.0) * xi * p - k * pm) / (k + 1.0);
    pm = p;
    p = pn;
  }
  return p;
}

}  // namespace mrcm
