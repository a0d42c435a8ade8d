// Internal declarations of the MRCM-OS library (host side).
#pragma once

#include <algorithm>
#include <array>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mrcm.h"

namespace mrcm {

enum Side { SW = 0, SE = 1, SS = 2, SN = 3 };

// Error carried to the C ABI as a return code plus message.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

struct Box {
  int x0, x1, y0, y1;
  int bx() const { return x1 - x0; }
  int by() const { return y1 - y0; }
  bool operator==(const Box& o) const {
    return x0 == o.x0 && x1 == o.x1 && y0 == o.y0 && y1 == o.y1;
  }
};

// Decomposition maps (Section 2.1): subdomains, oversampled regions,
// smoothing patches, interior edges, coarse dofs and coarse rows.
struct Maps {
  int nx = 0, ny = 0, sx = 0, sy = 0, mx = 0, my = 0, m = 0;
  int oversample = 0, overlap = 0, degree = 1;
  std::vector<Box> boxes, oboxes, pboxes;
  std::vector<int32_t> owner;
  std::vector<std::vector<int>> sides;        // interior sides per subdomain, W E S N order
  std::vector<std::array<int, 5>> edges;      // L, R, orientation, start, length
  std::vector<std::array<int, 3>> dofs;       // subdomain, side, q
  std::vector<int32_t> dof_offset;            // m + 1
  std::vector<std::array<int, 3>> rows;       // edge, kind (0 flux, 1 pressure), q
  std::vector<int32_t> row_offset;            // first coarse row of every edge, E + 1
  int nc() const { return dof_offset.empty() ? 0 : dof_offset.back(); }
  // Functions per side: P_0..P_degree, capped at the number of faces.
  int nbasis(int side_faces) const { return std::min(degree + 1, side_faces); }
  int dof_of(int i, int side, int q) const;   // -1 when absent
};

Maps build_maps(const mrcm_grid& g, const mrcm_params& p);
std::vector<int> interior_sides(const Box& b, int nx, int ny);
int side_len(const Box& b, int side);

// One face of the side of a cell box, in increasing coordinate.
struct Face {
  int inside, outside;  // global cell ids
  int kind;             // 0: x-face tx[row*(nx+1)+col], 1: y-face ty[row*nx+col]
  int row, col;
};
std::vector<Face> side_faces(const Box& b, int side, int nx);

// Legendre polynomial P_q at xi (three-term recurrence).
double legendre(int q, double xi);

// Message returned by mrcm_last_error() on the calling thread.
void set_last_error(const std::string& msg);

// The device allocator pair of mrcm_set_allocator (both null: hipMalloc /
// hipFree), read under its lock, for contexts being set up.
void current_allocator(mrcm_alloc_fn* alloc, mrcm_free_fn* release);

}  // namespace mrcm
