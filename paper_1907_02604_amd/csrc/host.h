// Host-only parts of libsgq: error messages, argument validation, and the geometry the
// set-up calls build on the CPU (node cube offsets, the cell lists that gather the per-node
// dV cubes, the tetrahedron buckets of a fine-grid mesh).  Plain C++17 with no HIP header,
// so the same sources also build with g++ under the host sanitizers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sgq.h"

namespace sgq {

constexpr int kMaxDepth = 128;       // largest Lanczos depth K

// Sets the calling thread's error message (sgq_last_error) and returns code.
int report_error(int code, const std::string& msg);

// Grid offsets d from an atom's nearest grid point that can lie within the projector
// cutoff rc: |d| h < rc + h/2 on each axis.
int box_half_width(double rc, double h);

// Points of each node's cube rounded up to 4 (16-byte aligned FP32 cubes), as offsets into
// one array of all cubes: off[q] .. off[q+1].  half_width < 0 is the whole grid of n_grid
// points.
std::vector<int64_t> cube_offsets(const std::vector<int32_t>& half_width, int64_t n_grid);

// For every cell of edge `cell` points of the periodic grid n, the nodes (ascending) whose
// cube meets it, as CSR: nodes of cell c are list[start[c] .. start[c+1]).  Cubes wrap
// periodically; an untruncated node (half_width < 0) meets every cell.
void gather_lists(const int32_t n[3], const std::vector<int32_t>& center,
                  const std::vector<int32_t>& half_width, int cell, std::vector<int32_t>& start,
                  std::vector<int32_t>& list);

// Geometry of a tetrahedral mesh over ESPs on grid points: ESP coordinates, positively
// oriented tetrahedra (zero-volume ones dropped), and the tetrahedra filed under the cubic
// buckets their bounding boxes touch.
struct FeGeometry {
  std::vector<int32_t> esp;      // [n_esp][4]: x, y, z, linear index
  std::vector<int32_t> tet;      // [max(n_tets,1)][4]: vertices, positively oriented (0 if dropped)
  std::vector<int32_t> bstart;   // [nbuckets + 1] CSR offsets
  std::vector<int32_t> blist;    // tetrahedron ids, ascending within a bucket
  int bucket = 0;                // bucket edge (points)
  int nb[3] = {0, 0, 0};         // buckets per axis
  int32_t kept = 0;              // tetrahedra of non-zero volume
};

// Validates the arguments of sgq_fe_mesh_create and builds the geometry; returns SGQ_OK or
// SGQ_EINVAL (with the message set).
int fe_geometry(const int32_t n[3], const int64_t* esp_center, int32_t n_esp, const int32_t* tets,
                int32_t n_tets, int32_t max_fields, FeGeometry* g);

}  // namespace sgq
