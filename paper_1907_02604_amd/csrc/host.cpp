// Host-only parts of libsgq (see host.h): error messages, argument validation, the host
// Gauss rule, the cluster lists of the energy sampling (Eq. eq:free_cg_sampling), and the
// geometry the set-up calls upload (node cube offsets, dV gather lists, FE mesh buckets).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

#include "host.h"
#include "sgq.h"

// The tridiagonal solver is written once for the kernels and the host; this file is built
// by the host compiler only, so its functions carry no device annotation here.
#define SGQ_HD
#include "tridiag.h"

namespace sgq {

static thread_local std::string g_error;

int report_error(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

int box_half_width(double rc, double h) {
  // grid offsets d from the nearest grid point that can lie within rc: d < rc/h + 1/2
  return (int)std::ceil(rc / h + 0.5) - 1;
}

std::vector<int64_t> cube_offsets(const std::vector<int32_t>& half_width, int64_t n_grid) {
  const size_t nq = half_width.size();
  std::vector<int64_t> off(nq + 1, 0);
  for (size_t q = 0; q < nq; ++q) {
    const int64_t s = 2 * (int64_t)half_width[q] + 1;
    const int64_t n = half_width[q] < 0 ? n_grid : s * s * s;
    off[q + 1] = off[q] + (n + 3) / 4 * 4;
  }
  return off;
}

void gather_lists(const int32_t n[3], const std::vector<int32_t>& center,
                  const std::vector<int32_t>& half_width, int cell, std::vector<int32_t>& start,
                  std::vector<int32_t>& list) {
  const int C = cell;
  const int nx = n[0], ny = n[1], nz = n[2];
  const int ncx = (nx + C - 1) / C, ncy = (ny + C - 1) / C, ncz = (nz + C - 1) / C;
  const int64_t ncells = (int64_t)ncx * ncy * ncz;
  const int nq = (int)center.size();
  // the cells one axis of a cube meets (each once, also when the cube wraps)
  auto axis_cells = [&](int c, int R, int na, int nc, std::vector<int>& out) {
    out.clear();
    if (R < 0) {
      for (int i = 0; i < nc; ++i) out.push_back(i);
      return;
    }
    std::vector<char> seen(nc, 0);
    for (int x = c - R; x <= c + R; ++x) {
      const int cx = ((x % na) + na) % na / C;
      if (!seen[cx]) {
        seen[cx] = 1;
        out.push_back(cx);
      }
    }
  };
  start.assign(ncells + 1, 0);
  std::vector<int> ax, ay, az;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fill;
    if (pass == 1) {
      list.assign(start[ncells], 0);
      fill.assign(start.begin(), start.end() - 1);
    }
    for (int q = 0; q < nq; ++q) {
      const int c = center[q], R = half_width[q];
      axis_cells(c % nx, R, nx, ncx, ax);
      axis_cells((c / nx) % ny, R, ny, ncy, ay);
      axis_cells(c / (nx * ny), R, nz, ncz, az);
      for (int kz : az)
        for (int ky : ay)
          for (int kx : ax) {
            const int64_t k = kx + (int64_t)ncx * (ky + (int64_t)ncy * kz);
            if (pass == 0) ++start[k + 1];
            else list[fill[k]++] = q;
          }
    }
    if (pass == 0)
      for (int64_t i = 0; i < ncells; ++i) start[i + 1] += start[i];
  }
}

int fe_geometry(const int32_t n[3], const int64_t* esp_center, int32_t n_esp, const int32_t* tets,
                int32_t n_tets, int32_t max_fields, FeGeometry* g) {
  if (!n) return report_error(SGQ_EINVAL, "n is null");
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || n[a] > 65536) return report_error(SGQ_EINVAL, "grid extents must be in [1, 65536]");
  const int64_t npts = (int64_t)n[0] * n[1] * n[2];
  if (npts >= 2147483647LL) return report_error(SGQ_EINVAL, "grid has 2^31 or more points");
  if (n_esp < 1 || !esp_center) return report_error(SGQ_EINVAL, "no ESPs");
  if (n_tets < 0 || (n_tets > 0 && !tets)) return report_error(SGQ_EINVAL, "bad tetrahedra");
  if (max_fields < 1 || max_fields > 4) return report_error(SGQ_EINVAL, "max_fields must be in [1, 4]");
  g->esp.assign((size_t)4 * n_esp, 0);
  for (int32_t q = 0; q < n_esp; ++q) {
    const int64_t c = esp_center[q];
    if (c < 0 || c >= npts)
      return report_error(SGQ_EINVAL, "ESP " + std::to_string(q) + ": centre outside the grid");
    g->esp[4 * (size_t)q] = (int32_t)(c % n[0]);
    g->esp[4 * (size_t)q + 1] = (int32_t)((c / n[0]) % n[1]);
    g->esp[4 * (size_t)q + 2] = (int32_t)(c / ((int64_t)n[0] * n[1]));
    g->esp[4 * (size_t)q + 3] = (int32_t)c;
  }
  // orient, drop zero volumes (D is an exact integer: extents below 2^16)
  const size_t ntet = (size_t)std::max(n_tets, 1);
  g->tet.assign(4 * ntet, 0);
  std::vector<char> keep(ntet, 0);
  auto coord = [&](int v, int a) { return (int64_t)g->esp[4 * (size_t)v + a]; };
  g->kept = 0;
  for (int32_t t = 0; t < n_tets; ++t) {
    int v[4];
    for (int i = 0; i < 4; ++i) {
      v[i] = tets[4 * (size_t)t + i];
      if (v[i] < 0 || v[i] >= n_esp)
        return report_error(SGQ_EINVAL, "tetrahedron " + std::to_string(t) + ": vertex out of range");
    }
    int64_t u[3][3];
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) u[k][a] = coord(v[k + 1], a) - coord(v[0], a);
    const int64_t D = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
                      u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
                      u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
    if (D == 0) continue;
    if (D < 0) std::swap(v[0], v[1]);
    for (int i = 0; i < 4; ++i) g->tet[4 * (size_t)t + i] = v[i];
    keep[t] = 1;
    ++g->kept;
  }
  // bucket edge: about one kept tetrahedron per 2 bucket points
  const double per = g->kept > 0 ? (double)npts / g->kept : (double)npts;
  int bucket = (int)std::lround(2.0 * std::cbrt(per));
  bucket = std::max(2, std::min(bucket, 32));
  g->bucket = bucket;
  for (int a = 0; a < 3; ++a) g->nb[a] = (n[a] + bucket - 1) / bucket;
  const int64_t nbuckets = (int64_t)g->nb[0] * g->nb[1] * g->nb[2];
  std::vector<int64_t> count(nbuckets + 1, 0);
  auto for_buckets = [&](int32_t t, auto&& fn) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      int64_t mn = coord(g->tet[4 * (size_t)t], a), mx = mn;
      for (int i = 1; i < 4; ++i) {
        mn = std::min(mn, coord(g->tet[4 * (size_t)t + i], a));
        mx = std::max(mx, coord(g->tet[4 * (size_t)t + i], a));
      }
      lo[a] = (int)(mn / bucket);
      hi[a] = (int)(mx / bucket);
    }
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
      for (int by = lo[1]; by <= hi[1]; ++by)
        for (int bx = lo[0]; bx <= hi[0]; ++bx)
          fn(bx + (int64_t)g->nb[0] * (by + (int64_t)g->nb[1] * bz));
  };
  for (int32_t t = 0; t < n_tets; ++t)
    if (keep[t]) for_buckets(t, [&](int64_t b) { ++count[b + 1]; });
  for (int64_t b = 0; b < nbuckets; ++b) count[b + 1] += count[b];
  if (count[nbuckets] >= 2147483647LL)
    return report_error(SGQ_EINVAL, "bucket lists exceed 2^31 entries");
  g->bstart.assign(nbuckets + 1, 0);
  g->blist.assign(std::max<int64_t>(count[nbuckets], 1), 0);
  for (int64_t b = 0; b <= nbuckets; ++b) g->bstart[b] = (int32_t)count[b];
  std::vector<int64_t> fill(count.begin(), count.end() - 1);
  for (int32_t t = 0; t < n_tets; ++t)
    if (keep[t]) for_buckets(t, [&](int64_t b) { g->blist[fill[b]++] = t; });
  return SGQ_OK;
}

}  // namespace sgq

using sgq::box_half_width;
using sgq::kMaxDepth;
using sgq::report_error;
using sgq::tridiag_gauss;

extern "C" const char* sgq_last_error(void) { return sgq::g_error.c_str(); }

extern "C" int sgq_validate(const sgq_problem* prob, const int64_t* center,
                            const int32_t* half_width, const int32_t* depth) {
  if (!prob) return report_error(SGQ_EINVAL, "problem is null");
  for (int a = 0; a < 3; ++a)
    if (prob->n[a] < 1) return report_error(SGQ_EINVAL, "grid extent must be >= 1");
  double ng = (double)prob->n[0] * prob->n[1] * prob->n[2];
  if (ng >= 2147483647.0) return report_error(SGQ_EINVAL, "grid has 2^31 or more points");
  if (!(prob->h > 0.0) || !std::isfinite(prob->h)) return report_error(SGQ_EINVAL, "h must be > 0");
  if (prob->n_atoms < 0) return report_error(SGQ_EINVAL, "n_atoms < 0");
  if (prob->n_proj != 0 && prob->n_proj != 4) return report_error(SGQ_EINVAL, "n_proj must be 0 or 4");
  if (prob->precision != SGQ_FP64 && prob->precision != SGQ_FP32)
    return report_error(SGQ_EINVAL, "precision must be SGQ_FP64 or SGQ_FP32");
  int m = 3;
  if (prob->n_proj == 4) {
    if (!(prob->proj_rc > 0.0) || !(prob->proj_rg > 0.0) || !std::isfinite(prob->proj_rc) ||
        !std::isfinite(prob->proj_rg))
      return report_error(SGQ_EINVAL, "projector radii must be > 0");
    m = std::max(3, box_half_width(prob->proj_rc, prob->h));
    if (2 * m + 1 > 33) return report_error(SGQ_EINVAL, "projector cutoff spans more than 33 points");
  }
  if (prob->n_nodes < 0) return report_error(SGQ_EINVAL, "n_nodes < 0");
  if (prob->n_nodes > 0 && (!center || !half_width || !depth))
    return report_error(SGQ_EINVAL, "node arrays are null");
  int nmin = std::min(prob->n[0], std::min(prob->n[1], prob->n[2]));
  for (int q = 0; q < prob->n_nodes; ++q) {
    if (center[q] < 0 || (double)center[q] >= ng)
      return report_error(SGQ_EINVAL, "node " + std::to_string(q) + ": centre outside the grid");
    if (depth[q] < 1 || depth[q] > kMaxDepth)
      return report_error(SGQ_EINVAL, "node " + std::to_string(q) + ": depth outside [1, 128]");
    int R = half_width[q];
    if (R < -1) return report_error(SGQ_EINVAL, "node " + std::to_string(q) + ": half_width < -1");
    if (R >= 0 && 2 * R + 1 > nmin - 2 * m)
      return report_error(SGQ_EINVAL, "node " + std::to_string(q) +
                                  ": cube side exceeds the grid minus the stencil/projector reach");
  }
  return SGQ_OK;
}

extern "C" int sgq_gauss_rule_host(const double* alpha, const double* beta, int K, double* theta,
                                   double* weight) {
  if (!alpha || !theta || !weight || K < 1 || K > kMaxDepth || (K > 1 && !beta))
    return report_error(SGQ_EINVAL, "bad arguments");
  double a[kMaxDepth], b[kMaxDepth], z[kMaxDepth];
  for (int i = 0; i < K; ++i) a[i] = alpha[i];
  for (int i = 0; i + 1 < K; ++i) b[i] = beta[i];
  if (!tridiag_gauss(a, b, z, K)) return report_error(SGQ_ENONFINITE, "tridiagonal QR did not converge");
  std::vector<int> idx(K);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return a[i] < a[j]; });
  for (int k = 0; k < K; ++k) {
    theta[k] = a[idx[k]];
    weight[k] = z[idx[k]] * z[idx[k]];
  }
  return SGQ_OK;
}

extern "C" int sgq_cluster_build(const int32_t n[3], double h, const int64_t* esp_center,
                                 int32_t n_esp, double radius, const double* esp_weight,
                                 int64_t node_capacity, int64_t member_capacity,
                                 int64_t* node_center, int32_t* node_esp, double* node_weight,
                                 int64_t* member_offset, int32_t* member_node, int64_t* n_nodes,
                                 int64_t* n_members) {
  if (!n || !n_nodes || !n_members) return report_error(SGQ_EINVAL, "null argument");
  if (n_esp < 0) return report_error(SGQ_EINVAL, "n_esp < 0");
  if (n_esp > 0 && !esp_center) return report_error(SGQ_EINVAL, "esp_center is null");
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1) return report_error(SGQ_EINVAL, "grid extent must be >= 1");
  const int64_t nx = n[0], ny = n[1], nz = n[2], ng = nx * ny * nz;
  if (ng >= 2147483647LL) return report_error(SGQ_EINVAL, "grid has 2^31 or more points");
  if (!(h > 0.0) || !std::isfinite(h)) return report_error(SGQ_EINVAL, "h must be finite and > 0");
  if (!(radius >= 0.0) || !std::isfinite(radius))
    return report_error(SGQ_EINVAL, "radius must be finite and >= 0");
  if (node_weight && !esp_weight)
    return report_error(SGQ_EINVAL, "node_weight needs esp_weight");
  for (int32_t q = 0; q < n_esp; ++q)
    if (esp_center[q] < 0 || esp_center[q] >= ng)
      return report_error(SGQ_EINVAL, "ESP " + std::to_string(q) + ": centre outside the grid");

  // Offsets of the ball: squared distance in grid units (an integer) against (r/h)^2
  // widened by a relative 1e-9, so a radius equal to a lattice distance keeps that shell.
  // Each axis offset is the minimum-image representative of its residue class, so every
  // grid point of the periodic box is reached at most once per cluster.
  const double lim = (radius / h) * (radius / h) * (1.0 + 1e-9);
  const int64_t reach = (int64_t)std::floor(std::sqrt(lim));
  const int64_t dims[3] = {nx, ny, nz};
  int64_t lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = std::max(-reach, -((dims[a] - 1) / 2));
    hi[a] = std::min(reach, dims[a] / 2);
  }
  std::vector<int64_t> off;   // (dx, dy, dz) triples
  for (int64_t dz = lo[2]; dz <= hi[2]; ++dz)
    for (int64_t dy = lo[1]; dy <= hi[1]; ++dy)
      for (int64_t dx = lo[0]; dx <= hi[0]; ++dx)
        if ((double)(dx * dx + dy * dy + dz * dz) <= lim) {
          off.push_back(dx);
          off.push_back(dy);
          off.push_back(dz);
        }
  const int64_t per = (int64_t)off.size() / 3;
  const int64_t total = per * n_esp;
  *n_members = total;

  // Members of every cluster as ascending linear indices.
  std::vector<int64_t> lin((size_t)total);
  for (int32_t q = 0; q < n_esp; ++q) {
    const int64_t c = esp_center[q];
    const int64_t cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
    int64_t* out = lin.data() + (size_t)q * per;
    for (int64_t i = 0; i < per; ++i) {
      const int64_t x = ((cx + off[3 * i]) % nx + nx) % nx;
      const int64_t y = ((cy + off[3 * i + 1]) % ny + ny) % ny;
      const int64_t z = ((cz + off[3 * i + 2]) % nz + nz) % nz;
      out[i] = x + nx * (y + ny * z);
    }
    std::sort(out, out + per);
  }
  std::vector<int64_t> nodes(lin);
  std::sort(nodes.begin(), nodes.end());
  nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
  *n_nodes = (int64_t)nodes.size();

  const bool want_nodes = node_center || node_esp || node_weight;
  const bool want_members = member_offset || member_node;
  if (want_nodes && node_capacity < *n_nodes)
    return report_error(SGQ_EINVAL, "node arrays hold " + std::to_string(node_capacity) +
                                        " entries, " + std::to_string(*n_nodes) + " needed");
  if (member_node && member_capacity < total)
    return report_error(SGQ_EINVAL, "member_node holds " + std::to_string(member_capacity) +
                                        " entries, " + std::to_string(total) + " needed");
  if (!want_nodes && !want_members) return SGQ_OK;

  if (node_center) std::copy(nodes.begin(), nodes.end(), node_center);
  if (node_esp) std::fill(node_esp, node_esp + nodes.size(), -1);
  if (node_weight) std::fill(node_weight, node_weight + nodes.size(), 0.0);
  if (member_offset) member_offset[0] = 0;
  for (int32_t q = 0; q < n_esp; ++q) {
    const int64_t* mem = lin.data() + (size_t)q * per;
    if (member_offset) member_offset[q + 1] = (int64_t)(q + 1) * per;
    const double share = esp_weight ? esp_weight[q] / (double)per : 0.0;
    for (int64_t i = 0; i < per; ++i) {
      const int32_t k =
          (int32_t)(std::lower_bound(nodes.begin(), nodes.end(), mem[i]) - nodes.begin());
      if (member_node) member_node[(size_t)q * per + i] = k;
      if (node_esp && node_esp[k] < 0) node_esp[k] = q;
      if (node_weight) node_weight[k] += share;
    }
  }
  return SGQ_OK;
}
