// Cluster sampling of the energy (Eq. eq:free_cg with the cluster averages of
// Eq. eq:free_cg_sampling).
//
// Host side: sgq_cluster_build enumerates, for each energy sampling point (ESP) q, the
// cluster C_q of grid points within a ball of radius r around it, merges the clusters into
// one ascending node list (so a point shared by several clusters is evaluated once) and
// writes the clusters as a CSR list of positions in that node list.
//
// Device side: the segmented mean Fbar_q = (1/|C_q|) sum_{p in C_q} e_p over the per-node
// energies of a band_energy call on that node list, one wavefront per cluster with a fixed
// summation order; the weighted total sum_q n_q Fbar_q reuses the node-weighted sum kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "sgq.h"
#include "sgq_common.h"

namespace sgq {

hipError_t launch_weighted_sum(const double* e, const double* w, int n, double* out,
                               hipStream_t s);
int report_error(int code, const std::string& msg);

__global__ void clear_status_kernel(int* status) { *status = 0; }

// One wavefront per cluster.  Lane l adds members l, l+64, ... in ascending order; the
// 64 partial sums are combined by a fixed butterfly, so the result does not depend on
// scheduling.  A cluster with no members, offsets that decrease or pass n_members, or a
// member outside [0, nq) latches kStatusIndex and gets NaN; a non-finite member energy
// latches kStatusNonFinite.
__global__ __launch_bounds__(256) void cluster_mean_kernel(const double* __restrict__ e_node,
                                                           int nq,
                                                           const int64_t* __restrict__ offset,
                                                           const int32_t* __restrict__ member,
                                                           int64_t n_members, int n_esp,
                                                           double* __restrict__ fbar,
                                                           int* status) {
  const int lane = threadIdx.x & (kWave - 1);
  const int q = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (q >= n_esp) return;
  const int64_t beg = offset[q], end = offset[q + 1];
  bool bad_index = !(end > beg) || beg < 0 || end > n_members;
  double s = 0.0;
  bool bad_value = false;
  if (!bad_index) {
    for (int64_t i = beg + lane; i < end; i += kWave) {
      const int32_t p = member[i];
      if (p < 0 || p >= nq) {
        bad_index = true;
        continue;
      }
      const double e = e_node[p];
      if (!isfinite(e)) bad_value = true;
      s += e;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  const bool any_index = __any(bad_index), any_value = __any(bad_value);
  if (lane == 0) {
    if (any_index) atomicOr(status, kStatusIndex);
    if (any_value) atomicOr(status, kStatusNonFinite);
    fbar[q] = any_index ? __builtin_nan("") : s / (double)(end - beg);
  }
}

hipError_t launch_cluster_energy(const double* e_node, int nq, const int64_t* offset,
                                 const int32_t* member, int64_t n_members, int n_esp,
                                 const double* esp_weight, double* fbar, double* energy,
                                 int* status, hipStream_t s) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, s, status);
  constexpr int kWavesPerBlock = 4;
  const int blocks = (n_esp + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(cluster_mean_kernel, dim3(blocks), dim3(kWavesPerBlock * kWave), 0, s,
                     e_node, nq, offset, member, n_members, n_esp, fbar, status);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && energy) e = launch_weighted_sum(fbar, esp_weight, n_esp, energy, s);
  return e;
}

}  // namespace sgq

using sgq::report_error;

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
