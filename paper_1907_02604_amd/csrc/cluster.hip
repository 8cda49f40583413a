// Cluster sampling of the energy (Eq. eq:free_cg with the cluster averages of
// Eq. eq:free_cg_sampling).
//
// The host side, sgq_cluster_build (the clusters C_q of grid points within a ball of radius
// r around each energy sampling point, merged into one ascending node list, and the
// clusters as CSR positions in it), lives in host.cpp.
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
