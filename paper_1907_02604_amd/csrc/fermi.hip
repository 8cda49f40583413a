// Fermi level of stored Gauss rules (Eq. Eqn:LSSGQ:Fermi_level:GQ with the node weights of
// Eq. eq:free_cg): the two pass kernels, their launcher for a plan, and the variant of the
// solve that allocates nothing, whose state lives in a file-scope device array.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "sgq.h"
#include "sgq_common.h"

namespace sgq {
int report_error(int code, const std::string& msg);

// Fermi level of stored Gauss rules: the mu at which
//   N(mu) = 2 sum_q n_q sum_k w_k g(theta_k; mu)
// equals ne.  N increases strictly with mu.  A first pass brackets the level by every rule
// point -+ 60 kT and totals the count; then safeguarded Newton steps (dN/dmu =
// 2 sum n w g (1 - g) / kT; a step that leaves the bracket is replaced by bisection) run
// until |N - ne| <= tol ne, the bracket shrinks to rounding, or kFermiSteps steps.
//
// Every pass spreads the rule points over the whole chip: fermi_partial_kernel writes one
// partial sum per workgroup, and fermi_update_kernel (one wavefront) combines them in a
// fixed order and takes the step.  The host enqueues kFermiSteps pass pairs; once the
// state says done, the remaining launches return at once.  Points more than 36 kT from mu
// count as fully occupied or empty (g differs from 0 or 1 by less than 2.4e-16 there).
// State ws[0..5] = mu, lo, hi, N, step, done (0 running, 1 finished, 2 error); partials
// from ws[16], four per workgroup.  out[0] = mu, out[1] = N(mu), out[2] = steps taken.
__global__ __launch_bounds__(kFermiThreads) void fermi_partial_kernel(
    const double* __restrict__ tw, const double* __restrict__ weight, int nq, int kmax,
    double kT, int mode, double* __restrict__ ws) {
  constexpr int NW = kFermiThreads / kWave;
  __shared__ double red[4][NW];
  if (mode == 1 && ws[5] != 0.0) return;   // the same value for every lane: uniform exit
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const unsigned ntot = (unsigned)nq * (unsigned)kmax;   // < 2^31 (checked by the host)
  const double mu = ws[0];
  double a0, a1, a2 = 0.0, a3 = 0.0;
  if (mode == 0) {
    a0 = __builtin_inf();    // lowest rule point
    a1 = -__builtin_inf();   // highest
  } else {
    a0 = 0.0;                // sum n w g
    a1 = 0.0;                // sum n w g (1 - g)
  }
  for (unsigned e = blockIdx.x * kFermiThreads + tid; e < ntot; e += gridDim.x * kFermiThreads) {
    const double th = tw[2 * e], w = tw[2 * e + 1], n = weight[e / (unsigned)kmax];
    if (mode == 0) {
      if (!isfinite(th) || !isfinite(w) || !isfinite(n)) a3 = 1.0;
      if (w > 0.0) {
        a0 = fmin(a0, th);
        a1 = fmax(a1, th);
        a2 += n * w;
      }
    } else if (w > 0.0) {
      const double x = (th - mu) / kT;
      const double nw = n * w;
      if (x < -36.0) {
        a0 += nw;
      } else if (x <= 36.0) {
        const double g = fermi_occ(x);
        a0 += nw * g;
        a1 += nw * g * (1.0 - g);
      }
    }
  }
  if (mode == 0) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      a0 = fmin(a0, __shfl_xor(a0, off, kWave));
      a1 = fmax(a1, __shfl_xor(a1, off, kWave));
      a3 = fmax(a3, __shfl_xor(a3, off, kWave));
    }
  } else {
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
  }
  a2 = wave_sum(a2);
  if (lane == 0) {
    red[0][wave] = a0;
    red[1][wave] = a1;
    red[2][wave] = a2;
    red[3][wave] = a3;
  }
  __syncthreads();
  if (tid == 0) {
    double b0 = red[0][0], b1 = red[1][0], b2 = red[2][0], b3 = red[3][0];
    for (int w = 1; w < NW; ++w) {
      b0 = mode == 0 ? fmin(b0, red[0][w]) : b0 + red[0][w];
      b1 = mode == 0 ? fmax(b1, red[1][w]) : b1 + red[1][w];
      b2 += red[2][w];
      b3 = fmax(b3, red[3][w]);
    }
    double* part = ws + 16 + 4 * blockIdx.x;
    part[0] = b0;
    part[1] = b1;
    part[2] = b2;
    part[3] = b3;
  }
}

__global__ __launch_bounds__(kWave) void fermi_update_kernel(int nparts, int mode, double ne,
                                                             double kT, double tol,
                                                             double* __restrict__ ws,
                                                             double* __restrict__ out,
                                                             int* status) {
  const int lane = threadIdx.x;
  if (mode == 1 && ws[5] != 0.0) return;
  const double* part = ws + 16;
  double a0, a1, a2 = 0.0, a3 = 0.0;
  if (mode == 0) {
    a0 = __builtin_inf();
    a1 = -__builtin_inf();
  } else {
    a0 = 0.0;
    a1 = 0.0;
  }
  for (int b = lane; b < nparts; b += kWave) {
    a0 = mode == 0 ? fmin(a0, part[4 * b]) : a0 + part[4 * b];
    a1 = mode == 0 ? fmax(a1, part[4 * b + 1]) : a1 + part[4 * b + 1];
    a2 += part[4 * b + 2];
    a3 = fmax(a3, part[4 * b + 3]);
  }
  if (mode == 0) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      a0 = fmin(a0, __shfl_xor(a0, off, kWave));
      a1 = fmax(a1, __shfl_xor(a1, off, kWave));
      a3 = fmax(a3, __shfl_xor(a3, off, kWave));
    }
  } else {
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
  }
  a2 = wave_sum(a2);
  if (lane != 0) return;
  if (mode == 0) {
    *status = 0;   // this call's latch
    const double total = 2.0 * a2 + (a3 != 0.0 ? __builtin_nan("") : 0.0);
    if (!(isfinite(total) && ne > 0.0 && ne < total)) {
      atomicOr(status, isfinite(total) ? kStatusRange : kStatusNonFinite);
      out[0] = out[1] = __builtin_nan("");
      out[2] = 0.0;
      ws[5] = 2.0;
      return;
    }
    const double lo = a0 - 60.0 * kT, hi = a1 + 60.0 * kT;
    ws[0] = 0.5 * (lo + hi);
    ws[1] = lo;
    ws[2] = hi;
    ws[3] = 0.0;
    ws[4] = 0.0;
    ws[5] = 0.0;
    return;
  }
  const double N = 2.0 * a0, dN = 2.0 * a1 / kT, f = N - ne;
  double mu = ws[0], lo = ws[1], hi = ws[2];
  const int it = (int)ws[4];
  bool done = fabs(f) <= tol * ne || it >= kFermiSteps - 1;
  if (!done) {
    if (f < 0.0) lo = mu; else hi = mu;
    done = hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(mu));
  }
  if (done) {
    out[0] = mu;
    out[1] = N;
    out[2] = (double)(it + 1);
    ws[5] = 1.0;
    return;
  }
  const double cand = mu - f / dN;
  ws[0] = (dN > 0.0 && cand > lo && cand < hi) ? cand : 0.5 * (lo + hi);
  ws[1] = lo;
  ws[2] = hi;
  ws[3] = N;
  ws[4] = (double)(it + 1);
}

// ------------------------------------------------------------------ host launcher
hipError_t launch_fermi_level(const double* tw, const double* weight, int nq, int kmax,
                              double ne, double kT, double tol, double* out, int* status,
                              double* ws, hipStream_t s) {
  // at most kFermiBlocks partial sums: the workspace holds 16 + 4 kFermiBlocks doubles
  const size_t ntot = (size_t)nq * kmax;
  const int parts = (int)std::min<size_t>(kFermiBlocks, (ntot + kFermiThreads - 1) / kFermiThreads);
  for (int step = -1; step < kFermiSteps; ++step) {
    const int mode = step < 0 ? 0 : 1;
    hipLaunchKernelGGL(fermi_partial_kernel, dim3(parts), dim3(kFermiThreads), 0, s, tw, weight, nq,
                       kmax, kT, mode, ws);
    hipLaunchKernelGGL(fermi_update_kernel, dim3(1), dim3(kWave), 0, s, parts, mode, ne, kT, tol, ws,
                       out, status);
  }
  return hipGetLastError();
}


// ------------------------------------------------------------------ allocation-free variant
// The state and partial sums of one solve (kFermiWs doubles) and the status word, in a
// file-scope device array: every GPU holds its own copy until the process ends, and every
// call on that GPU shares it.
constexpr int kFermiWs = 16 + 4 * kFermiBlocks;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kFermiWs + 1];

// Maps the status bits of the solve to an sgq_status code in the caller's word.
__global__ void fermi_status_code_kernel(const int* bits, int32_t* code) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int b = *bits;
  *code = (b & kStatusNonFinite) ? SGQ_ENONFINITE : (b & kStatusRange) ? SGQ_ERANGE : SGQ_OK;
}

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up once per device.  In host
// code the array's name is only a host-side stand-in; kernels get this address.
static int scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return report_error(SGQ_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return report_error(SGQ_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return report_error(SGQ_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return SGQ_OK;
}

}  // namespace sgq

extern "C" int sgq_fermi_level_noalloc(const double* theta_w, const double* node_weight,
                                       int32_t n_nodes, int32_t kmax, double n_electrons,
                                       double kT, double tol, double* result, int32_t* status,
                                       void* stream) {
  using namespace sgq;
  if (!theta_w || !node_weight || !result || !status) return report_error(SGQ_EINVAL, "null argument");
  if (n_nodes < 1 || kmax < 1) return report_error(SGQ_EINVAL, "n_nodes and kmax must be >= 1");
  if ((int64_t)n_nodes * kmax >= ((int64_t)1 << 31))
    return report_error(SGQ_EINVAL, "n_nodes * kmax must stay below 2^31 rule points");
  if (!(kT > 0.0) || !std::isfinite(kT)) return report_error(SGQ_EINVAL, "kT must be finite and > 0");
  if (!(n_electrons > 0.0) || !std::isfinite(n_electrons))
    return report_error(SGQ_EINVAL, "n_electrons must be finite and > 0");
  if (!(tol > 0.0) || !std::isfinite(tol)) return report_error(SGQ_EINVAL, "tol must be finite and > 0");
  double* ws = nullptr;
  int st = scratch_address(&ws);
  if (st != SGQ_OK) return st;
  int* bits = reinterpret_cast<int*>(ws + kFermiWs);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_fermi_level(theta_w, node_weight, n_nodes, kmax, n_electrons, kT, tol,
                                    result, bits, ws, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fermi_status_code_kernel, dim3(1), dim3(1), 0, s, bits, status);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return report_error(SGQ_EHIP, std::string("Fermi-level launch: ") + hipGetErrorString(e));
  return SGQ_OK;
}
