// Persistent Lanczos-Gauss forward kernel for gfx950.
//
// One workgroup owns one node at a time (nodes are popped, most expensive first,
// from a device counter), so every reduction of the Lanczos step is a workgroup
// reduction and no cross-workgroup synchronisation exists.  Per node q and step j
// (paper: Lanczos quadrature of Eq. eq:9, density of Eq.
// Eqn:LSSGQ:Electron_density:GQ):
//
//   S_j  u_j = H q_j            stencil + local potential + projector apply, writes U
//        alpha_j = q_j . u_j    (FP64 accumulation)
//   F_j  w = u_j - sum_{i<=j} c_i q_i, stored unnormalised as W_{j+1}; in the same
//        sweep  D_i = W_i . w  and |w|^2 (FP64 accumulation of FP32 products).
//        beta_j = |w|, q_{j+1} = w / beta_j (the scale is applied lazily).
//
// The full-reorthogonalisation coefficients c_i = q_i . u_j are obtained without a
// second sweep over the basis: c_j = alpha_j and, for i < j, from the symmetry of H
// and the three-term relation, c_i = beta_{i-1} G_{i-1} + alpha_i G_i + beta_i G_{i+1}
// with G_i = q_i . q_j the Gram column measured (exactly, in FP64) in the previous
// sweep and G_j = 1.  Every Lanczos step therefore reads the stored basis once.
// The Gauss rule comes from the FP64 tridiagonal eigensolver; quadrature in FP64.
// A node's basis and u_j rows live in its workgroup's slot, or, for a node given retained
// storage (sgq_plan_set_retain), in that storage, which the next backward call reads.
#include "lanczos_device.h"

namespace sgq {

template <typename T, int BLOCK, int KG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void lanczos_forward_kernel(LaunchParams P) {
  __shared__ NodeState<T, BLOCK> st_shared;
  SGQ_L NodeState<T, BLOCK>& st = *(SGQ_L NodeState<T, BLOCK>*)(&st_shared);
  const int tid = threadIdx.x;
  SGQ_G T* __restrict__ W = (SGQ_G T*)P.W + (size_t)blockIdx.x * P.slot_stride;
  SGQ_G T* __restrict__ U = (SGQ_G T*)P.U + (size_t)blockIdx.x * P.npad;
  if (tid == 0) st.orth_tol = sizeof(T) == 4 ? 3.4526698300124393e-4 : 1.4901161193847656e-8;

  for (;;) {
    if (tid == 0) st.node = atomicAdd(P.queue, 1);
    __syncthreads();
    const int qi = st.node;
    if (qi >= P.n_nodes) break;
    const int q = P.order[qi];
    node_setup<T, BLOCK>(P, st, q);
    const int K = P.depth[q];
    if (st.abort) {
      if (tid == 0) P.tri_k[q] = -1;
      __syncthreads();
      continue;
    }
    // a retained node's basis and its u_j rows go to its own storage
    const int rs = P.Wr ? P.ret_slot[q] : -1;
    const size_t roff = (size_t)(rs < 0 ? 0 : rs) * P.kmax_out * P.npad;
    const int keff = rs >= 0 ? run_lanczos<T, BLOCK, KG>(P, st, (SGQ_G T*)P.Wr + roff,
                                                         (SGQ_G T*)P.Ur + roff, P.npad, K)
                             : run_lanczos<T, BLOCK, KG>(P, st, W, U, 0, K);
    // ---- the tridiagonal of the node, for the Gauss-rule kernel
    double* tri = P.tri + (size_t)q * 2 * P.kmax_out;
    for (int k = tid; k < keff; k += BLOCK) {
      tri[k] = st.alpha[k];
      tri[P.kmax_out + k] = k + 1 < keff ? st.beta[k] : 0.0;
    }
    if (tid == 0) P.tri_k[q] = keff;
    __syncthreads();
  }
}

// LDS array of one thread: element i at p[i * stride].
struct LdsColumn {
  SGQ_L double* p;
  int stride;
  __device__ SGQ_L double& operator[](int i) const { return p[i * stride]; }
};

// Gauss rule and quadrature of every node (one thread per node, nodes in cost order so a
// wave holds tridiagonals of similar size): implicit-shift QR of T_K for the nodes
// lambda_k and the weights w_k = (first eigenvector component)^2, then
// rho = 2 h^-3 sum_k w_k g(lambda_k), e = 2 sum_k w_k F(lambda_k), and the sorted rule.
// LDS holds the thread's diagonal, off-diagonal and first-row arrays, interleaved by
// thread.
__global__ void gauss_rule_kernel(LaunchParams P) {
  extern __shared__ double lds_tri[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int i = blockIdx.x * nt + t;
  if (i >= P.n_nodes) return;
  const int q = P.order[i];
  const int kmax = P.kmax_out;
  const int keff = P.tri_k[q];
  if (keff < 0) {   // node skipped by the Lanczos kernel (status latched there)
    double nan = __builtin_nan("");
    if (P.rho) P.rho[q] = nan;
    if (P.e_node) P.e_node[q] = nan;
    if (P.k_eff) P.k_eff[q] = 0;
    // a NaN rule, so that a Fermi-level solve on these rules latches a non-finite input
    // even though it starts with a clear status word
    if (P.theta_w)
      for (int k = 0; k < 2 * kmax; ++k) P.theta_w[(size_t)q * kmax * 2 + k] = nan;
    return;
  }
  SGQ_L double* base = (SGQ_L double*)lds_tri;
  const LdsColumn a{base + t, nt}, b{base + (size_t)kmax * nt + t, nt},
      z{base + (size_t)2 * kmax * nt + t, nt};
  const double* tri = P.tri + (size_t)q * 2 * kmax;
  for (int k = 0; k < keff; ++k) {
    a[k] = tri[k];
    b[k] = tri[kmax + k];
  }
  if (!tridiag_gauss(a, b, z, keff)) atomicOr(P.status, kStatusNonFinite);
  const double h3 = P.h * P.h * P.h;
  double rho = 0.0, e = 0.0;
  for (int k = 0; k < keff; ++k) {
    const double wk = z[k] * z[k];
    const double th = a[k];
    rho += wk * fermi_occ((th - P.mu) / P.kT);
    if (P.e_node) e += wk * integrand_value(th, P.mu, P.kT, P.integrand);
  }
  if (P.rho) P.rho[q] = 2.0 / h3 * rho;
  if (P.e_node) P.e_node[q] = 2.0 * e;
  if (P.k_eff) P.k_eff[q] = keff;
  if (P.theta_w) {
    // ascending order of the nodes
    for (int k = 1; k < keff; ++k) {
      const double tk = a[k], zk = z[k];
      int m = k - 1;
      while (m >= 0 && a[m] > tk) {
        a[m + 1] = a[m];
        z[m + 1] = z[m];
        --m;
      }
      a[m + 1] = tk;
      z[m + 1] = zk;
    }
    double* out = P.theta_w + (size_t)q * kmax * 2;
    for (int k = 0; k < kmax; ++k) {
      out[2 * k] = k < keff ? a[k] : 0.0;
      out[2 * k + 1] = k < keff ? z[k] * z[k] : 0.0;
    }
  }
}

// ------------------------------------------------------------------ setup kernels
__global__ void reset_kernel(int* queue, int* status, double* vmax, unsigned long long* hash) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    queue[0] = 0;     // the persistent kernels' node queue
    queue[1] = 0;     // the backward's eigensolve pre-pass queue
    *status = 0;
    *vmax = 0.0;
    *hash = 0ull;
  }
}

// Potential in the storage precision, max |V| (order-independent), a finiteness check and
// the potential's part of the input hash (a wrapping sum of mixed (value, index) pairs, so
// the order of the additions does not matter).
template <typename T>
__global__ void prepare_potential_kernel(const double* __restrict__ v64, T* __restrict__ vout,
                                         size_t n, double* vmax, int* status,
                                         unsigned long long* hash) {
  __shared__ double red[1024 / kWave];
  __shared__ unsigned long long hred[1024 / kWave];
  double mx = 0.0;
  unsigned long long hs = 0ull;
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = v64[i];
    if (!isfinite(v)) bad = true;
    mx = fmax(mx, fabs(v));
    hs += mix64((unsigned long long)__double_as_longlong(v) ^ mix64(i));
    if (vout) vout[i] = (T)v;
  }
  if (bad) atomicOr(status, kStatusNonFinite);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, kWave));
    hs += __shfl_xor(hs, off, kWave);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[threadIdx.x / kWave] = mx;
    hred[threadIdx.x / kWave] = hs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
      mx = fmax(mx, red[w]);
      hs += hred[w];
    }
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(vmax),
              (unsigned long long)__double_as_longlong(mx));
    atomicAdd(hash, hs);
  }
}

// Projector samples chi_l on the (2m+1)^3 box around each atom's nearest grid point.
template <typename T>
__global__ void projector_table_kernel(LaunchParams P, T* __restrict__ chi, int32_t* g0) {
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
  const int J = blockIdx.x;
  if (J >= P.n_atoms) return;
  const double Rx = P.atom_R[3 * J], Ry = P.atom_R[3 * J + 1], Rz = P.atom_R[3 * J + 2];
  const int gx = (int)rint(Rx / P.h), gy = (int)rint(Ry / P.h), gz = (int)rint(Rz / P.h);
  if (threadIdx.x == 0) {
    bool bad = !(isfinite(Rx) && isfinite(Ry) && isfinite(Rz));
    for (int l = 0; l < 4; ++l) bad = bad || !isfinite(P.proj_E[4 * J + l]);
    if (bad) atomicOr(P.status, kStatusNonFinite);
    // the atom's part of the input hash: its position and projector energies
    unsigned long long hs = mix64(~(unsigned long long)J);
    for (int c = 0; c < 3; ++c) hs = mix64(hs ^ (unsigned long long)__double_as_longlong(P.atom_R[3 * J + c]));
    for (int l = 0; l < 4; ++l) hs = mix64(hs ^ (unsigned long long)__double_as_longlong(P.proj_E[4 * J + l]));
    atomicAdd(P.hash + P.hash_slot, hs);
    g0[3 * J] = bad ? 0 : gx;
    g0[3 * J + 1] = bad ? 0 : gy;
    g0[3 * J + 2] = bad ? 0 : gz;
  }
  const double rg2 = P.proj_rg * P.proj_rg, rc2 = P.proj_rc * P.proj_rc;
  for (int b = threadIdx.x; b < B3; b += blockDim.x) {
    int bx = b % B - P.box_m, by = (b / B) % B - P.box_m, bz = b / (B * B) - P.box_m;
    double dx = (gx + bx) * P.h - Rx, dy = (gy + by) * P.h - Ry, dz = (gz + bz) * P.h - Rz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double g = 0.0;
    if (r2 < rc2) {
      double t = 1.0 - r2 / rc2;
      g = exp(-r2 / (2.0 * rg2)) * t * t * t;
    }
    T* out = chi + ((size_t)J * B3 + b) * 4;
    out[0] = (T)(P.proj_norm_s * g);
    out[1] = (T)(P.proj_norm_p * dx / P.proj_rg * g);
    out[2] = (T)(P.proj_norm_p * dy / P.proj_rg * g);
    out[3] = (T)(P.proj_norm_p * dz / P.proj_rg * g);
  }
}

// Omega = sum_q n_q e_q in a fixed order (one workgroup).
__global__ void weighted_sum_kernel(const double* __restrict__ e, const double* __restrict__ w,
                                    int n, double* out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += w[i] * e[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------ host launchers
template <typename T, int BLOCK>
static hipError_t launch_forward_t(const LaunchParams& P, int grid, int kg, hipStream_t s) {
  switch (kg) {
    case 8:
      hipLaunchKernelGGL((lanczos_forward_kernel<T, BLOCK, 8>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
    case 16:
      hipLaunchKernelGGL((lanczos_forward_kernel<T, BLOCK, 16>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
    default:
      hipLaunchKernelGGL((lanczos_forward_kernel<T, BLOCK, 32>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const LaunchParams& P, bool fp64, int grid, int block, int kg,
                          hipStream_t s) {
  if (fp64) return launch_forward_t<double, 256>(P, grid, kg, s);
  if (block == 128) return launch_forward_t<float, 128>(P, grid, kg, s);
  if (block == 512) return launch_forward_t<float, 512>(P, grid, kg, s);
  return launch_forward_t<float, 256>(P, grid, kg, s);
}

hipError_t launch_setup(const LaunchParams& P, bool fp64, const double* v64, void* vstore,
                        void* chi, int32_t* g0, double* vmax, hipStream_t s) {
  unsigned long long* hash = P.hash + P.hash_slot;
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, P.queue, P.status, vmax, hash);
  size_t n = (size_t)P.nx * P.ny * P.nz;
  int blocks = (int)((n + 1023) / 1024);
  if (blocks > 1024) blocks = 1024;
  if (fp64) {
    hipLaunchKernelGGL(prepare_potential_kernel<double>, dim3(blocks), dim3(1024), 0, s, v64,
                       (double*)nullptr, n, vmax, P.status, hash);
  } else {
    hipLaunchKernelGGL(prepare_potential_kernel<float>, dim3(blocks), dim3(1024), 0, s, v64,
                       (float*)vstore, n, vmax, P.status, hash);
  }
  if (P.n_proj > 0 && P.n_atoms > 0) {
    if (fp64)
      hipLaunchKernelGGL(projector_table_kernel<double>, dim3(P.n_atoms), dim3(256), 0, s, P,
                         (double*)chi, g0);
    else
      hipLaunchKernelGGL(projector_table_kernel<float>, dim3(P.n_atoms), dim3(256), 0, s, P,
                         (float*)chi, g0);
  }
  return hipGetLastError();
}

hipError_t launch_gauss_rule(const LaunchParams& P, hipStream_t s) {
  if (P.n_nodes <= 0) return hipSuccess;
  // three K-arrays of doubles per thread; at most 61 KB of LDS per workgroup
  const int nt = P.kmax_out <= 40 ? 64 : (P.kmax_out <= 80 ? 32 : 16);
  const size_t lds = (size_t)3 * P.kmax_out * nt * sizeof(double);
  hipLaunchKernelGGL(gauss_rule_kernel, dim3((P.n_nodes + nt - 1) / nt), dim3(nt), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_weighted_sum(const double* e, const double* w, int n, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(weighted_sum_kernel, dim3(1), dim3(1024), 0, s, e, w, n, out);
  return hipGetLastError();
}

}  // namespace sgq
