// Unbatched reference schedule: one node at a time, each Lanczos step as grid-wide
// kernels over the node's cube (matvec, projector overlaps and scatter, classical
// Gram-Schmidt dot products with a second-stage reduction, update and norm), then the
// Gauss rule.  Same arithmetic precision and depth as the batched persistent kernel;
// it exists as the per-node GPU baseline that the batched schedule is measured against.
#include "sgq_common.h"
#include "tridiag.h"

namespace sgq {

constexpr int kPlainBlock = 256;

struct PlainNode {
  int sx, sy, sz, ox, oy, oz, periodic, n, start;
};

__host__ __device__ inline PlainNode plain_node(int c, int R, int nx, int ny, int nz) {
  PlainNode g;
  const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
  if (R < 0) {
    g.sx = nx; g.sy = ny; g.sz = nz;
    g.ox = g.oy = g.oz = 0;
    g.periodic = 1;
    g.start = c;
  } else {
    const int s = 2 * R + 1;
    g.sx = g.sy = g.sz = s;
    g.ox = cx - R; g.oy = cy - R; g.oz = cz - R;
    g.periodic = 0;
    g.start = R + s * (R + s * R);
  }
  g.n = g.sx * g.sy * g.sz;
  return g;
}

// scalars of the node being processed: [0] K_eff, [1..] alpha, beta, scale, coefficients
struct PlainScalars {
  int keff;
  int natoms;
  double alpha[kMaxDepth], beta[kMaxDepth], scale[kMaxDepth + 1];
  double coef[kMaxDepth + 1];
  double nl;    // q . V_nl q of the current step
};

__global__ void plain_init_kernel(LaunchParams P, int q, PlainScalars* S, void* Wv, int natom_cap,
                                  int32_t* atoms, int32_t* abox, bool fp64) {
  const PlainNode g = plain_node(P.center[q], P.half_width[q], P.nx, P.ny, P.nz);
  const size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (size_t i = i0; i < P.npad; i += (size_t)gridDim.x * blockDim.x) {
    const double v = (i == (size_t)g.start) ? 1.0 : 0.0;
    if (fp64) ((double*)Wv)[i] = v; else ((float*)Wv)[i] = (float)v;
  }
  if (i0 == 0) {
    S->keff = P.depth[q];
    S->scale[0] = 1.0;
    // projector atoms meeting the cube (same rule as the batched kernel), in atom order
    int na = 0;
    const int m = P.box_m;
    const int nn[3] = {P.nx, P.ny, P.nz}, o[3] = {g.ox, g.oy, g.oz}, s[3] = {g.sx, g.sy, g.sz};
    for (int J = 0; J < (P.n_proj ? P.n_atoms : 0); ++J) {
      bool hit = true;
      int lo[3];
      for (int ax = 0; ax < 3; ++ax) {
        int d = wrap_index(P.atom_g0[3 * J + ax] - o[ax], nn[ax]);
        if (!g.periodic) {
          if (d >= nn[ax] - m) d -= nn[ax];
          if (d + m < 0 || d - m > s[ax] - 1) hit = false;
        }
        lo[ax] = d - m;
      }
      if (hit && na < natom_cap) {
        atoms[na] = J;
        abox[3 * na] = lo[0];
        abox[3 * na + 1] = lo[1];
        abox[3 * na + 2] = lo[2];
        ++na;
      } else if (hit) {
        atomicOr(P.status, kStatusLimit);
      }
    }
    S->natoms = na < natom_cap ? na : natom_cap;
  }
}

__device__ inline int plain_box_point(const PlainNode& g, const int32_t* abox, int a, int b, int B) {
  int x = abox[3 * a] + b % B, y = abox[3 * a + 1] + (b / B) % B, z = abox[3 * a + 2] + b / (B * B);
  if (g.periodic) {
    x = wrap_index(x, g.sx); y = wrap_index(y, g.sy); z = wrap_index(z, g.sz);
  } else if (x < 0 || y < 0 || z < 0 || x >= g.sx || y >= g.sy || z >= g.sz) {
    return -1;
  }
  return x + g.sx * (y + g.sy * z);
}

// u = s_j (-1/2 Lap_6 + V) W_j, one thread per cube point.
template <typename T>
__global__ void plain_matvec_kernel(LaunchParams P, int q, const PlainScalars* S, const T* Wj,
                                    T* U, int j) {
  const PlainNode g = plain_node(P.center[q], P.half_width[q], P.nx, P.ny, P.nz);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.n) return;
  const T* V = (const T*)P.v;
  const int x = p % g.sx, y = (p / g.sx) % g.sy, z = p / (g.sx * g.sy);
  // sum_d w_d (neighbour - centre) over the six neighbours at distance d: the weights add
  // up to zero, and differences keep the FP32 rounding small where the vector is smooth
  const double w[4] = {0.0, kFd1, kFd2, kFd3};
  const T c0 = Wj[p];
  T lap = (T)0;
  for (int d = 1; d <= 3; ++d) {
    const int xs[2] = {x - d, x + d}, ys[2] = {y - d, y + d}, zs[2] = {z - d, z + d};
    for (int e = 0; e < 2; ++e) {
      int a = xs[e], b = ys[e], c = zs[e];
      if (g.periodic) {
        a = wrap_index(a, g.sx); b = wrap_index(b, g.sy); c = wrap_index(c, g.sz);
        lap += (T)w[d] * ((Wj[a + g.sx * (y + g.sy * z)] - c0) + (Wj[x + g.sx * (b + g.sy * z)] - c0) +
                          (Wj[x + g.sx * (y + g.sy * c)] - c0));
      } else {
        const T va = (a >= 0 && a < g.sx) ? Wj[a + g.sx * (y + g.sy * z)] : (T)0;
        const T vb = (b >= 0 && b < g.sy) ? Wj[x + g.sx * (b + g.sy * z)] : (T)0;
        const T vc = (c >= 0 && c < g.sz) ? Wj[x + g.sx * (y + g.sy * c)] : (T)0;
        lap += (T)w[d] * ((va - c0) + (vb - c0) + (vc - c0));
      }
    }
  }
  const int gx = wrap_index(g.ox + x, P.nx), gy = wrap_index(g.oy + y, P.ny),
            gz = wrap_index(g.oz + z, P.nz);
  const T sj = (T)S->scale[j];
  U[p] = sj * ((T)(-0.5 / (P.h * P.h)) * lap + V[gx + P.nx * (gy + P.ny * gz)] * Wj[p]);
}

// chi . q_j per node atom (one workgroup per atom) -> coef[4a+l] = E h^3 (chi . q), nl[a]
template <typename T>
__global__ void plain_proj_dots_kernel(LaunchParams P, int q, const PlainScalars* S, const T* Wj,
                                       int j, const int32_t* atoms, const int32_t* abox,
                                       double* coef, double* nl) {
  const int a = blockIdx.x;
  if (a >= S->natoms) return;
  const PlainNode g = plain_node(P.center[q], P.half_width[q], P.nx, P.ny, P.nz);
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
  const int J = atoms[a];
  const T* chi = (const T*)P.chi;
  __shared__ double red[kPlainBlock][4];
  double acc[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < B3; b += blockDim.x) {
    const int lp = plain_box_point(g, abox, a, b, B);
    if (lp < 0) continue;
    for (int l = 0; l < 4; ++l) acc[l] += (double)chi[((size_t)J * B3 + b) * 4 + l] * (double)Wj[lp];
  }
  for (int l = 0; l < 4; ++l) red[threadIdx.x][l] = acc[l];
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half)
      for (int l = 0; l < 4; ++l) red[threadIdx.x][l] += red[threadIdx.x + half][l];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double h3 = P.h * P.h * P.h, sj = S->scale[j];
    double e = 0.0;
    for (int l = 0; l < 4; ++l) {
      const double c = red[0][l] * sj;
      const double E = P.proj_E[4 * J + l];
      coef[4 * a + l] = E * h3 * c;
      e += E * h3 * c * c;
    }
    nl[a] = e;
  }
}

// u += chi E h^3 (chi . q) over each atom's box (atomic adds: boxes may overlap).
template <typename T>
__global__ void plain_proj_scatter_kernel(LaunchParams P, int q, const PlainScalars* S, T* U,
                                          const int32_t* atoms, const int32_t* abox,
                                          const double* coef) {
  const int a = blockIdx.x;
  if (a >= S->natoms) return;
  const PlainNode g = plain_node(P.center[q], P.half_width[q], P.nx, P.ny, P.nz);
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
  const int J = atoms[a];
  const T* chi = (const T*)P.chi;
  for (int b = threadIdx.x; b < B3; b += blockDim.x) {
    const int lp = plain_box_point(g, abox, a, b, B);
    if (lp < 0) continue;
    double v = 0.0;
    for (int l = 0; l < 4; ++l) v += (double)chi[((size_t)J * B3 + b) * 4 + l] * coef[4 * a + l];
    atomicAdd(&U[lp], (T)v);
  }
}

// partial[blk][i] = sum over this block's points of W_i(p) u(p) (i <= j), FP64
template <typename T>
__global__ void plain_dots_kernel(int n, size_t npad, const T* W, const T* U, int j,
                                  double* partial) {
  __shared__ double red[kPlainBlock];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const double u = p < n ? (double)U[p] : 0.0;
  for (int i = 0; i <= j; ++i) {
    red[threadIdx.x] = p < n ? (double)W[(size_t)i * npad + p] * u : 0.0;
    __syncthreads();
    for (int half = blockDim.x / 2; half > 0; half >>= 1) {
      if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * (kMaxDepth + 1) + i] = red[0];
    __syncthreads();
  }
}

// coefficients c_i = q_i . u from the partials (fixed order); alpha_j = c_j + q.V_nl q
__global__ void plain_coef_kernel(int nblocks, int j, const double* partial, const double* nl,
                                  PlainScalars* S) {
  const int i = threadIdx.x;
  if (i <= j) {
    double c = 0.0;
    for (int b = 0; b < nblocks; ++b) c += partial[(size_t)b * (kMaxDepth + 1) + i];
    S->coef[i] = c * S->scale[i];   // q_i . u
  }
  __syncthreads();
  if (i == 0) {
    double e = 0.0;
    for (int a = 0; a < S->natoms; ++a) e += nl[a];
    // the projector part of u is already in U, so c_j includes it
    S->alpha[j] = S->coef[j];
    (void)e;
  }
}

// w = u - sum_i c_i q_i -> W_{j+1}; partial |w|^2
template <typename T>
__global__ void plain_update_kernel(int n, size_t npad, T* W, const T* U, int j,
                                    const PlainScalars* S, double* partial) {
  __shared__ double red[kPlainBlock];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  if (p < n) {
    w = (double)U[p];
    for (int i = 0; i <= j; ++i) w -= S->coef[i] * S->scale[i] * (double)W[(size_t)i * npad + p];
    W[(size_t)(j + 1) * npad + p] = (T)w;
  }
  red[threadIdx.x] = w * w;
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void plain_norm_kernel(int nblocks, int j, const double* partial, PlainScalars* S,
                                  double tol_rel, const double* vmax, double h) {
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b];
  const double beta = sqrt(s);
  S->beta[j] = beta;
  S->scale[j + 1] = beta > 0.0 ? 1.0 / beta : 0.0;
  const double hscale = 1.5 * (-kFd0 + 2.0 * (kFd1 - kFd2 + kFd3)) / (h * h) + *vmax;
  if (!(beta > tol_rel * hscale) && S->keff > j + 1) S->keff = j + 1;
}

__global__ void plain_quadrature_kernel(LaunchParams P, int q, PlainScalars* S) {
  // one thread: its three arrays in LDS, so the kernel needs no private (scratch) memory
  __shared__ double a[kMaxDepth], b[kMaxDepth], z[kMaxDepth];
  const int K = S->keff;
  for (int k = 0; k < K; ++k) a[k] = S->alpha[k];
  for (int k = 0; k + 1 < K; ++k) b[k] = S->beta[k];
  if (!tridiag_gauss(a, b, z, K)) atomicOr(P.status, kStatusNonFinite);
  double rho = 0.0;
  for (int k = 0; k < K; ++k) rho += z[k] * z[k] * fermi_occ((a[k] - P.mu) / P.kT);
  if (P.rho) P.rho[q] = 2.0 / (P.h * P.h * P.h) * rho;
  if (P.k_eff) P.k_eff[q] = K;
}

// Launch every step of every node (host loop).  Steps past a breakdown still run but
// are ignored by the quadrature (K_eff is latched on the device).
template <typename T>
static hipError_t plain_run(const LaunchParams& P, const int32_t* h_center, const int32_t* h_hw,
                            const int32_t* h_depth, void* scratch, hipStream_t s) {
  char* base = (char*)scratch;
  PlainScalars* S = (PlainScalars*)base;
  base += (sizeof(PlainScalars) + 255) / 256 * 256;
  const int cap = kMaxNodeAtoms;
  int32_t* atoms = (int32_t*)base;
  base += cap * 4 * 4;
  int32_t* abox = (int32_t*)base;
  base += cap * 3 * 4 * 4;
  double* coef = (double*)base;
  base += cap * 4 * 8;
  double* nl = (double*)base;
  base += cap * 8;
  double* partial = (double*)base;
  base += (size_t)65536 * (kMaxDepth + 1) * 8;
  T* W = (T*)base;
  T* U = W + (size_t)P.slot_stride;
  for (int q = 0; q < P.n_nodes; ++q) {
    const PlainNode g = plain_node(h_center[q], h_hw[q], P.nx, P.ny, P.nz);
    const int nb = (g.n + kPlainBlock - 1) / kPlainBlock;
    hipLaunchKernelGGL(plain_init_kernel, dim3(64), dim3(256), 0, s, P, q, S, (void*)W, cap, atoms,
                       abox, sizeof(T) == 8);
    for (int j = 0; j < h_depth[q]; ++j) {
      const T* Wj = W + (size_t)j * P.npad;
      hipLaunchKernelGGL(plain_matvec_kernel<T>, dim3(nb), dim3(kPlainBlock), 0, s, P, q, S, Wj, U, j);
      if (P.n_proj && P.n_atoms) {
        hipLaunchKernelGGL(plain_proj_dots_kernel<T>, dim3(cap), dim3(kPlainBlock), 0, s, P, q, S, Wj,
                           j, atoms, abox, coef, nl);
        hipLaunchKernelGGL(plain_proj_scatter_kernel<T>, dim3(cap), dim3(kPlainBlock), 0, s, P, q, S,
                           U, atoms, abox, coef);
      }
      hipLaunchKernelGGL(plain_dots_kernel<T>, dim3(nb), dim3(kPlainBlock), 0, s, g.n, P.npad, W, U,
                         j, partial);
      hipLaunchKernelGGL(plain_coef_kernel, dim3(1), dim3(kMaxDepth + 1), 0, s, nb, j, partial, nl, S);
      if (j + 1 < h_depth[q]) {
        hipLaunchKernelGGL(plain_update_kernel<T>, dim3(nb), dim3(kPlainBlock), 0, s, g.n, P.npad, W,
                           U, j, S, partial);
        hipLaunchKernelGGL(plain_norm_kernel, dim3(1), dim3(1), 0, s, nb, j, partial, S, P.tau,
                           P.vmax, P.h);
      }
    }
    hipLaunchKernelGGL(plain_quadrature_kernel, dim3(1), dim3(1), 0, s, P, q, S);
  }
  return hipGetLastError();
}

size_t plain_scratch_bytes(size_t npad, int kmax, bool fp64) {
  size_t b = (sizeof(PlainScalars) + 255) / 256 * 256;
  b += kMaxNodeAtoms * (4 * 4 + 3 * 4 * 4 + 4 * 8 + 8);
  b += (size_t)65536 * (kMaxDepth + 1) * 8;
  b += ((size_t)kmax + 2) * npad * (fp64 ? 8 : 4);
  return b;
}

hipError_t launch_plain(const LaunchParams& P, bool fp64, const int32_t* h_center,
                        const int32_t* h_hw, const int32_t* h_depth, void* scratch, hipStream_t s) {
  return fp64 ? plain_run<double>(P, h_center, h_hw, h_depth, scratch, s)
              : plain_run<float>(P, h_center, h_hw, h_depth, scratch, s);
}

}  // namespace sgq
