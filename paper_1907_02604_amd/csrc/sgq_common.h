// Shared device/host definitions of the gfx950 spectral-quadrature library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "host.h"

// host and device code (the tridiagonal solver shared by the kernels and the host)
#define SGQ_HD __host__ __device__

// Address-space qualifiers for device functions that are not inlined: without them the
// compiler must use FLAT accesses (and wait on every memory counter at once).
#define SGQ_G __attribute__((address_space(1)))   // global memory
#define SGQ_L __attribute__((address_space(3)))   // LDS

namespace sgq {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kFermiBlocks = 512;    // Fermi-level passes: partial sums per pass
constexpr int kFermiThreads = 256;   //   lanes per workgroup of a pass
constexpr int kFermiSteps = 64;      //   Newton / bisection steps enqueued per call
constexpr int kMaxNodeAtoms = 256;   // atoms whose projector box meets one node cube

// Status bits latched by kernels (mapped to sgq_status by the host).
constexpr int kStatusNonFinite = 1;
constexpr int kStatusLimit = 2;
constexpr int kStatusRange = 4;
constexpr int kStatusIndex = 8;

// Sixth-order central weights of d^2/dx^2 at offsets 0, 1, 2, 3 (symmetric).
constexpr double kFd0 = -49.0 / 18.0;
constexpr double kFd1 = 3.0 / 2.0;
constexpr double kFd2 = -3.0 / 20.0;
constexpr double kFd3 = 1.0 / 90.0;

// Everything a launch needs; passed by value as the kernel argument.
struct LaunchParams {
  // grid and projectors
  int nx, ny, nz;
  double h;
  int n_atoms, n_proj;
  int box_m;           // projector box half-width (grid points); box side B = 2m+1
  double proj_norm_s, proj_norm_p, proj_rg, proj_rc;
  // nodes, cost-sorted
  int n_nodes;
  const int32_t* order;       // [Nq] node ids, most expensive first
  const int32_t* center;      // [Nq] by node id: linear grid index
  const int32_t* half_width;  // [Nq] by node id
  const int32_t* depth;       // [Nq] by node id
  // inputs
  const void* v;              // [nz*ny*nx] potential in the storage precision
  const double* atom_R;       // [M*3]
  const double* proj_E;       // [M*4]
  const void* chi;            // [M*B^3*4] projector samples in storage precision
  const int32_t* atom_g0;     // [M*3] nearest grid point (unwrapped)
  const double* vmax;         // device scalar max |V|
  double mu, kT;
  int integrand;
  double tau;                 // breakdown threshold relative to the spectral scale
  // workspace
  void* W;                    // [slots]: basis [npad/64][kmax][64] (point-blocked)
  void* U;                    // [slots][npad]
  size_t npad;
  size_t slot_stride;         // elements of W per slot
  int wbs;                    // element stride between 64-point blocks of the basis (kmax*64)
  int* queue;                 // node counter of the persistent launch
  int* status;                // latched error bits
  // outputs (by node id)
  double* rho;                // [Nq] or null
  double* e_node;             // [Nq] or null
  double* theta_w;            // [Nq*kmax_out*2] or null
  int32_t* k_eff;             // [Nq] or null
  int kmax_out;
  double* tri;                // [Nq][2*kmax_out]: alpha_0.. then beta_0.. of each node
  int32_t* tri_k;             // [Nq] K_eff of each node's tridiagonal (-1: node skipped)
  // backward extras
  const double* node_weight;  // [Nq]
  const double* grad_omega;   // device scalar
  void* P_cube;               // [Nq][cube points] per-node dV contribution (storage precision)
  const int64_t* cube_offset; // [Nq] offset of each node's cube in P_cube
  double* dR_part;            // [Nq][kMaxNodeAtoms][3] node partials of dR (nonlocal)
  double* dE_part;            // [Nq][kMaxNodeAtoms][4] node partials of dE
  int32_t* node_atoms;        // [Nq][1 + kMaxNodeAtoms]: count, then the node's atom ids
  double* zbuf;               // [slots][2*Kb*Kb] eigenvectors of T, then the weighted
                              // divided differences (per backward slot)
  void* Wr;                   // retained bases [R][npad/64][kmax][64] (NULL: slots only)
  void* Ur;                   // retained u_j = H q_j rows [R][kmax][npad]
  const int32_t* ret_slot;    // [Nq] each node's place among the R retained ones, or -1
  int use_retained;           // backward: take the retained basis instead of recomputing
  // 64-bit hashes of the inputs' contents (v_loc, atom_R, proj_E): [0] taken by the last
  // forward call, [1] by the current backward call; setup writes entry hash_slot.  The
  // backward takes retained bases only when the two agree.
  unsigned long long* hash;
  int hash_slot;
  // backward: alphabar / betabar of each node from the eigensolve pre-pass ([Nq][2*kmax_out])
  // and the K_eff it solved for (-1: not solved there); tbar_k NULL: no pre-pass
  double* tbar;
  int32_t* tbar_k;
};

// splitmix64 finaliser: mixes the bits of one input value with its index for the input hash.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Element index of point p in a vector stored in 64-point blocks with block stride bs
// (bs = 64: a plain vector; bs = kmax*64: one row of the point-blocked Lanczos basis).
__device__ __forceinline__ int bidx(int p, int bs) { return (p >> 6) * bs + (p & 63); }

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Fermi-Dirac occupation 1/(1+exp(x)), x = (lam - mu)/kT, without overflow.
__device__ __forceinline__ double fermi_occ(double x) {
  if (x > 0.0) {
    double e = exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(x));
}

__device__ __forceinline__ double softplus(double y) {
  return fmax(y, 0.0) + log1p(exp(-fabs(y)));
}

// F(lam) of the requested integrand (0 band, 1 Mermin free energy, 2 grand potential).
__device__ __forceinline__ double integrand_value(double lam, double mu, double kT, int kind) {
  double x = (lam - mu) / kT;
  double g = fermi_occ(x);
  if (kind == 0) return lam * g;
  double sp = kT * softplus(-x);
  return kind == 1 ? mu * g - sp : -sp;
}

__device__ __forceinline__ double integrand_deriv(double lam, double mu, double kT, int kind) {
  double x = (lam - mu) / kT;
  double g = fermi_occ(x);
  double dg = -g * (1.0 - g) / kT;
  if (kind == 0) return g + lam * dg;
  if (kind == 1) return g + mu * dg;
  return g;
}

}  // namespace sgq
