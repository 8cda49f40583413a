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
#include "sgq_common.h"
#include "tridiag.h"

namespace sgq {

template <typename T, int BLOCK>
struct NodeState {
  static constexpr int NW = BLOCK / kWave;
  int node;
  int sx, sy, sz, ox, oy, oz, periodic, n, start, natoms, abort;
  int atom[kMaxNodeAtoms];
  int abox[kMaxNodeAtoms][3];       // local coordinates of the projector box corner
  int aphase[kMaxNodeAtoms];        // 0: scatter with the parallel group, 1: alone
  int wcount[NW];
  T acoef[kMaxNodeAtoms][4];        // E h^3 (chi . q): weights of the projector scatter
  double anl[kMaxNodeAtoms];        // q . V_nl q contribution of each atom
  double alpha[kMaxDepth];
  double beta[kMaxDepth];
  double scale[kMaxDepth + 1];      // 1 / |W_i| (q_i = scale_i W_i)
  double gram[kMaxDepth + 1];       // q_i . q_j of the current vector
  T ct[kMaxDepth + 1];              // c_i * scale_i
  double red[NW][kMaxDepth + 2];
  double ta[kMaxDepth], tb[kMaxDepth], tz[kMaxDepth];
  double dsave[kMaxDepth + 1];      // D_i of the last sweep
  double orth_tol;
  int redo;
};

// local linear index -> (x, y, z) of a cube with extents sx, sy
__device__ __forceinline__ void unflatten(int p, int sx, int sxy, float inv_sx, float inv_sxy,
                                          int& x, int& y, int& z) {
  z = (int)(((float)p + 0.5f) * inv_sxy);
  int r = p - z * sxy;
  if (r < 0) { --z; r += sxy; } else if (r >= sxy) { ++z; r -= sxy; }
  y = (int)(((float)r + 0.5f) * inv_sx);
  x = r - y * sx;
  if (x < 0) { --y; x += sx; } else if (x >= sx) { ++y; x -= sx; }
}

// Projector box point b of node atom a -> local linear index, or -1 outside the cube.
template <typename S>
__device__ __forceinline__ int box_point(const S& st, int a, int b, int B) {
  int bx = b % B, by = (b / B) % B, bz = b / (B * B);
  int x = st.abox[a][0] + bx, y = st.abox[a][1] + by, z = st.abox[a][2] + bz;
  if (st.periodic) {
    x = wrap_index(x, st.sx);
    y = wrap_index(y, st.sy);
    z = wrap_index(z, st.sz);
  } else if (x < 0 || y < 0 || z < 0 || x >= st.sx || y >= st.sy || z >= st.sz) {
    return -1;
  }
  return x + st.sx * (y + st.sy * z);
}

// Sets up the cube geometry and the node's projector atom list (ordered by atom id).
template <typename T, int BLOCK>
__device__ void node_setup(const LaunchParams& P, NodeState<T, BLOCK>& st, int q) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  if (tid == 0) {
    int R = P.half_width[q];
    int c = P.center[q];
    int cx = c % P.nx, cy = (c / P.nx) % P.ny, cz = c / (P.nx * P.ny);
    if (R < 0) {
      st.sx = P.nx; st.sy = P.ny; st.sz = P.nz;
      st.ox = st.oy = st.oz = 0;
      st.periodic = 1;
      st.start = c;
    } else {
      int s = 2 * R + 1;
      st.sx = st.sy = st.sz = s;
      st.ox = cx - R; st.oy = cy - R; st.oz = cz - R;
      st.periodic = 0;
      st.start = R + s * (R + s * R);
    }
    st.n = st.sx * st.sy * st.sz;
    st.natoms = 0;
    st.abort = 0;
  }
  __syncthreads();
  if (P.n_proj == 0) return;
  const int m = P.box_m;
  const int nn[3] = {P.nx, P.ny, P.nz};
  for (int base = 0; base < P.n_atoms; base += BLOCK) {
    int J = base + tid;
    bool hit = false;
    int lo[3] = {0, 0, 0};
    if (J < P.n_atoms) {
      const int o[3] = {st.ox, st.oy, st.oz};
      const int s[3] = {st.sx, st.sy, st.sz};
      hit = true;
      for (int ax = 0; ax < 3; ++ax) {
        int d = wrap_index(P.atom_g0[3 * J + ax] - o[ax], nn[ax]);
        if (!st.periodic) {
          if (d >= nn[ax] - m) d -= nn[ax];
          if (d + m < 0 || d - m > s[ax] - 1) hit = false;
        }
        lo[ax] = d - m;
      }
    }
    uint64_t mask = __ballot(hit);
    int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) st.wcount[wave] = __popcll(mask);
    __syncthreads();
    int off = st.natoms;
    for (int w = 0; w < wave; ++w) off += st.wcount[w];
    if (hit) {
      int slot = off + before;
      if (slot < kMaxNodeAtoms) {
        st.atom[slot] = J;
        st.abox[slot][0] = lo[0];
        st.abox[slot][1] = lo[1];
        st.abox[slot][2] = lo[2];
      }
    }
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += st.wcount[w];
      st.natoms += tot;
    }
    __syncthreads();
  }
  if (st.natoms > kMaxNodeAtoms) {
    if (tid == 0) {
      st.abort = 1;
      atomicOr(P.status, kStatusLimit);
    }
    __syncthreads();
    return;
  }
  // Scatter groups: an atom whose box overlaps no earlier atom's box joins the
  // parallel group; the others are added one at a time, in atom order.
  const int B = 2 * m + 1;
  bool alias = st.periodic && (P.nx < B || P.ny < B || P.nz < B);
  for (int a = tid; a < st.natoms; a += BLOCK) {
    int ph = alias ? 1 : 0;
    for (int b = 0; b < a && ph == 0; ++b) {
      bool ov = true;
      for (int ax = 0; ax < 3; ++ax) {
        int d = st.abox[a][ax] - st.abox[b][ax];
        if (st.periodic) {
          int nax = nn[ax];
          d = wrap_index(d, nax);
          d = d > nax / 2 ? nax - d : d;
        }
        if (abs(d) > 2 * m) ov = false;
      }
      if (ov) ph = 1;
    }
    st.aphase[a] = ph;
  }
  __syncthreads();
}

// dst(p) = src(p) - sum_{i<=j} ct_i W_i(p) for every cube point, with the FP64 dots
// D_i = W_i . dst and |dst|^2 left per wave in st.red.  Four lanes share a point, each
// taking the basis vectors i = g (mod 4), so a wave reads 16 consecutive points of four
// vectors per load and each lane keeps ceil((j+1)/4) FP64 partial sums.
template <typename T, int BLOCK, int KG>
__device__ __forceinline__ void fused_sweep(NodeState<T, BLOCK>& st, const T* __restrict__ W,
                                            const T* src, T* dst, int j, int n, size_t npad) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int g = lane & 3;
  double D[KG];
  T qv[KG];
  T cg[KG];
#pragma unroll
  for (int m = 0; m < KG; ++m) {
    D[m] = 0.0;
    int i = 4 * m + g;
    cg[m] = (i <= j) ? st.ct[i] : (T)0;
  }
  double n2 = 0.0;
  const int mmax = j / 4;   // last lane group holding a live basis vector
  for (int p = tid >> 2; p < n; p += BLOCK / 4) {
    T acc = 0;
#pragma unroll
    for (int m = 0; m < KG; ++m) {
      if (m <= mmax) {
        int i = 4 * m + g;
        qv[m] = (i <= j) ? W[(size_t)i * npad + p] : (T)0;
        acc += cg[m] * qv[m];
      }
    }
    acc += __shfl_xor(acc, 1, kWave);
    acc += __shfl_xor(acc, 2, kWave);
    T w = src[p] - acc;
    if (g == 0) {
      dst[p] = w;
      n2 += (double)w * (double)w;
    }
    const double wd = (double)w;
#pragma unroll
    for (int m = 0; m < KG; ++m)
      if (m <= mmax) D[m] += (double)qv[m] * wd;
  }
#pragma unroll
  for (int m = 0; m < KG; ++m) {
    if (m <= mmax) {
      double v = D[m];
      v += __shfl_xor(v, 4, kWave);
      v += __shfl_xor(v, 8, kWave);
      v += __shfl_xor(v, 16, kWave);
      v += __shfl_xor(v, 32, kWave);
      int i = 4 * m + g;
      if (lane < 4 && i <= j) st.red[wave][i] = v;
    }
  }
  n2 = wave_sum(n2);
  if (lane == 0) st.red[wave][kMaxDepth + 1] = n2;
}

// Totals of a sweep: beta_j, the scale of the new vector, its Gram column against
// q_0..q_j and the semi-orthogonality flag.  Ends with a barrier.
template <typename T, int BLOCK>
__device__ __forceinline__ void finish_sweep(NodeState<T, BLOCK>& st, int j) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x;
  double dsum = 0.0;
  if (tid <= j) {
    for (int w = 0; w < NW; ++w) dsum += st.red[w][tid];
    st.dsave[tid] = dsum;
  }
  if (tid == 0) {
    double nn2 = 0.0;
    for (int w = 0; w < NW; ++w) nn2 += st.red[w][kMaxDepth + 1];
    double b = sqrt(nn2);
    st.beta[j] = b;
    st.scale[j + 1] = b > 0.0 ? 1.0 / b : 0.0;
  }
  __syncthreads();
  if (tid <= j) st.gram[tid] = st.scale[tid] * st.scale[j + 1] * dsum;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i <= j; ++i) mx = fmax(mx, fabs(st.gram[i]));
    st.redo = !(mx <= st.orth_tol);
  }
  __syncthreads();
}

template <typename T, int BLOCK, int KG>
__global__ __launch_bounds__(BLOCK) void lanczos_forward_kernel(LaunchParams P) {
  constexpr int NW = BLOCK / kWave;
  __shared__ NodeState<T, BLOCK> st;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const T* __restrict__ V = reinterpret_cast<const T*>(P.v);
  const T* __restrict__ chi = reinterpret_cast<const T*>(P.chi);
  T* __restrict__ W = reinterpret_cast<T*>(P.W) + (size_t)blockIdx.x * P.slot_stride;
  T* __restrict__ U = reinterpret_cast<T*>(P.U) + (size_t)blockIdx.x * P.npad;
  const size_t npad = P.npad;
  const double h = P.h;
  const double h3 = h * h * h;
  const T kin = (T)(-0.5 / (h * h));
  const T w0 = (T)(3.0 * kFd0), w1 = (T)kFd1, w2 = (T)kFd2, w3 = (T)kFd3;
  const double hscale = 1.5 * (-kFd0 + 2.0 * (kFd1 - kFd2 + kFd3)) / (h * h) + *P.vmax;
  const double tol = P.tau * hscale;
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
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
      if (tid == 0) {
        double nan = __builtin_nan("");
        if (P.rho) P.rho[q] = nan;
        if (P.e_node) P.e_node[q] = nan;
        if (P.k_eff) P.k_eff[q] = 0;
      }
      __syncthreads();
      continue;
    }
    const int n = st.n, sx = st.sx, sy = st.sy, sz = st.sz, sxy = sx * sy;
    const float inv_sx = 1.0f / (float)sx, inv_sxy = 1.0f / (float)sxy;
    const int periodic = st.periodic, natoms = st.natoms;
    for (int p = tid; p < n; p += BLOCK) W[p] = (T)0;
    __syncthreads();
    if (tid == 0) {
      W[st.start] = (T)1;
      st.scale[0] = 1.0;
    }
    __syncthreads();

    int keff = K;
    for (int j = 0; j < K; ++j) {
      const T* __restrict__ Wj = W + (size_t)j * npad;
      const double sjd = st.scale[j];
      const T sj = (T)sjd;
      // ---- projector overlaps chi_Jl . q_j (one wave per atom)
      for (int a = wave; a < natoms; a += NW) {
        const int J = st.atom[a];
        T acc[4] = {0, 0, 0, 0};
        for (int b = lane; b < B3; b += kWave) {
          int lp = box_point(st, a, b, B);
          if (lp >= 0) {
            T wv = Wj[lp];
            const T* c4 = chi + ((size_t)J * B3 + b) * 4;
            acc[0] += c4[0] * wv;
            acc[1] += c4[1] * wv;
            acc[2] += c4[2] * wv;
            acc[3] += c4[3] * wv;
          }
        }
        double nl = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          double cl = (double)wave_sum(acc[l]) * sjd;    // chi . q_j
          double El = P.proj_E[4 * J + l];
          if (lane == 0) st.acoef[a][l] = (T)(El * h3 * cl);
          nl += El * h3 * cl * cl;
        }
        if (lane == 0) st.anl[a] = nl;
      }
      // ---- stencil and local potential: u = s_j (-1/2 Lap_6 + V) W_j
      double apart = 0.0;
      for (int p = tid; p < n; p += BLOCK) {
        int x, y, z;
        unflatten(p, sx, sxy, inv_sx, inv_sxy, x, y, z);
        T wc = Wj[p];
        T lap = w0 * wc;
        if (!periodic) {
          if (x >= 1) lap += w1 * Wj[p - 1];
          if (x + 1 < sx) lap += w1 * Wj[p + 1];
          if (x >= 2) lap += w2 * Wj[p - 2];
          if (x + 2 < sx) lap += w2 * Wj[p + 2];
          if (x >= 3) lap += w3 * Wj[p - 3];
          if (x + 3 < sx) lap += w3 * Wj[p + 3];
          if (y >= 1) lap += w1 * Wj[p - sx];
          if (y + 1 < sy) lap += w1 * Wj[p + sx];
          if (y >= 2) lap += w2 * Wj[p - 2 * sx];
          if (y + 2 < sy) lap += w2 * Wj[p + 2 * sx];
          if (y >= 3) lap += w3 * Wj[p - 3 * sx];
          if (y + 3 < sy) lap += w3 * Wj[p + 3 * sx];
          if (z >= 1) lap += w1 * Wj[p - sxy];
          if (z + 1 < sz) lap += w1 * Wj[p + sxy];
          if (z >= 2) lap += w2 * Wj[p - 2 * sxy];
          if (z + 2 < sz) lap += w2 * Wj[p + 2 * sxy];
          if (z >= 3) lap += w3 * Wj[p - 3 * sxy];
          if (z + 3 < sz) lap += w3 * Wj[p + 3 * sxy];
        } else {
          const T wd[4] = {0, w1, w2, w3};
          for (int d = 1; d <= 3; ++d) {
            lap += wd[d] * (Wj[wrap_index(x - d, sx) + sx * (y + sy * z)] +
                            Wj[wrap_index(x + d, sx) + sx * (y + sy * z)]);
            lap += wd[d] * (Wj[x + sx * (wrap_index(y - d, sy) + sy * z)] +
                            Wj[x + sx * (wrap_index(y + d, sy) + sy * z)]);
            lap += wd[d] * (Wj[x + sx * (y + sy * wrap_index(z - d, sz))] +
                            Wj[x + sx * (y + sy * wrap_index(z + d, sz))]);
          }
        }
        int gx = st.ox + x, gy = st.oy + y, gz = st.oz + z;
        gx = gx < 0 ? gx + P.nx : (gx >= P.nx ? gx - P.nx : gx);
        gy = gy < 0 ? gy + P.ny : (gy >= P.ny ? gy - P.ny : gy);
        gz = gz < 0 ? gz + P.nz : (gz >= P.nz ? gz - P.nz : gz);
        T vloc = V[gx + P.nx * (gy + P.ny * gz)];
        T u = sj * (kin * lap + vloc * wc);
        U[p] = u;
        apart += (double)(sj * wc) * (double)u;
      }
      apart = wave_sum(apart);
      if (lane == 0) st.red[wave][0] = apart;
      __syncthreads();
      // ---- projector scatter u += sum_l chi_l E_l h^3 (chi_l . q)
      if (natoms > 0) {
        for (int a = wave; a < natoms; a += NW) {
          if (st.aphase[a]) continue;
          const int J = st.atom[a];
          for (int b = lane; b < B3; b += kWave) {
            int lp = box_point(st, a, b, B);
            if (lp >= 0) {
              const T* c4 = chi + ((size_t)J * B3 + b) * 4;
              U[lp] += c4[0] * st.acoef[a][0] + c4[1] * st.acoef[a][1] +
                       c4[2] * st.acoef[a][2] + c4[3] * st.acoef[a][3];
            }
          }
        }
        __syncthreads();
        const bool alias = periodic && (P.nx < B || P.ny < B || P.nz < B);
        for (int a = 0; a < natoms; ++a) {
          if (!st.aphase[a]) continue;
          const int J = st.atom[a];
          if (alias) {
            if (tid == 0) {
              for (int b = 0; b < B3; ++b) {
                int lp = box_point(st, a, b, B);
                const T* c4 = chi + ((size_t)J * B3 + b) * 4;
                U[lp] += c4[0] * st.acoef[a][0] + c4[1] * st.acoef[a][1] +
                         c4[2] * st.acoef[a][2] + c4[3] * st.acoef[a][3];
              }
            }
          } else {
            for (int b = tid; b < B3; b += BLOCK) {
              int lp = box_point(st, a, b, B);
              if (lp >= 0) {
                const T* c4 = chi + ((size_t)J * B3 + b) * 4;
                U[lp] += c4[0] * st.acoef[a][0] + c4[1] * st.acoef[a][1] +
                         c4[2] * st.acoef[a][2] + c4[3] * st.acoef[a][3];
              }
            }
          }
          __syncthreads();
        }
      }
      if (tid == 0) {
        double al = 0.0;
        for (int w = 0; w < NW; ++w) al += st.red[w][0];
        for (int a = 0; a < natoms; ++a) al += st.anl[a];
        st.alpha[j] = al;
      }
      __syncthreads();
      if (j == K - 1) break;
      // ---- reorthogonalisation coefficients (Gram column through the tridiagonal)
      for (int i = tid; i <= j; i += BLOCK) {
        double c;
        if (i == j) {
          c = st.alpha[j];
        } else {
          double gi1 = (i + 1 == j) ? 1.0 : st.gram[i + 1];
          c = st.alpha[i] * st.gram[i] + st.beta[i] * gi1;
          if (i > 0) c += st.beta[i - 1] * st.gram[i - 1];
        }
        st.ct[i] = (T)(c * st.scale[i]);
      }
      __syncthreads();
      // ---- fused sweep: w = u - sum c_i q_i, D_i = W_i . w, |w|^2
      T* __restrict__ Wn = W + (size_t)(j + 1) * npad;
      fused_sweep<T, BLOCK, KG>(st, W, U, Wn, j, n, npad);
      __syncthreads();
      finish_sweep<T, BLOCK>(st, j);
      // Semi-orthogonality guard: the coefficients above are exact up to O(G^2); when
      // the measured Gram column exceeds sqrt(eps) (only near an invariant subspace)
      // the projection is repeated once with the exact dots of this sweep.
      if (st.redo && st.beta[j] > tol) {
        for (int i = tid; i <= j; i += BLOCK)
          st.ct[i] = (T)(st.scale[i] * st.scale[i] * st.dsave[i]);
        __syncthreads();
        fused_sweep<T, BLOCK, KG>(st, W, Wn, Wn, j, n, npad);
        __syncthreads();
        finish_sweep<T, BLOCK>(st, j);
      }
      if (!(st.beta[j] > tol)) {   // breakdown (or NaN): the Krylov space is invariant
        keff = j + 1;
        break;
      }
    }
    // ---- Gauss rule and quadrature (one thread)
    if (tid == 0) {
      for (int k = 0; k < keff; ++k) st.ta[k] = st.alpha[k];
      for (int k = 0; k + 1 < keff; ++k) st.tb[k] = st.beta[k];
      bool ok = tridiag_gauss(st.ta, st.tb, st.tz, keff);
      if (!ok) atomicOr(P.status, kStatusNonFinite);
      double rho = 0.0, e = 0.0;
      for (int k = 0; k < keff; ++k) {
        double wk = st.tz[k] * st.tz[k];
        double th = st.ta[k];
        rho += wk * fermi_occ((th - P.mu) / P.kT);
        if (P.e_node) e += wk * integrand_value(th, P.mu, P.kT, P.integrand);
      }
      if (P.rho) P.rho[q] = 2.0 / h3 * rho;
      if (P.e_node) P.e_node[q] = 2.0 * e;
      if (P.k_eff) P.k_eff[q] = keff;
      if (P.theta_w) {
        // ascending order of nodes
        for (int k = 1; k < keff; ++k) {
          double tk = st.ta[k], zk = st.tz[k];
          int i = k - 1;
          while (i >= 0 && st.ta[i] > tk) {
            st.ta[i + 1] = st.ta[i];
            st.tz[i + 1] = st.tz[i];
            --i;
          }
          st.ta[i + 1] = tk;
          st.tz[i + 1] = zk;
        }
        double* out = P.theta_w + (size_t)q * P.kmax_out * 2;
        for (int k = 0; k < P.kmax_out; ++k) {
          out[2 * k] = k < keff ? st.ta[k] : 0.0;
          out[2 * k + 1] = k < keff ? st.tz[k] * st.tz[k] : 0.0;
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ setup kernels
__global__ void reset_kernel(int* queue, int* status, double* vmax) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *queue = 0;
    *status = 0;
    *vmax = 0.0;
  }
}

// Potential in the storage precision, max |V| (order-independent) and a finiteness check.
template <typename T>
__global__ void prepare_potential_kernel(const double* __restrict__ v64, T* __restrict__ vout,
                                         size_t n, double* vmax, int* status) {
  __shared__ double red[1024 / kWave];
  double mx = 0.0;
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = v64[i];
    if (!isfinite(v)) bad = true;
    mx = fmax(mx, fabs(v));
    if (vout) vout[i] = (T)v;
  }
  if (bad) atomicOr(status, kStatusNonFinite);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) mx = fmax(mx, red[w]);
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(vmax),
              (unsigned long long)__double_as_longlong(mx));
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
  if (fp64) {
    return block == 512 ? launch_forward_t<double, 512>(P, grid, kg, s)
                        : launch_forward_t<double, 256>(P, grid, kg, s);
  }
  return block == 512 ? launch_forward_t<float, 512>(P, grid, kg, s)
                      : launch_forward_t<float, 256>(P, grid, kg, s);
}

hipError_t launch_setup(const LaunchParams& P, bool fp64, const double* v64, void* vstore,
                        void* chi, int32_t* g0, double* vmax, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, P.queue, P.status, vmax);
  size_t n = (size_t)P.nx * P.ny * P.nz;
  int blocks = (int)((n + 1023) / 1024);
  if (blocks > 1024) blocks = 1024;
  if (fp64) {
    hipLaunchKernelGGL(prepare_potential_kernel<double>, dim3(blocks), dim3(1024), 0, s, v64,
                       (double*)nullptr, n, vmax, P.status);
  } else {
    hipLaunchKernelGGL(prepare_potential_kernel<float>, dim3(blocks), dim3(1024), 0, s, v64,
                       (float*)vstore, n, vmax, P.status);
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

hipError_t launch_weighted_sum(const double* e, const double* w, int n, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(weighted_sum_kernel, dim3(1), dim3(1024), 0, s, e, w, n, out);
  return hipGetLastError();
}

}  // namespace sgq
