// Adjoint of Omega = sum_q n_q e_q, e_q = 2 e_1^T F(T_q) e_1 (band / free-energy terms of
// the total-energy expression, weighted as in the coarse-grained energy sum), with
// respect to the local potential, the projector energies and the atom positions.
//
// Per node (one workgroup, persistent queue as in the forward kernel):
//   1. the forward Lanczos run is recomputed from the start vector, keeping every
//      u_j = H q_j; or, when the forward call retained the node's basis and u_j rows
//      (sgq_plan_set_retain, for all nodes or the costliest ones within a byte limit),
//      those are taken with alpha, beta and K_eff from the forward's tridiagonal buffer
//      (the same values bit for bit);
//   2. the eigenvectors S of T (wave-parallel QR sweeps, FP64, in LDS) give the
//      Daleckii-Krein adjoint Tbar = 2 n_q Omegabar S (D o s1 s1^T) S^T, D the divided
//      differences of F; alphabar_j = Tbar_jj, betabar_j = 2 Tbar_j,j+1;
//   3. the exact-arithmetic three-term recurrence is reversed, j = K-1 .. 0:
//        rbar = qbar_{j+1}/beta_j + (betabar_j - qbar_{j+1}.q_{j+1}/beta_j) q_{j+1}
//        ahat = alphabar_j - rbar.q_j,   ubar_j = rbar + ahat q_j
//        qbar_j += -alpha_j rbar + ahat u_j + H ubar_j
//        qbar_{j-1} = -beta_{j-1} rbar,  betabar_{j-1} -= rbar.q_{j-1}
//      accumulating the node's dV cube P_q = sum_j ubar_j o q_j; ubar_j replaces u_j in
//      the workspace once step j is done;
//   4. the projector adjoints Ebar_Jl = h^3 sum_j (chi.ubar_j)(chi.q_j) and
//      Rbar_J = h^3 E sum_j [(ubar_j.dchi)(chi.q_j) + (ubar_j.chi)(dchi.q_j)]
//      (dchi = d chi / d R) come from one dense product per atom,
//      M = [chi; d chi] (16 x box points) . [ubar_j | q_j], on the matrix cores (16x16x4
//      MFMA, accumulation in the storage precision), one wave per atom;
//   5. a gather kernel sums the node cubes into dV in a fixed order (deterministic,
//      no floating-point atomics) and a reduction kernel sums the atom adjoints.
#include "lanczos_device.h"

namespace sgq {

constexpr int kBwdMaxDepth = kMaxDepth;   // largest depth of the adjoint (eigenvector matrix K x K)
constexpr int kGatherCell = 8;     // dV gather cell edge (points)

struct BwdState {
  double abar[kBwdMaxDepth], bbar[kBwdMaxDepth];
  double Fv[kBwdMaxDepth], Fd[kBwdMaxDepth];
  double part[4 * kBwdMaxDepth];
  double sc[8];
};

// 16x16x4 matrix-core product of one wave: A (16 x 4) from lane i + 16k, B (4 x 16) from
// lane j + 16k; output element r of lane l is row row(l, r), column l % 16.
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  using V = float __attribute__((ext_vector_type(4)));
  __device__ static V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma16<double> {
  using V = double __attribute__((ext_vector_type(4)));
  __device__ static V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Projector adjoints of one node from its stored vectors: for every node atom (one wave
// per atom, the node's waves working side by side) the dense product
// M = [chi_0..3 ; d chi_l / d d_a] (16 x box points) times the box values of the columns
// [ubar_j | q_j] on the matrix cores, then
//   Ebar_l = h^3 sum_j M[l][ubar_j] M[l][q_j],
//   Rbar_a = -h^3 sum_l E_l sum_j (M[4+3l+a][ubar_j] M[l][q_j] + M[l][ubar_j] M[4+3l+a][q_j]).
// Column block b of the product holds ubar_j in its columns 0..7 and q_j in its columns
// 8..15, j = 8b .. 8b+7, so every pair the sums need lies in one 16 x 16 output tile: the
// wave stages a finished tile in its own 16 x 16 piece of `scratch` (LDS) and folds it into
// FP64 sums at once.  CB blocks are accumulated per pass over the box (CB MFMA accumulators
// in registers), so a depth of 8 CB or less takes one pass and the projector values are
// evaluated once.
template <typename T, int BLOCK, int CB>
__device__ __noinline__ void projector_gradients(const SGQ_G double* proj_E,
                                                 SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                                 const SGQ_G T* W, int wbs, const SGQ_G T* Ub,
                                                 int npad, int keff, double h3, int B, int B3,
                                                 SGQ_L T* scratch, double* dEp, double* dRp) {
  using M16 = Mfma16<T>;
  using V = typename M16::V;
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int fr = lane & 15, kk = lane >> 4;   // A row / B column, and the k index of the lane
  const int nblk = (keff + 7) / 8;
  SGQ_L T* Ms = scratch + wave * 256;          // this wave's 16 x 16 tile
  const int natoms = st.natoms;
  for (int a = wave; a < natoms; a += NW) {
    const int J = st.atom[a];
    double El[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) El[l] = proj_E[4 * J + l];
    double eb[4] = {0, 0, 0, 0}, rb[3] = {0, 0, 0};
    for (int b0 = 0; b0 < nblk; b0 += CB) {
      V acc[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[cb] = (V)(T)0;
      for (int k0 = 0; k0 < B3; k0 += 4) {
        const int b = k0 + kk;
        const int bx = b % B, by = (b / B) % B, bz = b / (B * B);
        const int lp = b < B3 ? box_point(st, a, bx, by, bz) : -1;
        T c[4], g[12];
        chi_grad_at(pe, st.afrac[a], bx, by, bz, c, g);
        T av = (T)0;
#pragma unroll
        for (int r = 0; r < 16; ++r) av = fr == r ? (r < 4 ? c[r] : g[r - 4]) : av;
        av = b < B3 ? av : (T)0;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          if (b0 + cb < nblk) {
            const int j = 8 * (b0 + cb) + (fr & 7);
            T bv = (T)0;
            if (lp >= 0 && j < keff)
              bv = fr < 8 ? Ub[(size_t)j * npad + lp]
                          : W[64 * j + bidx(lp, wbs)] * (T)st.scale[j];
            acc[cb] = M16::op(av, bv, acc[cb]);
          }
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (b0 + cb < nblk) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Ms[M16::row(lane, r) * 16 + fr] = acc[cb][r];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const int j = 8 * (b0 + cb) + lane;
          if (lane < 8 && j < keff) {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              const double cu = (double)Ms[l * 16 + lane], cq = (double)Ms[l * 16 + 8 + lane];
              eb[l] += cu * cq;
#pragma unroll
              for (int ax = 0; ax < 3; ++ax) {
                const int rr = 4 + 3 * l + ax;
                rb[ax] += El[l] * ((double)Ms[rr * 16 + lane] * cq + cu * (double)Ms[rr * 16 + 8 + lane]);
              }
            }
          }
          // the tile is read before the next block overwrites it
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) eb[l] = wave_sum(eb[l]);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) rb[ax] = wave_sum(rb[ax]);
    if (lane == 0) {
      for (int l = 0; l < 4; ++l) dEp[4 * a + l] = h3 * eb[l];
      for (int ax = 0; ax < 3; ++ax) dRp[3 * a + ax] = -h3 * rb[ax];
    }
  }
}

// Implicit-shift QR of the tridiagonal (a, b) accumulating all eigenvectors in Z.
// Run by one whole wave: every lane computes the same rotations from the LDS copies of
// a and b (lane 0 writes them back) and updates its rows of Z.
// Z (global, per workgroup slot): Z[i*K + k] is component i of eigenvector k.  Each lane
// owns rows i = lane (mod 64) of Z, so its updates need no synchronisation with the
// other lanes.
__device__ bool tridiag_eig_wave(SGQ_L double* a, SGQ_L double* b, SGQ_G double* Z, int K) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int i = lane; i < K; i += kWave)
    for (int k = 0; k < K; ++k) Z[i * K + k] = (i == k) ? 1.0 : 0.0;
  const double eps = 2.220446049250313e-16;
  int m = K - 1;
  int sweeps = 0;
  while (m > 0) {
    if (fabs(b[m - 1]) <= eps * (fabs(a[m - 1]) + fabs(a[m]))) {
      if (lane == 0) b[m - 1] = 0.0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && fabs(b[l - 1]) > eps * (fabs(a[l - 1]) + fabs(a[l]))) --l;
    if (l > 0 && lane == 0) b[l - 1] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (++sweeps > 40 * K) return false;
    double d = 0.5 * (a[m - 1] - a[m]);
    double bm = b[m - 1];
    double den = d + copysign(hypot(d, bm), d == 0.0 ? 1.0 : d);
    double shift = a[m] - bm * bm / den;
    double x = a[l] - shift;
    double y = b[l];
    for (int k = l; k < m; ++k) {
      double r = hypot(x, y);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -y / r;
      }
      double ak = a[k], ak1 = a[k + 1], bk = b[k];
      double bulge = 0.0, bk1 = 0.0;
      if (k + 1 < m) {
        bk1 = b[k + 1];
        bulge = -s * bk1;
      }
      const double nak = c * c * ak - 2.0 * c * s * bk + s * s * ak1;
      const double nak1 = s * s * ak + 2.0 * c * s * bk + c * c * ak1;
      const double nbk = c * s * (ak - ak1) + (c * c - s * s) * bk;
      if (lane == 0) {
        if (k > l) b[k - 1] = r;
        a[k] = nak;
        a[k + 1] = nak1;
        b[k] = nbk;
        if (k + 1 < m) b[k + 1] = c * bk1;
      }
      // lane 0's LDS writes must be ordered before the next rotation's reads by the
      // other lanes: without the fence the compiler may hoist those reads
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int i = lane; i < K; i += kWave) {
        double u0 = Z[i * K + k], u1 = Z[i * K + k + 1];
        Z[i * K + k] = c * u0 - s * u1;
        Z[i * K + k + 1] = s * u0 + c * u1;
      }
      x = nbk;
      y = bulge;
    }
  }
  return true;
}

template <typename T, int BLOCK, int KG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void lanczos_backward_kernel(LaunchParams P) {
  constexpr int NW = BLOCK / kWave;
  __shared__ NodeState<T, BLOCK> st_shared;
  __shared__ BwdState bs_shared;
  SGQ_L NodeState<T, BLOCK>& st = *(SGQ_L NodeState<T, BLOCK>*)(&st_shared);
  SGQ_L BwdState& bs = *(SGQ_L BwdState*)(&bs_shared);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const size_t npad = P.npad;
  const int kmax = P.kmax_out;
  const int wbs = P.wbs;
  SGQ_G T* __restrict__ W = (SGQ_G T*)P.W + (size_t)blockIdx.x * P.slot_stride;
  SGQ_G T* __restrict__ Ubase = W + (size_t)kmax * npad;
  SGQ_G double* __restrict__ Z = (SGQ_G double*)P.zbuf + (size_t)blockIdx.x * kBwdMaxDepth * kBwdMaxDepth;
  SGQ_G T* __restrict__ R[3] = {Ubase + (size_t)kmax * npad, Ubase + (size_t)(kmax + 1) * npad,
                                Ubase + (size_t)(kmax + 2) * npad};
  const SGQ_G T* __restrict__ V = (const SGQ_G T*)P.v;
  const ProjEval<T> pe = proj_eval<T>(P);
  const SGQ_G double* proj_E = (const SGQ_G double*)P.proj_E;
  const double h = P.h, h3 = h * h * h;
  const T kin = (T)(-0.5 / (h * h));
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
  const double gomega = *P.grad_omega;
  constexpr int VW = 16 / (int)sizeof(T);                    // points per 16-byte access
  typedef T VT __attribute__((ext_vector_type(VW)));
  if (tid == 0) st.orth_tol = sizeof(T) == 4 ? 3.4526698300124393e-4 : 1.4901161193847656e-8;

  for (;;) {
    if (tid == 0) st.node = atomicAdd(P.queue, 1);
    __syncthreads();
    const int qi = st.node;
    if (qi >= P.n_nodes) break;
    const int q = P.order[qi];
    node_setup<T, BLOCK>(P, st, q);
    SGQ_G T* __restrict__ Pq = (SGQ_G T*)P.P_cube + P.cube_offset[q];
    int32_t* natoms_out = P.node_atoms + (size_t)q * (kMaxNodeAtoms + 1);
    if (st.abort) {
      for (int p = tid; p < st.n; p += BLOCK) Pq[p] = (T)0;
      if (tid == 0) natoms_out[0] = 0;
      __syncthreads();
      continue;
    }
    const int n = st.n, natoms = st.natoms;
    // the node's basis and u_j rows: retained by the forward call, or recomputed here
    SGQ_G T* __restrict__ Wq = W;
    SGQ_G T* __restrict__ Uq = Ubase;
    int keff;
    // retained rows serve only inputs with the contents the forward call saw
    const int rs = P.use_retained && P.hash[0] == P.hash[1] ? P.ret_slot[q] : -1;
    if (rs >= 0) {
      const size_t roff = (size_t)rs * kmax * npad;
      Wq = (SGQ_G T*)P.Wr + roff;
      Uq = (SGQ_G T*)P.Ur + roff;
      keff = P.tri_k[q];
      const double* tri = P.tri + (size_t)q * 2 * kmax;
      for (int k = tid; k < keff; k += BLOCK) {
        st.alpha[k] = tri[k];
        if (k + 1 < keff) {
          const double b = tri[kmax + k];
          st.beta[k] = b;
          st.scale[k + 1] = b > 0.0 ? 1.0 / b : 0.0;   // as the forward's sweep sets it
        }
      }
      if (tid == 0) st.scale[0] = 1.0;
      __syncthreads();
    } else {
      keff = run_lanczos<T, BLOCK, KG>(P, st, W, Ubase, npad, P.depth[q]);
    }
    // ---- eigenvectors of T and the Daleckii-Krein adjoint
    for (int k = tid; k < keff; k += BLOCK) {
      st.ta[k] = st.alpha[k];
      st.tb[k] = k + 1 < keff ? st.beta[k] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      bool ok = tridiag_eig_wave(st.ta, st.tb, Z, keff);
      if (!ok && lane == 0) atomicOr(P.status, kStatusNonFinite);
    }
    __syncthreads();
    const double cscale = 2.0 * P.node_weight[q] * gomega;
    for (int k = tid; k < keff; k += BLOCK) {
      bs.Fv[k] = integrand_value(st.ta[k], P.mu, P.kT, P.integrand);
      bs.Fd[k] = integrand_deriv(st.ta[k], P.mu, P.kT, P.integrand);
    }
    __syncthreads();
    // output o < keff: alphabar_o; o >= keff: betabar_{o-keff}; two threads per output
    for (int t = tid; t < 2 * (2 * keff - 1); t += BLOCK) {
      const int o = t >> 1, half = t & 1;
      const int j = o < keff ? o : o - keff;
      const int m = o < keff ? o : o - keff + 1;
      double acc = 0.0;
      for (int k = half; k < keff; k += 2) {
        const double tk = st.ta[k];
        const double ak = Z[j * keff + k] * Z[k];
        double inner = 0.0;
        for (int l = 0; l < keff; ++l) {
          const double tl = st.ta[l];
          const double diff = tk - tl;
          double D;
          if (l == k) {
            D = bs.Fd[k];
          } else if (fabs(diff) <= 1e-6 * fmax(P.kT, fmax(fabs(tk), fabs(tl)))) {
            D = integrand_deriv(0.5 * (tk + tl), P.mu, P.kT, P.integrand);
          } else {
            D = (bs.Fv[k] - bs.Fv[l]) / diff;
          }
          inner += D * Z[l] * Z[m * keff + l];
        }
        acc += ak * inner;
      }
      bs.part[t] = acc;
    }
    __syncthreads();
    for (int o = tid; o < 2 * keff - 1; o += BLOCK) {
      const double v = cscale * (bs.part[2 * o] + bs.part[2 * o + 1]);
      if (o < keff) bs.abar[o] = v;
      else bs.bbar[o - keff] = 2.0 * v;
    }
    __syncthreads();
    // ---- reverse recurrence
    int r0 = 0, r1 = 1, r2 = 2;
    for (int j = keff - 1; j >= 0; --j) {
      // rows of the point-blocked basis (block stride wbs)
      const SGQ_G T* Wc = Wq + 64 * j;
      const SGQ_G T* Wn = Wq + 64 * (j + 1);
      const SGQ_G T* Wp = Wq + 64 * (j > 0 ? j - 1 : 0);
      SGQ_G T* Uj = Uq + (size_t)j * npad;      // u_j, replaced by ubar_j in pass B
      SGQ_G T* Q0 = R[r0];
      SGQ_G T* Q1 = R[r1];
      SGQ_G T* Q2 = R[r2];
      const double sc_ = st.scale[j];
      const double sn = (j + 1 < keff) ? st.scale[j + 1] : 0.0;
      const double sp = j > 0 ? st.scale[j - 1] : 0.0;
      const bool last = (j == keff - 1);
      // pass A: the dot products the recurrence needs (FP64).  Every row involved starts
      // 16-byte aligned and VW consecutive points of a basis row are adjacent in the
      // point-blocked layout, so each lane takes VW points per 16-byte load; points past
      // n read as zero.
      if (!last) {
        double d[5] = {0, 0, 0, 0, 0};
        for (int p = tid * VW; p < n; p += BLOCK * VW) {
          const VT q0 = *(const SGQ_G VT*)(Q0 + p);
          const VT wn = *(const SGQ_G VT*)(Wn + bidx(p, wbs));
          const VT wc = *(const SGQ_G VT*)(Wc + bidx(p, wbs));
          const VT wp = *(const SGQ_G VT*)(Wp + bidx(p, wbs));
#pragma unroll
          for (int k = 0; k < VW; ++k) {
            const bool in = p + k < n;
            const double qb = in ? (double)q0[k] : 0.0;
            const double qn = in ? sn * (double)wn[k] : 0.0;
            const double qc = in ? sc_ * (double)wc[k] : 0.0;
            const double qp = in ? sp * (double)wp[k] : 0.0;
            d[0] += qb * qn;
            d[1] += qb * qc;
            d[2] += qb * qp;
            d[3] += qn * qc;
            d[4] += qn * qp;
          }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          d[c] = wave_sum(d[c]);
          if (lane == 0) st.red[wave][c] = d[c];
        }
        __syncthreads();
        if (tid == 0) {
          double D[5] = {0, 0, 0, 0, 0};
          for (int w = 0; w < NW; ++w)
            for (int c = 0; c < 5; ++c) D[c] += st.red[w][c];
          const double bj = st.beta[j];
          const double bb = bs.bbar[j] - D[0] / bj;
          const double rqc = D[1] / bj + bb * D[3];
          const double rqp = D[2] / bj + bb * D[4];
          bs.sc[0] = 1.0 / bj;
          bs.sc[1] = bb;
          bs.sc[2] = bs.abar[j] - rqc;
          if (j > 0) bs.bbar[j - 1] -= rqp;
        }
      } else if (tid == 0) {
        bs.sc[0] = 0.0;
        bs.sc[1] = 0.0;
        bs.sc[2] = bs.abar[j];
      }
      __syncthreads();
      // pass B: ubar_j, the node dV cube, and the adjoint rows (VW points per lane as in
      // pass A; the padding past n, inside every row and cube, receives zeros)
      {
        const double ib = bs.sc[0], bb = bs.sc[1], ahat = bs.sc[2];
        const double al = st.alpha[j];
        const double bprev = j > 0 ? st.beta[j - 1] : 0.0;
        for (int p = tid * VW; p < n; p += BLOCK * VW) {
          const VT wc = *(const SGQ_G VT*)(Wc + bidx(p, wbs));
          const VT uj = *(const SGQ_G VT*)(Uj + p);
          VT q0 = {}, wn = {}, pq = {}, q1 = {};
          if (!last) {
            q0 = *(const SGQ_G VT*)(Q0 + p);
            wn = *(const SGQ_G VT*)(Wn + bidx(p, wbs));
            pq = *(const SGQ_G VT*)(Pq + p);
            q1 = *(const SGQ_G VT*)(Q1 + p);
          }
          VT o_u, o_p, o_q1, o_q2;
#pragma unroll
          for (int k = 0; k < VW; ++k) {
            const bool in = p + k < n;
            const double qc = sc_ * (double)wc[k];
            const double rb = (double)q0[k] * ib + bb * sn * (double)wn[k];
            const double ub = rb + ahat * qc;
            o_u[k] = in ? (T)ub : (T)0;
            o_p[k] = in ? (T)((double)pq[k] + ub * qc) : (T)0;
            o_q1[k] = in ? (T)((double)q1[k] - al * rb + ahat * (double)uj[k]) : (T)0;
            o_q2[k] = in ? (T)(-bprev * rb) : (T)0;
          }
          *(SGQ_G VT*)(Uj + p) = o_u;
          *(SGQ_G VT*)(Pq + p) = o_p;
          *(SGQ_G VT*)(Q1 + p) = o_q1;
          if (j > 0) *(SGQ_G VT*)(Q2 + p) = o_q2;
        }
      }
      __syncthreads();
      // pass C: qbar_j += H ubar_j (projector weights E h^3 chi.ubar_j for the scatter)
      // (in the FP32 march the projector group's term is added plane by plane, as in the
      // forward step, and the scatter then covers the remaining atoms)
      if (natoms > 0) projector_dots<T, BLOCK>(proj_E, st, pe, Uj, 64, 1.0, h3, B, B3);
      const bool fused = st.fuse && uses_march(st, BLOCK);
      apply_local<T, BLOCK, true>(P, st, V, Uj, 64, Q1, (T)1, kin, pe, B, fused);
      __syncthreads();
      apply_scatter<T, BLOCK>(P, st, pe, Q1, B, B3, !fused);
      __syncthreads();
      const int t0 = r0;
      r0 = r1;
      r1 = r2;
      r2 = t0;
    }
    // ---- per-node projector adjoints (matrix cores), staged through the march's plane
    // buffers, which are idle after the reverse recurrence
    double* dEp = P.dE_part + (size_t)q * kMaxNodeAtoms * 4;
    double* dRp = P.dR_part + (size_t)q * kMaxNodeAtoms * 3;
    if (natoms > 0) {
      static_assert(sizeof(st.plane) >= NW * 256 * sizeof(T),
                    "the plane buffers must hold a 16 x 16 tile per wave");
      __syncthreads();
      projector_gradients<T, BLOCK, 8>(proj_E, st, pe, Wq, wbs, Uq, (int)npad, keff, h3, B, B3,
                                       (SGQ_L T*)&st.plane[0][0], dEp, dRp);
    }
    for (int a = tid; a < natoms; a += BLOCK) natoms_out[1 + a] = st.atom[a];
    if (tid == 0) natoms_out[0] = natoms;
    __syncthreads();
  }
}

// dV(x) = sum over the nodes whose cube contains x of P_q(x), in ascending node order.
// One workgroup per 8^3 cell of the grid; cell_nodes lists the nodes meeting each cell.
template <typename T>
__global__ __launch_bounds__(512) void gather_dv_kernel(LaunchParams P, const int32_t* cell_start,
                                                      const int32_t* cell_nodes, double* dV) {
  const int C = kGatherCell;
  const int ncx = (P.nx + C - 1) / C, ncy = (P.ny + C - 1) / C;
  const int cell = blockIdx.x;
  const int cx = cell % ncx, cy = (cell / ncx) % ncy, cz = cell / (ncx * ncy);
  const int x = cx * C + (threadIdx.x % C);
  const int y = cy * C + (threadIdx.x / C) % C;
  const int z = cz * C + threadIdx.x / (C * C);
  const bool inside = x < P.nx && y < P.ny && z < P.nz;
  const SGQ_G T* Pc = (const SGQ_G T*)P.P_cube;
  double acc = 0.0;
  const int e0 = cell_start[cell], e1 = cell_start[cell + 1];
  for (int e = e0; e < e1; ++e) {
    const int q = cell_nodes[e];
    const int R = P.half_width[q];
    const int c = P.center[q];
    int lx, ly, lz, s;
    if (R < 0) {
      lx = x; ly = y; lz = z;
      if (!inside) continue;
      acc += (double)Pc[P.cube_offset[q] + lx + P.nx * (ly + P.ny * lz)];
      continue;
    }
    s = 2 * R + 1;
    lx = wrap_index(x - (c % P.nx - R), P.nx);
    ly = wrap_index(y - ((c / P.nx) % P.ny - R), P.ny);
    lz = wrap_index(z - (c / (P.nx * P.ny) - R), P.nz);
    if (inside && lx < s && ly < s && lz < s)
      acc += (double)Pc[P.cube_offset[q] + lx + s * (ly + s * lz)];
  }
  if (inside) dV[x + P.nx * (y + P.ny * z)] = acc;
}

// dE[J], dR_nl[J]: sum over nodes (ascending) of the node partials of atom J, found by
// binary search in each node's sorted atom list; fixed-order block reduction.
__global__ __launch_bounds__(256) void reduce_atom_adjoints_kernel(LaunchParams P, double* dR,
                                                                   double* dE) {
  __shared__ double red[256][8];
  const int J = blockIdx.x;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < P.n_nodes; q += blockDim.x) {
    const int32_t* lst = P.node_atoms + (size_t)q * (kMaxNodeAtoms + 1);
    int lo = 0, hi = lst[0] - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = lst[1 + mid];
      if (v == J) {
        const double* e = P.dE_part + ((size_t)q * kMaxNodeAtoms + mid) * 4;
        const double* r = P.dR_part + ((size_t)q * kMaxNodeAtoms + mid) * 3;
        for (int l = 0; l < 4; ++l) acc[l] += e[l];
        for (int c = 0; c < 3; ++c) acc[4 + c] += r[c];
        break;
      }
      if (v < J) lo = mid + 1; else hi = mid - 1;
    }
  }
  for (int c = 0; c < 7; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half)
      for (int c = 0; c < 7; ++c) red[threadIdx.x][c] += red[threadIdx.x + half][c];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (dE)
      for (int l = 0; l < 4; ++l) dE[4 * J + l] = red[0][l];
    if (dR)
      for (int c = 0; c < 3; ++c) dR[3 * J + c] = red[0][4 + c];
  }
}

// dR[J] += sum_x dV(x) dV_loc(x)/dR_J for the Gaussian local potential
// V(x) = depth sum_J sum_images exp(-|x - R_J - L m|^2 / (2 sigma^2)) (distance <= cutoff).
__global__ __launch_bounds__(256) void vloc_backward_kernel(const double* __restrict__ dV,
                                                            const double* __restrict__ R, int nx,
                                                            int ny, int nz, double h, double depth,
                                                            double sigma, double rcut, double* dR) {
  __shared__ double red[256][3];
  const int J = blockIdx.x;
  const double Rx = R[3 * J], Ry = R[3 * J + 1], Rz = R[3 * J + 2];
  const int w = (int)ceil(rcut / h) + 1;
  const int W = 2 * w + 1;
  const int gx = (int)floor(Rx / h), gy = (int)floor(Ry / h), gz = (int)floor(Rz / h);
  double acc[3] = {0, 0, 0};
  const double s2 = sigma * sigma;
  for (int b = threadIdx.x; b < W * W * W; b += blockDim.x) {
    const int ix = gx - w + b % W, iy = gy - w + (b / W) % W, iz = gz - w + b / (W * W);
    const double dx = ix * h - Rx, dy = iy * h - Ry, dz = iz * h - Rz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 > rcut * rcut) continue;
    const double g =
        depth * exp(-r2 / (2.0 * s2)) / s2 *
        dV[wrap_index(ix, nx) + nx * (wrap_index(iy, ny) + ny * wrap_index(iz, nz))];
    acc[0] += g * dx;
    acc[1] += g * dy;
    acc[2] += g * dz;
  }
  for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half)
      for (int c = 0; c < 3; ++c) red[threadIdx.x][c] += red[threadIdx.x + half][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) dR[3 * J + c] += red[0][c];
}

// ------------------------------------------------------------------ host launchers
template <typename T>
static hipError_t launch_backward_t(const LaunchParams& P, int grid, int kg, hipStream_t s) {
  switch (kg) {
    case 8:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, 256, 8>), dim3(grid), dim3(256), 0, s, P);
      break;
    case 16:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, 256, 16>), dim3(grid), dim3(256), 0, s, P);
      break;
    default:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, 256, 32>), dim3(grid), dim3(256), 0, s, P);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_backward(const LaunchParams& P, bool fp64, int grid, int block, int kg,
                           hipStream_t s) {
  (void)block;
  return fp64 ? launch_backward_t<double>(P, grid, kg, s) : launch_backward_t<float>(P, grid, kg, s);
}

hipError_t launch_backward_gather(const LaunchParams& P, bool fp64, const int32_t* cell_start,
                                  const int32_t* cell_nodes, int ncells, double* dV, double* dR,
                                  double* dE, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(gather_dv_kernel<double>, dim3(ncells), dim3(512), 0, s, P, cell_start,
                       cell_nodes, dV);
  else
    hipLaunchKernelGGL(gather_dv_kernel<float>, dim3(ncells), dim3(512), 0, s, P, cell_start,
                       cell_nodes, dV);
  if (P.n_proj > 0 && P.n_atoms > 0 && (dR || dE))
    hipLaunchKernelGGL(reduce_atom_adjoints_kernel, dim3(P.n_atoms), dim3(256), 0, s, P, dR, dE);
  return hipGetLastError();
}

hipError_t launch_vloc_backward(const double* dV, const double* R, int M, int nx, int ny, int nz,
                                double h, double depth, double sigma, double cutoff, double* dR,
                                hipStream_t s) {
  if (M > 0)
    hipLaunchKernelGGL(vloc_backward_kernel, dim3(M), dim3(256), 0, s, dV, R, nx, ny, nz, h,
                       depth, sigma, cutoff * sigma, dR);
  return hipGetLastError();
}

__global__ void zero_kernel(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0 || !p) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

int backward_max_depth() { return kBwdMaxDepth; }
int gather_cell() { return kGatherCell; }

}  // namespace sgq
