// Adjoint of Omega = sum_q n_q e_q, e_q = 2 e_1^T F(T_q) e_1 (band / free-energy terms of
// the total-energy expression, weighted as in the coarse-grained energy sum), with
// respect to the local potential, the projector energies and the atom positions.
//
// Per node (one workgroup, persistent queue as in the forward kernel; FP32 cubes of 37 to
// 49 points in a 512-lane launch, whose plane march takes planes that wide, then every
// other node in a 256-lane launch):
//   1. the forward Lanczos run is recomputed from the start vector, keeping every
//      u_j = H q_j; or, when the forward call retained the node's basis and u_j rows
//      (sgq_plan_set_retain, for all nodes or the costliest ones within a byte limit),
//      those are taken with alpha, beta and K_eff from the forward's tridiagonal buffer
//      (the same values bit for bit);
//   2. the eigenvectors S of T (wave-parallel QR sweeps, FP64, S in a global slot; in a
//      pre-pass over the forward's tridiagonals when it stored them) give the
//      Daleckii-Krein adjoint Tbar = 2 n_q Omegabar S (D o s1 s1^T) S^T, D the divided
//      differences of F; alphabar_j = Tbar_jj, betabar_j = 2 Tbar_j,j+1;
//   3. the exact-arithmetic three-term recurrence is reversed, j = K-1 .. 0:
//        rbar = qbar_{j+1}/beta_j + (betabar_j - qbar_{j+1}.q_{j+1}/beta_j) q_{j+1}
//        ahat = alphabar_j - rbar.q_j,   ubar_j = rbar + ahat q_j
//        qbar_j += -alpha_j rbar + ahat u_j + H ubar_j
//        qbar_{j-1} = -beta_{j-1} rbar,  betabar_{j-1} -= rbar.q_{j-1}
//      accumulating the node's dV cube P_q = sum_j ubar_j o q_j.  FP32 nodes on the
//      plane march run each step as one fused march (reverse_march); the others as
//      separate dot, update and operator passes, where ubar_j replaces u_j in the
//      workspace once step j is done;
//   4. the projector adjoints Ebar_Jl = h^3 sum_j (chi.ubar_j)(chi.q_j) and
//      Rbar_J = h^3 E sum_j [(ubar_j.dchi)(chi.q_j) + (ubar_j.chi)(dchi.q_j)]
//      (dchi = d chi / d R): in the fused steps from the box sums each step forms anyway
//      (ubar_coefs); otherwise from one dense product per atom,
//      M = [chi; d chi] (16 x box points) . [ubar_j | q_j], on the matrix cores (16x16x4
//      MFMA, accumulation in the storage precision), one wave per atom;
//   5. a gather kernel sums the node cubes into dV in a fixed order (deterministic,
//      no floating-point atomics) and a reduction kernel sums the atom adjoints.
#include "lanczos_device.h"

namespace sgq {

constexpr int kBwdMaxDepth = kMaxDepth;   // largest depth of the adjoint (eigenvector matrix K x K)
// per backward slot: the K x K eigenvector matrix, then the weighted divided differences
constexpr size_t kBwdSlotDoubles = 2 * (size_t)kBwdMaxDepth * kBwdMaxDepth;
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

// A wave-uniform value moved to scalar registers (arguments of a non-inlined call arrive
// in vector registers, where the fields of RevStep would stay for the whole march).
template <typename X>
__device__ __forceinline__ X to_sgpr(X v) {
  static_assert(sizeof(X) % 4 == 0, "whole dwords");
  union {
    X x;
    int i[sizeof(X) / 4];
  } u;
  u.x = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(X) / 4); ++k) u.i[k] = __builtin_amdgcn_readfirstlane(u.i[k]);
  return u.x;
}

// Projector terms of step j of the fused reverse recurrence, for
// ubar_j = ib qbar_{j+1} + bb q_{j+1} + ahat q_j.  For every node atom the sixteen box sums
// m_r(v) = phi_r . v, phi = [chi_0..3 ; d chi_l / d d_a] (the functions of the projector
// adjoints), are formed for v = qbar_{j+1} and v = q_j (accumulated in the storage
// precision); m_r(q_{j+1}) is carried in cq from the step before, and
// m_r(ubar_j) = ib m_r(qbar_{j+1}) + bb m_r(q_{j+1}) + ahat m_r(q_j).  Then
//   acoef[a][l] = E_l h^3 m_l(ubar_j)                      (weights of the scatter of H ubar_j)
//   Ebar_l += h^3 m_l(ubar_j) m_l(q_j),
//   Rbar_a -= h^3 sum_l E_l (m_{4+3l+a}(ubar_j) m_l(q_j) + m_l(ubar_j) m_{4+3l+a}(q_j)),
// the per-step terms of the projector adjoints, added into the node's partials (dEp, dRp;
// set on the last step j = K_eff - 1, which comes first), and cq takes m_r(q_j).  On the
// last step only the q_j term of ubar_j is present.
// The atoms are dealt round-robin to the waves, NA at a time.  A wave requests the box
// values of its NA atoms and their seven partials (one per lane) together, so the step
// waits on memory once per NA atoms; the totals and the step's terms pass through the
// wave's 64 doubles of wsb (LDS).
// The rows, coefficients and outputs of ubar_coefs.
template <typename T>
struct UbarArgs {
  const SGQ_G double* proj_E;
  const SGQ_G T* Q0;
  const SGQ_G T* Wc;
  double* dEp;
  double* dRp;
  double sc, ib, bb, ahat, h3;
  int wbs, B, B3, last;
};

template <typename T, int BLOCK>
__device__ __noinline__ void ubar_coefs(SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                        SGQ_L T (*cq)[16], SGQ_L double* wsb, UbarArgs<T> U) {
  // the arguments as one by-value aggregate: scalar arguments beyond the registers the
  // calling convention passes them in changed the register allocation to one that saved
  // four times as many registers through scratch on every call
  const SGQ_G double* proj_E = U.proj_E;
  const SGQ_G T* Q0 = U.Q0;
  const SGQ_G T* Wc = U.Wc;
  const int wbs = U.wbs, B = U.B, B3 = U.B3;
  const double sc = U.sc, ib = U.ib, bb = U.bb, ahat = U.ahat, h3 = U.h3;
  const bool last = U.last;
  double* dEp = U.dEp;
  double* dRp = U.dRp;
  constexpr int NW = BLOCK / kWave;
  constexpr int UNR = 6;    // 6 x 64 box points cover the 7^3 box of h = rc/3
  constexpr int NA = 3;     // atoms whose box values are requested together
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int natoms = st.natoms;
  SGQ_L double* ws = wsb + wave * 64;      // [0, 32): the totals; [32, 32 + 7 NA): terms
  auto atom_of = [&](int t) { return wave + NW * t; };
  // box value of atom a at box point b: (q_j, qbar_{j+1}), zero outside the cube
  auto load = [&](int a, int b, T& vw, T& vq) {
    const int lp = (b < B3 && a < natoms) ? box_point(st, a < natoms ? a : 0, b, B) : -1;
    const int lc = lp >= 0 ? lp : 0;
    vw = Wc[bidx(lc, wbs)] * (T)(lp >= 0);
    vq = last ? (T)0 : Q0[lc] * (T)(lp >= 0);
  };
  auto accumulate = [&](int a, int b, T vw, T vq, T (&aw)[16], T (&aq)[16]) {
    T c[4], g[12];
    chi_grad_at(pe, st.afrac[a], b % B, (b / B) % B, b / (B * B), c, g);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const T f = r < 4 ? c[r] : g[r - 4];
      aq[r] += f * vq;
      aw[r] += f * vw;
    }
  };
  // the sums of atom a (batch slot t) are complete: its weights, its step terms, the carry
  auto finish = [&](int a, int t, const T (&aw)[16], const T (&aq)[16]) {
    // the 32 wave totals by a transposed reduction: at each offset o = 32 .. 2 a lane keeps
    // half of its partial sums (the upper half when lane & o) and adds its partner's
    // partial of the same ones; a last exchange at offset 1 leaves total q in lanes 2q and
    // 2q + 1: 32 exchanges of one value, against 6 per total for a butterfly of each
    T v[32];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      v[r] = aw[r];
      v[16 + r] = aq[r];
    }
#pragma unroll
    for (int h = 16, o = 32; h >= 1; h >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const T give = up ? v[i] : v[i + h];
        const T keep = up ? v[i + h] : v[i];
        v[i] = keep + __shfl_xor(give, o, kWave);
      }
    }
    v[0] += __shfl_xor(v[0], 1, kWave);
    if ((lane & 1) == 0) ws[lane >> 1] = (double)v[0];   // ws[r]: q_j terms, ws[16 + r]: qbar
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // every lane reads the totals (one broadcast LDS read each, all in flight together)
    // and the atom's energies (one uniform address each), so that lane 0 below works from
    // registers instead of a chain of dependent reads
    const int J = to_sgpr(st.atom[a]);
    double El[4], mq[16], mu[16];
#pragma unroll
    for (int l = 0; l < 4; ++l) El[l] = proj_E[4 * J + l];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      mq[r] = sc * ws[r];                                                        // m_r(q_j)
      double m = ahat * mq[r];                                                   // m_r(ubar_j)
      if (!last) m += ib * ws[16 + r] + bb * (double)cq[a][r];
      mu[r] = m;
    }
    if (lane == 0) {
      double rb[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const double mql = mq[l], mul = mu[l];
        st.acoef[a][l] = (T)(El[l] * h3 * mul);
        ws[32 + 7 * t + l] = h3 * mul * mql;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int ra = 4 + 3 * l + ax;
          rb[ax] -= h3 * El[l] * (mu[ra] * mql + mul * mq[ra]);
        }
      }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) ws[32 + 7 * t + 4 + ax] = rb[ax];
#pragma unroll
      for (int r = 0; r < 16; ++r) cq[a][r] = (T)mq[r];
    }
    // ws[0, 32) is rewritten for the next atom only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  const int tl = lane / 7, il = lane - 7 * tl;        // the partial this lane carries
  for (int t0 = 0; atom_of(t0) < natoms; t0 += NA) {
    // partial il of the batch's atom tl (Ebar_0..3, then Rbar_x,y,z)
    const int al = atom_of(t0 + tl);
    const bool carry = lane < 7 * NA && al < natoms;
    double part = 0.0;
    if (carry && !last) part = il < 4 ? dEp[4 * al + il] : dRp[3 * al + il - 4];
    if (B3 <= UNR * kWave) {
      // one round covers the box: every box value of the batch is requested at once
      T vq[NA][UNR], vw[NA][UNR];
#pragma unroll
      for (int t = 0; t < NA; ++t)
#pragma unroll
        for (int u = 0; u < UNR; ++u) load(atom_of(t0 + t), u * kWave + lane, vw[t][u], vq[t][u]);
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        const int a = atom_of(t0 + t);
        if (a >= natoms) break;
        T aq[16], aw[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) aq[r] = aw[r] = (T)0;
#pragma unroll
        for (int u = 0; u < UNR; ++u) accumulate(a, u * kWave + lane, vw[t][u], vq[t][u], aw, aq);
        finish(a, t, aw, aq);
      }
    } else {
      // larger boxes: one atom at a time, UNR x 64 box points per round
      for (int t = 0; t < NA; ++t) {
        const int a = atom_of(t0 + t);
        if (a >= natoms) break;
        T aq[16], aw[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) aq[r] = aw[r] = (T)0;
        for (int b0 = 0; b0 < B3; b0 += UNR * kWave) {
          T vq[UNR], vw[UNR];
#pragma unroll
          for (int u = 0; u < UNR; ++u) load(a, b0 + u * kWave + lane, vw[u], vq[u]);
#pragma unroll
          for (int u = 0; u < UNR; ++u) accumulate(a, b0 + u * kWave + lane, vw[u], vq[u], aw, aq);
        }
        finish(a, t, aw, aq);
      }
    }
    if (carry) {
      const double v = part + ws[32 + 7 * tl + il];
      if (il < 4) dEp[4 * al + il] = v;
      else dRp[3 * al + il - 4] = v;
    }
    // ws is rewritten by the next batch only after every lane has read its term
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Rows and coefficients of one reversed step j for reverse_march.
template <typename T>
struct RevStep {
  const SGQ_G T* Q0;    // qbar_{j+1} (plain vector)
  const SGQ_G T* Wn;    // basis rows j+1, j, j-1, j-2 (block stride wbs)
  const SGQ_G T* Wc;
  const SGQ_G T* Wp;
  const SGQ_G T* Wpp;
  const SGQ_G T* Uj;    // u_j
  SGQ_G T* Q1;          // qbar_j so far, completed here
  SGQ_G T* Q2;          // receives qbar_{j-1} = -beta_{j-1} rbar
  SGQ_G T* Pq;          // the node dV cube
  double ib, bb, ahat, al, bprev;
  double sn, sc, sp, spp;   // scales of rows j+1, j, j-1, j-2 (zero where absent)
  int wbs;
  int last;             // j = K_eff - 1: no qbar_{j+1}, and P_q starts here
  int prev;             // j > 0: qbar_{j-1} is written
  int ldq1;             // Q1 holds a value to add to (else it starts from zero)
};

// Element i of a row addressed as a 32-bit byte offset from the row's base (indices of a
// node's rows stay far below 2^30), which lets a wave-uniform base stay in scalar registers.
template <typename T>
__device__ __forceinline__ T ld_off(const SGQ_G T* base, int i) {
  return *(const SGQ_G T*)((const SGQ_G char*)base + (unsigned)i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_off(SGQ_G T* base, int i, T v) {
  *(SGQ_G T*)((SGQ_G char*)base + (unsigned)i * (unsigned)sizeof(T)) = v;
}

// One reversed step of the recurrence as a single march through the z planes of a
// Dirichlet cube (FP32 nodes whose parallel projector group is added plane by plane; the
// other atoms, if any, were scattered into Q1 before).  When plane z+4 enters the register
// ring, each of its points gets
//   rbar = ib qbar_{j+1} + bb q_{j+1},  ubar_j = rbar + ahat q_j   (FP64, stored rounded),
// P_q += ubar_j q_j and qbar_{j-1} = -beta_{j-1} rbar are written, and
// qbar_j - alpha_j rbar + ahat u_j waits in a second register ring; when plane z is
// reached, H ubar_j (the stencil and potential on the ring of ubar_j, the group term from
// the plane correction) is added to it and qbar_j is stored.  ubar_j itself is not stored:
// the step's projector sums already hold what the adjoints need of it.  The same pass
// accumulates the FP64 products that step j-1 starts from (qbar_j . q_j, qbar_j . q_{j-1},
// qbar_j . q_{j-2}, q_j . q_{j-1}, q_j . q_{j-2}) into st.red.  Per step this reads nine rows
// and writes three, against ten reads and seven writes for separate dot, update and
// operator passes.  Plane order, ring lengths and the LDS plane as in stencil_march.
// What reverse_march needs of the caller besides the node state: the rows of the step and
// its index (the coefficients are read from the node state and the adjoint scalars in LDS).
template <typename T>
struct RevArgs {
  const SGQ_G T* Q0;
  const SGQ_G T* Wq;    // the basis (row j at Wq + 64 j, block stride wbs)
  const SGQ_G T* Uj;
  SGQ_G T* Q1;
  SGQ_G T* Q2;
  SGQ_G T* Pq;
  int j, keff, wbs;
};

template <typename T, int BLOCK, int PPT>
__device__ __noinline__ void reverse_march(int gnx, int gny, int gnz, SGQ_L NodeState<T, BLOCK>& st,
                                           const SGQ_G T* __restrict__ V, T kin, ProjEval<T> pe,
                                           int B, const SGQ_L double* sc3, RevArgs<T> A) {
  // the step's coefficients and basis rows are formed here from the step index, the node
  // state and the adjoint scalars (a by-value descriptor of all of them cost 160 bytes of
  // each lane's scratch memory per step)
  RevStep<T> S;
  const int jj = to_sgpr(A.j), ke = to_sgpr(A.keff);
  const SGQ_G T* Wb = to_sgpr(A.Wq);
  S.last = jj == ke - 1;
  S.prev = jj > 0;
  S.Q0 = to_sgpr(A.Q0);
  S.Wn = Wb + 64 * (S.last ? jj : jj + 1);     // (row j+1 does not exist on the last step)
  S.Wc = Wb + 64 * jj;
  S.Wp = Wb + 64 * (jj >= 1 ? jj - 1 : 0);
  S.Wpp = Wb + 64 * (jj >= 2 ? jj - 2 : 0);
  S.Uj = to_sgpr(A.Uj);
  S.Q1 = to_sgpr(A.Q1);
  S.Q2 = to_sgpr(A.Q2);
  S.Pq = to_sgpr(A.Pq);
  S.ib = to_sgpr(sc3[0]);
  S.bb = to_sgpr(sc3[1]);
  S.ahat = to_sgpr(sc3[2]);
  S.al = to_sgpr(st.alpha[jj]);
  S.bprev = jj > 0 ? to_sgpr(st.beta[jj - 1]) : 0.0;
  S.sn = (jj + 1 < ke) ? to_sgpr(st.scale[jj + 1]) : 0.0;
  S.sc = to_sgpr(st.scale[jj]);
  S.sp = jj >= 1 ? to_sgpr(st.scale[jj - 1]) : 0.0;
  S.spp = jj >= 2 ? to_sgpr(st.scale[jj - 2]) : 0.0;
  S.wbs = to_sgpr(A.wbs);
  S.ldq1 = !S.last || st.natoms > st.ngrp;
  constexpr int NQ = 8;    // ring of ubar planes z-3 .. z+4 (z+4 arrives after plane z)
  constexpr int LEAD = 4;  // plane z+LEAD is loaded while plane z is computed
  const int sx = st.sx, sy = st.sy, sz = st.sz, sxy = sx * sy;
  const int rx = sx + 6;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int vplane = gnx * gny;
  const T w1 = (T)kFd1, w2 = (T)kFd2, w3 = (T)kFd3;
  const bool proj = st.natoms > 0;
  for (int i = tid; i < 2 * NodeState<T, BLOCK>::kMarchPad; i += BLOCK) (&st.plane[0][0])[i] = (T)0;
  if (proj)
    for (int i = tid; i < 2 * NodeState<T, BLOCK>::kCorr; i += BLOCK) (&st.corr[0][0])[i] = (T)0;
  __syncthreads();
  if (proj) plane_group_term<T, BLOCK>(st, pe, 0, B, st.corr[0]);
  T ring[PPT][NQ];    // ubar_j
  T part[PPT][NQ];    // qbar_j - alpha_j rbar + ahat u_j
  T vcur[PPT];        // V on plane z
  int li[PPT], vrow[PPT];
  bool own[PPT];
  const int gz0 = st.oz < 0 ? st.oz + gnz : st.oz;
  auto vz = [&](int z) {   // global z of local plane z (clamped into the cube)
    int gz = gz0 + (z < sz ? z : sz - 1);
    return gz >= gnz ? gz - gnz : gz;
  };
  // Raw values of plane zf of point column k.  fill_load issues the loads at the top of
  // an iteration and fill_apply uses them after the plane's output, so they are in flight
  // while the plane is computed.  fill_apply gives the ring values and, for a plane inside
  // the cube, makes the point updates (planes outside are read clamped and only feed
  // masked neighbours).
  struct Raw {
    T wc, q0, wn, uj, q1, pq;
  };
  auto point_of = [&](int k, int zf) {
    const int zc = zf < 0 ? 0 : (zf < sz ? zf : sz - 1);
    return (own[k] ? tid + k * BLOCK : 0) + zc * sxy;
  };
  auto fill_load = [&](int k, int zf, Raw& w) {
    // every row is read (the absent ones point at rows that exist) and the values not
    // wanted are replaced by zero, so the loads of an iteration form one branch-free run
    const int p = point_of(k, zf);
    const int pb = bidx(p, S.wbs);
    w.wc = ld_off(S.Wc, pb);
    w.uj = ld_off(S.Uj, p);
    const T q0 = ld_off(S.Q0, p), wn = ld_off(S.Wn, pb), pq = ld_off(S.Pq, p);
    const T q1 = ld_off(S.Q1, p);
    w.q0 = S.last ? (T)0 : q0;
    w.wn = S.last ? (T)0 : wn;
    w.pq = S.last ? (T)0 : pq;
    w.q1 = S.ldq1 ? q1 : (T)0;
  };
  auto fill_apply = [&](int k, int zf, const Raw& w, T& u, T& pt) {
    const double qc = S.sc * (double)w.wc;
    // ib = bb = 0 on the last step, where the raw q0 and wn are zero
    const double rb = (double)w.q0 * S.ib + S.bb * S.sn * (double)w.wn;
    const double ub = rb + S.ahat * qc;
    u = (T)ub;
    pt = (T)((double)w.q1 - S.al * rb + S.ahat * (double)w.uj);
    if (own[k] && zf >= 0 && zf < sz) {
      const int p = point_of(k, zf);
      st_off(S.Pq, p, (T)((double)w.pq + ub * qc));
      if (S.prev) st_off(S.Q2, p, (T)(-S.bprev * rb));
    }
  };
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int p2 = tid + k * BLOCK;
    own[k] = p2 < sxy;
    const int pc = own[k] ? p2 : 0;
    const int y = pc / sx, x = pc - y * sx;
    li[k] = (y + 3) * rx + (x + 3);
    int gx = st.ox + x, gy = st.oy + y;
    gx = gx < 0 ? gx + gnx : (gx >= gnx ? gx - gnx : gx);
    gy = gy < 0 ? gy + gny : (gy >= gny ? gy - gny : gy);
    vrow[k] = gx + gnx * gy;
    // slot d holds plane d (d < LEAD) or plane d - NQ (below the cube); the planes below
    // are filled after plane 0, whose u_j they would read already replaced, and feed only
    // masked neighbours
#pragma unroll
    for (int d = 0; d < NQ; ++d) {
      const int zf = d < LEAD ? d : d - NQ;
      Raw w;
      fill_load(k, zf, w);
      fill_apply(k, zf, w, ring[k][d], part[k][d]);
    }
    vcur[k] = ld_off(V, vrow[k] + vplane * vz(0));
  }
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0, d4 = 0.0;
  for (int z0 = 0; z0 < sz; z0 += NQ) {
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int z = z0 + r;
      if (z < sz) {
        // loads first: plane z+LEAD for the ring, plane z of the basis rows for the
        // products, the potential of plane z+1
        const int zf = z + LEAD;
        Raw raw[PPT];
        T dwc[PPT], dwp[PPT], dwpp[PPT], vnext[PPT];
        const int gzn = vz(z + 1);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          fill_load(k, zf, raw[k]);
          vnext[k] = ld_off(V, vrow[k] + vplane * gzn);
          // (on step 0 the products are formed and not used)
          const int pb = bidx(point_of(k, z), S.wbs);
          dwc[k] = ld_off(S.Wc, pb);
          dwp[k] = ld_off(S.Wp, pb);
          dwpp[k] = ld_off(S.Wpp, pb);
        }
        SGQ_L T* plane = st.plane[z & 1];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
          if (own[k]) plane[li[k]] = ring[k][r];
        __syncthreads();
        const T mz1 = (T)(z >= 1), pz1 = (T)(z + 1 < sz);
        const T mz2 = (T)(z >= 2), pz2 = (T)(z + 2 < sz);
        const T mz3 = (T)(z >= 3), pz3 = (T)(z + 3 < sz);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const SGQ_L T* c0 = plane + li[k];
          const T c = ring[k][r];
          const T l1 = ((mz1 * ring[k][(r + NQ - 1) % NQ] - c) + (pz1 * ring[k][(r + 1) % NQ] - c)) +
                       ((c0[-1] - c) + (c0[1] - c)) + ((c0[-rx] - c) + (c0[rx] - c));
          const T l2 = ((mz2 * ring[k][(r + NQ - 2) % NQ] - c) + (pz2 * ring[k][(r + 2) % NQ] - c)) +
                       ((c0[-2] - c) + (c0[2] - c)) + ((c0[-2 * rx] - c) + (c0[2 * rx] - c));
          const T l3 = ((mz3 * ring[k][(r + NQ - 3) % NQ] - c) + (pz3 * ring[k][(r + 3) % NQ] - c)) +
                       ((c0[-3] - c) + (c0[3] - c)) + ((c0[-3 * rx] - c) + (c0[3 * rx] - c));
          const T lap = w1 * l1 + w2 * l2 + w3 * l3;
          T add = kin * lap + vcur[k] * c;
          if (own[k]) {
            const int p2 = tid + k * BLOCK;
            if (proj) {
              SGQ_L T* cz = st.corr[z & 1];
              add += cz[p2];
              cz[p2] = (T)0;
            }
            const T out = part[k][r] + add;
            st_off(S.Q1, p2 + z * sxy, out);
            const double qn = S.sc * (double)dwc[k];
            const double qc = S.sp * (double)dwp[k];
            const double qp = S.spp * (double)dwpp[k];
            const double qb = (double)out;
            d0 += qb * qn;
            d1 += qb * qc;
            d2 += qb * qp;
            d3 += qn * qc;
            d4 += qn * qp;
          }
        }
        if (proj && z + 1 < sz) plane_group_term<T, BLOCK>(st, pe, z + 1, B, st.corr[(z + 1) & 1]);
        // plane z+LEAD takes the slot of plane z+LEAD-NQ, which no later plane reads
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          fill_apply(k, zf, raw[k], ring[k][(r + LEAD) % NQ], part[k][(r + LEAD) % NQ]);
          vcur[k] = vnext[k];
        }
      }
    }
  }
  d0 = wave_sum(d0);
  d1 = wave_sum(d1);
  d2 = wave_sum(d2);
  d3 = wave_sum(d3);
  d4 = wave_sum(d4);
  if (lane == 0) {
    st.red[wave][0] = d0;
    st.red[wave][1] = d1;
    st.red[wave][2] = d2;
    st.red[wave][3] = d3;
    st.red[wave][4] = d4;
  }
}

// A node's K x K eigenvector matrix by columns, Z(i, k) = component i of eigenvector k at
// p[k K + i]: the lanes of a wave, one component each, read and write one contiguous run
// per column.  (By rows, each access of a wave touched 64 cache lines, and the pre-pass
// took twice as long; holding the matrix in LDS allowed a quarter as many nodes in flight
// and lost to this form at every depth.)
template <typename Ptr>
struct ZCols {
  Ptr p;
  int K;
  __device__ decltype(auto) operator()(int i, int k) const { return p[(size_t)k * K + i]; }
};

// Implicit-shift QR of the tridiagonal (a, b) accumulating all eigenvectors in Z.
// Run by one whole wave.  Each sweep first forms its chain of Givens rotations: every lane
// computes the same rotations from the LDS copies of a and b, carrying the entries the
// previous rotation changed in registers (a rotation reads only entries no earlier one of
// the sweep has written), and lane 0 writes the results back and the (c, s) pairs to rot.
// The rotations of up to four consecutive sweeps are then applied to Z in one pass over
// the columns: rotation k of a sweep needs only rotations k and k+1 of the sweep before it
// done, so at column position p sweep s of the batch applies its rotation p - s.  Each
// entry of Z gets the same operations in the same order as with one pass per sweep, with
// a batch's worth fewer reads and writes of Z.
// Z (ZCols): Z(i, k) is component i of eigenvector k; each lane owns the components
// i = lane (mod 64).  rot: 4 kBwdMaxDepth doubles of LDS, the (c, s) pairs of the batch.
template <typename ZA>
__device__ bool tridiag_eig_wave(SGQ_L double* a, SGQ_L double* b, ZA Z, int K,
                                 SGQ_L double* rot) {
  constexpr int kBatch = 4;   // most sweeps per pass over Z
  const int lane = threadIdx.x & (kWave - 1);
  for (int i = lane; i < K; i += kWave)
    for (int k = 0; k < K; ++k) Z(i, k) = (i == k) ? 1.0 : 0.0;
  // sweeps per pass: as many chains of 2 (K - 1) values as rot holds
  const int rs = 2 * (K > 1 ? K - 1 : 1);
  const int S = min(kBatch, (4 * kBwdMaxDepth) / rs);
  int ns = 0;                          // sweeps formed and not yet applied
  int wl[kBatch], wm[kBatch];          // their rotation windows [l, m)
#pragma unroll
  for (int t = 0; t < kBatch; ++t) wl[t] = wm[t] = 0;
  // applies the ns formed sweeps: column positions p = L .. M + 3, where sweep t applies
  // its rotation p - t to columns (p - t, p - t + 1); v[j] holds column p - 3 + j
  auto apply = [&]() {
    int L = wl[0], M = wm[0];
#pragma unroll
    for (int t = 1; t < kBatch; ++t)
      if (t < ns) {
        L = min(L, wl[t]);
        M = max(M, wm[t]);
      }
    for (int i = lane; i < K; i += kWave) {
      double v[kBatch + 1];
#pragma unroll
      for (int j = 0; j < kBatch + 1; ++j) v[j] = 0.0;
      v[kBatch - 1] = Z(i, L);
      for (int p0 = L; p0 <= M + kBatch - 1; p0 += 8) {
        // the new columns of eight positions are loaded together
        double u[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) u[t] = p0 + t + 1 <= M ? Z(i, p0 + t + 1) : 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int p = p0 + t;
          if (p <= M + kBatch - 1) {
            v[kBatch] = u[t];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
              const int k = p - q;
              if (q < ns && k >= wl[q] && k < wm[q]) {
                const SGQ_L double* rq = rot + q * rs + 2 * (k - wl[q]);
                const double c = rq[0], s = rq[1];
                const double u0 = v[kBatch - 1 - q], u1 = v[kBatch - q];
                v[kBatch - 1 - q] = c * u0 - s * u1;
                v[kBatch - q] = s * u0 + c * u1;
              }
            }
            const int done = p - (kBatch - 1);
            if (done >= L && done <= M) Z(i, done) = v[0];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) v[j] = v[j + 1];
          }
        }
      }
    }
    // rot is rewritten by the next batch only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    ns = 0;
  };
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
    // l: the start of the unreduced block ending at m, one split test per lane (index
    // i = w + 64 c tests b[i-1]); the largest split index below m wins
    int l = 0;
    for (int c0 = 0; c0 < m; c0 += kWave) {
      const int i = c0 + lane;
      const bool split = i >= 1 && i < m && fabs(b[i - 1]) <= eps * (fabs(a[i - 1]) + fabs(a[i]));
      const unsigned long long mask = __ballot(split);
      if (mask) l = c0 + 63 - __clzll(mask);
    }
    if (l > 0 && lane == 0) b[l - 1] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (++sweeps > 40 * K) return false;
    const double d = 0.5 * (a[m - 1] - a[m]);
    const double bm = b[m - 1];
    const double den = d + copysign(hypot(d, bm), d == 0.0 ? 1.0 : d);
    const double shift = a[m] - bm * bm / den;
    // the chain: (ak, bk) are a[k], b[k] as the previous rotation left them
    double x = a[l] - shift;
    double y = b[l];
    double ak = a[l], bk = b[l];
    // (a[k+1], b[k+1]) of the next rotation are read one rotation ahead; the entries of T
    // stay far inside the double range, so x^2 + y^2 needs no scaling.  One reciprocal
    // square root gives c, s and r: the chain's latency is the solve's time, and a square
    // root followed by a division is about four times as long a dependent sequence
    double ak1 = a[l + 1];
    double bk1 = l + 1 < m ? b[l + 1] : 0.0;
    SGQ_L double* rw = rot + ns * rs;
    for (int k = l; k < m; ++k) {
      const double ak1n = k + 2 <= m ? a[k + 2] : 0.0;
      const double bk1n = k + 2 < m ? b[k + 2] : 0.0;
      const double r2 = x * x + y * y;
      double c = 1.0, s = 0.0, r = 0.0;
      if (r2 != 0.0) {
        const double ir = rsqrt(r2);
        r = r2 * ir;
        c = x * ir;
        s = -y * ir;
      }
      const double nak = c * c * ak - 2.0 * c * s * bk + s * s * ak1;
      const double nak1 = s * s * ak + 2.0 * c * s * bk + c * c * ak1;
      const double nbk = c * s * (ak - ak1) + (c * c - s * s) * bk;
      if (lane == 0) {
        if (k > l) b[k - 1] = r;
        a[k] = nak;
        b[k] = nbk;
        rw[2 * (k - l)] = c;
        rw[2 * (k - l) + 1] = s;
      }
      x = nbk;
      y = -s * bk1;      // the bulge
      ak = nak1;
      bk = c * bk1;
      ak1 = ak1n;
      bk1 = bk1n;
    }
    if (lane == 0) a[m] = ak;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < kBatch; ++t)
      if (t == ns) {
        wl[t] = l;
        wm[t] = m;
      }
    if (++ns == S) apply();
  }
  if (ns > 0) apply();
  return true;
}

// alphabar_j = Tbar_jj and betabar_j = 2 Tbar_j,j+1 of one node, Tbar = cscale S (D o s1 s1^T) S^T
// (Daleckii-Krein), from the eigenvalues ta and eigenvectors S of T (Z[i*K + k]: component i
// of eigenvector k).  G_kl = s1_k D_kl s1_l (s1 the first row of S, D the divided
// differences of F, F' on the diagonal and for nearly equal eigenvalues) goes to G (K^2
// doubles, global); thread (j, c) then forms y_jl = sum_k S_jk G_lk (G is symmetric) for the
// columns l = c (mod nch) and its parts of alphabar_j and betabar_j, which are added in a
// fixed order.  Run by the NT threads of a workgroup; Fv, Fd: K values, part: 4 kBwdMaxDepth.
template <int NT, typename ZA>
__device__ void daleckii_krein(const LaunchParams& P, SGQ_L const double* ta, SGQ_L double* Fv,
                               SGQ_L double* Fd, SGQ_L double* part, ZA Z,
                               SGQ_G double* __restrict__ G, int keff, double cscale,
                               SGQ_L double* abar, SGQ_L double* bbar) {
  const int tid = threadIdx.x;
  for (int k = tid; k < keff; k += NT) {
    Fv[k] = integrand_value(ta[k], P.mu, P.kT, P.integrand);
    Fd[k] = integrand_deriv(ta[k], P.mu, P.kT, P.integrand);
  }
  __syncthreads();
  for (int t = tid; t < keff * keff; t += NT) {
    const int k = t / keff, l = t - k * keff;
    const double tk = ta[k], tl = ta[l];
    const double diff = tk - tl;
    double D;
    if (l == k) {
      D = Fd[k];
    } else if (fabs(diff) <= 1e-6 * fmax(P.kT, fmax(fabs(tk), fabs(tl)))) {
      D = integrand_deriv(0.5 * (tk + tl), P.mu, P.kT, P.integrand);
    } else {
      D = (Fv[k] - Fv[l]) / diff;
    }
    G[t] = Z(0, k) * D * Z(0, l);
  }
  __syncthreads();
  const int nch = keff * 8 <= 2 * kBwdMaxDepth ? 8 : (2 * kBwdMaxDepth) / keff;
  for (int t = tid; t < keff * nch; t += NT) {
    const int j = t / nch, c = t - j * nch;
    const int j1 = j + 1 < keff ? j + 1 : j;
    double pa = 0.0, pb = 0.0;
    for (int l = c; l < keff; l += nch) {
      const SGQ_G double* gl = G + (size_t)l * keff;
      double y = 0.0;
      for (int k = 0; k < keff; ++k) y += Z(j, k) * gl[k];
      pa += y * Z(j, l);
      pb += y * Z(j1, l);
    }
    part[2 * t] = pa;
    part[2 * t + 1] = pb;
  }
  __syncthreads();
  for (int j = tid; j < keff; j += NT) {
    double sa = 0.0, sb = 0.0;
    for (int c = 0; c < nch; ++c) {
      sa += part[2 * (j * nch + c)];
      sb += part[2 * (j * nch + c) + 1];
    }
    abar[j] = cscale * sa;
    if (j + 1 < keff) bbar[j] = 2.0 * cscale * sb;
  }
  __syncthreads();
}

// The eigensolve and Daleckii-Krein step of every node as a pass of its own, before the
// backward kernel: one wave per workgroup, many per CU, so the serial rotation chains of
// the QR sweeps of different nodes overlap.  Each node's tridiagonal is the one the forward
// call stored (alpha, beta, K_eff); it serves only when the forward saw these inputs
// (hash[0] == hash[1]), and the backward kernel takes a node's result only when its own
// K_eff agrees (tbar_k).  zscratch: 2 K_max^2 doubles per workgroup, the eigenvectors by
// columns and then G.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void tbar_kernel(LaunchParams P, double* zscratch,
                                                      size_t zstride, double* tbar,
                                                      int32_t* tbar_k) {
  __shared__ double ta_s[kBwdMaxDepth], tb_s[kBwdMaxDepth], Fv_s[kBwdMaxDepth], Fd_s[kBwdMaxDepth];
  __shared__ double part_s[4 * kBwdMaxDepth];
  __shared__ double abar_s[kBwdMaxDepth], bbar_s[kBwdMaxDepth];
  __shared__ int node;
  SGQ_L double* ta = (SGQ_L double*)ta_s;
  SGQ_L double* tb = (SGQ_L double*)tb_s;
  SGQ_L double* Fv = (SGQ_L double*)Fv_s;
  SGQ_L double* Fd = (SGQ_L double*)Fd_s;
  SGQ_L double* part = (SGQ_L double*)part_s;
  SGQ_L double* abar = (SGQ_L double*)abar_s;
  SGQ_L double* bbar = (SGQ_L double*)bbar_s;
  const int tid = threadIdx.x;
  const int kmax = P.kmax_out;
  SGQ_G double* Z = (SGQ_G double*)zscratch + (size_t)blockIdx.x * zstride;
  const bool same = P.hash[0] == P.hash[1];
  const double gomega = *P.grad_omega;
  for (;;) {
    if (tid == 0) node = atomicAdd(P.queue + 1, 1);
    __syncthreads();
    const int qi = node;
    if (qi >= P.n_nodes) break;
    const int q = P.order[qi];
    const int keff = same ? P.tri_k[q] : -1;
    if (keff < 1 || keff > kmax) {
      if (tid == 0) tbar_k[q] = -1;
      __syncthreads();
      continue;
    }
    const double* tri = P.tri + (size_t)q * 2 * kmax;
    for (int k = tid; k < keff; k += kWave) {
      ta[k] = tri[k];
      tb[k] = k + 1 < keff ? tri[kmax + k] : 0.0;
    }
    __syncthreads();
    const ZCols<SGQ_G double*> Zg{Z, keff};
    const bool ok = tridiag_eig_wave(ta, tb, Zg, keff, part);
    __syncthreads();
    if (ok) {
      daleckii_krein<kWave>(P, ta, Fv, Fd, part, Zg, Z + (size_t)keff * keff, keff,
                            2.0 * P.node_weight[q] * gomega, abar, bbar);
      double* out = tbar + (size_t)q * 2 * kmax;
      for (int k = tid; k < keff; k += kWave) {
        out[k] = abar[k];
        if (k + 1 < keff) out[kmax + k] = bbar[k];
      }
    }
    // (a node whose sweeps did not converge is left to the backward kernel, which reports it)
    if (tid == 0) tbar_k[q] = ok ? keff : -1;
    __syncthreads();
  }
}

template <typename T, int BLOCK, int KG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void lanczos_backward_kernel(LaunchParams P) {
  constexpr int NW = BLOCK / kWave;
  __shared__ NodeState<T, BLOCK> st_shared;
  __shared__ BwdState bs_shared;
  // the projector box sums of q_{j+1} of every node atom, carried between the fused
  // reverse steps
  __shared__ T cq_shared[NodeState<T, BLOCK>::kFuse ? kMaxNodeAtoms : 1][16];
  SGQ_L T(*cq)[16] = (SGQ_L T(*)[16])(&cq_shared[0][0]);
  SGQ_L NodeState<T, BLOCK>& st = *(SGQ_L NodeState<T, BLOCK>*)(&st_shared);
  SGQ_L BwdState& bs = *(SGQ_L BwdState*)(&bs_shared);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  // (the kernel-wide values in scalar registers, where the step calls do not make the
  // kernel save them through scratch)
  const size_t npad = to_sgpr(P.npad);
  const int kmax = to_sgpr(P.kmax_out);
  const int wbs = to_sgpr(P.wbs);
  SGQ_G T* __restrict__ W = to_sgpr((SGQ_G T*)P.W + (size_t)blockIdx.x * P.slot_stride);
  SGQ_G T* __restrict__ Ubase = to_sgpr(W + (size_t)kmax * npad);
  SGQ_G double* __restrict__ Z =
      to_sgpr((SGQ_G double*)P.zbuf + (size_t)blockIdx.x * kBwdSlotDoubles);
  // the three qbar rows follow the kmax u_j rows of the slot: row r at
  // Ubase + (kmax + r) npad
  const SGQ_G T* __restrict__ V = to_sgpr((const SGQ_G T*)P.v);
  const ProjEval<T> pe = to_sgpr(proj_eval<T>(P));
  const SGQ_G double* proj_E = to_sgpr((const SGQ_G double*)P.proj_E);
  const double h = to_sgpr(P.h), h3 = h * h * h;
  const T kin = (T)(-0.5 / (h * h));
  const int B = to_sgpr(2 * P.box_m + 1), B3 = B * B * B;
  const double gomega = to_sgpr(*P.grad_omega);
  constexpr int VW = 16 / (int)sizeof(T);                    // points per 16-byte access
  typedef T VT __attribute__((ext_vector_type(VW)));
  if (tid == 0) st.orth_tol = sizeof(T) == 4 ? 3.4526698300124393e-4 : 1.4901161193847656e-8;

  for (;;) {
    if (tid == 0) st.node = atomicAdd(P.queue, 1);
    __syncthreads();
    // node-level values are wave-uniform: in scalar registers they cost no vector registers
    // to keep across the step calls (where vector registers are saved through scratch)
    const int qi = to_sgpr(st.node);
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
    const int n = to_sgpr(st.n), natoms = to_sgpr(st.natoms);
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
      keff = to_sgpr(run_lanczos<T, BLOCK, KG>(P, st, W, Ubase, npad, P.depth[q]));
    }
    // ---- eigenvectors of T and the Daleckii-Krein adjoint: from the pre-pass when it
    // solved this node's tridiagonal (the forward's, for these inputs and this K_eff), else
    // here
    if (P.tbar_k && P.tbar_k[q] == keff) {
      const double* tq = P.tbar + (size_t)q * 2 * kmax;
      for (int k = tid; k < keff; k += BLOCK) {
        bs.abar[k] = tq[k];
        if (k + 1 < keff) bs.bbar[k] = tq[kmax + k];
      }
      __syncthreads();
    } else {
      for (int k = tid; k < keff; k += BLOCK) {
        st.ta[k] = st.alpha[k];
        st.tb[k] = k + 1 < keff ? st.beta[k] : 0.0;
      }
      __syncthreads();
      if (wave == 0) {
        bool ok = tridiag_eig_wave(st.ta, st.tb, ZCols<SGQ_G double*>{Z, keff}, keff, bs.part);
        if (!ok && lane == 0) atomicOr(P.status, kStatusNonFinite);
      }
      __syncthreads();
      daleckii_krein<BLOCK>(P, st.ta, bs.Fv, bs.Fd, bs.part, ZCols<SGQ_G double*>{Z, keff},
                            Z + (size_t)keff * keff, keff, 2.0 * P.node_weight[q] * gomega,
                            bs.abar, bs.bbar);
    }
    double* dEp = to_sgpr(P.dE_part + (size_t)q * kMaxNodeAtoms * 4);
    double* dRp = to_sgpr(P.dR_part + (size_t)q * kMaxNodeAtoms * 3);
    Wq = to_sgpr(Wq);
    Uq = to_sgpr(Uq);
    // ---- reverse recurrence: one fused march per step where the node's stencil is the
    // FP32 plane march and its projector group is added inside it; otherwise separate
    // dot, update and operator passes
    bool rev_fused = false;
    if constexpr (NodeState<T, BLOCK>::kFuse)
      rev_fused = !st.periodic && uses_march(st, BLOCK) && (natoms == 0 || st.fuse);
    if constexpr (NodeState<T, BLOCK>::kFuse) {
      if (rev_fused) {
        int r0 = 0, r1 = 1, r2 = 2;
        for (int j = keff - 1; j >= 0; --j) {
          const bool last = (j == keff - 1);
          if (tid == 0) {
            if (!last) {
              // the products step j+1's march left in st.red
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
            } else {
              bs.sc[0] = 0.0;
              bs.sc[1] = 0.0;
              bs.sc[2] = bs.abar[j];
            }
          }
          __syncthreads();
          RevStep<T> S;
          // (the qbar rows by their index: R[r] with r varying would be a select the
          // compiler keeps in vector registers)
          S.Q0 = to_sgpr(Ubase + (size_t)(kmax + r0) * npad);
          S.Wn = Wq + 64 * (last ? j : j + 1);     // (row j+1 does not exist on the last step)
          S.Wc = Wq + 64 * j;
          S.Wp = Wq + 64 * (j >= 1 ? j - 1 : 0);
          S.Wpp = Wq + 64 * (j >= 2 ? j - 2 : 0);
          S.Uj = Uq + (size_t)j * npad;
          S.Q1 = to_sgpr(Ubase + (size_t)(kmax + r1) * npad);
          S.Q2 = to_sgpr(Ubase + (size_t)(kmax + r2) * npad);
          S.Pq = to_sgpr(Pq);
          S.ib = bs.sc[0];
          S.bb = bs.sc[1];
          S.ahat = bs.sc[2];
          S.al = st.alpha[j];
          S.bprev = j > 0 ? st.beta[j - 1] : 0.0;
          S.sn = (j + 1 < keff) ? st.scale[j + 1] : 0.0;
          S.sc = st.scale[j];
          S.sp = j >= 1 ? st.scale[j - 1] : 0.0;
          S.spp = j >= 2 ? st.scale[j - 2] : 0.0;
          S.wbs = wbs;
          S.last = last;
          S.prev = j > 0;
          S.ldq1 = !last || natoms > st.ngrp;
          if (natoms > 0) {
            ubar_coefs<T, BLOCK>(st, pe, cq, bs.part,
                                 UbarArgs<T>{proj_E, S.Q0, S.Wc, dEp, dRp, S.sc, S.ib, S.bb,
                                             S.ahat, h3, wbs, B, B3, (int)last});
            __syncthreads();
            if (natoms > st.ngrp) {
              // the atoms outside the group are added to qbar_j before the march
              if (last) {
                for (int p = tid; p < n; p += BLOCK) S.Q1[p] = (T)0;
                __syncthreads();
              }
              apply_scatter<T, BLOCK>(P, st, pe, S.Q1, B, B3, false);
            }
          }
          reverse_march<T, BLOCK, 5>(P.nx, P.ny, P.nz, st, V, kin, pe, B, bs.sc,
                                     RevArgs<T>{S.Q0, Wq, S.Uj, S.Q1, S.Q2, S.Pq, j, keff, wbs});
          __syncthreads();
          const int t0 = r0;
          r0 = r1;
          r1 = r2;
          r2 = t0;
        }
      }
    }
    int r0 = 0, r1 = 1, r2 = 2;
    for (int j = rev_fused ? -1 : keff - 1; j >= 0; --j) {
      // rows of the point-blocked basis (block stride wbs)
      const SGQ_G T* Wc = Wq + 64 * j;
      const SGQ_G T* Wn = Wq + 64 * (j + 1);
      const SGQ_G T* Wp = Wq + 64 * (j > 0 ? j - 1 : 0);
      SGQ_G T* Uj = Uq + (size_t)j * npad;      // u_j, replaced by ubar_j in pass B
      SGQ_G T* Q0 = to_sgpr(Ubase + (size_t)(kmax + r0) * npad);
      SGQ_G T* Q1 = to_sgpr(Ubase + (size_t)(kmax + r1) * npad);
      SGQ_G T* Q2 = to_sgpr(Ubase + (size_t)(kmax + r2) * npad);
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
    // buffers, which are idle after the reverse recurrence (the fused steps added them
    // step by step)
    if (natoms > 0 && !rev_fused) {
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

// dV(x) = sum over the nodes whose cube contains x of P_q(x).  One workgroup per 8^3 cell
// of the grid; cell_nodes lists the nodes meeting each cell in ascending order.  Wave w of
// the eight takes the nodes w, w + 8, ... of the cell's list, in that order, and each lane
// adds the eight points of one column of the cell (x = lane % 8, y = lane / 8, every z)
// per node, four nodes' loads at a time: where one lane per point and the whole workgroup
// on each node made the loop one chain of dependent loads per node.  The eight partial
// sums are added in wave order, so dV is reproducible bit for bit.
template <typename T>
__global__ __launch_bounds__(512) void gather_dv_kernel(LaunchParams P, const int32_t* cell_start,
                                                      const int32_t* cell_nodes, double* dV) {
  constexpr int C = kGatherCell;
  constexpr int NW = 512 / kWave;
  static_assert(C * C == kWave && C == NW, "a lane per column of the cell, a wave per eighth");
  __shared__ double part_s[NW][C * C * C];
  const int ncx = (P.nx + C - 1) / C, ncy = (P.ny + C - 1) / C;
  const int cell = blockIdx.x;
  const int cx = cell % ncx, cy = (cell / ncx) % ncy, cz = cell / (ncx * ncy);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int x = cx * C + lane % C, y = cy * C + lane / C, z0 = cz * C;
  const bool col = x < P.nx && y < P.ny;
  const SGQ_G T* Pc = (const SGQ_G T*)P.P_cube;
  double acc[C];
#pragma unroll
  for (int k = 0; k < C; ++k) acc[k] = 0.0;
  // the loads of U nodes are issued together and their values added in list order
  constexpr int U = 4;
  const int e0 = cell_start[cell], e1 = cell_start[cell + 1];
  for (int e = e0 + wave; e < e1; e += U * NW) {
    T v[U][C];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int eu = e + u * NW;
      const int q = cell_nodes[eu < e1 ? eu : e];
      const int R = P.half_width[q];
      const SGQ_G T* Pq = Pc + P.cube_offset[q];
      const int c = P.center[q];
      const int s = 2 * R + 1;
      const int lx = wrap_index(x - (c % P.nx - R), P.nx);
      const int ly = wrap_index(y - ((c / P.nx) % P.ny - R), P.ny);
      const int lz0 = wrap_index(z0 - (c / (P.nx * P.ny) - R), P.nz);   // cube plane of z0
      const bool live = eu < e1 && col;
      const bool in = live && lx < s && ly < s;
      const SGQ_G T* rq = Pq + lx + s * ly;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const int z = z0 + k;
        if (R < 0) {   // the whole periodic grid
          v[u][k] = live && z < P.nz ? Pq[x + P.nx * (y + P.ny * z)] : (T)0;
        } else {
          const int lz = lz0 + k < P.nz ? lz0 + k : lz0 + k - P.nz;
          v[u][k] = in && z < P.nz && lz < s ? rq[(size_t)s * s * lz] : (T)0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < C; ++k) acc[k] += (double)v[u][k];
  }
  SGQ_L double(*part)[C * C * C] = (SGQ_L double(*)[C * C * C])part_s;
#pragma unroll
  for (int k = 0; k < C; ++k) part[wave][lane + kWave * k] = acc[k];
  __syncthreads();
  const int t = threadIdx.x;
  const int px = cx * C + t % C, py = cy * C + (t / C) % C, pz = z0 + t / (C * C);
  if (px < P.nx && py < P.ny && pz < P.nz) {
    double sum = 0.0;
    for (int w = 0; w < NW; ++w) sum += part[w][t];
    dV[px + P.nx * (py + P.ny * pz)] = sum;
  }
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
template <typename T, int BLOCK>
static hipError_t launch_backward_t(const LaunchParams& P, int grid, int kg, hipStream_t s) {
  switch (kg) {
    case 8:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, BLOCK, 8>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
    case 16:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, BLOCK, 16>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
    default:
      hipLaunchKernelGGL((lanczos_backward_kernel<T, BLOCK, 32>), dim3(grid), dim3(BLOCK), 0, s, P);
      break;
  }
  return hipGetLastError();
}

// FP32 Dirichlet nodes whose planes only the 512-lane march takes: wider than the 256-lane
// march allows (35 points), at most 49 (the same test as uses_march on the device).  The
// backward reverses them in a 512-lane launch and every other node in a 256-lane one.
bool backward_wide_node(int half_width) {
  if (half_width < 0) return false;
  const int side = 2 * half_width + 1;
  auto fits = [side](int block, int pad) {
    return side * side <= 5 * block && (side + 6) * (side + 6) <= pad;
  };
  return !fits(256, NodeState<float, 256>::kMarchPad) && fits(512, NodeState<float, 512>::kMarchPad);
}

__global__ void queue_reset_kernel(int* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

hipError_t launch_queue_reset(int* queue, hipStream_t s) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, s, queue);
  return hipGetLastError();
}

// 256 lanes per node (two workgroups per CU) or, in FP32, 512 (one per CU: the wide-plane
// march of cubes up to 49 points across); FP64 nodes take 256.
hipError_t launch_backward(const LaunchParams& P, bool fp64, int grid, int block, int kg,
                           hipStream_t s) {
  if (fp64) return launch_backward_t<double, 256>(P, grid, kg, s);
  if (block == 512) return launch_backward_t<float, 512>(P, grid, kg, s);
  return launch_backward_t<float, 256>(P, grid, kg, s);
}

hipError_t launch_tbar(const LaunchParams& P, int grid, double* zscratch, size_t zstride,
                       double* tbar, int32_t* tbar_k, hipStream_t s) {
  hipLaunchKernelGGL(tbar_kernel, dim3(grid), dim3(kWave), 0, s, P, zscratch, zstride, tbar,
                     tbar_k);
  return hipGetLastError();
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
size_t backward_slot_doubles() { return kBwdSlotDoubles; }
int gather_cell() { return kGatherCell; }

}  // namespace sgq
