// Device building blocks of the Lanczos-Gauss kernels (forward and adjoint): the node
// state in LDS, node geometry and projector atom lists, the fused reorthogonalisation
// sweep, the stencil passes and the projector passes, and one full Lanczos run.
#pragma once

#include "sgq_common.h"
#include "tridiag.h"

namespace sgq {


constexpr int kFnzBlocks = 2048;   // 64-point blocks tracked per node (cubes up to 131072 points)
constexpr int kNoRow = 255;        // no nonzero row in the block yet

template <typename T, int BLOCK>
struct NodeState {
  static constexpr int NW = BLOCK / kWave;
  // FP32 nodes add the parallel projector group inside the stencil march (per-plane atom
  // lists and a double-buffered plane correction); FP64 keeps the separate scatter so that
  // two FP64 workgroups still fit a CU's LDS
  static constexpr bool kFuse = sizeof(T) == 4;
  // widest plane of the march: 49 points for the FP32 512-lane state (one workgroup per
  // CU: five points per lane cover 49^2), 35 otherwise (two workgroups per CU must fit)
  static constexpr int kMarchEdge = kFuse && BLOCK >= 512 ? 49 : 35;
  static constexpr int kMarchPad = (kMarchEdge + 6) * (kMarchEdge + 6);   // zero halo of 3
  static constexpr int kPlanes = kFuse ? kMarchEdge : 1;   // cube edges of the plane march
  static constexpr int kPlaneAtoms = 32;                   // group atoms crossing one plane
  static constexpr int kCorr = kFuse ? kMarchEdge * kMarchEdge : 1;
  int node;
  int sx, sy, sz, ox, oy, oz, periodic, n, start, natoms, abort;
  int atom[kMaxNodeAtoms];
  int abox[kMaxNodeAtoms][3];       // local coordinates of the projector box corner
  int aphase[kMaxNodeAtoms];        // scatter layer (0: the parallel group)
  int grp[kMaxNodeAtoms];           // the atoms by layer, in atom order within a layer
  unsigned short lstart[kMaxNodeAtoms + 1];   // layer L is grp[lstart[L], lstart[L + 1])
  int nlayer;                       // layers, the group included
  int lchange;                      // a layer changed in the last relaxation round
  int ngrp;                         // atoms of the group (layer 0)
  int wcount[NW];
  T afrac[kMaxNodeAtoms][4];        // g0 h - R of each node atom (x, y, z): box offsets
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
  int wflag[NW];
  T plane[2][kMarchPad];            // z planes of the cube (zero halo of 3) for the march
  int fuse;                         // the group scatter runs inside the march
  int pl_count[kPlanes];            // group atoms whose box crosses plane z
  unsigned char pl_atom[kPlanes][kPlaneAtoms];
  T corr[2][kCorr];                 // projector term of the next plane, by in-plane index
  // first basis row with a nonzero value in each 64-point block (kNoRow: none yet); a
  // Krylov vector is exactly zero outside the reach of the earlier ones, so the sweep skips
  // the leading rows of a block that are still zero there
  unsigned char fnz[kFnzBlocks];
  int fnz_on;                       // the node's blocks fit fnz
};

// Whether the node's stencil runs as the plane march (the condition apply_local uses).
template <typename T, int BLOCK>
__device__ __forceinline__ bool uses_march(const SGQ_L NodeState<T, BLOCK>& st, int block) {
  return !st.periodic && st.sx * st.sy <= 5 * block &&
         (st.sx + 6) * (st.sy + 6) <= NodeState<T, BLOCK>::kMarchPad;
}

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

// Projector box point (bx, by, bz) of node atom a -> local linear index, or -1 outside
// the cube.
template <typename S>
__device__ __forceinline__ int box_point(const S& st, int a, int bx, int by, int bz) {
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

template <typename S>
__device__ __forceinline__ int box_point(const S& st, int a, int b, int B) {
  return box_point(st, a, b % B, (b / B) % B, b / (B * B));
}

// The four projectors of one atom (s, px, py, pz: Gaussian of width rg times the
// smooth cutoff (1 - r^2/rc^2)^3, continuum-normalised), evaluated at a box point from
// the atom's offset f = g0 h - R instead of being read from a table.
template <typename T>
struct ProjEval {
  T h, ns, npr, inv_rc2, k2;
  int m;
};

template <typename T>
__host__ __device__ inline ProjEval<T> proj_eval(const LaunchParams& P) {
  ProjEval<T> e;
  e.h = (T)P.h;
  e.ns = (T)P.proj_norm_s;
  e.npr = (T)(P.proj_norm_p / P.proj_rg);
  e.inv_rc2 = (T)(1.0 / (P.proj_rc * P.proj_rc));
  e.k2 = (T)(0.5 / (P.proj_rg * P.proj_rg));
  e.m = P.box_m;
  return e;
}

__device__ __forceinline__ float exp_neg(float x) { return __expf(-x); }
__device__ __forceinline__ double exp_neg(double x) { return exp(-x); }

// The four projectors and their derivatives with respect to the displacement d = x - R
// of the point from the atom: g[3 l + a] = d chi_l / d d_a (the derivative with respect to
// the atom position is its negative).
template <typename T, typename F>
__device__ __forceinline__ void chi_grad_at(const ProjEval<T>& pe, const F& f, int bx, int by,
                                            int bz, T (&c)[4], T (&g)[12]) {
  const T d[3] = {(T)(bx - pe.m) * pe.h + f[0], (T)(by - pe.m) * pe.h + f[1],
                  (T)(bz - pe.m) * pe.h + f[2]};
  const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const T t = (T)1 - r2 * pe.inv_rc2;
  const bool in = t > (T)0;
  const T e = in ? exp_neg(r2 * pe.k2) : (T)0;
  const T gv = e * (t * t * t);                                              // e t^3
  const T gd = in ? e * (-(T)2 * pe.k2 * (t * t * t) - (T)6 * pe.inv_rc2 * (t * t)) : (T)0;
  c[0] = pe.ns * gv;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[1 + a] = pe.npr * d[a] * gv;
    g[a] = pe.ns * gd * d[a];
  }
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      g[3 * (l + 1) + a] = pe.npr * (d[l] * gd * d[a] + (l == a ? gv : (T)0));
}

template <typename T, typename F>
__device__ __forceinline__ void chi_at(const ProjEval<T>& pe, const F& f, int bx, int by, int bz,
                                       T (&c)[4]) {
  const T dx = (T)(bx - pe.m) * pe.h + f[0];
  const T dy = (T)(by - pe.m) * pe.h + f[1];
  const T dz = (T)(bz - pe.m) * pe.h + f[2];
  const T r2 = dx * dx + dy * dy + dz * dz;
  const T t = (T)1 - r2 * pe.inv_rc2;
  const T g = t > (T)0 ? exp_neg(r2 * pe.k2) * (t * t * t) : (T)0;
  const T gp = pe.npr * g;
  c[0] = pe.ns * g;
  c[1] = gp * dx;
  c[2] = gp * dy;
  c[3] = gp * dz;
}

// Sets up the cube geometry and the node's projector atom list (ordered by atom id).
template <typename T, int BLOCK>
__device__ __noinline__ void node_setup(const LaunchParams& P, SGQ_L NodeState<T, BLOCK>& st, int q) {
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
    st.ngrp = 0;
    st.nlayer = 0;
    st.abort = 0;
    st.fuse = 0;
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
        for (int ax = 0; ax < 3; ++ax)
          st.afrac[slot][ax] = (T)(P.atom_g0[3 * J + ax] * P.h - P.atom_R[3 * J + ax]);
        st.afrac[slot][3] = (T)0;
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
  // Scatter layers: an atom whose box overlaps no earlier atom's box joins the parallel
  // group (layer 0); any other atom takes the layer one above the highest layer among the
  // earlier atoms whose boxes overlap its own.  No two atoms of a layer overlap, so each
  // layer is scattered in parallel, and at every point the layers add their terms in atom
  // order, as scattering the atoms one at a time would.  Where the grid is narrower than a
  // box, a box overlaps itself: every atom is then scattered alone, by one thread.
  const int B = 2 * m + 1;
  const bool alias = st.periodic && (P.nx < B || P.ny < B || P.nz < B);
  auto overlap = [&](int a, int b) {
    for (int ax = 0; ax < 3; ++ax) {
      int d = st.abox[a][ax] - st.abox[b][ax];
      if (st.periodic) {
        int nax = nn[ax];
        d = wrap_index(d, nax);
        d = d > nax / 2 ? nax - d : d;
      }
      if (abs(d) > 2 * m) return false;
    }
    return true;
  };
  for (int a = tid; a < st.natoms; a += BLOCK) {
    int ph = alias ? 1 : 0;
    for (int b = 0; b < a && ph == 0; ++b)
      if (overlap(a, b)) ph = 1;
    st.aphase[a] = ph;
  }
  __syncthreads();
  if (!alias) {
    // rounds of L(a) = 1 + max L(b) over the overlapping earlier atoms b, each from the
    // layers of the round before; the layers only grow, and a round that changes none has
    // reached the (unique) solution
    constexpr int IT = (kMaxNodeAtoms + BLOCK - 1) / BLOCK;
    for (;;) {
      int nl[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int a = tid + i * BLOCK;
        int L = 0;
        if (a < st.natoms && st.aphase[a]) {
          L = 1;
          for (int b = 0; b < a; ++b)
            if (st.aphase[b] >= L && overlap(a, b)) L = st.aphase[b] + 1;
        }
        nl[i] = L;
      }
      __syncthreads();
      if (tid == 0) st.lchange = 0;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int a = tid + i * BLOCK;
        if (a < st.natoms && nl[i] != st.aphase[a]) {
          st.aphase[a] = nl[i];
          st.lchange = 1;
        }
      }
      __syncthreads();
      if (!st.lchange) break;
    }
  }
  if (threadIdx.x == 0) {
    // counting sort of the atoms by layer, stable in atom order
    int nlay = 0;
    for (int a = 0; a < st.natoms; ++a) nlay = max(nlay, st.aphase[a] + 1);
    for (int L = 0; L <= nlay; ++L) st.lstart[L] = 0;
    for (int a = 0; a < st.natoms; ++a) ++st.lstart[st.aphase[a] + 1];
    for (int L = 0; L < nlay; ++L) st.lstart[L + 1] += st.lstart[L];
    for (int a = 0; a < st.natoms; ++a) st.grp[st.lstart[st.aphase[a]]++] = a;
    // lstart[L] now ends layer L: shift to the starts
    for (int L = nlay - 1; L >= 1; --L) st.lstart[L] = st.lstart[L - 1];
    st.lstart[0] = 0;
    st.nlayer = nlay;
    st.ngrp = nlay > 0 ? st.lstart[1] : 0;
  }
  __syncthreads();
  if constexpr (NodeState<T, BLOCK>::kFuse) {
    constexpr int KP = NodeState<T, BLOCK>::kPlanes, KA = NodeState<T, BLOCK>::kPlaneAtoms;
    const bool march = uses_march(st, BLOCK) && st.sz <= KP;
    if (march) {
      for (int z = tid; z < st.sz; z += BLOCK) {
        int c = 0;
        for (int i = 0; i < st.ngrp; ++i) {
          const int a = st.grp[i], z0 = st.abox[a][2];
          if (z >= z0 && z < z0 + B) {
            if (c < KA) st.pl_atom[z][c] = (unsigned char)a;
            ++c;
          }
        }
        st.pl_count[z] = c;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int ok = march && st.ngrp > 0;
      for (int z = 0; ok && z < st.sz; ++z) ok = st.pl_count[z] <= KA;
      st.fuse = ok;
    }
    __syncthreads();
  } else {
    if (tid == 0) st.fuse = 0;
    __syncthreads();
  }
}

// Buffer resource over `bytes` bytes from `base` (raw, unswizzled): loads at offsets at
// or beyond `bytes` return zero without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// Streaming (non-temporal) load of the basis: each row is read once per Lanczos step and
// not again before the next step's sweep, so it should not displace the vectors and
// potential the other phases reuse from L2.
constexpr int kLoadNT = 2;

template <typename V>
__device__ __forceinline__ V buffer_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(V) == 16)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kLoadNT));
  else if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kLoadNT));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kLoadNT));
}

// dst(p) = src(p) - sum_{i<=j} ct_i W_i(p) for every cube point, with the FP64 dots
// D_i = W_i . dst and |dst|^2 left per wave in st.red.
//
// The basis is stored in 64-point blocks, [npad/64][kmax][64] (block stride bs), so rows
// 0..j of one block are a single contiguous run.  Four lanes share a point group of VEC
// consecutive points, each lane taking the rows i = g (mod 4), i.e. KS "slots"
// i = 4m + g; with VEC = 4 one load instruction of a wave reads four whole 256-byte rows
// of a block.  A lane handles PU point groups per iteration, so one iteration issues
// KS*PU vector loads before any of them is consumed.  Rows are addressed through a
// buffer resource: one 32-bit lane offset plus a uniform per-slot offset.  Rows i > j of
// the last slot are read from row j (finite data) and weighted zero.  Slots whose rows all
// precede the block's first nonzero row (st.fnz) are not read: they hold exact zeros in
// that block, which contribute nothing to w or D.  src and dst are row views with block
// strides sbs and bs.
template <typename T, int BLOCK, int KS, int PU, int VEC, int G = 4>
__device__ __noinline__ void fused_sweep_v(SGQ_L NodeState<T, BLOCK>& st,
                                           const SGQ_G T* __restrict__ W, int bs, int wbytes,
                                           const SGQ_G T* src, int sbs, SGQ_G T* dst, int j,
                                           int n) {
  using V = T __attribute__((ext_vector_type(VEC)));
  static_assert(G == 4 || G == 8, "lane groups of 4 or 8");
  constexpr int ES = (int)sizeof(T);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int g = lane & (G - 1);
  const __amdgpu_buffer_rsrc_t rw = buffer_over((const void*)W, wbytes);
  const int mlast = j / G;        // last slot holding a row <= j
  const int rlast = G * mlast + g <= j ? G * mlast + g : j;
  const int dlast = (rlast - g - G * mlast) * 64 * ES;
  double D[KS];
  T cg[KS];
#pragma unroll
  for (int m = 0; m < KS; ++m) {
    D[m] = 0.0;
    const int i = G * m + g;
    cg[m] = (i <= j) ? st.ct[i] : (T)0;
  }
  double n2 = 0.0;
  const int ngroups = (n + VEC - 1) / VEC;
  constexpr int STRIDE = BLOCK / G;
  // A wave's point groups lie in one 64-point block (all of it, or half of it when a wave
  // covers 32 points), so the first nonzero row of the block is uniform over the wave.
  const bool skip = st.fnz_on;
  for (int pg0 = tid / G; pg0 < ngroups; pg0 += STRIDE * PU) {
    V qv[PU][KS];
    V sv[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int pg = pg0 + u * STRIDE;
      const int p0 = (pg < ngroups ? pg : 0) * VEC;
      const int voff = (bidx(p0, bs) + 64 * g) * ES;
      // slots whose G rows all precede the block's first nonzero row hold zeros there
      const int mfirst = skip ? (int)st.fnz[p0 >> 6] / G : 0;
#pragma unroll
      for (int m = 0; m < KS; ++m) {
        if (m < mfirst)
          qv[u][m] = (V)(T)0;
        else if (m < mlast)
          qv[u][m] = buffer_load<V>(rw, voff, m * 64 * G * ES);
        else if (m == mlast)
          qv[u][m] = buffer_load<V>(rw, voff + dlast, m * 64 * G * ES);
        else
          qv[u][m] = (V)(T)0;
      }
      sv[u] = *reinterpret_cast<const SGQ_G V*>(src + bidx(p0, sbs));
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int pg = pg0 + u * STRIDE;
      const int p0 = pg * VEC;
      V acc = (V)(T)0;
#pragma unroll
      for (int m = 0; m < KS; ++m) acc += cg[m] * qv[u][m];
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        acc[k] += __shfl_xor(acc[k], 1, kWave);
        acc[k] += __shfl_xor(acc[k], 2, kWave);
        if (G == 8) acc[k] += __shfl_xor(acc[k], 4, kWave);
      }
      V w = sv[u] - acc;
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (pg >= ngroups || p0 + k >= n) w[k] = (T)0;
      bool nz = false;
      if (g == 0 && pg < ngroups) {
        *reinterpret_cast<SGQ_G V*>(dst + bidx(p0, bs)) = w;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          n2 += (double)w[k] * (double)w[k];
          nz = nz || w[k] != (T)0;
        }
      }
      // record the first nonzero row j + 1 of the block (the same value from every wave
      // that covers part of it; rows up to j stay zero there either way)
      if (skip && __any(nz) && lane == 0 && st.fnz[(pg * VEC) >> 6] > j + 1)
        st.fnz[(pg * VEC) >> 6] = (unsigned char)(j + 1);
#pragma unroll
      for (int m = 0; m < KS; ++m) {
#pragma unroll
        for (int k = 0; k < VEC; ++k) D[m] += (double)qv[u][m][k] * (double)w[k];
      }
    }
  }
#pragma unroll
  for (int m = 0; m < KS; ++m) {
    double v = D[m];
    if (G == 4) v += __shfl_xor(v, 4, kWave);
    v += __shfl_xor(v, 8, kWave);
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    const int i = G * m + g;
    if (lane < G && i <= j) st.red[wave][i] = v;
  }
  n2 = wave_sum(n2);
  if (lane == 0) st.red[wave][kMaxDepth + 1] = n2;
}

// Picks the sweep variant for step j (slots KS >= (j+1)/4, at most KG).  The FP32
// variants read 16 bytes per lane and row (a wave reads four whole 256-byte block rows
// per instruction), which measured fastest at every depth.
template <typename T, int BLOCK, int KG>
__device__ __forceinline__ void fused_sweep(SGQ_L NodeState<T, BLOCK>& st,
                                            const SGQ_G T* __restrict__ W, int bs, int wbytes,
                                            const SGQ_G T* src, int sbs, SGQ_G T* dst, int j,
                                            int n) {
  const int need = j / 4 + 1;
  if constexpr (sizeof(T) == 4) {
    if (need <= 2) return fused_sweep_v<T, BLOCK, 2, 4, 4>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (need <= 4) return fused_sweep_v<T, BLOCK, 4, 2, 4>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (need <= 8) return fused_sweep_v<T, BLOCK, 8, 1, 4>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (need <= 12) return fused_sweep_v<T, BLOCK, 12, 1, 4>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (KG <= 16 || need <= 16) return fused_sweep_v<T, BLOCK, 16, 1, 4>(st, W, bs, wbytes, src, sbs, dst, j, n);
    // deeper steps: eight lanes per point group, rows i = g (mod 8)
    const int need8 = j / 8 + 1;
    if (need8 <= 12) return fused_sweep_v<T, BLOCK, 12, 1, 4, 8>(st, W, bs, wbytes, src, sbs, dst, j, n);
    return fused_sweep_v<T, BLOCK, 16, 1, 4, 8>(st, W, bs, wbytes, src, sbs, dst, j, n);
  } else {
    if (need <= 2) return fused_sweep_v<T, BLOCK, 2, 4, 2>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (need <= 4) return fused_sweep_v<T, BLOCK, 4, 2, 2>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (need <= 8) return fused_sweep_v<T, BLOCK, 8, 2, 1>(st, W, bs, wbytes, src, sbs, dst, j, n);
    if (KG <= 16 || need <= 16) return fused_sweep_v<T, BLOCK, 16, 1, 1>(st, W, bs, wbytes, src, sbs, dst, j, n);
    return fused_sweep_v<T, BLOCK, 32, 1, 1>(st, W, bs, wbytes, src, sbs, dst, j, n);
  }
}

// Totals of a sweep: beta_j, the scale of the new vector, its Gram column against
// q_0..q_j and the semi-orthogonality flag.  Ends with a barrier.
template <typename T, int BLOCK>
__device__ __forceinline__ void finish_sweep(SGQ_L NodeState<T, BLOCK>& st, int j) {
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
  double gi = 0.0;
  if (tid <= j) {
    gi = st.scale[tid] * st.scale[j + 1] * dsum;
    st.gram[tid] = gi;
  }
  // semi-orthogonality test: any |G_i| above sqrt(eps) (or not finite)
  int bad = (tid <= j) && !(fabs(gi) <= st.orth_tol);
  bad = __any(bad);
  if ((tid & (kWave - 1)) == 0) st.wflag[tid / kWave] = bad;
  __syncthreads();
  if (tid == 0) {
    int r = 0;
    for (int w = 0; w < NW; ++w) r |= st.wflag[w];
    st.redo = r;
  }
  __syncthreads();
}

// chi . q_j of every node atom (projector overlaps).  A wave takes NA atoms at a time
// with every box point of all of them unrolled, so their loads are in flight together;
// the projector values are evaluated in registers.
template <typename T, int BLOCK>
__device__ __noinline__ void projector_dots(const SGQ_G double* proj_E,
                                            SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                            const SGQ_G T* Wj, int bs, double sjd, double h3,
                                            int B, int B3) {
  constexpr int NW = BLOCK / kWave;
  constexpr int UNR = 6;    // 6 x 64 box points cover the 7^3 box of h = rc/3
  constexpr int NA = sizeof(T) == 4 ? 3 : 1;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int natoms = st.natoms;
  for (int a0 = NA * wave; a0 < natoms; a0 += NA * NW) {
    T acc[NA][4];
#pragma unroll
    for (int t = 0; t < NA; ++t)
#pragma unroll
      for (int l = 0; l < 4; ++l) acc[t][l] = (T)0;
    for (int b0 = 0; b0 < B3; b0 += UNR * kWave) {
      int bc[UNR][3];
      T wv[NA][UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int b = b0 + u * kWave + lane;
        bc[u][0] = b % B;
        bc[u][1] = (b / B) % B;
        bc[u][2] = b / (B * B);
#pragma unroll
        for (int t = 0; t < NA; ++t) {
          const int a = a0 + t;
          const bool live = (b < B3) && (a < natoms);
          const int lp = live ? box_point(st, a, bc[u][0], bc[u][1], bc[u][2]) : -1;
          wv[t][u] = Wj[bidx(lp >= 0 ? lp : 0, bs)] * (T)(lp >= 0);
        }
      }
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        const int a = a0 + t < natoms ? a0 + t : a0;
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          T c[4];
          chi_at(pe, st.afrac[a], bc[u][0], bc[u][1], bc[u][2], c);
#pragma unroll
          for (int l = 0; l < 4; ++l) acc[t][l] += c[l] * wv[t][u];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int a = a0 + t;
      if (a >= natoms) break;
      const int J = st.atom[a];
      double nl = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        double cl = (double)wave_sum(acc[t][l]) * sjd;     // chi_l . q_j
        double El = proj_E[4 * J + l];
        if (lane == 0) st.acoef[a][l] = (T)(El * h3 * cl);
        nl += El * h3 * cl * cl;
      }
      if (lane == 0) st.anl[a] = nl;
    }
  }
}

// u += sum_l chi_l E_l h^3 (chi_l . q) over the box of atom a, one point at a time by the
// calling thread (grids narrower than the box, where box points alias).
template <typename T, int BLOCK>
__device__ __noinline__ void scatter_atom(SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                          SGQ_G T* U, int a, int B, int B3) {
  const T coef[4] = {st.acoef[a][0], st.acoef[a][1], st.acoef[a][2], st.acoef[a][3]};
  for (int b = 0; b < B3; ++b) {
    const int bx = b % B, by = (b / B) % B, bz = b / (B * B);
    int lp = box_point(st, a, bx, by, bz);
    if (lp < 0) continue;
    T c[4];
    chi_at(pe, st.afrac[a], bx, by, bz, c);
    U[lp] += c[0] * coef[0] + c[1] * coef[1] + c[2] * coef[2] + c[3] * coef[3];
  }
}

// One scatter layer, the atoms st.grp[first, end): their boxes are disjoint, so their
// updates never touch the same point.  A wave takes NA of them per round with all the
// loads of the round issued before any update.
template <typename T, int BLOCK>
__device__ __noinline__ void scatter_group(SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                           SGQ_G T* U, int B, int B3, int first, int end) {
  constexpr int NW = BLOCK / kWave;
  constexpr int NA = sizeof(T) == 4 ? 3 : 1;
  constexpr int UNR = 6;    // 6 x 64 box points cover the 7^3 box of h = rc/3
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  // the layer's atoms (in atom order) dealt round-robin to the waves
  const int na = end - first;
  const int cnt = na > wave ? (na - wave + NW - 1) / NW : 0;
  auto mine = [&](int i) { return st.grp[first + wave + NW * i]; };
  for (int i0 = 0; i0 < cnt; i0 += NA) {
    for (int b0 = 0; b0 < B3; b0 += UNR * kWave) {
      int bc[UNR][3];
      int lp[NA][UNR];
      T old[NA][UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int b = b0 + u * kWave + lane;
        bc[u][0] = b % B;
        bc[u][1] = (b / B) % B;
        bc[u][2] = b / (B * B);
#pragma unroll
        for (int t = 0; t < NA; ++t) {
          const int a = i0 + t < cnt ? mine(i0 + t) : mine(i0);
          lp[t][u] = (b < B3 && i0 + t < cnt) ? box_point(st, a, bc[u][0], bc[u][1], bc[u][2]) : -1;
          old[t][u] = U[lp[t][u] >= 0 ? lp[t][u] : 0];
        }
      }
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        const int a = i0 + t < cnt ? mine(i0 + t) : mine(i0);
        const T coef[4] = {st.acoef[a][0], st.acoef[a][1], st.acoef[a][2], st.acoef[a][3]};
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          if (lp[t][u] >= 0) {
            T c[4];
            chi_at(pe, st.afrac[a], bc[u][0], bc[u][1], bc[u][2], c);
            U[lp[t][u]] = old[t][u] +
                          (c[0] * coef[0] + c[1] * coef[1] + c[2] * coef[2] + c[3] * coef[3]);
          }
        }
      }
    }
  }
}

// The three stencil forms below take the Laplacian as sum_d w_d ((v_-d - v) + (v_+d - v)),
// which equals the usual weighted sum because the sixth-order weights add up to zero.
// Forming each neighbour difference first keeps the FP32 rounding of the matvec
// proportional to those differences, not to the point values: on the smooth parts of a
// vector the usual form loses the Laplacian to cancellation of terms up to 8 |v|, and
// that rounding, seen by the Lanczos rule as a perturbation of H, was the largest error of
// the FP32 adjoint.
//
// u = s_j (-1/2 Lap_6 + V) W_j on a Dirichlet cube, four points per thread with every
// load issued unconditionally (out-of-cube neighbours read the centre and are masked).
// Returns this thread's part of q_j . u.
template <typename T, int BLOCK, bool ACC = false>
__device__ __noinline__ double stencil_cube(int gnx, int gny, int gnz,
                                            const SGQ_L NodeState<T, BLOCK>& st,
                                            const SGQ_G T* __restrict__ V,
                                            const SGQ_G T* __restrict__ Wj, int vbs,
                                            SGQ_G T* __restrict__ U, T sj, T kin) {
  const int n = st.n, sx = st.sx, sy = st.sy, sz = st.sz, sxy = sx * sy;
  const float inv_sx = 1.0f / (float)sx, inv_sxy = 1.0f / (float)sxy;
  const T w1 = (T)kFd1, w2 = (T)kFd2, w3 = (T)kFd3;
  const int ox = st.ox, oy = st.oy, oz = st.oz;
  double apart = 0.0;
  constexpr int UNR = 4;
  for (int base = threadIdx.x; base < n; base += UNR * BLOCK) {
    T u[UNR], wc[UNR];
    int pk[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const int p = base + k * BLOCK;
      const int pc = p < n ? p : 0;
      pk[k] = p;
      int x, y, z;
      unflatten(pc, sx, sxy, inv_sx, inv_sxy, x, y, z);
      const T c = Wj[bidx(pc, vbs)];
      wc[k] = c;
      // neighbour minus centre (zero outside the cube, so the difference is -c there)
      auto nb = [&](bool ok, int idx) -> T {
        T v = Wj[bidx(ok ? idx : pc, vbs)];
        return (ok ? v : (T)0) - c;
      };
      T l1 = (nb(x >= 1, pc - 1) + nb(x + 1 < sx, pc + 1)) + (nb(y >= 1, pc - sx) +
             nb(y + 1 < sy, pc + sx)) + (nb(z >= 1, pc - sxy) + nb(z + 1 < sz, pc + sxy));
      T l2 = (nb(x >= 2, pc - 2) + nb(x + 2 < sx, pc + 2)) + (nb(y >= 2, pc - 2 * sx) +
             nb(y + 2 < sy, pc + 2 * sx)) + (nb(z >= 2, pc - 2 * sxy) + nb(z + 2 < sz, pc + 2 * sxy));
      T l3 = (nb(x >= 3, pc - 3) + nb(x + 3 < sx, pc + 3)) + (nb(y >= 3, pc - 3 * sx) +
             nb(y + 3 < sy, pc + 3 * sx)) + (nb(z >= 3, pc - 3 * sxy) + nb(z + 3 < sz, pc + 3 * sxy));
      int gx = ox + x, gy = oy + y, gz = oz + z;
      gx = gx < 0 ? gx + gnx : (gx >= gnx ? gx - gnx : gx);
      gy = gy < 0 ? gy + gny : (gy >= gny ? gy - gny : gy);
      gz = gz < 0 ? gz + gnz : (gz >= gnz ? gz - gnz : gz);
      const T vloc = V[gx + gnx * (gy + gny * gz)];
      const T lap = w1 * l1 + w2 * l2 + w3 * l3;
      u[k] = sj * (kin * lap + vloc * c);
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      if (pk[k] < n) {
        if (ACC) U[pk[k]] += u[k]; else U[pk[k]] = u[k];
        apart += (double)(sj * wc[k]) * (double)u[k];
      }
    }
  }
  return apart;
}

// u = s_j (-1/2 Lap_6 + V) W_j on a Dirichlet cube by marching through the z planes.
// Thread t owns the in-plane points t + k*BLOCK (k < PPT) of every plane.  Their values
// at planes z-3 .. z+NQ-4 live in a register ring indexed statically (the z loop is
// unrolled by the ring length), so a plane is loaded NQ-6 planes before it is first
// used; the potential is loaded NV planes ahead.  The x/y neighbours of plane z come
// from a double-buffered copy of the plane in LDS with a zero halo three points wide,
// which makes every neighbour a fixed offset (no clamping, no masks); one barrier per
// plane.  Returns this thread's part of q_j . u.
// Projector term of the parallel group on local plane zc, added into buf (in-plane index
// x + sx*y): the group's boxes are disjoint, so no two (atom, point) pairs meet.
template <typename T, int BLOCK>
__device__ __forceinline__ void plane_group_term(SGQ_L NodeState<T, BLOCK>& st, ProjEval<T> pe,
                                                 int zc, int B, SGQ_L T* buf) {
  const int BB = B * B, na = st.pl_count[zc], sx = st.sx, sy = st.sy;
  for (int t = threadIdx.x; t < na * BB; t += BLOCK) {
    const int i = t / BB, sp = t - i * BB;
    const int a = st.pl_atom[zc][i];
    const int bx = sp % B, by = sp / B, bz = zc - st.abox[a][2];
    const int x = st.abox[a][0] + bx, y = st.abox[a][1] + by;
    if (x >= 0 && x < sx && y >= 0 && y < sy) {
      T c[4];
      chi_at(pe, st.afrac[a], bx, by, bz, c);
      buf[x + sx * y] += c[0] * st.acoef[a][0] + c[1] * st.acoef[a][1] + c[2] * st.acoef[a][2] +
                         c[3] * st.acoef[a][3];
    }
  }
}

template <typename T, int BLOCK, int PPT, bool ACC = false, bool PROJ = false>
__device__ __noinline__ double stencil_march(int gnx, int gny, int gnz,
                                             SGQ_L NodeState<T, BLOCK>& st,
                                             const SGQ_G T* __restrict__ V,
                                             const SGQ_G T* __restrict__ Wj, int vbs,
                                             SGQ_G T* __restrict__ U, T sj, T kin,
                                             ProjEval<T> pe, int B) {
  constexpr int NQ = 8;    // ring of W planes z-3 .. z+4
  constexpr int NV = 4;    // ring of V planes z .. z+3
  static_assert(NQ % NV == 0, "the unrolled z loop indexes both rings by r = z mod NQ");
  const int sx = st.sx, sy = st.sy, sz = st.sz, sxy = sx * sy;
  const int rx = sx + 6;   // padded row
  const int tid = threadIdx.x;
  const int vplane = gnx * gny;
  const T w1 = (T)kFd1, w2 = (T)kFd2, w3 = (T)kFd3;
  for (int i = tid; i < 2 * NodeState<T, BLOCK>::kMarchPad; i += BLOCK) (&st.plane[0][0])[i] = (T)0;
  if (PROJ)
    for (int i = tid; i < 2 * NodeState<T, BLOCK>::kCorr; i += BLOCK) (&st.corr[0][0])[i] = (T)0;
  __syncthreads();
  // the group term of a plane is built during the previous plane (plane 0 here) into the
  // other half of corr; each lane clears its entries after reading them
  if (PROJ) plane_group_term<T, BLOCK>(st, pe, 0, B, st.corr[0]);
  T ring[PPT][NQ];
  T vring[PPT][NV];
  int li[PPT], vrow[PPT];
  bool own[PPT];
  int gz0 = st.oz < 0 ? st.oz + gnz : st.oz;     // global z of local plane 0
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
#pragma unroll
    for (int d = 0; d < NQ; ++d) {
      // slot d holds plane d (d <= NQ-4) or plane d - NQ (below the cube: masked at
      // use); planes outside the cube are read clamped and masked where they are used
      const int z = d <= NQ - 4 ? d : d - NQ;
      const int zc = z < 0 ? 0 : (z < sz ? z : sz - 1);
      ring[k][d] = Wj[bidx(pc + zc * sxy, vbs)];
    }
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      int gz = gz0 + (d < sz ? d : sz - 1);
      gz = gz >= gnz ? gz - gnz : gz;
      vring[k][d] = V[vrow[k] + vplane * gz];
    }
  }
  double apart = 0.0;
  for (int z0 = 0; z0 < sz; z0 += NQ) {
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int z = z0 + r;
      if (z < sz) {
        SGQ_L T* plane = st.plane[z & 1];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
          if (own[k]) plane[li[k]] = ring[k][r];
        __syncthreads();
        // uniform masks of the z neighbours (zero outside the cube)
        const T mz1 = (T)(z >= 1), pz1 = (T)(z + 1 < sz);
        const T mz2 = (T)(z >= 2), pz2 = (T)(z + 2 < sz);
        const T mz3 = (T)(z >= 3), pz3 = (T)(z + 3 < sz);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const SGQ_L T* c0 = plane + li[k];
          const T c = ring[k][r];
          // neighbour minus centre; the halo and the masked z planes are zero
          const T l1 = ((mz1 * ring[k][(r + NQ - 1) % NQ] - c) + (pz1 * ring[k][(r + 1) % NQ] - c)) +
                       ((c0[-1] - c) + (c0[1] - c)) + ((c0[-rx] - c) + (c0[rx] - c));
          const T l2 = ((mz2 * ring[k][(r + NQ - 2) % NQ] - c) + (pz2 * ring[k][(r + 2) % NQ] - c)) +
                       ((c0[-2] - c) + (c0[2] - c)) + ((c0[-2 * rx] - c) + (c0[2 * rx] - c));
          const T l3 = ((mz3 * ring[k][(r + NQ - 3) % NQ] - c) + (pz3 * ring[k][(r + 3) % NQ] - c)) +
                       ((c0[-3] - c) + (c0[3] - c)) + ((c0[-3 * rx] - c) + (c0[3 * rx] - c));
          const T lap = w1 * l1 + w2 * l2 + w3 * l3;
          const T u = sj * (kin * lap + vring[k][r % NV] * c);
          if (own[k]) {
            const int p2 = tid + k * BLOCK;
            if (ACC) {
              T add = u;
              if (PROJ) {
                SGQ_L T* cz = st.corr[z & 1];
                add += cz[p2];
                cz[p2] = (T)0;
              }
              U[p2 + z * sxy] += add;
            } else if (PROJ) {
              SGQ_L T* cz = st.corr[z & 1];
              U[p2 + z * sxy] = u + cz[p2];
              cz[p2] = (T)0;
            } else {
              U[p2 + z * sxy] = u;
            }
            apart += (double)(sj * c) * (double)u;
          }
        }
        if (PROJ && z + 1 < sz) plane_group_term<T, BLOCK>(st, pe, z + 1, B, st.corr[(z + 1) & 1]);
        // refill: plane z+NQ-3 replaces plane z-3, the potential of plane z+NV replaces z
        const int zw = z + NQ - 3, zv = z + NV < sz ? z + NV : sz - 1;
        int gz = gz0 + zv;
        gz = gz >= gnz ? gz - gnz : gz;
        gz = gz >= gnz ? gz - gnz : gz;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int pc = own[k] ? tid + k * BLOCK : 0;
          ring[k][(r + NQ - 3) % NQ] = Wj[bidx(pc + (zw < sz ? zw : sz - 1) * sxy, vbs)];
          vring[k][r % NV] = V[vrow[k] + vplane * gz];
        }
      }
    }
  }
  return apart;
}

// The same operator on the whole periodic grid (untruncated nodes), UNR points per thread
// with every load issued unconditionally (points past the end read point 0 and store
// nothing), in the same order of operations per point.  A neighbour coordinate c +- d
// (d <= 3) wraps with one conditional add or subtract on an axis longer than 3 points, and
// by the full remainder on a shorter one.
template <typename T, int BLOCK, bool ACC = false>
__device__ __noinline__ double stencil_periodic(const SGQ_L NodeState<T, BLOCK>& st,
                                                const SGQ_G T* __restrict__ V,
                                                const SGQ_G T* __restrict__ Wj, int vbs,
                                                SGQ_G T* __restrict__ U, T sj, T kin) {
  const int n = st.n, sx = st.sx, sy = st.sy, sz = st.sz, sxy = sx * sy;
  const float inv_sx = 1.0f / (float)sx, inv_sxy = 1.0f / (float)sxy;
  const T wd[4] = {(T)0, (T)kFd1, (T)kFd2, (T)kFd3};
  const bool fx = sx > 3, fy = sy > 3, fz = sz > 3;
  auto wrap = [](int v, int m, bool fast) {
    return fast ? (v < 0 ? v + m : (v >= m ? v - m : v)) : wrap_index(v, m);
  };
  constexpr int UNR = sizeof(T) == 4 ? 4 : 2;
  double apart = 0.0;
  for (int base = threadIdx.x; base < n; base += UNR * BLOCK) {
    T u[UNR], wc[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const int p = base + k * BLOCK;
      const int pc = p < n ? p : 0;
      int x, y, z;
      unflatten(pc, sx, sxy, inv_sx, inv_sxy, x, y, z);
      const T c = Wj[bidx(pc, vbs)];
      wc[k] = c;
      T lap = (T)0;
#pragma unroll
      for (int d = 1; d <= 3; ++d) {
        // neighbour minus centre, as in the cube forms
        lap += wd[d] * ((Wj[bidx(wrap(x - d, sx, fx) + sx * (y + sy * z), vbs)] - c) +
                        (Wj[bidx(wrap(x + d, sx, fx) + sx * (y + sy * z), vbs)] - c));
        lap += wd[d] * ((Wj[bidx(x + sx * (wrap(y - d, sy, fy) + sy * z), vbs)] - c) +
                        (Wj[bidx(x + sx * (wrap(y + d, sy, fy) + sy * z), vbs)] - c));
        lap += wd[d] * ((Wj[bidx(x + sx * (y + sy * wrap(z - d, sz, fz)), vbs)] - c) +
                        (Wj[bidx(x + sx * (y + sy * wrap(z + d, sz, fz)), vbs)] - c));
      }
      u[k] = sj * (kin * lap + V[pc] * c);
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const int p = base + k * BLOCK;
      if (p < n) {
        if (ACC) U[p] += u[k]; else U[p] = u[k];
        apart += (double)(sj * wc[k]) * (double)u[k];
      }
    }
  }
  return apart;
}


// u = (-1/2 Lap_6 + V) s v for one vector of the node cube (v a row view with block
// stride vbs, u a plain vector): dispatches the stencil form.  ACC adds into U instead of
// storing.  Returns this thread's part of (s v) . u.
// With `group` set and st.fuse on, the march also adds the parallel projector group
// (weights st.acoef, set by the caller before the call).
template <typename T, int BLOCK, bool ACC>
__device__ __forceinline__ double apply_local(const LaunchParams& P, SGQ_L NodeState<T, BLOCK>& st,
                                              const SGQ_G T* V, const SGQ_G T* v, int vbs,
                                              SGQ_G T* U, T s, T kin, ProjEval<T> pe, int B,
                                              bool group) {
  if (st.periodic) return stencil_periodic<T, BLOCK, ACC>(st, V, v, vbs, U, s, kin);
  if (uses_march(st, BLOCK)) {
    if constexpr (NodeState<T, BLOCK>::kFuse) {
      if (group && st.fuse)
        return stencil_march<T, BLOCK, 5, ACC, true>(P.nx, P.ny, P.nz, st, V, v, vbs, U, s,
                                                     kin, pe, B);
    }
    return stencil_march<T, BLOCK, 5, ACC, false>(P.nx, P.ny, P.nz, st, V, v, vbs, U, s, kin,
                                                  pe, B);
  }
  return stencil_cube<T, BLOCK, ACC>(P.nx, P.ny, P.nz, st, V, v, vbs, U, s, kin);
}

// u += V_nl v with the weights st.acoef: the parallel group (unless the march added it,
// `group` false), then the other scatter layers in order, each in parallel.
template <typename T, int BLOCK>
__device__ __forceinline__ void apply_scatter(const LaunchParams& P, SGQ_L NodeState<T, BLOCK>& st,
                                              ProjEval<T> pe, SGQ_G T* U, int B, int B3,
                                              bool group = true) {
  if (st.natoms == 0) return;
  if (group) {
    scatter_group<T, BLOCK>(st, pe, U, B, B3, 0, st.ngrp);
    __syncthreads();
  }
  if (st.periodic && (P.nx < B || P.ny < B || P.nz < B)) {
    for (int a = 0; a < st.natoms; ++a) {
      if (!st.aphase[a]) continue;
      if (threadIdx.x == 0) scatter_atom<T, BLOCK>(st, pe, U, a, B, B3);
      __syncthreads();
    }
    return;
  }
  for (int L = 1; L < st.nlayer; ++L) {
    scatter_group<T, BLOCK>(st, pe, U, B, B3, st.lstart[L], st.lstart[L + 1]);
    __syncthreads();
  }
}

// One K-step Lanczos run of the current node (after node_setup): rows 0..K_eff-1 of the
// point-blocked basis W (block stride P.wbs) hold the unnormalised vectors
// (q_i = st.scale[i] W_i), st.alpha / st.beta the tridiagonal.
// u_j = H q_j is written to U + j*ustride (ustride 0: one reused row).  Returns K_eff.
template <typename T, int BLOCK, int KG>
__device__ int run_lanczos(const LaunchParams& P, SGQ_L NodeState<T, BLOCK>& st,
                           SGQ_G T* __restrict__ W, SGQ_G T* __restrict__ Ubase, size_t ustride,
                           int K) {
  constexpr int NW = BLOCK / kWave;
  constexpr int VEC = sizeof(T) == 4 ? 4 : 2;   // widest point group of the sweeps
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const SGQ_G T* __restrict__ V = (const SGQ_G T*)P.v;
  const ProjEval<T> pe = proj_eval<T>(P);
  const SGQ_G double* proj_E = (const SGQ_G double*)P.proj_E;
  const size_t npad = P.npad;
  const double h = P.h;
  const double h3 = h * h * h;
  const T kin = (T)(-0.5 / (h * h));
  const double hscale = 1.5 * (-kFd0 + 2.0 * (kFd1 - kFd2 + kFd3)) / (h * h) + *P.vmax;
  const double tol = P.tau * hscale;
  const int B = 2 * P.box_m + 1, B3 = B * B * B;
  const int n = st.n;
  const int natoms = st.natoms;
  const int bs = P.wbs;
  const int wbytes = (int)((npad / 64) * (size_t)bs * sizeof(T));
  const int nzero = ((n + VEC - 1) / VEC) * VEC;
  for (int p = tid; p < nzero; p += BLOCK) W[bidx(p, bs)] = (T)0;
  const int nblk = (int)(npad / 64);
  const bool fnz_on = nblk <= kFnzBlocks;
  if (fnz_on)
    for (int b = tid; b < nblk; b += BLOCK) st.fnz[b] = (unsigned char)kNoRow;
  __syncthreads();
  if (tid == 0) {
    W[bidx(st.start, bs)] = (T)1;
    st.scale[0] = 1.0;
    st.fnz_on = fnz_on;
    if (fnz_on) st.fnz[st.start >> 6] = 0;   // row 0: the unit vector at the node
  }
  __syncthreads();

  int keff = K;
  for (int j = 0; j < K; ++j) {
    const SGQ_G T* __restrict__ Wj = W + 64 * j;     // row j (block stride bs)
    SGQ_G T* __restrict__ U = Ubase + (size_t)j * ustride;
    const double sjd = st.scale[j];
    const T sj = (T)sjd;
    // ---- H q_j: projector overlaps, stencil + local potential, projector scatter
    projector_dots<T, BLOCK>(proj_E, st, pe, Wj, bs, sjd, h3, B, B3);
    const bool fused = st.fuse && uses_march(st, BLOCK);
    double apart = apply_local<T, BLOCK, false>(P, st, V, Wj, bs, U, sj, kin, pe, B, true);
    apart = wave_sum(apart);
    if (lane == 0) st.red[wave][0] = apart;
    __syncthreads();
    apply_scatter<T, BLOCK>(P, st, pe, U, B, B3, !fused);
    if (tid < kWave) {
      double al = 0.0;
      for (int a = tid; a < natoms; a += kWave) al += st.anl[a];
      al = wave_sum(al);
      if (tid == 0) {
        for (int w = 0; w < NW; ++w) al += st.red[w][0];
        st.alpha[j] = al;
      }
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
    SGQ_G T* __restrict__ Wn = W + 64 * (j + 1);
    fused_sweep<T, BLOCK, KG>(st, W, bs, wbytes, U, 64, Wn, j, n);
    __syncthreads();
    finish_sweep<T, BLOCK>(st, j);
    // Semi-orthogonality guard: the coefficients above are exact up to O(G^2); when
    // the measured Gram column exceeds sqrt(eps) (only near an invariant subspace)
    // the projection is repeated once with the exact dots of this sweep.
    if (st.redo && st.beta[j] > tol) {
      for (int i = tid; i <= j; i += BLOCK)
        st.ct[i] = (T)(st.scale[i] * st.scale[i] * st.dsave[i]);
      __syncthreads();
      fused_sweep<T, BLOCK, KG>(st, W, bs, wbytes, Wn, bs, Wn, j, n);
      __syncthreads();
      finish_sweep<T, BLOCK>(st, j);
    }
    if (!(st.beta[j] > tol)) {   // breakdown (or NaN): the Krylov space is invariant
      keff = j + 1;
      break;
    }
  }
  return keff;
}

}  // namespace sgq
