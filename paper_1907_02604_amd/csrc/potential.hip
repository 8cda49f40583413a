// Self-consistency ingredients of the Hamiltonian's potential (Eq. Eqn:Hamiltonian):
// the LDA exchange-correlation energy and potential (Eq. eq:xc, Perdew-Wang correlation)
// and the electrostatic potential of the periodic Poisson problem (Eq. eq:poisson),
// discretised with the sixth-order FD Laplacian of the Hamiltonian and solved exactly for
// that operator by FFT.
//
// The 3-D FFT is a sequence of line passes.  A pass loads a tile of lines along one axis
// into LDS (the tile groups lines adjacent in x, or in y for the x axis, so that global
// accesses are contiguous runs), runs a mixed-radix (4, 2, 3, 5) Stockham FFT on them in
// LDS (one buffer: each stage reads its inputs into registers before writing), and writes
// the lines back in place.  The work grid holds the half spectrum along x (nx/2 + 1
// complex columns): the X passes carry two real lines per complex transform.  Five passes
// solve the problem:
//   X forward, reading the real source rho + b;
//   Y forward;
//   Z forward, multiply by -4 pi / (N lambda(k)), Z inverse (one LDS tile, one HBM round
//   trip);
//   Y inverse;
//   X inverse, writing phi and, fused, V = phi + u(rho) and e_xc(rho).
// lambda(k) = lx[kx] + ly[ky] + lz[kz] is the FD Laplacian's eigenvalue; the k = 0 mode
// (the mean of the source) is dropped and reported.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "sgq.h"
#include "sgq_common.h"

namespace sgq {
int report_error(int code, const std::string& msg);
}
using sgq::report_error;

namespace {
constexpr int kMaxStages = 12;
constexpr int kPassBlock = 256;
constexpr int kLdsComplex = 1024;   // complex doubles per LDS tile (16 KB, plus the twiddles)
constexpr int kRowAlign = 8;        // complex values per 128-byte cache line

// Row stride of the work grid: the nx/2 + 1 half-spectrum columns rounded up to whole cache
// lines, so that every column tile of the Y and Z passes starts on a line boundary and no
// line is fetched by two tiles.
int row_stride(int nx) { return (nx / 2 + 1 + kRowAlign - 1) / kRowAlign * kRowAlign; }
}  // namespace

struct AxisPlan {
  int n = 1;
  int nstages = 0;
  int radix[kMaxStages] = {};
};

struct sgq_potential {
  int device = 0;
  int32_t n[3] = {1, 1, 1};
  int64_t npts = 0;
  double h = 1.0;
  AxisPlan axis[3];
  double2* d_work = nullptr;    // half-spectrum complex grid, [z][y][row_stride(nx)]
  double2* d_tw[3] = {};        // exp(-2 pi i m / n_a), m < n_a
  double* d_lam[3] = {};        // per-axis FD eigenvalues
};

namespace sgq {
namespace {

// Perdew-Wang (1992) unpolarised correlation (Hartree) and Slater exchange.
constexpr double kPwA = 0.031091, kPwA1 = 0.21370;
constexpr double kPwB1 = 7.5957, kPwB2 = 3.5876, kPwB3 = 1.6382, kPwB4 = 0.49294;

// 1/x for a normal, finite x: the hardware reciprocal refined by two Newton steps
// (error below an ulp).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// log(1 + x) for finite x >= 0.  With y = 1 + x rounded and c = x - (y - 1) its rounding
// error, log(1 + x) = log y + c / y to first order.  y = m 2^e with m in [sqrt(1/2),
// sqrt(2)), log y = e ln 2 + 2 atanh(s) with s = (m - 1) / (m + 1), |s| <= 0.1716, and atanh
// from its odd series to s^21, whose remainder is below 2^-53 of the sum.
__device__ __forceinline__ double log1p_nonneg(double x) {
  const double y = 1.0 + x;
  const double c = x - (y - 1.0);
  int e;
  double m = frexp(y, &e);                     // y = m 2^e, m in [1/2, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) * recip(m + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = 2.0 * s;
  const double log_m = fma(s2 * z, p, s2);
  return fma((double)e, 0.6931471805599453, log_m) + c * __builtin_amdgcn_rcp(y);
}

// e_xc per volume and u = d e_xc / d rho; zero for rho <= 0.  z = rho^(-1/6) comes from an
// FP32 seed (hardware log2 / exp2) and two division-free Newton steps for z^-6 = rho,
// z <- z (7 - rho z^6) / 6, whose relative error squares (1e-7 -> 1e-14 -> rounding).  Then
// rho^(-1/3) = z^2, rs = (3/(4 pi))^(1/3) z^2 and sqrt(rs) = (3/(4 pi))^(1/6) z, with no FP64
// square root.  Outside [1e-30, 1e30] z is taken from the library cube root instead.
__device__ __forceinline__ void lda_xc(double rho, double& e, double& u) {
  if (!(rho > 0.0)) {
    e = 0.0;
    u = 0.0;
    return;
  }
  double z;
  if (rho > 1e-30 && rho < 1e30) {
    const float lf = __builtin_amdgcn_logf((float)rho);          // log2, FP32
    z = (double)__builtin_amdgcn_exp2f(lf * (-1.0f / 6.0f));
    double z2 = z * z;
    z = z * (7.0 - rho * (z2 * z2 * z2)) * (1.0 / 6.0);
    z2 = z * z;
    z = z * (7.0 - rho * (z2 * z2 * z2)) * (1.0 / 6.0);
  } else {
    z = sqrt(1.0 / cbrt(rho));
  }
  const double cx = 0.98474502184269641;            // (3/pi)^(1/3)
  const double crs = 0.62035049089940001;           // (3/(4 pi))^(1/3)
  const double crs2 = 0.7876233178997433;           // (3/(4 pi))^(1/6)
  const double y = z * z;                           // rho^(-1/3)
  const double r13 = rho * y * y;
  const double ex = -0.75 * cx * rho * r13, ux = -cx * r13;
  const double rs = crs * y;
  const double sq = crs2 * z;                       // sqrt(rs)
  const double isq = sq * r13 * (1.0 / crs);        // 1/sqrt(rs) = sqrt(rs) / rs
  const double Q = 2.0 * kPwA * (kPwB1 * sq + kPwB2 * rs + kPwB3 * rs * sq + kPwB4 * rs * rs);
  const double dQ = 2.0 * kPwA * (0.5 * kPwB1 * isq + kPwB2 + 1.5 * kPwB3 * sq + 2.0 * kPwB4 * rs);
  const double iQ = recip(Q), iQ1 = recip(Q + 1.0);
  const double L = log1p_nonneg(iQ);
  const double ec = -2.0 * kPwA * (1.0 + kPwA1 * rs) * L;
  const double dec = -2.0 * kPwA * kPwA1 * L + 2.0 * kPwA * (1.0 + kPwA1 * rs) * dQ * iQ * iQ1;
  e = ex + rho * ec;
  u = ux + ec - rs * (1.0 / 3.0) * dec;
}

__global__ __launch_bounds__(256) void xc_kernel(const double* __restrict__ rho, int64_t n,
                                                 double* __restrict__ exc, double* __restrict__ vxc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double e, u;
    lda_xc(rho[i], e, u);
    if (exc) exc[i] = e;
    vxc[i] = u;
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by sign * i
__device__ __forceinline__ double2 cmuli(double2 a, double sign) { return make_double2(-sign * a.y, sign * a.x); }

// In-place R-point DFT with exponent sign (-1 forward, +1 inverse).
template <int R>
__device__ __forceinline__ void dft(double2* u, double sign) {
  if constexpr (R == 2) {
    const double2 a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 a0 = cadd(u[0], u[2]), a1 = csub(u[0], u[2]);
    const double2 b0 = cadd(u[1], u[3]), b1 = cmuli(csub(u[1], u[3]), sign);
    u[0] = cadd(a0, b0);
    u[2] = csub(a0, b0);
    u[1] = cadd(a1, b1);
    u[3] = csub(a1, b1);
  } else if constexpr (R == 3) {
    const double c = -0.5, s = sign * 0.86602540378443865;   // cos(2 pi/3), sign sin(2 pi/3)
    const double2 t = cadd(u[1], u[2]), d = csub(u[1], u[2]);
    const double2 m = make_double2(u[0].x + c * t.x, u[0].y + c * t.y);
    const double2 r = make_double2(-s * d.y, s * d.x);
    u[0] = cadd(u[0], t);
    u[1] = cadd(m, r);
    u[2] = csub(m, r);
  } else {   // R == 5
    const double c1 = 0.30901699437494742, c2 = -0.80901699437494742;   // cos(2 pi/5), cos(4 pi/5)
    const double s1 = sign * 0.95105651629515357, s2 = sign * 0.58778525229247313;
    const double2 t1 = cadd(u[1], u[4]), d1 = csub(u[1], u[4]);
    const double2 t2 = cadd(u[2], u[3]), d2 = csub(u[2], u[3]);
    const double2 m1 = make_double2(u[0].x + c1 * t1.x + c2 * t2.x, u[0].y + c1 * t1.y + c2 * t2.y);
    const double2 m2 = make_double2(u[0].x + c2 * t1.x + c1 * t2.x, u[0].y + c2 * t1.y + c1 * t2.y);
    // i (s1 d1 + s2 d2) and i (s2 d1 - s1 d2)
    const double2 r1 = make_double2(-(s1 * d1.y + s2 * d2.y), s1 * d1.x + s2 * d2.x);
    const double2 r2 = make_double2(-(s2 * d1.y - s1 * d2.y), s2 * d1.x - s1 * d2.x);
    u[0] = cadd(u[0], cadd(t1, t2));
    u[1] = cadd(m1, r1);
    u[4] = csub(m1, r1);
    u[2] = cadd(m2, r2);
    u[3] = csub(m2, r2);
  }
}

// One Stockham stage of radix R over nl lines of length N held in one LDS buffer: every
// lane reads its butterflies' inputs into registers, the workgroup synchronises, and the
// outputs are written back in place.  A lane takes at most MAXIT butterflies
// (nl * N <= kLdsComplex and 256 lanes).
template <int R>
__device__ __forceinline__ void stage(double2* __restrict__ buf, int N, int nl, int p,
                                      const double2* __restrict__ tw, double sign) {
  constexpr int MAXIT = (kLdsComplex / R + kPassBlock - 1) / kPassBlock;
  const int m = N / R, total = nl * m, step = N / (p * R);
  double2 u[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int idx = threadIdx.x + it * kPassBlock;
    if (idx < total) {
      const int l = idx / m, i = idx - l * m;
      const double2* s = buf + l * N;
#pragma unroll
      for (int q = 0; q < R; ++q) u[it][q] = s[i + q * m];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int idx = threadIdx.x + it * kPassBlock;
    if (idx < total) {
      const int l = idx / m, i = idx - l * m;
      const int k = i % p;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        double2 w = tw[q * k * step];       // exp(-2 pi i q k / (p R))
        w.y *= -sign;                       // conjugate for the inverse
        u[it][q] = cmul(u[it][q], w);
      }
      dft<R>(u[it], sign);
      double2* d = buf + l * N;
      const int j = (i / p) * p * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) d[j + q * p] = u[it][q];
    }
  }
  __syncthreads();
}

// In-place FFT of nl lines held in buf.
__device__ void lds_fft(double2* buf, const AxisPlan& ap, int nl, const double2* __restrict__ tw,
                        double sign) {
  int p = 1;
  for (int s = 0; s < ap.nstages; ++s) {
    const int R = ap.radix[s];
    if (R == 4) stage<4>(buf, ap.n, nl, p, tw, sign);
    else if (R == 2) stage<2>(buf, ap.n, nl, p, tw, sign);
    else if (R == 3) stage<3>(buf, ap.n, nl, p, tw, sign);
    else stage<5>(buf, ap.n, nl, p, tw, sign);
    p *= R;
  }
}

enum PassMode { kFwdReal = 0, kFwd = 1, kSolve = 2, kInv = 3, kInvReal = 4 };

struct PassArgs {
  AxisPlan ap;
  int axis, tl, nx, ny, nz;
  int nxc;               // complex columns of the work grid, nx/2 + 1
  int nxs;               // its row stride, row_stride(nx)
  int64_t npts;
  double2* work;         // [nz][ny][nxs] complex; columns nxc and up are not used
  const double2* tw;
  const double* src_a;   // kFwdReal: rho (or the source)
  const double* src_b;   // kFwdReal: b (optional)
  const double* lx;      // kSolve: per-axis eigenvalues
  const double* ly;
  const double* lz;
  double scale;          // kSolve: -4 pi / npts
  double* mean;          // kSolve: mean of the source (optional)
  const double* rho;     // kInvReal: density for the fused xc term (optional)
  double* phi;           // kInvReal outputs (each optional)
  double* v;
  double* exc;
};

// X passes (MODE kFwdReal, kInvReal): a tile is TL = 2 * pairs consecutive y lines at
// fixed z.  Two real lines a, b travel as one complex line a + i b; forward, its transform Z
// unpacks into the half spectra A(k) = (Z(k) + conj Z(N-k)) / 2 and B(k) = (Z(k) -
// conj Z(N-k)) / 2i, k <= N/2; inverse, A + i B (continued to k > N/2 by conjugate
// symmetry) transforms back to a + i b.  Y and Z passes (kFwd, kSolve, kInv): a tile is TL
// consecutive complex columns.
template <int MODE>
__global__ __launch_bounds__(kPassBlock) void fft_pass_kernel(PassArgs a) {
  extern __shared__ double2 lds[];
  constexpr bool XPASS = MODE == kFwdReal || MODE == kInvReal;
  const int N = a.ap.n, TL = a.tl;
  const int nx = a.nx, ny = a.ny, nxc = a.nxc, nxs = a.nxs;
  const int64_t nxy = (int64_t)nx * ny, nxys = (int64_t)nxs * ny;
  const double sign = (MODE == kFwdReal || MODE == kFwd || MODE == kSolve) ? -1.0 : 1.0;
  if constexpr (XPASS) {
    const int pairs = TL / 2;
    double2* buf = lds;
    double2* twl = lds + pairs * N;
    for (int m = threadIdx.x; m < N; m += blockDim.x) twl[m] = a.tw[m];
    const int tiles_y = (ny + TL - 1) / TL;
    const int z = blockIdx.x / tiles_y;
    const int y0 = (blockIdx.x % tiles_y) * TL;
    const int nl = min(TL, ny - y0);
    const int np = (nl + 1) / 2;
    const int64_t rbase = (int64_t)y0 * nx + z * nxy;     // real grid, line y0
    const int64_t cbase = (int64_t)y0 * nxs + z * nxys;   // complex grid, line y0
    const int total = np * N;
    if constexpr (MODE == kFwdReal) {
      for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx / N, j = idx - p * N;
        const int64_t g0 = rbase + (int64_t)(2 * p) * nx + j;
        const double re = a.src_a[g0] + (a.src_b ? a.src_b[g0] : 0.0);
        double im = 0.0;
        if (2 * p + 1 < nl) im = a.src_a[g0 + nx] + (a.src_b ? a.src_b[g0 + nx] : 0.0);
        buf[p * N + j] = make_double2(re, im);
      }
    } else {
      const int half = N / 2;
      for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx / N, k = idx - p * N;
        const bool lo = k <= half;
        const int src = lo ? k : N - k;
        const int64_t g0 = cbase + (int64_t)(2 * p) * nxs + src;
        double2 A = a.work[g0];
        double2 B = 2 * p + 1 < nl ? a.work[g0 + nxs] : make_double2(0.0, 0.0);
        if (!lo) {
          A.y = -A.y;
          B.y = -B.y;
        }
        buf[p * N + k] = make_double2(A.x - B.y, A.y + B.x);   // A + i B
      }
    }
    __syncthreads();
    lds_fft(buf, a.ap, np, twl, sign);
    if constexpr (MODE == kFwdReal) {
      const int ntot = np * nxc;
      for (int idx = threadIdx.x; idx < ntot; idx += blockDim.x) {
        const int p = idx / nxc, k = idx - p * nxc;
        const double2 Zk = buf[p * N + k];
        const double2 Zm = buf[p * N + (k == 0 ? 0 : N - k)];
        // A = (Zk + conj Zm) / 2, B = (Zk - conj Zm) / 2i
        const double2 A = make_double2(0.5 * (Zk.x + Zm.x), 0.5 * (Zk.y - Zm.y));
        const double2 B = make_double2(0.5 * (Zk.y + Zm.y), -0.5 * (Zk.x - Zm.x));
        const int64_t g0 = cbase + (int64_t)(2 * p) * nxs + k;
        a.work[g0] = A;
        if (2 * p + 1 < nl) a.work[g0 + nxs] = B;
      }
    } else {
      for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx / N, j = idx - p * N;
        const double2 c = buf[p * N + j];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (2 * p + h >= nl) break;
          const int64_t g = rbase + (int64_t)(2 * p + h) * nx + j;
          const double ph = h == 0 ? c.x : c.y;
          if (a.phi) a.phi[g] = ph;
          if (a.v) {
            double e = 0.0, u = 0.0;
            if (a.rho) lda_xc(a.rho[g], e, u);
            a.v[g] = ph + u;
            if (a.exc) a.exc[g] = e;
          }
        }
      }
    }
    return;
  } else {
    double2* buf = lds;
    double2* twl = lds + TL * N;   // the twiddle table, read by every stage
    for (int m = threadIdx.x; m < N; m += blockDim.x) twl[m] = a.tw[m];
    // lines along y or z; tile = TL consecutive complex columns
    const int tiles_x = (nxc + TL - 1) / TL;
    const int other = blockIdx.x / tiles_x;   // z for the y axis, y for the z axis
    const int line0 = (blockIdx.x % tiles_x) * TL;
    const int nl = min(TL, nxc - line0);
    int64_t base, sj;
    if (a.axis == 1) {
      base = line0 + other * nxys;
      sj = nxs;
    } else {
      base = line0 + (int64_t)other * nxs;
      sj = nxys;
    }
    const int total = nl * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int j = idx / nl, l = idx - j * nl;
      buf[l * N + j] = a.work[base + l + j * sj];
    }
    __syncthreads();
    lds_fft(buf, a.ap, nl, twl, sign);
    if constexpr (MODE == kSolve) {
      // lines along z at fixed (kx = line0 + l, ky = other)
      for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int l = idx / N, kz = idx - l * N;
        const int kx = line0 + l, ky = other;
        double2 c = buf[l * N + kz];
        if (kx == 0 && ky == 0 && kz == 0) {
          if (a.mean) *a.mean = c.x / (double)a.npts;
          c = make_double2(0.0, 0.0);
        } else {
          const double g = a.scale / (a.lx[kx] + a.ly[ky] + a.lz[kz]);
          c = make_double2(c.x * g, c.y * g);
        }
        buf[l * N + kz] = c;
      }
      __syncthreads();
      lds_fft(buf, a.ap, nl, twl, 1.0);
    }
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int j = idx / nl, l = idx - j * nl;
      a.work[base + l + j * sj] = buf[l * N + j];
    }
  }
}

// Lines per tile: complex lines of the Y and Z passes, real lines (an even count) of the
// X passes, so that every tile's LDS stays within kLdsComplex complex values.
int pass_tl(int n, bool xpass) {
  if (xpass) return 2 * std::max(1, std::min(8, kLdsComplex / std::max(n, 1)));
  return std::max(1, std::min(16, kLdsComplex / std::max(n, 1)));
}

int pass_tiles(const sgq_potential* P, int axis, int tl) {
  const int nxc = P->n[0] / 2 + 1, ny = P->n[1], nz = P->n[2];
  if (axis == 0) return ((ny + tl - 1) / tl) * nz;
  if (axis == 1) return ((nxc + tl - 1) / tl) * nz;
  return ((nxc + tl - 1) / tl) * ny;
}

template <int MODE>
hipError_t launch_pass(const sgq_potential* P, int axis, PassArgs a, hipStream_t s) {
  constexpr bool XPASS = MODE == kFwdReal || MODE == kInvReal;
  a.ap = P->axis[axis];
  a.axis = axis;
  a.tl = pass_tl(P->axis[axis].n, XPASS);
  a.tw = P->d_tw[axis];
  const size_t lines = XPASS ? (size_t)a.tl / 2 : (size_t)a.tl;
  const size_t lds = sizeof(double2) * (lines + 1) * P->axis[axis].n;
  hipLaunchKernelGGL(fft_pass_kernel<MODE>, dim3(pass_tiles(P, axis, a.tl)), dim3(kPassBlock), lds,
                     s, a);
  return hipGetLastError();
}

// rho + b -> phi (and V = phi + u(rho), e_xc when v is given).
hipError_t solve(const sgq_potential* P, const double* src_a, const double* src_b,
                 const double* rho_xc, double* phi, double* v, double* exc, double* mean,
                 hipStream_t s) {
  PassArgs a{};
  a.nx = P->n[0];
  a.ny = P->n[1];
  a.nz = P->n[2];
  a.nxc = P->n[0] / 2 + 1;
  a.nxs = row_stride(P->n[0]);
  a.npts = P->npts;
  a.work = P->d_work;
  a.src_a = src_a;
  a.src_b = src_b;
  a.lx = P->d_lam[0];
  a.ly = P->d_lam[1];
  a.lz = P->d_lam[2];
  a.scale = -4.0 * M_PI / (double)P->npts;
  a.mean = mean;
  a.rho = rho_xc;
  a.phi = phi;
  a.v = v;
  a.exc = exc;
  hipError_t e = launch_pass<kFwdReal>(P, 0, a, s);
  if (e == hipSuccess) e = launch_pass<kFwd>(P, 1, a, s);
  if (e == hipSuccess) e = launch_pass<kSolve>(P, 2, a, s);
  if (e == hipSuccess) e = launch_pass<kInv>(P, 1, a, s);
  if (e == hipSuccess) e = launch_pass<kInvReal>(P, 0, a, s);
  return e;
}

bool factor_axis(int n, AxisPlan& ap) {
  ap.n = n;
  ap.nstages = 0;
  int m = n;
  while (m > 1) {
    int r = (m % 4 == 0) ? 4 : (m % 2 == 0) ? 2 : (m % 3 == 0) ? 3 : (m % 5 == 0) ? 5 : 0;
    if (r == 0 || ap.nstages == kMaxStages) return false;
    ap.radix[ap.nstages++] = r;
    m /= r;
  }
  return true;
}

void free_potential(sgq_potential* P) {
  (void)hipFree(P->d_work);
  for (int a = 0; a < 3; ++a) {
    (void)hipFree(P->d_tw[a]);
    (void)hipFree(P->d_lam[a]);
  }
  delete P;
}

}  // namespace
}  // namespace sgq

#define POT_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      sgq::free_potential(P);                                                            \
      return report_error(SGQ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    }                                                                                    \
  } while (0)

extern "C" int sgq_potential_create(const int32_t n[3], double h, sgq_potential** out) {
  if (!out) return report_error(SGQ_EINVAL, "out is null");
  *out = nullptr;
  if (!n) return report_error(SGQ_EINVAL, "n is null");
  if (!(h > 0.0) || !std::isfinite(h)) return report_error(SGQ_EINVAL, "h must be finite and > 0");
  AxisPlan ap[3];
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > kLdsComplex)
      return report_error(SGQ_EINVAL, "grid extents must be in [1, 1024]");
    if (!sgq::factor_axis(n[a], ap[a]))
      return report_error(SGQ_EINVAL, "grid extents must be products of 2, 3 and 5");
  }
  const int64_t npts = (int64_t)n[0] * n[1] * n[2];
  if (npts >= 2147483647LL) return report_error(SGQ_EINVAL, "grid has 2^31 or more points");
  sgq_potential* P = new sgq_potential;
  for (int a = 0; a < 3; ++a) {
    P->n[a] = n[a];
    P->axis[a] = ap[a];
  }
  P->npts = npts;
  P->h = h;
  POT_HIP(hipGetDevice(&P->device));
  POT_HIP(hipMalloc(&P->d_work, sizeof(double2) * (size_t)row_stride(n[0]) * n[1] * n[2]));
  // sixth-order FD weights of the Laplacian (per axis, over h^2)
  const double w[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};
  for (int a = 0; a < 3; ++a) {
    const int na = n[a];
    std::vector<double2> tw(na);
    std::vector<double> lam(na);
    for (int m = 0; m < na; ++m) {
      const double ang = 2.0 * M_PI * (double)m / (double)na;
      tw[m] = make_double2(std::cos(ang), -std::sin(ang));
      double l = w[0];
      for (int d = 1; d <= 3; ++d) l += 2.0 * w[d] * std::cos(2.0 * M_PI * (double)((int64_t)d * m % na) / na);
      lam[m] = l / (h * h);
    }
    POT_HIP(hipMalloc(&P->d_tw[a], sizeof(double2) * na));
    POT_HIP(hipMalloc(&P->d_lam[a], sizeof(double) * na));
    POT_HIP(hipMemcpy(P->d_tw[a], tw.data(), sizeof(double2) * na, hipMemcpyHostToDevice));
    POT_HIP(hipMemcpy(P->d_lam[a], lam.data(), sizeof(double) * na, hipMemcpyHostToDevice));
  }
  *out = P;
  return SGQ_OK;
}

extern "C" int sgq_potential_destroy(sgq_potential* pot) {
  if (!pot) return SGQ_OK;
  (void)hipSetDevice(pot->device);
  (void)hipDeviceSynchronize();
  sgq::free_potential(pot);
  return SGQ_OK;
}

extern "C" int sgq_poisson(sgq_potential* pot, const double* source, double* phi, double* mean,
                           void* stream) {
  if (!pot || !source || !phi) return report_error(SGQ_EINVAL, "null argument");
  hipError_t e = hipSetDevice(pot->device);
  if (e == hipSuccess)
    e = sgq::solve(pot, source, nullptr, nullptr, phi, nullptr, nullptr, mean, (hipStream_t)stream);
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  return SGQ_OK;
}

extern "C" int sgq_effective_potential(sgq_potential* pot, const double* rho, const double* b,
                                       double* v, double* phi, double* exc, double* mean,
                                       void* stream) {
  if (!pot || !rho || !v) return report_error(SGQ_EINVAL, "null argument");
  hipError_t e = hipSetDevice(pot->device);
  if (e == hipSuccess) e = sgq::solve(pot, rho, b, rho, phi, v, exc, mean, (hipStream_t)stream);
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  return SGQ_OK;
}

extern "C" int sgq_lda_xc(const double* rho, int64_t n, double* exc, double* vxc, void* stream) {
  if (n < 0) return report_error(SGQ_EINVAL, "n < 0");
  if (n == 0) return SGQ_OK;
  if (!rho || !vxc) return report_error(SGQ_EINVAL, "null argument");
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(sgq::xc_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, rho, n,
                     exc, vxc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  return SGQ_OK;
}
