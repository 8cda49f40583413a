// Gauss rule of a symmetric tridiagonal (Golub-Welsch): eigenvalues and the first
// component of each eigenvector, by implicit-shift QR sweeps with Wilkinson shifts.
// Written for one thread; the arrays may live in LDS or global memory.
// SGQ_HD marks it for both the host and the device in the HIP sources (sgq_common.h); the
// host-only build defines it empty.
#pragma once

#include <cmath>

#ifndef SGQ_HD
#error "define SGQ_HD (include sgq_common.h) before tridiag.h"
#endif

namespace sgq {

// a[0..K)   in: diagonal, out: eigenvalues (unordered)
// b[0..K-1) in: off-diagonal (destroyed)
// z[0..K)   out: first row of the eigenvector matrix (weights are z^2)
// Z         optional [K*K] (row-major, Z[i*ld + k] = component i of eigenvector k): if
//           non-null the full eigenvector matrix is accumulated as well.
// Returns false if an unreduced block failed to converge in 40*K sweeps.
template <typename PA, typename PZ = double*>
SGQ_HD inline bool tridiag_gauss(PA a, PA b, PA z, int K, PZ Z = nullptr,
                                              int ld = 0) {
  for (int k = 0; k < K; ++k) z[k] = (k == 0) ? 1.0 : 0.0;
  if (Z) {
    for (int i = 0; i < K; ++i)
      for (int k = 0; k < K; ++k) Z[i * ld + k] = (i == k) ? 1.0 : 0.0;
  }
  const double eps = 2.220446049250313e-16;
  int m = K - 1;
  int sweeps = 0;
  while (m > 0) {
    // deflate negligible couplings at the bottom of the active block
    if (fabs(b[m - 1]) <= eps * (fabs(a[m - 1]) + fabs(a[m]))) {
      b[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && fabs(b[l - 1]) > eps * (fabs(a[l - 1]) + fabs(a[l]))) --l;
    if (l > 0) b[l - 1] = 0.0;
    if (++sweeps > 40 * K) return false;
    // Wilkinson shift from the trailing 2x2 block
    double d = 0.5 * (a[m - 1] - a[m]);
    double bm = b[m - 1];
    double den = d + copysign(hypot(d, bm), d == 0.0 ? 1.0 : d);
    double shift = a[m] - bm * bm / den;
    double x = a[l] - shift;
    double y = b[l];
    for (int k = l; k < m; ++k) {
      // rotation in the (k, k+1) plane that zeroes y against x
      double r = hypot(x, y);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -y / r;
      }
      if (k > l) b[k - 1] = r;
      double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak - 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak - ak1) + (c * c - s * s) * bk;
      double bulge = 0.0;
      if (k + 1 < m) {
        bulge = -s * b[k + 1];
        b[k + 1] = c * b[k + 1];
      }
      double zk = z[k], zk1 = z[k + 1];
      z[k] = c * zk - s * zk1;
      z[k + 1] = s * zk + c * zk1;
      if (Z) {
        for (int i = 0; i < K; ++i) {
          double u0 = Z[i * ld + k], u1 = Z[i * ld + k + 1];
          Z[i * ld + k] = c * u0 - s * u1;
          Z[i * ld + k + 1] = s * u0 + c * u1;
        }
      }
      x = b[k];
      y = bulge;
    }
  }
  return true;
}

}  // namespace sgq
