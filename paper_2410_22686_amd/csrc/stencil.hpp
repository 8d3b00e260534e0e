// E u = (I + tau K) u at one grid point, shared by the KKT matvec and the
// post-solve residual.
#pragma once

#include "common.hpp"

namespace pcop {

// E u at point i with E = I + tau K.  Constant coefficient: E = ediag I +
// eoff * (sum of existing neighbours).  Variable coefficient: per-point
// values ecoef[0][i] (diagonal) and ecoef[1 + 2d][i] / ecoef[2 + 2d][i]
// (the minus / plus neighbour along axis d, zero at the boundary).
template <int DIM, bool VAR>
__device__ __forceinline__ double apply_E(const double* __restrict__ u, int i, int c1, int c2, int c3,
                                          int nx, int m, const double* __restrict__ ecoef,
                                          double ediag, double eoff) {
  const int s2 = nx, s3 = nx * nx;
  if (!VAR) {
    double nb = 0.0;
    if (c1 > 0) nb += u[i - 1];
    if (c1 < nx - 1) nb += u[i + 1];
    if (c2 > 0) nb += u[i - s2];
    if (c2 < nx - 1) nb += u[i + s2];
    if (DIM == 3) {
      if (c3 > 0) nb += u[i - s3];
      if (c3 < nx - 1) nb += u[i + s3];
    }
    return ediag * u[i] + eoff * nb;
  } else {
    double acc = ecoef[i] * u[i];
    if (c1 > 0) acc += ecoef[(size_t)1 * m + i] * u[i - 1];
    if (c1 < nx - 1) acc += ecoef[(size_t)2 * m + i] * u[i + 1];
    if (c2 > 0) acc += ecoef[(size_t)3 * m + i] * u[i - s2];
    if (c2 < nx - 1) acc += ecoef[(size_t)4 * m + i] * u[i + s2];
    if (DIM == 3) {
      if (c3 > 0) acc += ecoef[(size_t)5 * m + i] * u[i - s3];
      if (c3 < nx - 1) acc += ecoef[(size_t)6 * m + i] * u[i + s3];
    }
    return acc;
  }
}

// the stencil weights of E at one point, loaded once for a march over time
// levels: diagonal, and minus / plus neighbour along each axis
struct StencilW {
  double d, lo[3], hi[3];
};

template <int DIM, bool VAR>
__device__ __forceinline__ StencilW load_stencil(int i, int m, const double* __restrict__ ecoef, double ediag,
                                                 double eoff) {
  StencilW w;
  if (!VAR) {
    w.d = ediag;
#pragma unroll
    for (int a = 0; a < 3; ++a) w.lo[a] = w.hi[a] = eoff;
  } else {
    w.d = ecoef[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      w.lo[a] = (a < DIM) ? ecoef[(size_t)(1 + 2 * a) * m + i] : 0.0;
      w.hi[a] = (a < DIM) ? ecoef[(size_t)(2 + 2 * a) * m + i] : 0.0;
    }
  }
  return w;
}

// E u at point i with preloaded weights (same sums, same order as apply_E).
// Every neighbour is loaded (a point on the boundary reads itself instead)
// and a missing one adds zero, so no branches surround the loads and they
// can all be issued together; the sums equal apply_E's (x + 0 = x).
template <int DIM, bool VAR>
__device__ __forceinline__ double apply_E_w(const double* __restrict__ u, int i, int c1, int c2, int c3, int nx,
                                            const StencilW& w) {
  const int s2 = nx, s3 = nx * nx;
  const bool h1 = c1 > 0, g1 = c1 < nx - 1, h2 = c2 > 0, g2 = c2 < nx - 1;
  const bool h3 = DIM == 3 && c3 > 0, g3 = DIM == 3 && c3 < nx - 1;
  const double uc = u[i];
  const double m1 = u[h1 ? i - 1 : i], p1 = u[g1 ? i + 1 : i];
  const double m2 = u[h2 ? i - s2 : i], p2 = u[g2 ? i + s2 : i];
  double m3 = 0.0, p3 = 0.0;
  if (DIM == 3) {
    m3 = u[h3 ? i - s3 : i];
    p3 = u[g3 ? i + s3 : i];
  }
  if (!VAR) {
    double nb = 0.0;
    nb += h1 ? m1 : 0.0;
    nb += g1 ? p1 : 0.0;
    nb += h2 ? m2 : 0.0;
    nb += g2 ? p2 : 0.0;
    if (DIM == 3) {
      nb += h3 ? m3 : 0.0;
      nb += g3 ? p3 : 0.0;
    }
    return w.d * uc + w.lo[0] * nb;
  } else {
    double acc = w.d * uc;
    acc += w.lo[0] * (h1 ? m1 : 0.0);
    acc += w.hi[0] * (g1 ? p1 : 0.0);
    acc += w.lo[1] * (h2 ? m2 : 0.0);
    acc += w.hi[1] * (g2 ? p2 : 0.0);
    if (DIM == 3) {
      acc += w.lo[2] * (h3 ? m3 : 0.0);
      acc += w.hi[2] * (g3 ? p3 : 0.0);
    }
    return acc;
  }
}

}  // namespace pcop
