// Q1 finite elements on the uniform grid (a = 1, zero Dirichlet data): the
// 1-D matrices M1 = (h/6) tridiag(1, 4, 1) and K1 = (1/h) tridiag(-1, 2, -1)
// and the tensor-product stencils of M and K built from them.
#pragma once

#include "common.hpp"

namespace pcop {

struct Q1W {
  double m0, m1;  // M1 diagonal and off-diagonal: 4h/6, h/6
  double k0, k1;  // K1 diagonal and off-diagonal: 2/h, -1/h
};

__host__ __device__ inline Q1W q1_weights(int nx) {
  const double h = 1.0 / (nx + 1);
  return Q1W{4.0 * h / 6.0, h / 6.0, 2.0 / h, -1.0 / h};
}

// (M u)_i and (K u)_i at grid point (c1, c2, c3) of one spatial slice u:
// sums along x1 first, then folded along x2 (and x3) with the mass weight on
// the axes that are not differentiated
template <int DIM>
__device__ __forceinline__ void q1_apply(const double* __restrict__ u, int c1, int c2, int c3, int nx,
                                         const Q1W& w, double& Mu, double& Ku) {
  double Pm = 0.0, Pk = 0.0;
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
    const int z = c3 + dz;
    if (DIM == 3 && (z < 0 || z >= nx)) continue;
    double Qm = 0.0, Qk = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = c2 + dy;
      if (yy < 0 || yy >= nx) continue;
      const double* row = u + ((size_t)z * nx + yy) * nx;
      const double ul = c1 > 0 ? row[c1 - 1] : 0.0;
      const double uc = row[c1];
      const double ur = c1 + 1 < nx ? row[c1 + 1] : 0.0;
      const double rm = w.m0 * uc + w.m1 * (ul + ur);
      const double rk = w.k0 * uc + w.k1 * (ul + ur);
      const double my = dy == 0 ? w.m0 : w.m1, ky = dy == 0 ? w.k0 : w.k1;
      Qm += my * rm;
      Qk += my * rk + ky * rm;
    }
    if (DIM == 3) {
      const double mz = dz == 0 ? w.m0 : w.m1, kz = dz == 0 ? w.k0 : w.k1;
      Pm += mz * Qm;
      Pk += mz * Qk + kz * Qm;
    } else {
      Pm = Qm;
      Pk = Qk;
    }
  }
  Mu = Pm;
  Ku = Pk;
}

}  // namespace pcop
