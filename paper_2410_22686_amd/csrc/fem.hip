// Finite-element form of the KKT system (Section 1 with M_m != I): bilinear
// (2-D) or trilinear (3-D) elements on the uniform grid, a = 1, zero
// Dirichlet data.  The mass and stiffness matrices are tensor products of
// the 1-D matrices M1 = (h/6) tridiag(1, 4, 1) and K1 = (1/h) tridiag(-1, 2, -1):
//   M = M1 (x) M1 (x) M1,  K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1
// (2-D: drop one factor), so both act as 9-point (27-point) stencils.
#include <algorithm>

#include "common.hpp"
#include "fem.hpp"
#include "launch.hpp"

namespace pcop {

// y = c - s A x (c != nullptr) or y = s A x with A of eq. matrix_A (sgn = 1)
// or A^T (sgn = -1), E = M + tau K:
//   y_1^j = alpha M x_1^j + sgn (E x_2^j - M x_2^{j+1}),
//   y_2^j = alpha M x_2^j - sgn (E x_1^j - M x_1^{j-1}),  x^0 = x^{n+1} = 0.
// One thread per spatial point and chunk of time levels; the products with
// M x_2^{j+1} and M x_1^j are carried to the next level.  JC > 0: chunks of
// JC levels (compile time, unrolled); JC = 0: jchunk levels at run time.
template <int DIM, int JC>
__global__ void __launch_bounds__(256) kkt_fem_kernel(Geo g, const double* __restrict__ x, double* __restrict__ y,
                                                      const double* __restrict__ c, const double* __restrict__ alpha,
                                                      const double* __restrict__ xscale, int xs_stride,
                                                      const int* __restrict__ active, double sgn, int jchunk) {
  // logical block (x: spatial tile, y: time chunk, z: member) in XCD-aware
  // order, so that tiles sharing neighbour rows run on one XCD's L2
  const int total = gridDim.x * gridDim.y * gridDim.z;
  const int hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int lg = xcd_remap(hw, total);
  const int bx = lg % gridDim.x;
  const int by = (lg / gridDim.x) % gridDim.y;
  const int b = lg / (gridDim.x * gridDim.y);
  if (active && !active[b]) return;
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= g.m) return;
  const int nx = g.nx, n = g.n, m = g.m;
  const int c1 = i % nx, c2 = (i / nx) % nx, c3 = (DIM == 3) ? i / (nx * nx) : 0;
  const int j0 = by * jchunk;
  const int j1 = min(n, j0 + jchunk);
  const Q1W w = q1_weights(nx);
  const double a = alpha[b];
  const double s = xscale ? xscale[(size_t)b * xs_stride] : 1.0;
  const size_t mb = (size_t)b * (size_t)g.vs;
  const double* x1 = x + mb;
  const double* x2 = x + mb + (size_t)n * m;
  double* y1 = y + mb;
  double* y2 = y + mb + (size_t)n * m;
  const double* cc1 = c ? c + mb : nullptr;
  const double* cc2 = c ? c + mb + (size_t)n * m : nullptr;
  // slices are addressed from their first point; q1_apply adds the row offset
  auto slice = [&](const double* base, int j) { return base + (size_t)j * m; };
  double Mx1prev = 0.0, dummy = 0.0;
  if (j0 > 0) q1_apply<DIM>(slice(x1, j0 - 1), c1, c2, c3, nx, w, Mx1prev, dummy);
  double Mx2c, Kx2c;
  q1_apply<DIM>(slice(x2, j0), c1, c2, c3, nx, w, Mx2c, Kx2c);
  auto level = [&](int j, bool has_next) {
    double Mx1, Kx1;
    q1_apply<DIM>(slice(x1, j), c1, c2, c3, nx, w, Mx1, Kx1);
    double Mx2n = 0.0, Kx2n = 0.0;
    if (has_next) q1_apply<DIM>(slice(x2, j + 1), c1, c2, c3, nx, w, Mx2n, Kx2n);
    double r1 = a * Mx1 + sgn * (Mx2c + g.tau * Kx2c - Mx2n);
    double r2 = a * Mx2c - sgn * (Mx1 + g.tau * Kx1 - Mx1prev);
    r1 *= s;
    r2 *= s;
    const size_t o = (size_t)j * m + i;
    if (c) {
      r1 = cc1[o] - r1;
      r2 = cc2[o] - r2;
    }
    y1[o] = r1;
    y2[o] = r2;
    Mx1prev = Mx1;
    Mx2c = Mx2n;
    Kx2c = Kx2n;
  };
  if (JC > 0 && j0 + JC < n) {
    // a full chunk followed by another level: straight-line code, so the
    // stencil loads of every level can be issued up front
#pragma unroll
    for (int jj = 0; jj < (JC > 0 ? JC : 1); ++jj) level(j0 + jj, true);
  } else {
    for (int j = j0; j < j1; ++j) level(j, j + 1 < n);
  }
}

// 2-D version with LDS tiles: a block owns PT * 256 consecutive points and
// marches over a chunk of levels; per level the segments of x_1^j and
// x_2^{j+1} covering its points and one grid row plus one point on either
// side are staged in LDS (zero outside the grid, which supplies the
// Dirichlet zeros above the first and below the last row), and the 9-point
// stencils read LDS, with the neighbours across a row end masked by x1.
// Same operations per point as kkt_fem_kernel<2>.
template <int PT>
__global__ void __launch_bounds__(256) kkt_fem_lds_kernel(Geo g, const double* __restrict__ x, double* __restrict__ y,
                                                          const double* __restrict__ c,
                                                          const double* __restrict__ alpha,
                                                          const double* __restrict__ xscale, int xs_stride,
                                                          const int* __restrict__ active, double sgn, int jchunk) {
  extern __shared__ double sm[];
  const int total = gridDim.x * gridDim.y * gridDim.z;
  const int hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int lg = xcd_remap(hw, total);
  const int bx = lg % gridDim.x;
  const int by = (lg / gridDim.x) % gridDim.y;
  const int b = lg / (gridDim.x * gridDim.y);
  if (active && !active[b]) return;
  const int nx = g.nx, n = g.n, m = g.m;
  constexpr int TP = 256 * PT;
  const int i0 = bx * TP;
  const int H = nx + 1;          // halo: one row and one point
  const int seg = TP + 2 * H;
  double* s1 = sm;
  double* s2 = sm + seg;
  const int j0 = by * jchunk;
  const int j1 = min(n, j0 + jchunk);
  const Q1W w = q1_weights(nx);
  const double a = alpha[b];
  const double s = xscale ? xscale[(size_t)b * xs_stride] : 1.0;
  const size_t mb = (size_t)b * (size_t)g.vs;
  const double* x1 = x + mb;
  const double* x2 = x + mb + (size_t)n * m;
  double* y1 = y + mb;
  double* y2 = y + mb + (size_t)n * m;
  const double* cc1 = c ? c + mb : nullptr;
  const double* cc2 = c ? c + mb + (size_t)n * m : nullptr;
  auto stage = [&](double* dst, const double* src) {
    for (int t = threadIdx.x; t < seg; t += 256) {
      const int gi = i0 - H + t;
      dst[t] = (gi >= 0 && gi < m) ? src[gi] : 0.0;
    }
  };
  auto stencil = [&](const double* sg, int p, double& Mu, double& Ku) {
    const int i = i0 + threadIdx.x + 256 * p;
    const int li = H + threadIdx.x + 256 * p;
    const int c1 = i % nx;
    double Qm = 0.0, Qk = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const double* r = sg + li + dy * nx;
      const double ul = c1 > 0 ? r[-1] : 0.0;
      const double uc = r[0];
      const double ur = c1 + 1 < nx ? r[1] : 0.0;
      const double rm = w.m0 * uc + w.m1 * (ul + ur);
      const double rk = w.k0 * uc + w.k1 * (ul + ur);
      const double my = dy == 0 ? w.m0 : w.m1, ky = dy == 0 ? w.k0 : w.k1;
      Qm += my * rm;
      Qk += my * rk + ky * rm;
    }
    Mu = Qm;
    Ku = Qk;
  };
  double Mx1prev[PT], Mx2c[PT], Kx2c[PT];
  if (j0 > 0) stage(s1, x1 + (size_t)(j0 - 1) * m);
  stage(s2, x2 + (size_t)j0 * m);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    double dummy;
    Mx1prev[p] = 0.0;
    if (j0 > 0) stencil(s1, p, Mx1prev[p], dummy);
    stencil(s2, p, Mx2c[p], Kx2c[p]);
  }
  // the segments of the next level are fetched into registers while the
  // current level's stencils run (NS slots: seg <= 256 NS for nx <= 511)
  constexpr int NS = (TP + 2 * 512 + 255) / 256;
  double p1[NS], p2[NS];
  auto fetch = [&](int j) {
    const double* a1 = x1 + (size_t)j * m;
    const double* a2 = x2 + (size_t)(j + 1) * m;
    const bool nxt = j + 1 < n;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int t = threadIdx.x + 256 * q;
      const int gi = i0 - H + t;
      const bool in = t < seg && gi >= 0 && gi < m;
      p1[q] = in ? a1[gi] : 0.0;
      p2[q] = (in && nxt) ? a2[gi] : 0.0;
    }
  };
  fetch(j0);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();
    const bool has_next = j + 1 < n;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int t = threadIdx.x + 256 * q;
      if (t < seg) {
        s1[t] = p1[q];
        s2[t] = p2[q];
      }
    }
    __syncthreads();
    if (j + 1 < j1) fetch(j + 1);
    const size_t o = (size_t)j * m;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      double Mx1, Kx1, Mx2n = 0.0, Kx2n = 0.0;
      stencil(s1, p, Mx1, Kx1);
      if (has_next) stencil(s2, p, Mx2n, Kx2n);
      double r1 = a * Mx1 + sgn * (Mx2c[p] + g.tau * Kx2c[p] - Mx2n);
      double r2 = a * Mx2c[p] - sgn * (Mx1 + g.tau * Kx1 - Mx1prev[p]);
      const int i = i0 + threadIdx.x + 256 * p;
      if (i < m) {
        r1 *= s;
        r2 *= s;
        if (c) {
          r1 = cc1[o + i] - r1;
          r2 = cc2[o + i] - r2;
        }
        y1[o + i] = r1;
        y2[o + i] = r2;
      }
      Mx1prev[p] = Mx1;
      Mx2c[p] = Mx2n;
      Kx2c[p] = Kx2n;
    }
  }
}

// y = M x on spatial slices: slice q of group k = q / spg starts at
// x + k sgs + (q mod spg) m and y + k dgs + (q mod spg) m
template <int DIM>
__global__ void __launch_bounds__(256) mass_apply_kernel(Geo g, const double* __restrict__ x, long long sgs,
                                                         double* __restrict__ y, long long dgs, int spg,
                                                         long long nslices) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.m) return;
  const int nx = g.nx, m = g.m;
  const int c1 = i % nx, c2 = (i / nx) % nx, c3 = (DIM == 3) ? i / (nx * nx) : 0;
  const Q1W w = q1_weights(nx);
  for (long long q = blockIdx.y; q < nslices; q += gridDim.y) {
    const long long k = q / spg, r = q - k * spg;
    const double* u = x + k * sgs + r * (long long)m;
    double Mu, Ku;
    q1_apply<DIM>(u, c1, c2, c3, nx, w, Mu, Ku);
    y[k * dgs + r * (long long)m + i] = Mu;
  }
}

void launch_kkt_fem(const Geo& g, const double* x, double* y, const double* c, const double* alpha,
                    const double* xscale, int xs_stride, const int* active, bool transpose, hipStream_t st) {
  // 16 levels per thread with a run-time loop: unrolled 8-level chunks
  // (JC = 8) measured slower on the 2-D nx = 255, n = 255 workload
  constexpr int jc = 16;
  const dim3 grid((g.m + 255) / 256, (g.n + jc - 1) / jc, g.B);
  const double sgn = transpose ? -1.0 : 1.0;
  if (g.dim == 2 && g.nx <= 511) {
    // LDS tiles (the prefetch slots cover a halo of up to 512 points)
    constexpr int PT = 4;
    const dim3 gl((g.m + 256 * PT - 1) / (256 * PT), (g.n + jc - 1) / jc, g.B);
    const size_t lds = 2 * sizeof(double) * (256 * PT + 2 * (size_t)(g.nx + 1));
    kkt_fem_lds_kernel<PT><<<gl, 256, lds, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn, jc);
  } else if (g.dim == 2) {
    kkt_fem_kernel<2, 0><<<grid, 256, 0, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn, jc);
  } else {
    kkt_fem_kernel<3, 0><<<grid, 256, 0, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn, jc);
  }
}

void launch_mass_apply(const Geo& g, const double* x, long long sgs, double* y, long long dgs, int spg,
                       int ngroups, hipStream_t st) {
  const long long ns = (long long)spg * ngroups;
  if (ns <= 0) return;
  const dim3 grid((g.m + 255) / 256, (unsigned)std::min<long long>(ns, 65535));
  if (g.dim == 2)
    mass_apply_kernel<2><<<grid, 256, 0, st>>>(g, x, sgs, y, dgs, spg, ns);
  else
    mass_apply_kernel<3><<<grid, 256, 0, st>>>(g, x, sgs, y, dgs, spg, ns);
}

}  // namespace pcop
