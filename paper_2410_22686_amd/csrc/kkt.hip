// KKT matvec (eq. matrix_A) and the element-wise maps between the data
// (g, f, y0) and the all-at-once vectors (eq. main_system_before,
// eq. main_system).  All FP64 and HBM-bound.
#include "common.hpp"
#include "launch.hpp"
#include "stencil.hpp"

namespace pcop {

// y = c - s A x  (c != nullptr)  or  y = s A x, with A or A^T (sgn = -1).
// One thread per spatial point, marching over a chunk of time blocks so that
// x1^{j-1} and x2^{j+1} are loaded once.  JC > 0: the chunk is JC levels, a
// compile-time count, so the loop unrolls and the loads of every level are
// issued before the first result is formed; JC = 0: jchunk levels at run time.
template <int DIM, bool VAR, int JC>
__global__ void __launch_bounds__(256) kkt_apply_kernel(
    Geo g, const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ c,
    const double* __restrict__ alpha, const double* __restrict__ xscale, int xs_stride,
    const int* __restrict__ active, double sgn, const double* __restrict__ ecoef, double ediag,
    double eoff, int jchunk) {
  // logical block (x: spatial tile, y: time chunk, z: member) in XCD-friendly order
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
  const double a = alpha[b];
  const double s = xscale ? xscale[(size_t)b * xs_stride] : 1.0;
  const size_t mb = (size_t)b * (size_t)g.vs;
  const double* x1 = x + mb;
  const double* x2 = x + mb + (size_t)n * m;
  double* y1 = y + mb;
  double* y2 = y + mb + (size_t)n * m;
  const double* cc1 = c ? c + mb : nullptr;
  const double* cc2 = c ? c + mb + (size_t)n * m : nullptr;

  const StencilW sw = load_stencil<DIM, VAR>(i, m, ecoef, ediag, eoff);
  double x1prev = (j0 > 0) ? x1[(size_t)(j0 - 1) * m + i] : 0.0;
  double x2cur = x2[(size_t)j0 * m + i];
  // one time level: block row 1 alpha x1 + T^T x2, block row 2 -T x1 + alpha x2
  auto level = [&](int j, double x2next) {
    const size_t o = (size_t)j * m;
    const double x1cur = x1[o + i];
    const double ex2 = apply_E_w<DIM, VAR>(x2 + o, i, c1, c2, c3, nx, sw);
    const double ex1 = apply_E_w<DIM, VAR>(x1 + o, i, c1, c2, c3, nx, sw);
    double r1 = a * x1cur + sgn * (ex2 - x2next);
    double r2 = a * x2cur - sgn * (ex1 - x1prev);
    r1 *= s;
    r2 *= s;
    if (c) {
      r1 = cc1[o + i] - r1;
      r2 = cc2[o + i] - r2;
    }
    y1[o + i] = r1;
    y2[o + i] = r2;
    x1prev = x1cur;
    x2cur = x2next;
  };
  if (JC > 0 && j0 + JC < n) {
    // a full chunk followed by another level: no guards, so every load of
    // the chunk can be issued up front
#pragma unroll
    for (int jj = 0; jj < (JC > 0 ? JC : 1); ++jj) level(j0 + jj, x2[(size_t)(j0 + jj + 1) * m + i]);
  } else {
    for (int j = j0; j < j1; ++j) level(j, (j + 1 < n) ? x2[(size_t)(j + 1) * m + i] : 0.0);
  }
}

// E u at a staged point: the value and its in-plane neighbours from the LDS
// tile s (local index li, row length nx), the neighbours across planes (3-D)
// from the level's global values u.  Same selects and sums as apply_E_w.
template <int DIM, bool VAR>
__device__ __forceinline__ double apply_E_lds(const double* s, int li, const double* __restrict__ u, int i, int c1,
                                              int c2, int c3, int nx, const StencilW& w) {
  const bool h1 = c1 > 0, g1 = c1 < nx - 1, h2 = c2 > 0, g2 = c2 < nx - 1;
  const bool h3 = DIM == 3 && c3 > 0, g3 = DIM == 3 && c3 < nx - 1;
  const double uc = s[li];
  const double m1 = s[li - 1], p1 = s[li + 1];
  const double m2 = s[li - nx], p2 = s[li + nx];
  double m3 = 0.0, p3 = 0.0;
  if (DIM == 3) {
    const int s3 = nx * nx;
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

// LDS-tiled matvec: a block owns TS = 256 PT consecutive spatial points and
// a chunk of time levels.  Per level, x1 and x2 over the tile and nx points
// on either side (every in-plane neighbour) are staged in LDS with
// coalesced loads, the next level's being fetched into registers
// meanwhile; the stencils then read LDS.  Block row 1 of level j needs
// x2^{j+1}, so it is completed at level j + 1 from that level's staged
// values.  The operations per element are those of kkt_apply_kernel.
template <int DIM, bool VAR, int PT, int HQ>
__global__ void __launch_bounds__(256) kkt_lds_kernel(
    Geo g, const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ c,
    const double* __restrict__ alpha, const double* __restrict__ xscale, int xs_stride,
    const int* __restrict__ active, double sgn, const double* __restrict__ ecoef, double ediag,
    double eoff, int jchunk) {
  constexpr int NT = 256, TS = NT * PT;
  constexpr int QW = PT + HQ;  // staging slots per thread: TS + 2 nx <= QW NT (nx <= 128 HQ)
  extern __shared__ double kkt_sm[];
  const int total = gridDim.x * gridDim.y * gridDim.z;
  const int hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int lg = xcd_remap(hw, total);
  const int bx = lg % gridDim.x;
  const int by = (lg / gridDim.x) % gridDim.y;
  const int b = lg / (gridDim.x * gridDim.y);
  if (active && !active[b]) return;
  const int nx = g.nx, n = g.n, m = g.m, H = nx;
  const int W = TS + 2 * H;
  double* s1 = kkt_sm;
  double* s2 = kkt_sm + W;
  const int i0 = bx * TS;
  const int j0 = by * jchunk;
  const int j1 = min(n, j0 + jchunk);
  const double a = alpha[b];
  const double sc = xscale ? xscale[(size_t)b * xs_stride] : 1.0;
  const size_t mb = (size_t)b * (size_t)g.vs;
  const double* x1 = x + mb;
  const double* x2 = x + mb + (size_t)n * m;
  double* y1 = y + mb;
  double* y2 = y + mb + (size_t)n * m;
  const double* cc1 = c ? c + mb : nullptr;
  const double* cc2 = c ? c + mb + (size_t)n * m : nullptr;

  StencilW sw[PT];
  double x1prev[PT], pex2[PT], px1[PT];
  int cr1[PT], cr2[PT], cr3[PT];  // grid coordinates of the thread's points
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    const int i = i0 + threadIdx.x + NT * r;
    const int ii = i < m ? i : 0;
    cr1[r] = ii % nx;
    cr2[r] = (ii / nx) % nx;
    cr3[r] = (DIM == 3) ? ii / (nx * nx) : 0;
    sw[r] = load_stencil<DIM, VAR>(ii, m, ecoef, ediag, eoff);
    x1prev[r] = (j0 > 0 && i < m) ? x1[(size_t)(j0 - 1) * m + i] : 0.0;
    pex2[r] = px1[r] = 0.0;
  }
  double p1[QW], p2[QW];
  auto fetch = [&](int j) {
    const size_t o = (size_t)j * m;
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int e = threadIdx.x + NT * q;
      const int gi = i0 - H + e;
      const bool ok = e < W && gi >= 0 && gi < m;
      p1[q] = ok ? x1[o + gi] : 0.0;
      p2[q] = ok ? x2[o + gi] : 0.0;
    }
  };
  // block row 1 of level j: alpha x1 + T^T x2 with x2^{j+1} = x2n
  auto finish_row1 = [&](int r, int j, int i, double x2n) {
    double r1 = a * px1[r] + sgn * (pex2[r] - x2n);
    r1 *= sc;
    if (c) r1 = cc1[(size_t)j * m + i] - r1;
    y1[(size_t)j * m + i] = r1;
  };
  if (j0 < j1) fetch(j0);
  for (int j = j0; j < j1; ++j) {
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int e = threadIdx.x + NT * q;
      if (e < W) {
        s1[e] = p1[q];
        s2[e] = p2[q];
      }
    }
    __syncthreads();
    if (j + 1 < j1) fetch(j + 1);
    const size_t o = (size_t)j * m;
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int i = i0 + threadIdx.x + NT * r;
      if (i < m) {
        const int li = H + threadIdx.x + NT * r;
        const int c1 = cr1[r], c2 = cr2[r], c3 = cr3[r];
        const double x2c = s2[li];
        if (j > j0) finish_row1(r, j - 1, i, x2c);
        const double ex2 = apply_E_lds<DIM, VAR>(s2, li, x2 + o, i, c1, c2, c3, nx, sw[r]);
        const double ex1 = apply_E_lds<DIM, VAR>(s1, li, x1 + o, i, c1, c2, c3, nx, sw[r]);
        const double x1c = s1[li];
        // block row 2: -T x1 + alpha x2
        double r2 = a * x2c - sgn * (ex1 - x1prev[r]);
        r2 *= sc;
        if (c) r2 = cc2[o + i] - r2;
        y2[o + i] = r2;
        pex2[r] = ex2;
        px1[r] = x1c;
        x1prev[r] = x1c;
      }
    }
    __syncthreads();
  }
  if (j0 < j1) {
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int i = i0 + threadIdx.x + NT * r;
      if (i < m) finish_row1(r, j1 - 1, i, (j1 < n) ? x2[(size_t)j1 * m + i] : 0.0);
    }
  }
}

// The 2-D matvec with the residual form a compile-time switch and no store
// behind a per-lane branch (operations per element as in kkt_lds_kernel).
// A lane past the last point repeats the last point, the first level is
// peeled off the level loop, and the staging loads use clamped indices
// with the zeros outside the grid applied at the LDS commit; the wait for
// the next level's prefetched values then leaves this level's stores in
// flight.  (In 3-D the same structure took more registers, one wave per
// SIMD fewer, and ran slower; kkt_lds_kernel serves 3-D.)
template <bool VAR, int PT, int HQ, bool RES>
__global__ void __launch_bounds__(256) kkt_lds2_kernel(
    Geo g, const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ c,
    const double* __restrict__ alpha, const double* __restrict__ xscale, int xs_stride,
    const int* __restrict__ active, double sgn, const double* __restrict__ ecoef, double ediag,
    double eoff, int jchunk) {
  constexpr int DIM = 2, NT = 256, TS = NT * PT;
  constexpr int QW = PT + HQ;  // staging slots per thread: TS + 2 nx <= QW NT (nx <= 128 HQ)
  extern __shared__ double kkt_sm[];
  const int total = gridDim.x * gridDim.y * gridDim.z;
  const int hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int lg = xcd_remap(hw, total);
  const int bx = lg % gridDim.x;
  const int by = (lg / gridDim.x) % gridDim.y;
  const int b = lg / (gridDim.x * gridDim.y);
  if (active && !active[b]) return;
  const int nx = g.nx, n = g.n, m = g.m, H = nx;
  const int W = TS + 2 * H;
  double* s1 = kkt_sm;
  double* s2 = kkt_sm + W;
  const int i0 = bx * TS;
  const int j0 = by * jchunk;
  const int j1 = min(n, j0 + jchunk);
  if (j0 >= j1) return;
  const double a = alpha[b];
  const double sc = xscale ? xscale[(size_t)b * xs_stride] : 1.0;
  const size_t mb = (size_t)b * (size_t)g.vs;
  const double* x1 = x + mb;
  const double* x2 = x + mb + (size_t)n * m;
  double* y1 = y + mb;
  double* y2 = y + mb + (size_t)n * m;
  const double* cc1 = RES ? c + mb : nullptr;
  const double* cc2 = RES ? c + mb + (size_t)n * m : nullptr;

  // A lane past the last point takes the last point (m - 1) and repeats its
  // owner's arithmetic and stores (the same values to the same places), so
  // that no store sits behind a per-lane branch: the wait for the next
  // level's prefetched values then leaves this level's stores in flight.
  StencilW sw[PT];
  double x1prev[PT], pex2[PT], px1[PT];
  int cr1[PT], cr2[PT], cr3[PT];  // grid coordinates of the thread's points
  int ip[PT];                      // the thread's points (clamped)
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    const int ii = min(i0 + threadIdx.x + NT * r, m - 1);
    ip[r] = ii;
    cr1[r] = ii % nx;
    cr2[r] = (ii / nx) % nx;
    cr3[r] = 0;
    sw[r] = load_stencil<DIM, VAR>(ii, m, ecoef, ediag, eoff);
    x1prev[r] = (j0 > 0) ? x1[(size_t)(j0 - 1) * m + ii] : 0.0;
    pex2[r] = px1[r] = 0.0;
  }
  // staging slot e holds point i0 - H + e (zero outside the grid); the
  // loads use a clamped in-bounds index and the zeros are applied when the
  // values are committed to LDS, so no select waits on a load
  double p1[QW], p2[QW];
  auto fetch = [&](int j) {
    const size_t o = (size_t)j * m;
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int gi = min(max(i0 - H + (int)threadIdx.x + NT * q, 0), m - 1);
      p1[q] = x1[o + gi];
      p2[q] = x2[o + gi];
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int e = threadIdx.x + NT * q;
      const int gi = i0 - H + e;
      const bool ok = gi >= 0 && gi < m;
      if (e < W) {
        s1[e] = ok ? p1[q] : 0.0;
        s2[e] = ok ? p2[q] : 0.0;
      }
    }
  };
  // block row 1 of level j: alpha x1 + T^T x2 with x2^{j+1} = x2n
  auto finish_row1 = [&](int r, int j, int i, double x2n) {
    double r1 = a * px1[r] + sgn * (pex2[r] - x2n);
    r1 *= sc;
    if constexpr (RES) r1 = cc1[(size_t)j * m + i] - r1;
    y1[(size_t)j * m + i] = r1;
  };
  // level j's stencils; row 1 of level j - 1 is completed when FIRST is false
  auto level = [&](int j, bool first) {
    const size_t o = (size_t)j * m;
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int i = ip[r];
      const int li = H + (i - i0);
      const int c1 = cr1[r], c2 = cr2[r], c3 = cr3[r];
      const double x2c = s2[li];
      if (!first) finish_row1(r, j - 1, i, x2c);
      const double ex2 = apply_E_lds<DIM, VAR>(s2, li, x2 + o, i, c1, c2, c3, nx, sw[r]);
      const double ex1 = apply_E_lds<DIM, VAR>(s1, li, x1 + o, i, c1, c2, c3, nx, sw[r]);
      const double x1c = s1[li];
      // block row 2: -T x1 + alpha x2
      double r2 = a * x2c - sgn * (ex1 - x1prev[r]);
      r2 *= sc;
      if constexpr (RES) r2 = cc2[o + i] - r2;
      y2[o + i] = r2;
      pex2[r] = ex2;
      px1[r] = x1c;
      x1prev[r] = x1c;
    }
  };
  // the first level is peeled off the loop (no row 1 to complete), so that
  // inside it every level follows the previous level's stores
  fetch(j0);
  commit();
  __syncthreads();
  if (j0 + 1 < j1) fetch(j0 + 1);
  level(j0, true);
  __syncthreads();
  for (int j = j0 + 1; j < j1; ++j) {
    commit();
    __syncthreads();
    if (j + 1 < j1) fetch(j + 1);
    level(j, false);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < PT; ++r) finish_row1(r, j1 - 1, ip[r], (j1 < n) ? x2[(size_t)j1 * m + ip[r]] : 0.0);
}

void launch_kkt_apply(const Geo& g, const double* x, double* y, const double* c, const double* alpha,
                      const double* xscale, int xs_stride, const int* active, bool transpose,
                      const double* ecoef, double ediag, double eoff, int jchunk, hipStream_t st) {
  if (g.fem) {
    launch_kkt_fem(g, x, y, c, alpha, xscale, xs_stride, active, transpose, st);
    return;
  }
  const double sgn = transpose ? -1.0 : 1.0;
  if (jchunk < 0 && g.nx <= 1024) {
    // LDS-tiled kernel, -jchunk levels per block
    constexpr int PT = 4;
    const int jc = -jchunk;
    dim3 grid((g.m + 256 * PT - 1) / (256 * PT), (g.n + jc - 1) / jc, g.B);
    const size_t lds = 2 * sizeof(double) * (256 * PT + 2 * (size_t)g.nx);
#define PCOP_KKT_LDS_H(D, V, HQ)                                                                                  \
  if (D == 3)                                                                                                     \
    kkt_lds_kernel<3, V, PT, HQ><<<grid, 256, lds, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn, ecoef,  \
                                                         ediag, eoff, jc);                                        \
  else if (c)                                                                                                     \
    kkt_lds2_kernel<V, PT, HQ, true><<<grid, 256, lds, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn,     \
                                                             ecoef, ediag, eoff, jc);                             \
  else                                                                                                            \
    kkt_lds2_kernel<V, PT, HQ, false><<<grid, 256, lds, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn,    \
                                                              ecoef, ediag, eoff, jc)
#define PCOP_KKT_LDS(D, V)                                        \
  if (g.nx <= 256) PCOP_KKT_LDS_H(D, V, 2);                       \
  else if (g.nx <= 512) PCOP_KKT_LDS_H(D, V, 4);                  \
  else PCOP_KKT_LDS_H(D, V, 8);
    if (g.dim == 2) {
      if (ecoef) {
        PCOP_KKT_LDS(2, true)
      } else {
        PCOP_KKT_LDS(2, false)
      }
    } else {
      if (ecoef) {
        PCOP_KKT_LDS(3, true)
      } else {
        PCOP_KKT_LDS(3, false)
      }
    }
#undef PCOP_KKT_LDS
#undef PCOP_KKT_LDS_H
    return;
  }
  if (jchunk < 1) jchunk = 16;
  dim3 grid((g.m + 255) / 256, (g.n + jchunk - 1) / jchunk, g.B);
#define PCOP_KKT(D, V, J) \
  kkt_apply_kernel<D, V, J><<<grid, 256, 0, st>>>(g, x, y, c, alpha, xscale, xs_stride, active, sgn, ecoef, ediag, eoff, jchunk)
#define PCOP_KKT_J(D, V)        \
  switch (jchunk) {             \
    case 1: PCOP_KKT(D, V, 1); break; \
    case 2: PCOP_KKT(D, V, 2); break; \
    case 4: PCOP_KKT(D, V, 4); break; \
    case 8: PCOP_KKT(D, V, 8); break; \
    case 16: PCOP_KKT(D, V, 16); break; \
    default: PCOP_KKT(D, V, 0); break; \
  }
  if (g.dim == 2) {
    if (ecoef) {
      PCOP_KKT_J(2, true)
    } else {
      PCOP_KKT_J(2, false)
    }
  } else {
    if (ecoef) {
      PCOP_KKT_J(3, true)
    } else {
      PCOP_KKT_J(3, false)
    }
  }
#undef PCOP_KKT_J
#undef PCOP_KKT
}

// ---------------------------------------------------------------------------
// element-wise maps
// ---------------------------------------------------------------------------

// b_1^j = tau g^j,  b_2^j = -sqrt(gamma) (tau f^j + [j == 0] y0)
__global__ void rhs_kernel(Geo g, const double* __restrict__ gg, const double* __restrict__ ff,
                           const double* __restrict__ y0, const double* __restrict__ sg,
                           double* __restrict__ bvec) {
  const long long nm = (long long)g.n * g.m;
  const long long total = nm * g.B;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nm);
    const long long r = t - (long long)b * nm;
    const int i = (int)(r % g.m);
    const bool first = r < g.m;
    double fv = g.tau * ff[t] + (first ? y0[(size_t)b * g.m + i] : 0.0);
    double* out = bvec + (size_t)b * g.vs;
    out[r] = g.tau * gg[t];
    out[nm + r] = -sg[b] * fv;
  }
}

// y = x_1 / sqrt(gamma), p = x_2
__global__ void unpack_kernel(Geo g, const double* __restrict__ x, const double* __restrict__ sg,
                              double* __restrict__ y, double* __restrict__ p) {
  const long long nm = (long long)g.n * g.m;
  const long long total = nm * g.B;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nm);
    const long long r = t - (long long)b * nm;
    const double* in = x + (size_t)b * g.vs;
    y[t] = in[r] / sg[b];
    p[t] = in[nm + r];
  }
}

// r = [ybar / sqrt(gamma); pbar]
__global__ void pack_cot_kernel(Geo g, const double* __restrict__ yb, const double* __restrict__ pb,
                                const double* __restrict__ sg, double* __restrict__ r) {
  const long long nm = (long long)g.n * g.m;
  const long long total = nm * g.B;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nm);
    const long long q = t - (long long)b * nm;
    double* out = r + (size_t)b * g.vs;
    out[q] = yb ? yb[t] / sg[b] : 0.0;
    out[nm + q] = pb ? pb[t] : 0.0;
  }
}

// dg = tau lam_1, df = -sqrt(gamma) tau lam_2, dy0 = -sqrt(gamma) lam_2^1
__global__ void data_grad_kernel(Geo g, const double* __restrict__ lam, const double* __restrict__ sg,
                                 double* __restrict__ dg, double* __restrict__ df,
                                 double* __restrict__ dy0) {
  const long long nm = (long long)g.n * g.m;
  const long long total = nm * g.B;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nm);
    const long long q = t - (long long)b * nm;
    const double* in = lam + (size_t)b * g.vs;
    if (dg) dg[t] = g.tau * in[q];
    if (df) df[t] = -sg[b] * g.tau * in[nm + q];
    if (dy0 && q < g.m) dy0[(size_t)b * g.m + q] = -sg[b] * in[nm + q];
  }
}

// dst = src or J src = [src_1; -src_2], member b at dst + b dvs and
// src + b svs (copies between the caller's layout and the padded one)
__global__ void restride_kernel(Geo g, const double* __restrict__ src, long long svs, double* __restrict__ dst,
                                long long dvs, int flip) {
  const long long nm = (long long)g.n * g.m;
  const long long total = 2 * nm * g.B;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / (2 * nm));
    const long long r = t - (long long)b * 2 * nm;
    const double v = src[(size_t)b * svs + r];
    dst[(size_t)b * dvs + r] = (flip && r >= nm) ? -v : v;
  }
}

static int ew_blocks(const Geo& g) {
  long long total = (long long)g.n * g.m * g.B;
  long long blk = (total + 255) / 256;
  return (int)(blk < 8192 ? (blk < 1 ? 1 : blk) : 8192);
}

void launch_restride(const Geo& g, const double* src, long long svs, double* dst, long long dvs, bool flip,
                     hipStream_t st) {
  restride_kernel<<<ew_blocks(g), 256, 0, st>>>(g, src, svs, dst, dvs, flip ? 1 : 0);
}
void launch_rhs(const Geo& g, const double* gg, const double* ff, const double* y0, const double* sg,
                double* b, hipStream_t st) {
  rhs_kernel<<<ew_blocks(g), 256, 0, st>>>(g, gg, ff, y0, sg, b);
}
void launch_unpack(const Geo& g, const double* x, const double* sg, double* y, double* p,
                   hipStream_t st) {
  unpack_kernel<<<ew_blocks(g), 256, 0, st>>>(g, x, sg, y, p);
}
void launch_pack_cotangent(const Geo& g, const double* yb, const double* pb, const double* sg,
                           double* r, hipStream_t st) {
  pack_cot_kernel<<<ew_blocks(g), 256, 0, st>>>(g, yb, pb, sg, r);
}
void launch_data_grad(const Geo& g, const double* lam, const double* sg, double* dg, double* df,
                      double* dy0, hipStream_t st) {
  data_grad_kernel<<<ew_blocks(g), 256, 0, st>>>(g, lam, sg, dg, df, dy0);
}

}  // namespace pcop
