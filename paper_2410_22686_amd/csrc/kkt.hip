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

void launch_kkt_apply(const Geo& g, const double* x, double* y, const double* c, const double* alpha,
                      const double* xscale, int xs_stride, const int* active, bool transpose,
                      const double* ecoef, double ediag, double eoff, int jchunk, hipStream_t st) {
  if (jchunk < 1) jchunk = 16;
  dim3 grid((g.m + 255) / 256, (g.n + jchunk - 1) / jchunk, g.B);
  const double sgn = transpose ? -1.0 : 1.0;
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
