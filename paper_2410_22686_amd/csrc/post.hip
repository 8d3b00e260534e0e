// End levels of the discrete solution and the error e_h (Section 1, the two
// formulas after eq. Toeplitz_Mat_B; Section 3 for e_h):
//   (M + tau K) y^N = M (y^{N-1} + tau f^N + (tau/gamma) p^N),   p^N = 0,
//   (M + tau K) p^0 = M (p^1 + tau (g^0 - y^0)),
// with M = I for finite differences (E = I + tau K below; with Q1 elements
// E = M + tau K and the caller applies M to the right-hand sides).
// E = I + tau K is real, so both right-hand sides ride in one complex slice
// per member, r = r_y + i r_p, solved by iterative refinement
//   z <- z + S (rhs - E z),
// with the residual in FP64 and S one spatial solve with the shift 1 (sine
// transforms: exact in FP64; multigrid: one V-cycle in the context's
// precision).  Buffers: rhs and z planar [B][2][m] FP64, the correction slice
// [B][m] complex.
#include <cmath>

#include "common.hpp"
#include "fem.hpp"
#include "launch.hpp"
#include "stencil.hpp"

namespace pcop {

// rhs_y = x_1^n / sqrt(gamma) + tau f^N, rhs_p = x_2^1 + tau (g^0 - y^0); z = 0
__global__ void __launch_bounds__(256) post_rhs_kernel(Geo g, const double* __restrict__ x,
                                                       const double* __restrict__ fN, const double* __restrict__ g0,
                                                       const double* __restrict__ y0, const double* __restrict__ sg,
                                                       double* __restrict__ rhs, double* __restrict__ z) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n, m = g.m;
  if (i >= m) return;
  const double* x1 = x + (size_t)b * g.vs;
  const double* x2 = x1 + (size_t)n * m;
  const size_t o = (size_t)b * m + i;
  double* rb = rhs + (size_t)b * 2 * m;
  rb[i] = x1[(size_t)(n - 1) * m + i] / sg[b] + g.tau * fN[o];
  rb[m + i] = x2[i] + g.tau * (g0[o] - y0[o]);
  double* zb = z + (size_t)b * 2 * m;
  zb[i] = 0.0;
  zb[m + i] = 0.0;
}

// fixed-order block sum of v over 256 threads
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double part[256 / kWave];
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < 256 / kWave; ++k) s += part[k];
  return s;
}

// s = rhs - E z as a complex slice; part[b][blk] = block sum of |s|^2 (FP64)
template <class T, int DIM, bool VAR>
__global__ void __launch_bounds__(256) post_resid_kernel(Geo g, const double* __restrict__ rhs,
                                                         const double* __restrict__ z, cx<T>* __restrict__ s,
                                                         double* __restrict__ part, const double* __restrict__ ecoef,
                                                         double ediag, double eoff) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = g.nx, m = g.m;
  double r2 = 0.0;
  if (i < m) {
    const int c1 = i % nx, c2 = (i / nx) % nx, c3 = (DIM == 3) ? i / (nx * nx) : 0;
    const double* rb = rhs + (size_t)b * 2 * m;
    const double* zb = z + (size_t)b * 2 * m;
    const double re = rb[i] - apply_E<DIM, VAR>(zb, i, c1, c2, c3, nx, m, ecoef, ediag, eoff);
    const double im = rb[m + i] - apply_E<DIM, VAR>(zb + m, i, c1, c2, c3, nx, m, ecoef, ediag, eoff);
    s[(size_t)b * m + i] = cx<T>{(T)re, (T)im};
    r2 = re * re + im * im;
  }
  const double tot = block_sum256(r2);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = tot;
}

// the same residual with E = M + tau K of Q1 finite elements
template <class T, int DIM>
__global__ void __launch_bounds__(256) post_resid_fem_kernel(Geo g, const double* __restrict__ rhs,
                                                             const double* __restrict__ z, cx<T>* __restrict__ s,
                                                             double* __restrict__ part) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = g.nx, m = g.m;
  double r2 = 0.0;
  if (i < m) {
    const int c1 = i % nx, c2 = (i / nx) % nx, c3 = (DIM == 3) ? i / (nx * nx) : 0;
    const Q1W w = q1_weights(nx);
    const double* rb = rhs + (size_t)b * 2 * m;
    const double* zb = z + (size_t)b * 2 * m;
    double Mr, Kr, Mi, Ki;
    q1_apply<DIM>(zb, c1, c2, c3, nx, w, Mr, Kr);
    q1_apply<DIM>(zb + m, c1, c2, c3, nx, w, Mi, Ki);
    const double re = rb[i] - (Mr + g.tau * Kr);
    const double im = rb[m + i] - (Mi + g.tau * Ki);
    s[(size_t)b * m + i] = cx<T>{(T)re, (T)im};
    r2 = re * re + im * im;
  }
  const double tot = block_sum256(r2);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = tot;
}

// z += s
template <class T>
__global__ void __launch_bounds__(256) post_correct_kernel(Geo g, const cx<T>* __restrict__ s, double* __restrict__ z) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = g.m;
  if (i >= m) return;
  const cx<T> v = s[(size_t)b * m + i];
  double* zb = z + (size_t)b * 2 * m;
  zb[i] += (double)v.x;
  zb[m + i] += (double)v.y;
}

// out[b] = sum of part[b][0..nblk) in a fixed order
__global__ void __launch_bounds__(256) post_norm_kernel(const double* __restrict__ part, int nblk,
                                                        double* __restrict__ out) {
  const int b = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) v += part[(size_t)b * nblk + k];
  const double tot = block_sum256(v);
  if (threadIdx.x == 0) out[b] = tot;
}

// y^N = Re z, p^0 = Im z
__global__ void __launch_bounds__(256) post_store_kernel(Geo g, const double* __restrict__ z, double* __restrict__ yN,
                                                         double* __restrict__ p0) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = g.m;
  if (i >= m) return;
  const double* zb = z + (size_t)b * 2 * m;
  yN[(size_t)b * m + i] = zb[i];
  p0[(size_t)b * m + i] = zb[m + i];
}

template <class T>
static void resid_launch(const Geo& g, const PostArgs& a, cx<T>* s, int nblk, hipStream_t st) {
  dim3 grid(nblk, g.B);
  if (g.fem) {
    if (g.dim == 2) post_resid_fem_kernel<T, 2><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part);
    else post_resid_fem_kernel<T, 3><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part);
    return;
  }
  const bool var = a.ecoef != nullptr;
  if (g.dim == 2) {
    if (var) post_resid_kernel<T, 2, true><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part, a.ecoef, a.ediag, a.eoff);
    else post_resid_kernel<T, 2, false><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part, a.ecoef, a.ediag, a.eoff);
  } else {
    if (var) post_resid_kernel<T, 3, true><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part, a.ecoef, a.ediag, a.eoff);
    else post_resid_kernel<T, 3, false><<<grid, 256, 0, st>>>(g, a.rhs, a.z, s, a.part, a.ecoef, a.ediag, a.eoff);
  }
}

void launch_post_rhs(const Geo& g, const double* x, const double* fN, const double* g0, const double* y0,
                     const double* sg, const PostArgs& a, hipStream_t st) {
  dim3 grid((g.m + 255) / 256, g.B);
  post_rhs_kernel<<<grid, 256, 0, st>>>(g, x, fN, g0, y0, sg, a.rhs, a.z);
}

bool launch_post_step(const Geo& g, const PostArgs& a, void* slice, bool fp32, int spatial,
                      const PrecondTables& tb, const double* unit, hipStream_t st) {
  const int nblk = (g.m + 255) / 256;
  // sine transforms always in FP64; the multigrid cycle in the context's precision
  const bool f32 = (spatial != 0) && fp32;
  if (f32) resid_launch<float>(g, a, reinterpret_cast<cx<float>*>(slice), nblk, st);
  else resid_launch<double>(g, a, reinterpret_cast<cx<double>*>(slice), nblk, st);
  post_norm_kernel<<<g.B, 256, 0, st>>>(a.part, nblk, a.norm2);
  const bool ok = (spatial == 0) ? launch_dst_solve(g, slice, false, tb, 1, unit, st)
                                 : launch_mg_solve(g, slice, f32, tb, 1, unit, st);
  if (!ok) return false;
  dim3 grid(nblk, g.B);
  if (f32) post_correct_kernel<float><<<grid, 256, 0, st>>>(g, reinterpret_cast<const cx<float>*>(slice), a.z);
  else post_correct_kernel<double><<<grid, 256, 0, st>>>(g, reinterpret_cast<const cx<double>*>(slice), a.z);
  return true;
}

void launch_post_residual(const Geo& g, const PostArgs& a, void* slice, hipStream_t st) {
  const int nblk = (g.m + 255) / 256;
  resid_launch<double>(g, a, reinterpret_cast<cx<double>*>(slice), nblk, st);
  post_norm_kernel<<<g.B, 256, 0, st>>>(a.part, nblk, a.norm2);
}

void launch_post_store(const Geo& g, const PostArgs& a, double* yN, double* p0, hipStream_t st) {
  dim3 grid((g.m + 255) / 256, g.B);
  post_store_kernel<<<grid, 256, 0, st>>>(g, a.z, yN, p0);
}

// ---------------------------------------------------------------------------
// e_h = h^{d/2} max_{1 <= j <= N} max(||y^j - y(t_j)||_2, ||p^{j-1} - p(t_{j-1})||_2)
// sq[b][j][0] = ||y^{j+1} - y(t_{j+1})||^2, sq[b][j][1] = ||p^j - p(t_j)||^2, j = 0..N-1
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) eh_level_kernel(Geo g, const double* __restrict__ x,
                                                       const double* __restrict__ yN, const double* __restrict__ p0,
                                                       const double* __restrict__ sg, const double* __restrict__ yex,
                                                       const double* __restrict__ pex, double* __restrict__ sq) {
  const int j = blockIdx.x;  // 0..N-1
  const int b = blockIdx.y;
  const int n = g.n, m = g.m, N = g.n + 1;
  const double* x1 = x + (size_t)b * g.vs;
  const double* x2 = x1 + (size_t)n * m;
  const double* ye = yex + ((size_t)b * (N + 1) + (j + 1)) * m;
  const double* pe = pex + ((size_t)b * (N + 1) + j) * m;
  double sy = 0.0, sp = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double yv = (j + 1 <= n) ? x1[(size_t)j * m + i] / sg[b] : yN[(size_t)b * m + i];
    const double pv = (j == 0) ? p0[(size_t)b * m + i] : x2[(size_t)(j - 1) * m + i];
    const double dy = yv - ye[i], dp = pv - pe[i];
    sy += dy * dy;
    sp += dp * dp;
  }
  const double ty = block_sum256(sy);
  const double tp = block_sum256(sp);
  if (threadIdx.x == 0) {
    sq[((size_t)b * N + j) * 2] = ty;
    sq[((size_t)b * N + j) * 2 + 1] = tp;
  }
}

__global__ void eh_max_kernel(int B, int N, const double* __restrict__ sq, double scale, double* __restrict__ eh) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double mx = 0.0;
  for (int j = 0; j < N; ++j) {
    mx = fmax(mx, sq[((size_t)b * N + j) * 2]);
    mx = fmax(mx, sq[((size_t)b * N + j) * 2 + 1]);
  }
  eh[b] = scale * sqrt(mx);
}

void launch_error_eh(const Geo& g, const double* x, const double* yN, const double* p0, const double* sg,
                     const double* yex, const double* pex, double* sq, double* eh, hipStream_t st) {
  const int N = g.n + 1;
  dim3 grid(N, g.B);
  eh_level_kernel<<<grid, 256, 0, st>>>(g, x, yN, p0, sg, yex, pex, sq);
  const double h = 1.0 / (g.nx + 1.0);
  const double scale = std::pow(h, g.dim / 2.0);
  eh_max_kernel<<<(g.B + 63) / 64, 64, 0, st>>>(g.B, N, sq, scale, eh);
}

}  // namespace pcop
