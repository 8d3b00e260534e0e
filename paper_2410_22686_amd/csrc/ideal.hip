// The ideal RBD preconditioner w = P^{-1} v of eq. matrix_P (Section 2):
// P^{-1} = G^{-1} blockdiag(T^T + alpha I, T + alpha I)^{-1}, so
//   (T + alpha I) z_2 = v_2  by forward substitution in time,
//   (T^T + alpha I) z_1 = v_1 by backward substitution,
//   w_1 = z_1 - z_2, w_2 = z_1 + z_2,
// each substitution step a solve with T_0 = (1 + alpha) I + tau K.  T_0 is
// real, so step s carries both recurrences in one complex slice per member:
//   c = (v_2^s + z_2^{s-1}) + i (v_1^{n-1-s} + z_1^{n-s}),  T_0 c' = c,
//   z_2^s = Re c', z_1^{n-1-s} = Im c'.
// The n steps are sequential (one spatial solve launch sequence each); this
// is the method the epsilon-circulant preconditioner parallelises in time.
// Storage inside the spectrum buffer: z[b][2][n][m] (type T) followed by the
// slice buffer c[b][m] (complex T).
#include "common.hpp"
#include "launch.hpp"

namespace pcop {

// step s in 0..n: store the solved slice of step s-1, pack the slice of step s
template <class T>
__global__ void __launch_bounds__(256) ideal_step_kernel(Geo g, int s, const double* __restrict__ v, T* __restrict__ z,
                                                         cx<T>* __restrict__ c, const double* __restrict__ vscale,
                                                         int vs_stride, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n, m = g.m;
  if (i >= m) return;
  T* z1 = z + (size_t)b * 2 * n * m;
  T* z2 = z1 + (size_t)n * m;
  cx<T>* cb = c + (size_t)b * m;
  T p2 = 0, p1 = 0;  // z_2^{s-1}, z_1^{n-s}
  if (s > 0) {
    const cx<T> r = cb[i];
    p2 = r.x;
    p1 = r.y;
    z2[(size_t)(s - 1) * m + i] = p2;
    z1[(size_t)(n - s) * m + i] = p1;
  }
  if (s < n) {
    const double sc = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)n * m;
    const double a2 = sc * v2[(size_t)s * m + i] + (double)p2;
    const double a1 = sc * v1[(size_t)(n - 1 - s) * m + i] + (double)p1;
    cb[i] = cx<T>{(T)a2, (T)a1};
  }
}

// w = [z_1 - z_2; z_1 + z_2] (added to w when accum)
template <class T>
__global__ void __launch_bounds__(256) ideal_combine_kernel(Geo g, const T* __restrict__ z, double* __restrict__ w,
                                                            int accum, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long nm = (long long)g.n * g.m;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nm) return;
  const T* z1 = z + (size_t)b * 2 * nm;
  const double a = (double)z1[e], d = (double)z1[nm + e];
  double* w1 = w + (size_t)b * g.vs;
  double* w2 = w1 + nm;
  if (accum) {
    w1[e] += a - d;
    w2[e] += a + d;
  } else {
    w1[e] = a - d;
    w2[e] = a + d;
  }
}

template <class T>
static bool ideal_apply(const Geo& g, const double* v, double* w, void* spec, int spatial, const PrecondTables& tb,
                        const double* unit, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  T* z = reinterpret_cast<T*>(spec);
  const size_t zbytes = sizeof(T) * (size_t)g.B * 2 * g.n * g.m;
  cx<T>* c = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(spec) + ((zbytes + 255) & ~(size_t)255));
  const bool fp32 = sizeof(T) == 4;
  dim3 gs((g.m + 255) / 256, g.B);
  const double step_bytes = (8.0 + 2.0 * sizeof(cx<T>)) * g.m * tb.nact;
  for (int s = 0; s <= g.n; ++s) {
    tbeg(tb.timer, KF_IDEAL_STEP, step_bytes);
    ideal_step_kernel<T><<<gs, 256, 0, st>>>(g, s, v, z, c, vscale, vs_stride, tb.active);
    tend(tb.timer);
    if (s == g.n) break;
    // one slice per member, shift lam_0 + alpha_b with lam_0 = 1: T_0 = (1 + alpha) I + tau K
    const bool ok = (spatial == 0) ? launch_dst_solve(g, c, fp32, tb, 1, unit, st)
                                   : launch_mg_solve(g, c, fp32, tb, 1, unit, st);
    if (!ok) return false;
  }
  const long long nm = (long long)g.n * g.m;
  dim3 gc((unsigned)((nm + 255) / 256), g.B);
  tbeg(tb.timer, KF_COMBINE, (sizeof(T) * 2.0 + (accum ? 32.0 : 16.0)) * nm * tb.nact);
  ideal_combine_kernel<T><<<gc, 256, 0, st>>>(g, z, w, accum, tb.active);
  tend(tb.timer);
  return true;
}

size_t ideal_spec_bytes(const Geo& g, bool fp32) {
  const size_t t = fp32 ? 4 : 8;
  const size_t zbytes = t * (size_t)g.B * 2 * g.n * g.m;
  return ((zbytes + 255) & ~(size_t)255) + 2 * t * (size_t)g.B * g.m;
}

bool launch_ideal_precond(const Geo& g, const double* v, double* w, void* spec, bool fp32, int spatial,
                          const PrecondTables& tb, const double* unit, const double* vscale, int vs_stride,
                          int accum, hipStream_t st) {
  if (fp32) return ideal_apply<float>(g, v, w, spec, spatial, tb, unit, vscale, vs_stride, accum, st);
  return ideal_apply<double>(g, v, w, spec, spatial, tb, unit, vscale, vs_stride, accum, st);
}

}  // namespace pcop
