// Time passes for lengths with a prime factor above 17: chirp-z (Bluestein)
// transform with power-of-two convolutions in LDS.
#include "time_common.hpp"

namespace pcop {

template <class T, int P, int M>
__global__ void __launch_bounds__(256) time_fwd_bl(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, TimeTables tt,
                                                   const double* __restrict__ vscale, int vs_stride,
                                                   const int* __restrict__ active) {
  constexpr int LD = M + 1;
  __shared__ cx<T> buf[P * LD];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  const cx<T>* twM = reinterpret_cast<const cx<T>*>(tt.twM);
  const cx<T>* chirp = reinterpret_cast<const cx<T>*>(tt.chirp);
  const cx<T>* bhat = reinterpret_cast<const cx<T>*>(tt.bhat);
  const int i0 = bx * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vs;
  const double* v2 = v1 + (size_t)n * m;
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    cx<T> a{0, 0};
    if (j < n) a = pack_input<T>(v1, v2, dpow, s, j, i0 + p, m) * chirp[j];
    buf[p * LD + j] = a;
  }
  __syncthreads();
  p2_fft<T, -1, M, P, 256>(buf, LD, twM);
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int p = t / M, k = t - p * M;
    buf[p * LD + k] = buf[p * LD + k] * bhat[k];
  }
  __syncthreads();
  p2_fft<T, 1, M, P, 256>(buf, LD, twM);
  const T invM = (T)1 / (T)M;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int p = t / n, k = t - p * n;
    buf[p * LD + k] = scale(buf[p * LD + k] * chirp[k], invM);
  }
  __syncthreads();
  cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
  unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return buf[p * LD + k]; });
}

// inverse DFT through the forward chirp transform: e = conj(DFT(conj(E)))
template <class T, int P, int M>
__global__ void __launch_bounds__(256) time_inv_bl(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, TimeTables tt, int accum,
                                                   const int* __restrict__ active) {
  constexpr int LD = M + 1;
  __shared__ cx<T> buf[P * LD];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  const cx<T>* twM = reinterpret_cast<const cx<T>*>(tt.twM);
  const cx<T>* chirp = reinterpret_cast<const cx<T>*>(tt.chirp);
  const cx<T>* bhat = reinterpret_cast<const cx<T>*>(tt.bhat);
  const int i0 = bx * P;
  const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
  for (int t = threadIdx.x; t < (M - n) * P; t += blockDim.x) {
    const int j = n + t / P, p = t - (t / P) * P;
    buf[p * LD + j] = cx<T>{0, 0};
  }
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    cx<T> z2{0, 0}, z1{0, 0};
    if (i < m) {
      z2 = in[(size_t)(2 * k) * m + i];
      z1 = in[(size_t)(2 * k + 1) * m + i];
    }
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1)
    const cx<T> ek{z2.x - z1.y, -(z2.y + z1.x)};
    buf[p * LD + k] = ek * chirp[k];
    if (k != 0 && 2 * k != n) {
      const cx<T> enk{z2.x + z1.y, -(z1.x - z2.y)};
      buf[p * LD + (n - k)] = enk * chirp[n - k];
    }
  }
  __syncthreads();
  p2_fft<T, -1, M, P, 256>(buf, LD, twM);
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int p = t / M, k = t - p * M;
    buf[p * LD + k] = buf[p * LD + k] * bhat[k];
  }
  __syncthreads();
  p2_fft<T, 1, M, P, 256>(buf, LD, twM);
  double* w1 = w + (size_t)b * g.vs;
  double* w2 = w1 + (size_t)n * m;
  const double invM = 1.0 / (double)M;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    const int i = i0 + p;
    if (i >= m) continue;
    const cx<T> e = buf[p * LD + j] * chirp[j];
    // e_j = conj(chirp_j c_j / M)
    combine_store(w1, w2, dpow, n, m, j, i, (double)e.x * invM, -(double)e.y * invM, accum);
  }
}

template <class T, int P, int M>
static void bl_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  // only shapes whose LDS tile fits kBlueLds are instantiated (time_cols_bl
  // picks P accordingly); fewer than 4 columns only for the longest lengths
  if constexpr ((size_t)(M + 1) * P * sizeof(cx<T>) <= kBlueLds && (P >= 4 || M >= 2048)) {
    dim3 grid((g.m + P - 1) / P, g.B);
    if (fwd)
      time_fwd_bl<T, P, M><<<grid, 256, 0, st>>>(g, v, spec, tb.dpow, tt, vscale, vs_stride, tb.active);
    else
      time_inv_bl<T, P, M><<<grid, 256, 0, st>>>(g, spec, w, tb.dpow, tt, accum, tb.active);
  }
}

template <class T, int P>
static bool bl_dispatch_M(bool fwd, int M, const Geo& g, const double* v, cx<T>* spec, double* w,
                          const PrecondTables& tb, const TimeTables& tt, const double* vscale, int vs_stride,
                          int accum, hipStream_t st) {
  switch (M) {
    case 8: bl_launch<T, P, 8>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 16: bl_launch<T, P, 16>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 32: bl_launch<T, P, 32>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 64: bl_launch<T, P, 64>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 128: bl_launch<T, P, 128>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 256: bl_launch<T, P, 256>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 512: bl_launch<T, P, 512>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 1024: bl_launch<T, P, 1024>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 2048: bl_launch<T, P, 2048>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 4096: bl_launch<T, P, 4096>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    default: return false;
  }
}


template <class T>
bool launch_time_bl(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (P == 16) return bl_dispatch_M<T, 16>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  if (P == 8) return bl_dispatch_M<T, 8>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  if (P == 4) return bl_dispatch_M<T, 4>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  if (P == 2) return bl_dispatch_M<T, 2>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  if (P == 1) return bl_dispatch_M<T, 1>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  return false;
}

template bool launch_time_bl<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const TimeTables&, const double*, int, int, hipStream_t);
template bool launch_time_bl<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const TimeTables&, const double*, int, int, hipStream_t);

}  // namespace pcop
