// Time passes, Stockham kernels with two ping-pong LDS buffers.
#include "time_common.hpp"

namespace pcop {

template <class T, int P>
__global__ void __launch_bounds__(256) time_fwd_sk(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, const double* __restrict__ vscale, int vs_stride,
                                                   const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  const int i0 = bx * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vl;
  const double* v2 = v1 + (size_t)n * m;
  auto ld0 = [&](int j, int p) { return pack_input<T>(v1, v2, dpow, s, j, i0 + p, m); };
  auto stA = [&](int j, int p, cx<T> val) { bufA[j * P + p] = val; };
  sk_stage_rt<T, P, -1>(plan.rad[0], n, 1, twn, ld0, stA);
  __syncthreads();
  cx<T>* src = bufA;
  cx<T>* dst = bufB;
  int Ns = plan.rad[0];
  for (int st = 1; st < plan.nrad; ++st) {
    auto ld = [&](int j, int p) { return src[j * P + p]; };
    auto sto = [&](int j, int p, cx<T> val) { dst[j * P + p] = val; };
    sk_stage_rt<T, P, -1>(plan.rad[st], n, Ns, twn, ld, sto);
    __syncthreads();
    Ns *= plan.rad[st];
    cx<T>* t = src;
    src = dst;
    dst = t;
  }
  cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
  unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return src[k * P + p]; });
}

template <class T, int P>
__global__ void __launch_bounds__(256) time_inv_sk(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, int accum, const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  const int i0 = bx * P;
  const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    cx<T> z2{0, 0}, z1{0, 0};
    if (i < m) {
      z2 = in[(size_t)(2 * k) * m + i];
      z1 = in[(size_t)(2 * k + 1) * m + i];
    }
    // e_k = Z2 + i Z1 and, for the mirrored frequency, e_{n-k} = conj Z2 + i conj Z1
    bufA[k * P + p] = cx<T>{z2.x - z1.y, z2.y + z1.x};
    if (k != 0 && 2 * k != n) bufA[(n - k) * P + p] = cx<T>{z2.x + z1.y, z1.x - z2.y};
  }
  __syncthreads();
  double* w1 = w + (size_t)b * g.vl;
  double* w2 = w1 + (size_t)n * m;
  cx<T>* src = bufA;
  cx<T>* dst = bufB;
  int Ns = 1;
  for (int st = 0; st < plan.nrad; ++st) {
    auto ld = [&](int j, int p) { return src[j * P + p]; };
    if (st + 1 < plan.nrad) {
      auto sto = [&](int j, int p, cx<T> val) { dst[j * P + p] = val; };
      sk_stage_rt<T, P, 1>(plan.rad[st], n, Ns, twn, ld, sto);
      __syncthreads();
      cx<T>* t = src;
      src = dst;
      dst = t;
    } else {
      auto sto = [&](int j, int p, cx<T> val) {
        const int i = i0 + p;
        if (i < m) combine_store(w1, w2, dpow, n, m, j, i, (double)val.x, (double)val.y, accum);
      };
      sk_stage_rt<T, P, 1>(plan.rad[st], n, Ns, twn, ld, sto);
    }
    Ns *= plan.rad[st];
  }
}


template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  dim3 grid((g.m + P - 1) / P, g.B);
  const size_t lds = (size_t)2 * g.n * P * sizeof(cx<T>);
#define PCOP_TIME_SK(PP)                                                                                       \
  if (fwd)                                                                                                     \
    time_fwd_sk<T, PP><<<grid, 256, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tb.active); \
  else                                                                                                         \
    time_inv_sk<T, PP><<<grid, 256, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, accum, tb.active);
  if (P == 16) {
    PCOP_TIME_SK(16)
  } else if (P == 8) {
    PCOP_TIME_SK(8)
  } else {
    PCOP_TIME_SK(4)
  }
#undef PCOP_TIME_SK
}

template void launch_time_sk<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const cx<double>*, const double*, int, int, hipStream_t);
template void launch_time_sk<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const cx<float>*, const double*, int, int, hipStream_t);

}  // namespace pcop
