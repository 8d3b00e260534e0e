// Time passes, in-place Stockham kernels (one LDS buffer).  Each stage
// dispatches over the radix and the butterflies per thread at run time, so
// the kernels are large: every (precision, direction) pair is compiled in a
// translation unit of its own (time_ip_*.hip).
#pragma once

#include "time_common.hpp"

namespace pcop {

// In-place variants: one [n][P] LDS buffer, butterflies held in registers
// across the barrier of each stage (half the LDS of the ping-pong kernels).
template <class T, int P>
__global__ void __launch_bounds__(256) time_fwd_ip(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, const double* __restrict__ vscale, int vs_stride,
                                                   const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int i0 = bx * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vs;
  const double* v2 = v1 + (size_t)n * m;
  auto ldg = [&](int j, int p) { return pack_input<T>(v1, v2, dpow, s, j, i0 + p, m); };
  auto lds = [&](int j, int p) { return buf[j * P + p]; };
  auto sts = [&](int j, int p, cx<T> val) { buf[j * P + p] = val; };
  ip_stage_rt<T, P, -1>(plan.rad[0], n, 1, twn, false, ldg, sts);
  __syncthreads();
  int Ns = plan.rad[0];
  for (int st = 1; st < plan.nrad; ++st) {
    ip_stage_rt<T, P, -1>(plan.rad[st], n, Ns, twn, true, lds, sts);
    __syncthreads();
    Ns *= plan.rad[st];
  }
  cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
  unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return buf[k * P + p]; });
}

template <class T, int P>
__global__ void __launch_bounds__(256) time_inv_ip(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, int accum, const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
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
    buf[k * P + p] = cx<T>{z2.x - z1.y, z2.y + z1.x};
    if (k != 0 && 2 * k != n) buf[(n - k) * P + p] = cx<T>{z2.x + z1.y, z1.x - z2.y};
  }
  __syncthreads();
  double* w1 = w + (size_t)b * g.vs;
  double* w2 = w1 + (size_t)n * m;
  auto lds = [&](int j, int p) { return buf[j * P + p]; };
  auto sts = [&](int j, int p, cx<T> val) { buf[j * P + p] = val; };
  auto stg = [&](int j, int p, cx<T> val) {
    const int i = i0 + p;
    if (i < m) combine_store(w1, w2, dpow, n, m, j, i, (double)val.x, (double)val.y, accum);
  };
  int Ns = 1;
  for (int st = 0; st < plan.nrad; ++st) {
    if (st + 1 < plan.nrad) {
      ip_stage_rt<T, P, 1>(plan.rad[st], n, Ns, twn, true, lds, sts);
      __syncthreads();
    } else {
      ip_stage_rt<T, P, 1>(plan.rad[st], n, Ns, twn, false, lds, stg);
    }
    Ns *= plan.rad[st];
  }
}
template <class T, bool FWD>
void launch_time_ip_dir(int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                        const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  dim3 grid((g.m + P - 1) / P, g.B);
  const size_t lds = (size_t)g.n * P * sizeof(cx<T>);
#define PCOP_TIME_IP(PP)                                                                                       \
  if constexpr (FWD)                                                                                           \
    time_fwd_ip<T, PP><<<grid, 256, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tb.active); \
  else                                                                                                         \
    time_inv_ip<T, PP><<<grid, 256, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, accum, tb.active);
  if (P == 16) {
    PCOP_TIME_IP(16)
  } else if (P == 8) {
    PCOP_TIME_IP(8)
  } else {
    PCOP_TIME_IP(4)
  }
#undef PCOP_TIME_IP
}

}  // namespace pcop
