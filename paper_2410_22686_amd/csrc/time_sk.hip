// Time passes, Stockham kernels with two ping-pong LDS buffers.
#include <algorithm>

#include "time_common.hpp"

namespace pcop {

// Persistent blocks: each block walks column tiles lb, lb + grid, ... and
// fetches the global inputs of its next tile into registers before running
// the FFT stages of the current one in LDS, so HBM traffic overlaps the
// stages (two [n][P] buffers allow only a few blocks per CU).
//
// Tile t covers member t / tiles_per_member and spatial points
// i0 .. i0 + P - 1 with i0 = (t mod tiles_per_member) P.
struct TileWalk {
  int tpm;     // tiles per member
  int ntiles;  // B * tpm
  const int* active;
  // first tile at or after t whose member is active (ntiles if none)
  __device__ __forceinline__ int next(int t, int stride) const {
    while (t < ntiles && active && !active[t / tpm]) t += stride;
    return t;
  }
};

// Q = register slots per thread for one tile's inputs: n P <= Q * 256
template <class T, int P, int Q>
__global__ void __launch_bounds__(256) time_fwd_sk(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, const double* __restrict__ vscale, int vs_stride,
                                                   TileWalk tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int nP = n * P;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + nP;
  // consecutive logical blocks (whose tiles share 128-byte lines) on one XCD
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[Q], r2[Q];  // v_1, v_2 at element e = threadIdx.x + q * 256 of the tile
  auto fetch = [&](int t) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const double* v1 = v + (size_t)b * g.vl;
    const double* v2 = v1 + (size_t)n * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * 256;
      const int j = e / P, i = i0 + (e % P);
      const bool in = e < nP && i < m;
      r1[q] = in ? v1[(size_t)j * m + i] : 0.0;
      r2[q] = in ? v2[(size_t)j * m + i] : 0.0;
    }
  };
  if (tile < tw.ntiles) fetch(tile);
  while (tile < tw.ntiles) {
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    // c_j = s (d_j v2_j + i v1_j / d_j), stored at [j][p] = element e
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < nP) {
        const double d = dpow[e / P];
        bufA[e] = cx<T>{(T)(s * d * r2[q]), (T)(s * r1[q] / d)};
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt);
    cx<T>* src = bufA;
    cx<T>* dst = bufB;
    int Ns = 1;
    for (int st = 0; st < plan.nrad; ++st) {
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
    __syncthreads();
    tile = nxt;
  }
}

// Q = register slots per thread for one tile's spectrum: K P <= Q * 256
template <class T, int P, int Q>
__global__ void __launch_bounds__(256) time_inv_sk(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, int accum, TileWalk tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int KP = K * P;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[Q], r1[Q];  // Z_2, Z_1 at element e = threadIdx.x + q * 256 = k P + p
  auto fetch = [&](int t) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * 256;
      const int k = e / P, i = i0 + (e % P);
      const bool ok = e < KP && i < m;
      r2[q] = ok ? in[(size_t)(2 * k) * m + i] : cx<T>{0, 0};
      r1[q] = ok ? in[(size_t)(2 * k + 1) * m + i] : cx<T>{0, 0};
    }
  };
  if (tile < tw.ntiles) fetch(tile);
  while (tile < tw.ntiles) {
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < KP) {
        const int k = e / P, p = e % P;
        const cx<T> z2 = r2[q], z1 = r1[q];
        // e_k = Z2 + i Z1 and, for the mirrored frequency, e_{n-k} = conj Z2 + i conj Z1
        bufA[e] = cx<T>{z2.x - z1.y, z2.y + z1.x};
        if (k != 0 && 2 * k != n) bufA[(n - k) * P + p] = cx<T>{z2.x + z1.y, z1.x - z2.y};
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt);
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
    __syncthreads();
    tile = nxt;
  }
}

// register slots: the two [n][P] buffers fit 64 KiB, so n P <= 2048 (FP64)
// or 4096 (FP32) and K P <= n P / 2 + P
template <class T>
constexpr int sk_q_fwd() { return sizeof(T) == 8 ? 8 : 16; }
template <class T>
constexpr int sk_q_inv() { return sizeof(T) == 8 ? 5 : 9; }

template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  const size_t lds = (size_t)2 * g.n * P * sizeof(cx<T>);
  TileWalk tw{(g.m + P - 1) / P, 0, tb.active};
  tw.ntiles = tw.tpm * g.B;
  // persistent grid: as many blocks as stay resident on every CU
#define PCOP_TIME_SK(PP)                                                                                      \
  if (fwd) {                                                                                                  \
    auto kern = time_fwd_sk<T, PP, sk_q_fwd<T>()>;                                                            \
    const int grid = std::min(tw.ntiles, resident_blocks(kern, 256, lds) * std::max(1, tb.ncu));              \
    kern<<<grid, 256, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tw);                    \
  } else {                                                                                                    \
    auto kern = time_inv_sk<T, PP, sk_q_inv<T>()>;                                                            \
    const int grid = std::min(tw.ntiles, resident_blocks(kern, 256, lds) * std::max(1, tb.ncu));              \
    kern<<<grid, 256, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, accum, tw);                               \
  }
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
