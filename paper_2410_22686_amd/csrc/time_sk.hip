// Time passes, Stockham kernels with two ping-pong LDS buffers.
#include <algorithm>

#include "time_common.hpp"

namespace pcop {

// Persistent blocks: each block walks column tiles lb, lb + G, ... and
// fetches the global inputs of its next tile into registers before running
// the FFT stages of the current one in LDS, so HBM traffic overlaps the
// stages (two [n][P] buffers allow only a few blocks per CU).  A tile covers
// P consecutive points of every row (64 bytes in FP64), so a 128-byte line
// is shared by neighbouring tiles; consecutive logical blocks sit on one XCD
// and process neighbouring tiles at the same time, so the halves of a line
// meet in that XCD's L2.
//
// Tile t covers member t / tiles_per_member and spatial points
// i0 .. i0 + P - 1 with i0 = (t mod tiles_per_member) P.

// Q = register slots per thread for one tile's inputs: n P <= Q * NT
template <class T, int P, int Q, int NT>
__global__ void __launch_bounds__(NT) time_fwd_sk(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, const double* __restrict__ vscale, int vs_stride,
                                                   TileWalk tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int nP = n * P;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + nP;
  // twiddles and D_eps powers live in LDS, so that inside the loop the only
  // global loads are the prefetch (loads retire in order)
  cx<T>* tw_l = bufB + nP;
  double* dp_l = reinterpret_cast<double*>(tw_l + n);  // d_j
  double* di_l = dp_l + n;                              // 1 / d_j
  for (int t = threadIdx.x; t < n; t += NT) {
    tw_l[t] = twn[t];
    dp_l[t] = dpow[t];
    di_l[t] = 1.0 / dpow[t];
  }
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[Q], r2[Q];  // v_1, v_2 at element e = threadIdx.x + q * NT of the tile
  auto fetch = [&](int t) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)n * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
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
      const int e = threadIdx.x + q * NT;
      if (e < nP) {
        const int j = e / P;
        bufA[e] = cx<T>{(T)(s * dp_l[j] * r2[q]), (T)(s * di_l[j] * r1[q])};
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
      sk_stage_rt<T, P, -1>(plan.rad[st], n, Ns, tw_l, ld, sto);
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

// Q = register slots per thread for one tile's spectrum: K P <= Q * NT.
// ACC: add into w instead of overwriting it (a compile-time switch, so the
// common kernel issues no global loads besides the prefetch)
template <class T, int P, int Q, int ACC, int NT>
__global__ void __launch_bounds__(NT) time_inv_sk(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, TileWalk tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int KP = K * P;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  cx<T>* tw_l = bufB + n * P;
  double* dn_l = reinterpret_cast<double*>(tw_l + n);  // d_j / n
  double* di_l = dn_l + n;                              // 1 / (n d_j)
  for (int t = threadIdx.x; t < n; t += NT) {
    tw_l[t] = twn[t];
    dn_l[t] = dpow[t] / (double)n;
    di_l[t] = 1.0 / ((double)n * dpow[t]);
  }
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[Q], r1[Q];  // Z_2, Z_1 at element e = threadIdx.x + q * NT = k P + p
  auto fetch = [&](int t) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
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
      const int e = threadIdx.x + q * NT;
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
    double* w1 = w + (size_t)b * g.vs;
    double* w2 = w1 + (size_t)n * m;
    cx<T>* src = bufA;
    cx<T>* dst = bufB;
    int Ns = 1;
    for (int st = 0; st < plan.nrad; ++st) {
      auto ld = [&](int j, int p) { return src[j * P + p]; };
      if (st + 1 < plan.nrad) {
        auto sto = [&](int j, int p, cx<T> val) { dst[j * P + p] = val; };
        sk_stage_rt<T, P, 1>(plan.rad[st], n, Ns, tw_l, ld, sto);
        __syncthreads();
        cx<T>* t = src;
        src = dst;
        dst = t;
      } else {
        auto sto = [&](int j, int p, cx<T> val) {
          const int i = i0 + p;
          if (i < m) {
            // z_2 = Re(e) / (n d_j), z_1 = Im(e) d_j / n; w_1 = z_1 - z_2, w_2 = z_1 + z_2
            const double z2 = (double)val.x * di_l[j], z1 = (double)val.y * dn_l[j];
            const size_t o = (size_t)j * m + i;
            if (ACC) {
              w1[o] += z1 - z2;
              w2[o] += z1 + z2;
            } else {
              w1[o] = z1 - z2;
              w2[o] = z1 + z2;
            }
          }
        };
        sk_stage_rt<T, P, 1>(plan.rad[st], n, Ns, tw_l, ld, sto);
      }
      Ns *= plan.rad[st];
    }
    __syncthreads();
    tile = nxt;
  }
}

// register slots: with 256 threads the two [n][P] buffers fit 64 KiB, so
// n P <= 2048 (FP64) or 4096 (FP32) and K P <= n P / 2 + P; the wide kernels
// (512 threads, two buffers of up to 128 KiB) keep the same slots per thread
template <class T>
constexpr int sk_q_fwd() { return sizeof(T) == 8 ? 8 : 16; }
template <class T>
constexpr int sk_q_inv() { return sizeof(T) == 8 ? 5 : 9; }

template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  const size_t lds = sk_lds_bytes(g.n, P, sizeof(cx<T>));
  TileWalk tw{(g.m + P - 1) / P, 0, tb.active};
  tw.ntiles = tw.tpm * g.B;
  // persistent grid: as many blocks as stay resident on every CU
#define PCOP_TIME_SK_NT(PP, NTT)                                                                              \
  if (fwd) {                                                                                                  \
    auto kern = time_fwd_sk<T, PP, sk_q_fwd<T>(), NTT>;                                                       \
    const int grid = std::min(tw.ntiles, resident_blocks(kern, NTT, lds) * std::max(1, tb.ncu));              \
    kern<<<grid, NTT, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tw);                   \
  } else {                                                                                                    \
    auto kern = accum ? time_inv_sk<T, PP, sk_q_inv<T>(), 1, NTT> : time_inv_sk<T, PP, sk_q_inv<T>(), 0, NTT>; \
    const int grid = std::min(tw.ntiles, resident_blocks(kern, NTT, lds) * std::max(1, tb.ncu));              \
    kern<<<grid, NTT, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, tw);                                      \
  }
#define PCOP_TIME_SK(PP) PCOP_TIME_SK_NT(PP, 256)
  if (P == 16 && (size_t)2 * g.n * P * sizeof(cx<T>) > 65536) {
    // wide tiles: two buffers above 64 KiB, 512 threads, one block per CU
    static bool attr_set = false;
    if (!attr_set) {
      attr_set = true;
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(time_fwd_sk<T, 16, sk_q_fwd<T>(), 512>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(time_inv_sk<T, 16, sk_q_inv<T>(), 0, 512>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(time_inv_sk<T, 16, sk_q_inv<T>(), 1, 512>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
    }
    PCOP_TIME_SK_NT(16, 512)
  } else if (P == 16) {
    PCOP_TIME_SK(16)
  } else if (P == 8) {
    PCOP_TIME_SK(8)
  } else {
    PCOP_TIME_SK(4)
  }
#undef PCOP_TIME_SK_NT
#undef PCOP_TIME_SK
}

template void launch_time_sk<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const cx<double>*, const double*, int, int, hipStream_t);
template void launch_time_sk<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const cx<float>*, const double*, int, int, hipStream_t);

}  // namespace pcop
