// Time passes, Stockham kernels with two ping-pong LDS buffers.
#include <algorithm>
#include <initializer_list>

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

// Stage sequences of the two-buffer kernels, ping-ponging between LDS
// buffers src and dst; they return the buffer holding the result.  With
// LASTOUT the last stage writes through `last` instead (the inverse pass
// stores it to HBM).  PlanRT follows the host plan's radices at run time;
// PlanCT<R...> is a fixed radix list (the plan of a common length), so each
// stage is straight-line code with its sizes known at compile time.
struct PlanRT {};
template <int... R>
struct PlanCT {};

// the transform length of a compile-time plan (0 for the run-time plan)
template <class PL>
struct plan_len {
  static constexpr int value = 0;
};
template <int... R>
struct plan_len<PlanCT<R...>> {
  static constexpr int value = (R * ...);
};

template <class T, int P, int SG, bool LASTOUT, int NS, int R, int... RS>
struct StagesCT {
  template <class LAST>
  static __device__ __forceinline__ cx<T>* run(const cx<T>* tw, cx<T>* src, cx<T>* dst, LAST last) {
    constexpr int N = (R * ... * RS) * NS;
    auto ld = [&](int j, int p) { return src[j * P + p]; };
    if constexpr (sizeof...(RS) == 0 && LASTOUT) {
      sk_stage<T, R, P, SG>(N, NS, tw, ld, last);
      return src;
    } else {
      auto sto = [&](int j, int p, cx<T> val) { dst[j * P + p] = val; };
      sk_stage<T, R, P, SG>(N, NS, tw, ld, sto);
      __syncthreads();
      if constexpr (sizeof...(RS) == 0) return dst;
      else return StagesCT<T, P, SG, LASTOUT, NS * R, RS...>::run(tw, dst, src, last);
    }
  }
};

template <class T, int P, int SG, bool LASTOUT, class LAST>
__device__ __forceinline__ cx<T>* run_stages(PlanRT, const FftPlan& plan, int n, const cx<T>* tw, cx<T>* src,
                                             cx<T>* dst, LAST last) {
  int Ns = 1;
  for (int st = 0; st < plan.nrad; ++st) {
    auto ld = [&](int j, int p) { return src[j * P + p]; };
    if (LASTOUT && st + 1 == plan.nrad) {
      sk_stage_rt<T, P, SG>(plan.rad[st], n, Ns, tw, ld, last);
    } else {
      auto sto = [&](int j, int p, cx<T> val) { dst[j * P + p] = val; };
      sk_stage_rt<T, P, SG>(plan.rad[st], n, Ns, tw, ld, sto);
      __syncthreads();
      cx<T>* t = src;
      src = dst;
      dst = t;
    }
    Ns *= plan.rad[st];
  }
  return src;
}

template <class T, int P, int SG, bool LASTOUT, class LAST, int... R>
__device__ __forceinline__ cx<T>* run_stages(PlanCT<R...>, const FftPlan&, int, const cx<T>* tw, cx<T>* src,
                                             cx<T>* dst, LAST last) {
  return StagesCT<T, P, SG, LASTOUT, 1, R...>::run(tw, src, dst, last);
}

// Q = register slots per thread for one tile's inputs: n P <= Q * NT
template <class T, int P, int Q, int NT, class PL>
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
      // a wave past the tile's last element skips the round (a uniform
      // branch); the others load from a clamped in-bounds index (elements
      // e >= nP are not committed and columns i >= m are never stored)
      if (__builtin_amdgcn_readfirstlane(e) >= nP) continue;
      const int j = min(e / P, n - 1), i = min(i0 + (e % P), m - 1);
      r1[q] = v1[(size_t)j * m + i];
      r2[q] = v2[(size_t)j * m + i];
    }
  };
  // c_j = s (d_j v2_j + i v1_j / d_j), stored at [j][p] = element e
  auto stage0 = [&](int t) {
    const int b = t / tw.tpm;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < nP) {
        const int j = e / P;
        bufA[e] = cx<T>{(T)(s * dp_l[j] * r2[q]), (T)(s * di_l[j] * r1[q])};
      }
    }
  };
  // The first tile's stage 0 is peeled off the loop: inside it stage 0
  // follows the previous tile's stores, and with the compile-time plan
  // (every store unconditional) its wait for the prefetched inputs leaves
  // those stores in flight.
  if (tile < tw.ntiles) {
    fetch(tile);
    stage0(tile);
  }
  while (tile < tw.ntiles) {
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt);
    auto none = [](int, int, cx<T>) {};
    cx<T>* src = run_stages<T, P, -1, false>(PL{}, plan, n, tw_l, bufA, bufB, none);
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    // the unrolled store rounds cost registers: only the 512-thread tiles
    // (one block per CU, below 256 registers either way) take them
    constexpr int NL = plan_len<PL>::value;
    if constexpr (NL > 0 && NT == 512)
      unpack_store_u<T, NT, NL / 2 + 1, P>(out, n, i0, m, threadIdx.x, [&](int k, int p) { return src[k * P + p]; });
    else
      unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return src[k * P + p]; });
    __syncthreads();
    tile = nxt;
    if (tile < tw.ntiles) stage0(tile);
  }
}

// Q = register slots per thread for one tile's spectrum: K P <= Q * NT.
// ACC: add into w instead of overwriting it (a compile-time switch, so the
// common kernel issues no global loads besides the prefetch)
template <class T, int P, int Q, int ACC, int NT, class PL>
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
    auto sto_out = [&](int j, int p, cx<T> val) {
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
    run_stages<T, P, 1, true>(PL{}, plan, n, tw_l, bufA, bufB, sto_out);
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

// launch one kernel pair with stage runner PL (persistent grid: as many
// blocks as stay resident on every CU)
template <class T, int P, int NT, class PL>
static void sk_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const cx<T>* twn, const double* vscale, int vs_stride, int accum, const TileWalk& tw,
                      size_t lds, hipStream_t st) {
  auto kf = time_fwd_sk<T, P, sk_q_fwd<T>(), NT, PL>;
  auto ki0 = time_inv_sk<T, P, sk_q_inv<T>(), 0, NT, PL>;
  auto ki1 = time_inv_sk<T, P, sk_q_inv<T>(), 1, NT, PL>;
  if (lds > 65536) {
    // above 64 KiB of dynamic LDS the kernels must opt in (once each)
    static bool attr_set = false;
    if (!attr_set) {
      attr_set = true;
      for (const void* k : {reinterpret_cast<const void*>(kf), reinterpret_cast<const void*>(ki0),
                            reinterpret_cast<const void*>(ki1)})
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
    }
  }
  if (fwd) {
    const int grid = std::min(tw.ntiles, resident_blocks(kf, NT, lds) * std::max(1, tb.ncu));
    kf<<<grid, NT, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tw);
  } else {
    auto ki = accum ? ki1 : ki0;
    const int grid = std::min(tw.ntiles, resident_blocks(ki, NT, lds) * std::max(1, tb.ncu));
    ki<<<grid, NT, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, tw);
  }
}

static bool plan_is(const FftPlan& pl, std::initializer_list<int> r) {
  if (pl.nrad != (int)r.size()) return false;
  int k = 0;
  for (int x : r)
    if (pl.rad[k++] != x) return false;
  return true;
}

template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  const size_t lds = sk_lds_bytes(g.n, P, sizeof(cx<T>));
  TileWalk tw{(g.m + P - 1) / P, 0, tb.active};
  tw.ntiles = tw.tpm * g.B;
  const bool wide = P == 16 && (size_t)2 * g.n * P * sizeof(cx<T>) > 65536;
  // compile-time stage lists for common lengths (n = 255 = 3 * 5 * 17)
  const bool ct255 = P == 16 && plan_is(tb.plan, {3, 5, 17});
  using CT255 = PlanCT<3, 5, 17>;
#define PCOP_SK(PP, NTT, PL) sk_launch<T, PP, NTT, PL>(fwd, g, v, spec, w, tb, twn, vscale, vs_stride, accum, tw, lds, st)
  if (wide) {
    // wide tiles: two buffers above 64 KiB, 512 threads, one block per CU
    if (ct255) PCOP_SK(16, 512, CT255);
    else PCOP_SK(16, 512, PlanRT);
  } else if (P == 16) {
    if (ct255) PCOP_SK(16, 256, CT255);
    else PCOP_SK(16, 256, PlanRT);
  } else if (P == 8) {
    PCOP_SK(8, 256, PlanRT);
  } else {
    PCOP_SK(4, 256, PlanRT);
  }
#undef PCOP_SK
}

template void launch_time_sk<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const cx<double>*, const double*, int, int, hipStream_t);
template void launch_time_sk<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const cx<float>*, const double*, int, int, hipStream_t);

}  // namespace pcop
