// Time passes for lengths with a prime factor above 17 (and long smooth
// lengths whose Stockham tiles exceed LDS): chirp-z (Bluestein) transform
// with power-of-two convolutions in LDS.
//
// Persistent blocks walk column tiles lb, lb + G, ... (round robin, so that
// neighbouring tiles, which share 128-byte lines, run at the same time on one
// XCD) and fetch the global inputs of their next tile into registers before
// the convolution of the current one runs in LDS.  Twiddles, the filter
// spectrum, the chirp and the D_eps factors are copied to LDS once per block
// when they fit, so that inside the loop the prefetch is the only global load
// (loads retire in order: any other load would wait for the prefetch).
#include <algorithm>

#include "time_common.hpp"

namespace pcop {

// register slots per thread: n P (forward inputs) and (n/2 + 1) P (inverse
// spectra) elements over NT threads, with n <= M/2
constexpr int bl_q_fwd(int M, int P, int NT) { return std::max(1, (M / 2 * P + NT - 1) / NT); }
constexpr int bl_q_inv(int M, int P, int NT) { return std::max(1, ((M / 4 + 1) * P + NT - 1) / NT); }

// the chirp-z tables a block reads: in LDS (LT) or straight from global memory
template <class T, int M, bool LT>
struct BlTables {
  const cx<T>* tw;   // exp(-2 pi i t/M)
  const cx<T>* bh;   // filter spectrum, index min(k, M - k)
  const cx<T>* ch;   // chirp
  const double* da;  // forward: d_j;      inverse: d_j / n
  const double* db;  // forward: 1 / d_j;  inverse: 1 / (n d_j)

  __device__ __forceinline__ BlTables(unsigned char* tail, const TimeTables& tt, const double* dpow, int n,
                                      bool fwd, int NT) {
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(tt.twM);
    const cx<T>* bhg = reinterpret_cast<const cx<T>*>(tt.bhat);
    const cx<T>* chg = reinterpret_cast<const cx<T>*>(tt.chirp);
    if constexpr (LT) {
      // FP64 stages use exp(-2 pi i t/M) for t < M/2 only (successive powers)
      constexpr int ntw = sizeof(T) == 8 ? M / 2 : M;
      cx<T>* tw_l = reinterpret_cast<cx<T>*>(tail);
      cx<T>* bh_l = tw_l + ntw;
      cx<T>* ch_l = bh_l + (M / 2 + 1);
      double* da_l = reinterpret_cast<double*>(ch_l + n);
      double* db_l = da_l + n;
      for (int t = threadIdx.x; t < ntw; t += NT) tw_l[t] = twg[t];
      for (int t = threadIdx.x; t <= M / 2; t += NT) bh_l[t] = bhg[t];
      for (int t = threadIdx.x; t < n; t += NT) {
        ch_l[t] = chg[t];
        const double d = dpow[t];
        da_l[t] = fwd ? d : d / (double)n;
        db_l[t] = fwd ? 1.0 / d : 1.0 / ((double)n * d);
      }
      tw = tw_l;
      bh = bh_l;
      ch = ch_l;
      da = da_l;
      db = db_l;
    } else {
      // (the widest tiles of the longest lengths)
      (void)tail;
      tw = twg;
      bh = bhg;
      ch = chg;
      da = dpow;
      db = nullptr;
    }
  }
  __device__ __forceinline__ cx<T> filter(int k) const { return bh[k <= M / 2 ? k : M - k]; }
  // forward input scale factors s d_j and s / d_j
  __device__ __forceinline__ double fwd_d(int j) const { return da[j]; }
  __device__ __forceinline__ double fwd_dinv(int j) const {
    if constexpr (LT) return db[j];
    else return 1.0 / da[j];
  }
  // inverse output scale factors d_j / n and 1 / (n d_j)
  __device__ __forceinline__ double inv_dn(int j, int n) const {
    if constexpr (LT) return da[j];
    else return da[j] / (double)n;
  }
  __device__ __forceinline__ double inv_di(int j, int n) const {
    if constexpr (LT) return db[j];
    else return 1.0 / ((double)n * da[j]);
  }
};

template <class T, int P, int M, int NT>
__global__ void __launch_bounds__(NT) time_fwd_bl(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, TimeTables tt,
                                                   const double* __restrict__ vscale, int vs_stride, TileWalk tw) {
  constexpr int LD = M + 1;
  constexpr int Q = bl_q_fwd(M, P, NT);
  constexpr bool LT = bl_tables_in_lds(M, P, (int)sizeof(cx<T>));
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int nP = n * P;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const BlTables<T, M, LT> tb(smem + sizeof(cx<T>) * P * LD, tt, dpow, n, true, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[Q], r2[Q];  // v_1, v_2 at element e = threadIdx.x + q NT = j P + p of the tile
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
  const T invM = (T)1 / (T)M;
  while (tile < tw.ntiles) {
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    // x_j w_j with x_j = s (d_j v2_j + i v1_j / d_j), zero-padded to M
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < nP) {
        const int j = e / P, p = e - j * P;
        const cx<T> x{(T)(s * tb.fwd_d(j) * r2[q]), (T)(s * tb.fwd_dinv(j) * r1[q])};
        buf[p * LD + j] = x * tb.ch[j];
      }
    }
    // zero padding up to M/2 (n <= M/2; the first stage takes the upper half as zero)
    for (int t = threadIdx.x; t < (M / 2 - n) * P; t += NT) {
      const int j = n + t / P, p = t % P;
      buf[p * LD + j] = cx<T>{0, 0};
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt);
    // convolution with the chirp filter: FFT, filter spectrum (in the last
    // stage), inverse FFT of which only the first n < M/2 outputs are used
    p2_fft_x<T, -1, M, P, NT, true, false>(buf, LD, tb.tw, [&](int k, cx<T> x) { return x * tb.filter(k); });
    p2_fft_x<T, 1, M, P, NT, false, true>(buf, LD, tb.tw, P2Keep{});
    // X_k = w_k (x w * conj w)_k: the chirp again and 1/M of the inverse FFT
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return scale(buf[p * LD + k] * tb.ch[k], invM); });
    __syncthreads();
    tile = nxt;
  }
}

// inverse DFT through the forward chirp transform: e = conj(DFT(conj(E)))
template <class T, int P, int M, int NT>
__global__ void __launch_bounds__(NT) time_inv_bl(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, TimeTables tt, int accum,
                                                   TileWalk tw) {
  constexpr int LD = M + 1;
  constexpr int Q = bl_q_inv(M, P, NT);
  constexpr bool LT = bl_tables_in_lds(M, P, (int)sizeof(cx<T>));
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int KP = K * P;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const BlTables<T, M, LT> tb(smem + sizeof(cx<T>) * P * LD, tt, dpow, n, false, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[Q], r1[Q];  // Z_2, Z_1 at element e = threadIdx.x + q NT = k P + p
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
  const double invM = 1.0 / (double)M;
  while (tile < tw.ntiles) {
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < KP) {
        const int k = e / P, p = e - k * P;
        const cx<T> z2 = r2[q], z1 = r1[q];
        // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1)
        const cx<T> ek{z2.x - z1.y, -(z2.y + z1.x)};
        buf[p * LD + k] = ek * tb.ch[k];
        if (k != 0 && 2 * k != n) {
          const cx<T> enk{z2.x + z1.y, -(z1.x - z2.y)};
          buf[p * LD + (n - k)] = enk * tb.ch[n - k];
        }
      }
    }
    // zero padding up to M/2 (n <= M/2; the first stage takes the upper half as zero)
    for (int t = threadIdx.x; t < (M / 2 - n) * P; t += NT) {
      const int j = n + t / P, p = t % P;
      buf[p * LD + j] = cx<T>{0, 0};
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt);
    // convolution with the chirp filter: FFT, filter spectrum (in the last
    // stage), inverse FFT of which only the first n < M/2 outputs are used
    p2_fft_x<T, -1, M, P, NT, true, false>(buf, LD, tb.tw, [&](int k, cx<T> x) { return x * tb.filter(k); });
    p2_fft_x<T, 1, M, P, NT, false, true>(buf, LD, tb.tw, P2Keep{});
    double* w1 = w + (size_t)b * g.vs;
    double* w2 = w1 + (size_t)n * m;
    for (int t = threadIdx.x; t < n * P; t += NT) {
      const int j = t / P, p = t - j * P;
      const int i = i0 + p;
      if (i >= m) continue;
      // e_j = conj(w_j c_j / M); z_2 = Re(e)/(n d_j), z_1 = Im(e) d_j/n
      const cx<T> e = buf[p * LD + j] * tb.ch[j];
      const double z2 = ((double)e.x * invM) * tb.inv_di(j, n);
      const double z1 = (-(double)e.y * invM) * tb.inv_dn(j, n);
      const size_t o = (size_t)j * m + i;
      if (accum) {
        w1[o] += z1 - z2;
        w2[o] += z1 + z2;
      } else {
        w1[o] = z1 - z2;
        w2[o] = z1 + z2;
      }
    }
    __syncthreads();
    tile = nxt;
  }
}

template <class T, int P, int M, int NT>
static bool bl_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if constexpr (bl_shape_ok(M, P, NT, (int)sizeof(cx<T>))) {
    const size_t lds = bl_lds_bytes(M, P, g.n, (int)sizeof(cx<T>));
    auto kf = time_fwd_bl<T, P, M, NT>;
    auto ki = time_inv_bl<T, P, M, NT>;
    if (lds > 65536) {
      // above 64 KiB of dynamic LDS the kernels must opt in (once each)
      static bool attr_set = false;
      if (!attr_set) {
        attr_set = true;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kf), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLdsMax);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(ki), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLdsMax);
        (void)hipGetLastError();
      }
    }
    TileWalk twk{(g.m + P - 1) / P, 0, tb.active};
    twk.ntiles = twk.tpm * g.B;
    // persistent grid: as many blocks as stay resident on every CU
    if (fwd) {
      const int grid = std::min(twk.ntiles, resident_blocks(kf, NT, lds) * std::max(1, tb.ncu));
      kf<<<std::max(grid, 1), NT, lds, st>>>(g, v, spec, tb.dpow, tt, vscale, vs_stride, twk);
    } else {
      const int grid = std::min(twk.ntiles, resident_blocks(ki, NT, lds) * std::max(1, tb.ncu));
      ki<<<std::max(grid, 1), NT, lds, st>>>(g, spec, w, tb.dpow, tt, accum, twk);
    }
    return true;
  } else {
    return false;
  }
}

template <class T, int P, int NT>
static bool bl_dispatch_M(bool fwd, int M, const Geo& g, const double* v, cx<T>* spec, double* w,
                          const PrecondTables& tb, const TimeTables& tt, const double* vscale, int vs_stride,
                          int accum, hipStream_t st) {
#define PCOP_BL_M(MM) \
  case MM: return bl_launch<T, P, MM, NT>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  switch (M) {
    PCOP_BL_M(64)
    PCOP_BL_M(128)
    PCOP_BL_M(256)
    PCOP_BL_M(512)
    PCOP_BL_M(1024)
    PCOP_BL_M(2048)
    PCOP_BL_M(4096)
    default: return false;
  }
#undef PCOP_BL_M
}

// shape of a choice c: +P (256 threads) or -P (512 threads)
static bool bl_exists(int M, int csz, int c) {
  const int P = c < 0 ? -c : c, NT = c < 0 ? 512 : 256;
  return P >= 1 && P <= 16 && (P & (P - 1)) == 0 && bl_shape_ok(M, P, NT, csz);
}

int bl_choice(int M, int n, int csz, int req) {
  if (req == 64 || req == -64) {
    if (pr_exists(n, csz, req)) return req;
    req = 0;
  }
  if (req == 32 || req == -32) {
    if (cz_exists(M, csz, req)) return req;
    req = 0;
  }
  if (req > 0 || req < -1) {
    // at most |req| points, with the requested thread count
    for (int P = req > 0 ? req : -req; P >= 1; P /= 2) {
      const int c = req > 0 ? P : -P;
      if (bl_exists(M, csz, c)) return c;
    }
  }
  // automatic: the prime-factor kernels where they were measured faster
  // (16-point tiles at n = 511, in both precisions), else the three-stage
  // kernels (256 threads, else 512), else the two-FFT kernels with 256
  // threads and the widest tile that keeps two blocks per CU, else the
  // widest that fits at all
  if (const int c = pr_auto(n, csz)) return c;
  if (const int c = cz_auto(M, csz)) return c;
  for (int P = 16; P >= 1; P /= 2)
    if (bl_exists(M, csz, P) && bl_lds_bytes(M, P, n, csz) <= kLdsMax / 2) return P;
  for (int P = 16; P >= 1; P /= 2)
    if (bl_exists(M, csz, P) && bl_lds_bytes(M, P, n, csz) <= kLdsMax) return P;
  return 0;
}

template <class T>
bool launch_time_bl(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (bl_lds_bytes(tb.plan.M, c < 0 ? -c : c, g.n, (int)sizeof(cx<T>)) > kLdsMax) return false;
#define PCOP_BL_P(CC, PP, NTT) \
  if (c == CC) return bl_dispatch_M<T, PP, NTT>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  PCOP_BL_P(16, 16, 256)
  PCOP_BL_P(8, 8, 256)
  PCOP_BL_P(4, 4, 256)
  PCOP_BL_P(2, 2, 256)
  PCOP_BL_P(1, 1, 256)
  PCOP_BL_P(-16, 16, 512)
  PCOP_BL_P(-8, 8, 512)
  PCOP_BL_P(-4, 4, 512)
#undef PCOP_BL_P
  return false;
}

template bool launch_time_bl<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const TimeTables&, const double*, int, int, hipStream_t);
template bool launch_time_bl<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const TimeTables&, const double*, int, int, hipStream_t);

}  // namespace pcop
