// Time passes for chirp-z lengths (n with a prime factor above 17) with the
// convolution of length M = RA RB <= 1024 done in three LDS stages.
//
// The zero-padded chirp-multiplied column x (n <= M/2 values) is convolved
// with the chirp filter by FFT_M, a pointwise product with the filter
// spectrum F and an inverse FFT_M.  With j = RB jA + jB, k = kA + RA kB and
// W = exp(-2 pi i / M):
//   stage A   for each jB: RA-point DFT over jA of x[RB jA + jB] (the upper
//             half of jA is zero), times W^{jB kA}, stored at kA RB + jB;
//   stage B   for each kA: RB-point DFT over the contiguous group kA RB + jB
//             gives X[kA + RA kB]; times F[kA + RA kB]; RB-point inverse DFT;
//             times W^{-jB kA}; stored back in place;
//   stage A'  for each jB: RA-point inverse DFT over kA gives the convolution
//             at j = RB jA + jB (only jA < RA/2 is needed: j < M/2).
// The forward DFT's last stage and the inverse DFT's first stage act on the
// same groups, so they run back to back in registers (one LDS round trip
// instead of two), every stage keeps a whole group in one thread's registers
// (fft_reg.hpp), and there are four barriers per tile.  The forward pass
// feeds stage A straight from the prefetch registers; the inverse pass
// writes stage A' straight to HBM.
//
// Persistent blocks walk column tiles of P = NT / RB spatial points and
// prefetch the next tile's global inputs into registers during the LDS
// stages.  Twiddles, the filter spectrum, the chirp and the D_eps factors
// live in LDS, so inside the loop the prefetch is the only global load
// (loads retire in order: any other load would wait for the prefetch).
#include <algorithm>

#include "fft_reg.hpp"
#include "time_common.hpp"

namespace pcop {

// With ON, v passes through an empty asm statement at the top of every tile:
// the compiler can no longer prove it loop-invariant, so the many per-lane
// addresses derived from it are formed where they are used instead of being
// hoisted out of the tile loop into registers held (and spilled) for the
// whole loop.  Only the lane-pair inverse kernel needs it (without it, it
// spills and runs 1.4x slower); the other kernels run as fast or faster
// with the hoisted addresses (measured on the 127- and 511-point workloads).
template <bool ON>
__device__ __forceinline__ int per_tile(int v) {
  if constexpr (ON) asm volatile("" : "+v"(v));
  return v;
}

// M = RA RB with RA in {RB, 2 RB}
template <int M>
struct CzSplit;
template <>
struct CzSplit<64> {
  static constexpr int RA = 8, RB = 8;
};
template <>
struct CzSplit<128> {
  static constexpr int RA = 16, RB = 8;
};
template <>
struct CzSplit<256> {
  static constexpr int RA = 16, RB = 16;
};
template <>
struct CzSplit<512> {
  static constexpr int RA = 32, RB = 16;
};
template <>
struct CzSplit<1024> {
  static constexpr int RA = 32, RB = 32;
};

constexpr int cz_ra(int M) { return M == 64 ? 8 : M == 128 ? 16 : M == 256 ? 16 : 32; }
constexpr int cz_rb(int M) { return M / cz_ra(M); }

// LDS of one block: the [P][M+1] tile, the twiddles (FP64: W^t for t < RA,
// raised to powers; FP32: W^t for all t < M), the M/2 + 1 filter values, and
// n <= M/2 chirp values and pairs of D_eps factors
constexpr size_t cz_lds_bytes(int M, int NT, int csz) {
  return (size_t)(NT / cz_rb(M)) * (M + 1) * csz + (size_t)(csz == 16 ? cz_ra(M) : M) * csz +
         (size_t)(M / 2 + 1) * csz + (size_t)(M / 2) * csz + (size_t)M * 8;
}
constexpr bool cz_shape_ok(int M, int NT, int csz) {
  return (M == 64 || M == 128 || M == 256 || M == 512 || M == 1024) && (NT == 256 || NT == 512) &&
         NT / cz_rb(M) >= 1 && cz_lds_bytes(M, NT, csz) <= kLdsMax;
}

template <class T, int M>
struct CzTables {
  static constexpr int NTW = sizeof(T) == 8 ? CzSplit<M>::RA : M;
  const cx<T>* tw;   // W^t, t < NTW
  const cx<T>* flt;  // filter spectrum F[k] = bhat[min(k, M - k)], k <= M/2
  const cx<T>* ch;   // chirp, t < n
  const double* da;  // forward: d_j;      inverse: d_j / n
  const double* db;  // forward: 1 / d_j;  inverse: 1 / (n d_j)

  __device__ __forceinline__ CzTables(unsigned char* tail, const TimeTables& tt, const double* dpow, int n, bool fwd,
                                      int NT) {
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(tt.twM);
    const cx<T>* bhg = reinterpret_cast<const cx<T>*>(tt.bhat);
    const cx<T>* chg = reinterpret_cast<const cx<T>*>(tt.chirp);
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(tail);
    cx<T>* flt_l = tw_l + NTW;
    cx<T>* ch_l = flt_l + (M / 2 + 1);
    double* da_l = reinterpret_cast<double*>(ch_l + M / 2);
    double* db_l = da_l + M / 2;
    for (int t = threadIdx.x; t < NTW; t += NT) tw_l[t] = twg[t];
    for (int t = threadIdx.x; t <= M / 2; t += NT) flt_l[t] = bhg[t];
    for (int t = threadIdx.x; t < n; t += NT) {
      ch_l[t] = chg[t];
      const double d = dpow[t];
      da_l[t] = fwd ? d : d / (double)n;
      db_l[t] = fwd ? 1.0 / d : 1.0 / ((double)n * d);
    }
    tw = tw_l;
    flt = flt_l;
    ch = ch_l;
    da = da_l;
    db = db_l;
  }
  __device__ __forceinline__ cx<T> filter(int k) const { return flt[k <= M / 2 ? k : M - k]; }
};

// a[r] *= W^{SG base r}, r = 1..R-1 (W = exp(-2 pi i/M); SG = +1 conjugates)
template <class T, int M, int SG, int R>
__device__ __forceinline__ void cz_twiddle(cx<T>* a, int base, const CzTables<T, M>& tb) {
  if (base == 0) return;
  if constexpr (sizeof(T) == 8) {
    // FP64: powers of one looked-up twiddle
    cx<T> w1 = tb.tw[base];
    if (SG > 0) w1.y = -w1.y;
    cx<T> w = w1;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      a[r] = a[r] * w;
      w = w * w1;
    }
  } else {
    // FP32: every twiddle from the correctly rounded table
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cx<T> w = tb.tw[(r * base) & (M - 1)];
      if (SG > 0) w.y = -w.y;
      a[r] = a[r] * w;
    }
  }
}

// stage B + filter + B' on the groups of this thread (in place)
template <class T, int M, int NT>
__device__ __forceinline__ void cz_stage_b(cx<T>* buf, const CzTables<T, M>& tb, int lane) {
  constexpr int RA = CzSplit<M>::RA, RB = CzSplit<M>::RB, P = NT / RB, LDM = M + 1;
  constexpr int QB = (P * RA + NT - 1) / NT;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int gb = lane + qb * NT;
    if (gb >= P * RA) break;
    const int p = gb % P, kA = gb / P;
    cx<T>* row = buf + p * LDM + kA * RB;
    cx<T> c[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) c[r] = row[r];
    dft_reg<T, -1, RB>(c);  // X[kA + RA kB] = c[kB]
#pragma unroll
    for (int r = 0; r < RB; ++r) c[r] = c[r] * tb.filter(kA + RA * r);
    dft_reg<T, 1, RB>(c);
    cz_twiddle<T, M, 1, RB>(c, kA, tb);
#pragma unroll
    for (int r = 0; r < RB; ++r) row[r] = c[r];
  }
}

template <class T, int M, int NT>
__global__ void __launch_bounds__(NT) time_fwd_cz(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, TimeTables tt,
                                                   const double* __restrict__ vscale, int vs_stride, TileWalk tw) {
  constexpr int RA = CzSplit<M>::RA, RB = CzSplit<M>::RB, P = NT / RB, LDM = M + 1, H = RA / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const CzTables<T, M> tb(smem + sizeof(cx<T>) * P * LDM, tt, dpow, n, true, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[H], r2[H];  // v_1, v_2 at level j = RB jA + jb of column pa
  // this thread's stage-A (and A') group: column pa, residue jb
  auto fetch = [&](int t, int pa, int jb) {
    const int b = t / tw.tpm;
    const int i = (t - b * tw.tpm) * P + pa;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)n * m;
#pragma unroll
    for (int ja = 0; ja < H; ++ja) {
      const int j = RB * ja + jb;
      // an unconditional load from an in-bounds index (a conditional load,
      // or a select on the loaded value, waits for the load here); levels
      // j >= n are skipped in stage A and columns i >= m are never stored
      const size_t o = (j < n && i < m) ? (size_t)j * m + i : 0;
      r1[ja] = v1[o];
      r2[ja] = v2[o];
    }
  };
  if (tile < tw.ntiles) fetch(tile, threadIdx.x % P, threadIdx.x / P);
  const T invM = (T)1 / (T)M;
  while (tile < tw.ntiles) {
    const int lane = per_tile<false>(threadIdx.x);
    const int pa = lane % P, jb = lane / P;
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    // stage A from registers: x_j w_j with x_j = s (d_j v2_j + i v1_j / d_j)
    {
      cx<T> a[RA];
#pragma unroll
      for (int ja = 0; ja < H; ++ja) {
        const int j = RB * ja + jb;
        a[ja] = cx<T>{0, 0};
        if (j < n) {
          const cx<T> x{(T)(s * tb.da[j] * r2[ja]), (T)(s * tb.db[j] * r1[ja])};
          a[ja] = x * tb.ch[j];
        }
      }
      dft_reg_half_in<T, -1, RA>(a);
      cz_twiddle<T, M, -1, RA>(a, jb, tb);
      cx<T>* col = buf + pa * LDM + jb;
#pragma unroll
      for (int ka = 0; ka < RA; ++ka) col[ka * RB] = a[ka];
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, pa, jb);
    cz_stage_b<T, M, NT>(buf, tb, lane);
    __syncthreads();
    // stage A': convolution outputs j = RB jA + jb < n, times the chirp and 1/M
    {
      cx<T> c[RA];
      cx<T>* col = buf + pa * LDM + jb;
#pragma unroll
      for (int ka = 0; ka < RA; ++ka) c[ka] = col[ka * RB];
      dft_reg<T, 1, RA>(c);
#pragma unroll
      for (int ja = 0; ja < H; ++ja) {
        const int j = RB * ja + jb;
        if (j < n) col[ja * RB] = scale(c[ja] * tb.ch[j], invM);
      }
    }
    __syncthreads();
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return buf[p * LDM + k]; });
    __syncthreads();
    tile = nxt;
  }
}

// inverse DFT through the forward chirp transform: e = conj(DFT(conj(E)))
template <class T, int M, int NT>
__global__ void __launch_bounds__(NT) time_inv_cz(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, TimeTables tt, int accum,
                                                   TileWalk tw) {
  constexpr int RA = CzSplit<M>::RA, RB = CzSplit<M>::RB, P = NT / RB, LDM = M + 1, H = RA / 2;
  // prefetch slots: the K <= M/4 + 1 spectrum rows of P columns over NT threads
  constexpr int Q = ((M / 4 + 1) * P + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int KP = K * P;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const CzTables<T, M> tb(smem + sizeof(cx<T>) * P * LDM, tt, dpow, n, false, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[Q], r1[Q];  // Z_2, Z_1 at element e = lane + q NT = k P + p
  auto fetch = [&](int t, int lane) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = lane + q * NT;
      const int k = e / P, i = i0 + (e % P);
      // unconditional loads from an in-bounds index: slots e >= K P are not
      // committed and columns i >= m are never stored
      const size_t o = (e < KP && i < m) ? (size_t)(2 * k) * m + i : 0;
      r2[q] = in[o];
      r1[q] = in[o + m];
    }
  };
  if (tile < tw.ntiles) fetch(tile, threadIdx.x);
  const double invM = 1.0 / (double)M;
  while (tile < tw.ntiles) {
    const int lane = per_tile<false>(threadIdx.x);
    const int pa = lane % P, jb = lane / P;
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1), times the chirp
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = lane + q * NT;
      if (e < KP) {
        const int k = e / P, p = e - k * P;
        const cx<T> z2 = r2[q], z1 = r1[q];
        const cx<T> ek{z2.x - z1.y, -(z2.y + z1.x)};
        buf[p * LDM + k] = ek * tb.ch[k];
        if (k != 0 && 2 * k != n) {
          const cx<T> enk{z2.x + z1.y, -(z1.x - z2.y)};
          buf[p * LDM + (n - k)] = enk * tb.ch[n - k];
        }
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    // stage A: the inputs j = RB jA + jb < n of this thread's group (levels
    // n .. M/2 - 1 are zero), written back over the same residue class
    {
      cx<T> a[RA];
      cx<T>* col = buf + pa * LDM + jb;
#pragma unroll
      for (int ja = 0; ja < H; ++ja) {
        const int j = RB * ja + jb;
        a[ja] = j < n ? col[ja * RB] : cx<T>{0, 0};
      }
      dft_reg_half_in<T, -1, RA>(a);
      cz_twiddle<T, M, -1, RA>(a, jb, tb);
#pragma unroll
      for (int ka = 0; ka < RA; ++ka) col[ka * RB] = a[ka];
    }
    __syncthreads();
    cz_stage_b<T, M, NT>(buf, tb, lane);
    __syncthreads();
    // stage A' and the output: e_j = conj(w_j c_j / M); z_2 = Re(e)/(n d_j),
    // z_1 = Im(e) d_j / n; w_1 = z_1 - z_2, w_2 = z_1 + z_2
    {
      cx<T> c[RA];
      const cx<T>* col = buf + pa * LDM + jb;
#pragma unroll
      for (int ka = 0; ka < RA; ++ka) c[ka] = col[ka * RB];
      dft_reg<T, 1, RA>(c);
      const int i = i0 + pa;
      double* w1 = w + (size_t)b * g.vs;
      double* w2 = w1 + (size_t)n * m;
#pragma unroll
      for (int ja = 0; ja < H; ++ja) {
        const int j = RB * ja + jb;
        if (j < n && i < m) {
          const cx<T> e = c[ja] * tb.ch[j];
          const double z2 = ((double)e.x * invM) * tb.db[j];
          const double z1 = (-(double)e.y * invM) * tb.da[j];
          const size_t o = (size_t)j * m + i;
          if (accum) {
            w1[o] += z1 - z2;
            w2[o] += z1 + z2;
          } else {
            w1[o] = z1 - z2;
            w2[o] = z1 + z2;
          }
        }
      }
    }
    __syncthreads();
    tile = nxt;
  }
}

// ---------------------------------------------------------------------------
// M = 1024 = 32 x 32 with every 32-point group split over a lane pair
// (lanes 2g and 2g + 1 of a wave, h = lane & 1), each lane holding 16
// values: twice the threads per column of the kernels above for the same
// LDS tile (8 columns, 512 threads, where whole groups per thread allow 256)
// and half the data registers per thread.  The halves meet through a
// quad-permute (DPP) exchange inside the wave.  In FP32 these run the
// n = 511 workload's time passes 1.3x faster than whole groups; in FP64
// their stage B still spills registers and whole groups are faster.
// ---------------------------------------------------------------------------

// the partner lane's value (lane ^ 1)
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <class T>
__device__ __forceinline__ cx<T> pair_swap(cx<T> v) {
  return cx<T>{pair_swap(v.x), pair_swap(v.y)};
}

// 32-point DFT over a lane pair by decimation in time: on entry lane h holds
// x[2j + h] (j < 16; with HALF_IN only j < 8 is read, x[16..31] being zero),
// on exit X[16h + k] (k < 16).  X[k] = E[k] + w^k O[k], X[k+16] = E[k] - w^k O[k]
// with E, O the 16-point DFTs of the even and odd inputs.
template <class T, int SG, bool HALF_IN>
__device__ __forceinline__ void dft32_pair_dit(cx<T>* a, int h) {
  if constexpr (HALF_IN) dft_reg_half_in<T, SG, 16>(a);
  else dft_reg<T, SG, 16>(a);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const cx<T> t = h ? rot_root<T, SG>(a[k], k, 32) : a[k];
    const cx<T> o = pair_swap(t);
    a[k] = h ? o - t : t + o;
  }
}

// 32-point DFT over a lane pair by decimation in frequency: on entry lane h
// holds x[16h + j] (j < 16), on exit X[2k + h] (k < 16):
// X[2k] = DFT16(x[j] + x[j+16]), X[2k+1] = DFT16((x[j] - x[j+16]) w^j).
template <class T, int SG>
__device__ __forceinline__ void dft32_pair_dif(cx<T>* a, int h) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const cx<T> o = pair_swap(a[j]);
    a[j] = h ? rot_root<T, SG>(o - a[j], j, 32) : a[j] + o;
  }
  dft_reg<T, SG, 16>(a);
}

// LDS of the paired kernels: the [P][M+1] tile with P = NT/64, twiddles
// (FP64: W^t and W^{16t} for t < 64, raised to powers; FP32: W^t for all
// t < M), the filter, n chirp values and pairs of D_eps factors
constexpr size_t czp_lds_bytes(int NT, int csz) {
  return (size_t)(NT / 64) * 1025 * csz + (size_t)(csz == 16 ? 128 : 1024) * csz + (size_t)513 * csz +
         (size_t)512 * csz + (size_t)1024 * 8;
}
constexpr bool czp_shape_ok(int NT, int csz) { return NT == 512 && czp_lds_bytes(NT, csz) <= kLdsMax; }

template <class T>
struct CzpTables {
  static constexpr int M = 1024, NTW = sizeof(T) == 8 ? 128 : M;
  const cx<T>* tw;   // FP64: W^t (t < 64) then W^{16t} (t < 64); FP32: W^t, t < M
  const cx<T>* flt;  // filter spectrum, k <= M/2
  const cx<T>* ch;   // chirp, t < n
  const double* da;  // forward: d_j;      inverse: d_j / n
  const double* db;  // forward: 1 / d_j;  inverse: 1 / (n d_j)

  __device__ __forceinline__ CzpTables(unsigned char* tail, const TimeTables& tt, const double* dpow, int n,
                                       bool fwd, int NT) {
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(tt.twM);
    const cx<T>* bhg = reinterpret_cast<const cx<T>*>(tt.bhat);
    const cx<T>* chg = reinterpret_cast<const cx<T>*>(tt.chirp);
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(tail);
    cx<T>* flt_l = tw_l + NTW;
    cx<T>* ch_l = flt_l + (M / 2 + 1);
    double* da_l = reinterpret_cast<double*>(ch_l + M / 2);
    double* db_l = da_l + M / 2;
    for (int t = threadIdx.x; t < NTW; t += NT) {
      if constexpr (sizeof(T) == 8) tw_l[t] = twg[t < 64 ? t : 16 * (t - 64)];
      else tw_l[t] = twg[t];
    }
    for (int t = threadIdx.x; t <= M / 2; t += NT) flt_l[t] = bhg[t];
    for (int t = threadIdx.x; t < n; t += NT) {
      ch_l[t] = chg[t];
      const double d = dpow[t];
      da_l[t] = fwd ? d : d / (double)n;
      db_l[t] = fwd ? 1.0 / d : 1.0 / ((double)n * d);
    }
    tw = tw_l;
    flt = flt_l;
    ch = ch_l;
    da = da_l;
    db = db_l;
  }
  __device__ __forceinline__ cx<T> filter(int k) const { return flt[k <= M / 2 ? k : M - k]; }
  // a[r] *= W^{e0 + r step}, r < 16 (W = exp(-2 pi i/M); conjugated for
  // SG = +1), step < 64; FP64 starts from w0 = W^{e0} (from the tables)
  __device__ __forceinline__ void twiddle(cx<T>* a, int e0, cx<T> w0, int step, int SG) const {
    if constexpr (sizeof(T) == 8) {
      // FP64: powers of one looked-up twiddle
      cx<T> w = w0, w1 = tw[step];
      if (SG > 0) {
        w.y = -w.y;
        w1.y = -w1.y;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        a[r] = a[r] * w;
        w = w * w1;
      }
    } else {
      // FP32: every twiddle from the correctly rounded table
      (void)w0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cx<T> w = tw[(e0 + r * step) & (M - 1)];
        if (SG > 0) w.y = -w.y;
        a[r] = a[r] * w;
      }
    }
  }
  // W^{16 t} (FP64 table; t < 64) and W^t (t < 64)
  __device__ __forceinline__ cx<T> w16(int t) const { return sizeof(T) == 8 ? tw[64 + t] : tw[16 * t]; }
  __device__ __forceinline__ cx<T> w1(int t) const { return tw[t]; }
};

template <class T, int NT>
__global__ void __launch_bounds__(NT) time_fwd_czp(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                    const double* __restrict__ dpow, TimeTables tt,
                                                    const double* __restrict__ vscale, int vs_stride, TileWalk tw) {
  constexpr int M = 1024, R = 32, P = NT / 64, LDM = M + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const CzpTables<T> tb(smem + sizeof(cx<T>) * P * LDM, tt, dpow, n, true, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[8], r2[8];  // v_1, v_2 at level j = R (2q + h) + jb of column pa
  // lane h of the pair of group gp; stage A / A' group: column pa, residue jb
  auto fetch = [&](int t, int h, int pa, int jb) {
    const int b = t / tw.tpm;
    const int i = (t - b * tw.tpm) * P + pa;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)n * m;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = R * (2 * q + h) + jb;
      // unconditional load from an in-bounds index (see time_fwd_cz)
      const size_t o = (j < n && i < m) ? (size_t)j * m + i : 0;
      r1[q] = v1[o];
      r2[q] = v2[o];
    }
  };
  if (tile < tw.ntiles) fetch(tile, threadIdx.x & 1, (threadIdx.x >> 1) % P, (threadIdx.x >> 1) / P);
  const T invM = (T)1 / (T)M;
  while (tile < tw.ntiles) {
    const int lane = per_tile<false>(threadIdx.x);
    const int h = lane & 1, gp = lane >> 1;
    const int pa = gp % P, jb = gp / P;
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    cx<T>* col = buf + pa * LDM + jb;
    // stage A: x_j w_j, x_j = s (d_j v2_j + i v1_j / d_j), j = R jA + jb,
    // jA = 2q + h < 16; outputs kA = 16h + k times W^{jb kA}
    {
      cx<T> a[16];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = R * (2 * q + h) + jb;
        a[q] = cx<T>{0, 0};
        if (j < n) {
          const cx<T> x{(T)(s * tb.da[j] * r2[q]), (T)(s * tb.db[j] * r1[q])};
          a[q] = x * tb.ch[j];
        }
      }
      dft32_pair_dit<T, -1, true>(a, h);
      tb.twiddle(a, 16 * h * jb, tb.w16(h * jb), jb, -1);
#pragma unroll
      for (int k = 0; k < 16; ++k) col[(16 * h + k) * R] = a[k];
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, h, pa, jb);
    // stage B: group kA (contiguous row kA R .. kA R + 31 of column p)
    {
      const int p = gp % P, ka = gp / P;
      cx<T>* row = buf + p * LDM + ka * R;
      cx<T> c[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) c[j] = row[2 * j + h];
      dft32_pair_dit<T, -1, false>(c, h);  // X[kA + R (16h + k)]
#pragma unroll
      for (int k = 0; k < 16; ++k) c[k] = c[k] * tb.filter(ka + R * (16 * h + k));
      dft32_pair_dif<T, 1>(c, h);  // u[jB], jB = 2j + h
      tb.twiddle(c, h * ka, tb.w1(h * ka), 2 * ka, 1);  // W^{-jB kA}
#pragma unroll
      for (int j = 0; j < 16; ++j) row[2 * j + h] = c[j];
    }
    __syncthreads();
    // stage A': inverse DFT over kA = 16h + k; outputs jA = 2j + h < 16,
    // times the chirp and 1/M, at j = R jA + jb
    {
      cx<T> c[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) c[k] = col[(16 * h + k) * R];
      dft32_pair_dif<T, 1>(c, h);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int ja = 2 * q + h, j = R * ja + jb;
        if (j < n) col[ja * R] = scale(c[q] * tb.ch[j], invM);
      }
    }
    __syncthreads();
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return buf[p * LDM + k]; });
    __syncthreads();
    tile = nxt;
  }
}

template <class T, int NT>
__global__ void __launch_bounds__(NT) time_inv_czp(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                    const double* __restrict__ dpow, TimeTables tt, int accum,
                                                    TileWalk tw) {
  constexpr int M = 1024, R = 32, P = NT / 64, LDM = M + 1;
  constexpr int Q = ((M / 4 + 1) * P + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, m = g.m, K = g.K;
  const int KP = K * P;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const CzpTables<T> tb(smem + sizeof(cx<T>) * P * LDM, tt, dpow, n, false, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[Q], r1[Q];  // Z_2, Z_1 at element e = lane + q NT = k P + p
  auto fetch = [&](int t, int lane) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * P;
    const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = lane + q * NT;
      const int k = e / P, i = i0 + (e % P);
      // unconditional loads from an in-bounds index: slots e >= K P are not
      // committed and columns i >= m are never stored
      const size_t o = (e < KP && i < m) ? (size_t)(2 * k) * m + i : 0;
      r2[q] = in[o];
      r1[q] = in[o + m];
    }
  };
  if (tile < tw.ntiles) fetch(tile, threadIdx.x);
  const double invM = 1.0 / (double)M;
  while (tile < tw.ntiles) {
    const int lane = per_tile<true>(threadIdx.x);
    const int h = lane & 1, gp = lane >> 1;
    const int pa = gp % P, jb = gp / P;
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * P;
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1), times the chirp
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = lane + q * NT;
      if (e < KP) {
        const int k = e / P, p = e - k * P;
        const cx<T> z2 = r2[q], z1 = r1[q];
        const cx<T> ek{z2.x - z1.y, -(z2.y + z1.x)};
        buf[p * LDM + k] = ek * tb.ch[k];
        if (k != 0 && 2 * k != n) {
          const cx<T> enk{z2.x + z1.y, -(z1.x - z2.y)};
          buf[p * LDM + (n - k)] = enk * tb.ch[n - k];
        }
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    cx<T>* col = buf + pa * LDM + jb;
    // stage A: inputs j = R jA + jb < n, jA = 2q + h < 16 (levels n .. M/2 - 1
    // are zero); outputs kA = 16h + k times W^{jb kA}, over the same residue class
    {
      cx<T> a[16];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = R * (2 * q + h) + jb;
        a[q] = j < n ? col[(2 * q + h) * R] : cx<T>{0, 0};
      }
      dft32_pair_dit<T, -1, true>(a, h);
      tb.twiddle(a, 16 * h * jb, tb.w16(h * jb), jb, -1);
#pragma unroll
      for (int k = 0; k < 16; ++k) col[(16 * h + k) * R] = a[k];
    }
    __syncthreads();
    {
      const int p = gp % P, ka = gp / P;
      cx<T>* row = buf + p * LDM + ka * R;
      cx<T> c[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) c[j] = row[2 * j + h];
      dft32_pair_dit<T, -1, false>(c, h);
#pragma unroll
      for (int k = 0; k < 16; ++k) c[k] = c[k] * tb.filter(ka + R * (16 * h + k));
      dft32_pair_dif<T, 1>(c, h);  // u[jB], jB = 2j + h
      tb.twiddle(c, h * ka, tb.w1(h * ka), 2 * ka, 1);  // W^{-jB kA}
#pragma unroll
      for (int j = 0; j < 16; ++j) row[2 * j + h] = c[j];
    }
    __syncthreads();
    // stage A' and the output: e_j = conj(w_j c_j / M); z_2 = Re(e)/(n d_j),
    // z_1 = Im(e) d_j / n; w_1 = z_1 - z_2, w_2 = z_1 + z_2
    {
      cx<T> c[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) c[k] = col[(16 * h + k) * R];
      dft32_pair_dif<T, 1>(c, h);
      const int i = i0 + pa;
      double* w1 = w + (size_t)b * g.vs;
      double* w2 = w1 + (size_t)n * m;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = R * (2 * q + h) + jb;
        if (j < n && i < m) {
          const cx<T> e = c[q] * tb.ch[j];
          const double z2 = ((double)e.x * invM) * tb.db[j];
          const double z1 = (-(double)e.y * invM) * tb.da[j];
          const size_t o = (size_t)j * m + i;
          if (accum) {
            w1[o] += z1 - z2;
            w2[o] += z1 + z2;
          } else {
            w1[o] = z1 - z2;
            w2[o] = z1 + z2;
          }
        }
      }
    }
    __syncthreads();
    tile = nxt;
  }
}

template <class T, int NT>
static bool czp_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                       const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if constexpr (czp_shape_ok(NT, (int)sizeof(cx<T>))) {
    constexpr size_t lds = czp_lds_bytes(NT, (int)sizeof(cx<T>));
    constexpr int P = NT / 64;
    auto kf = time_fwd_czp<T, NT>;
    auto ki = time_inv_czp<T, NT>;
    if constexpr (lds > 65536) {
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

template <class T, int M, int NT>
static bool cz_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if constexpr (cz_shape_ok(M, NT, (int)sizeof(cx<T>))) {
    constexpr size_t lds = cz_lds_bytes(M, NT, (int)sizeof(cx<T>));
    constexpr int P = NT / CzSplit<M>::RB;
    auto kf = time_fwd_cz<T, M, NT>;
    auto ki = time_inv_cz<T, M, NT>;
    if constexpr (lds > 65536) {
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

// c = 32: whole groups per thread, 256 threads; c = -32: 512 threads (for
// M = 1024, the lane-pair kernels)
bool cz_exists(int M, int csz, int c) {
  const int NT = c == 32 ? 256 : c == -32 ? 512 : 0;
  if (NT == 0) return false;
  switch (M) {
    case 64: return cz_shape_ok(64, NT, csz);
    case 128: return cz_shape_ok(128, NT, csz);
    case 256: return cz_shape_ok(256, NT, csz);
    case 512: return cz_shape_ok(512, NT, csz);
    case 1024: return c == 32 ? cz_shape_ok(1024, 256, csz) : czp_shape_ok(512, csz);
    default: return false;
  }
}

// the automatic three-stage kernel: lane pairs for M = 1024 in FP32 (measured
// faster there); whole groups with 256 threads otherwise (FP64 lane pairs
// spill registers)
int cz_auto(int M, int csz) {
  if (M == 1024 && csz == 8 && cz_exists(M, csz, -32)) return -32;
  if (cz_exists(M, csz, 32)) return 32;
  return cz_exists(M, csz, -32) ? -32 : 0;
}

template <class T>
bool launch_time_cz(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (!cz_exists(tb.plan.M, (int)sizeof(cx<T>), c) || 2 * g.n > tb.plan.M) return false;
#define PCOP_CZ(MM)                                                                                           \
  case MM:                                                                                                    \
    return c == 32 ? cz_launch<T, MM, 256>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st)        \
                   : cz_launch<T, MM, 512>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  switch (tb.plan.M) {
    PCOP_CZ(64)
    PCOP_CZ(128)
    PCOP_CZ(256)
    PCOP_CZ(512)
    case 1024:
      return c == 32 ? cz_launch<T, 1024, 256>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st)
                     : czp_launch<T, 512>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
    default: return false;
  }
#undef PCOP_CZ
}

template bool launch_time_cz<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const TimeTables&, const double*, int, int, hipStream_t);
template bool launch_time_cz<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const TimeTables&, const double*, int, int, hipStream_t);

}  // namespace pcop
