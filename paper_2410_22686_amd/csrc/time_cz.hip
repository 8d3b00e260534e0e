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
__device__ __forceinline__ void cz_stage_b(cx<T>* buf, const CzTables<T, M>& tb) {
  constexpr int RA = CzSplit<M>::RA, RB = CzSplit<M>::RB, P = NT / RB, LDM = M + 1;
  constexpr int QB = (P * RA + NT - 1) / NT;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int gb = threadIdx.x + qb * NT;
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
  // this thread's stage-A (and A') group: column pa, residue jb
  const int pa = threadIdx.x % P, jb = threadIdx.x / P;
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  double r1[H], r2[H];  // v_1, v_2 at level j = RB jA + jb of column pa
  auto fetch = [&](int t) {
    const int b = t / tw.tpm;
    const int i = (t - b * tw.tpm) * P + pa;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)n * m;
#pragma unroll
    for (int ja = 0; ja < H; ++ja) {
      const int j = RB * ja + jb;
      const bool in = j < n && i < m;
      r1[ja] = in ? v1[(size_t)j * m + i] : 0.0;
      r2[ja] = in ? v2[(size_t)j * m + i] : 0.0;
    }
  };
  if (tile < tw.ntiles) fetch(tile);
  const T invM = (T)1 / (T)M;
  while (tile < tw.ntiles) {
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
    if (nxt < tw.ntiles) fetch(nxt);
    cz_stage_b<T, M, NT>(buf, tb);
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
  const int pa = threadIdx.x % P, jb = threadIdx.x / P;
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
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1), times the chirp
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + q * NT;
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
    if (nxt < tw.ntiles) fetch(nxt);
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
    cz_stage_b<T, M, NT>(buf, tb);
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

bool cz_exists(int M, int csz, int c) {
  const int NT = c == 32 ? 256 : c == -32 ? 512 : 0;
  if (NT == 0) return false;
  switch (M) {
    case 64: return cz_shape_ok(64, NT, csz);
    case 128: return cz_shape_ok(128, NT, csz);
    case 256: return cz_shape_ok(256, NT, csz);
    case 512: return cz_shape_ok(512, NT, csz);
    case 1024: return cz_shape_ok(1024, NT, csz);
    default: return false;
  }
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
    PCOP_CZ(1024)
    default: return false;
  }
#undef PCOP_CZ
}

template bool launch_time_cz<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const TimeTables&, const double*, int, int, hipStream_t);
template bool launch_time_cz<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const TimeTables&, const double*, int, int, hipStream_t);

}  // namespace pcop
