// Time passes for lengths n = N1 PR (N1 and PR coprime, PR prime) by the
// prime-factor (Good-Thomas) split and Rader's algorithm for the PR-point
// transforms; built for n = 511 = 7 x 73.
//
// Index maps (t1 = PR^-1 mod N1, t2 = N1^-1 mod PR):
//   input   j = (PR j1 + N1 j2) mod n,          j1 < N1, j2 < PR
//   output  k = (PR t1 k1 + N1 t2 k2) mod n,    k1 < N1, k2 < PR
// turn the n-point DFT into an N1 x PR two-dimensional DFT with no twiddles:
//   X[k] = sum_{j2} W_PR^{j2 k2} y[k1][j2],   y[k1][j2] = sum_{j1} W_N1^{j1 k1} x[j].
// Rader, with g a generator of the multiplicative group mod PR, j2 = g^-p
// and k2 = g^q (p, q < RC = PR - 1):
//   X[g^q] = y_0 + sum_p a_p b_{q-p},   a_p = y[g^-p],  b_m = W_PR^{g^m},
//   X[0]   = y_0 + sum_p a_p,
// a cyclic convolution of length RC = RA RB, computed as in the chirp-z
// kernels (time_cz.hip) in three LDS stages with j = RB jA + jB and
// k = kA + RA kB:
//   stage A   RA-point DFT over jA for each jB, times W_RC^{jB kA};
//   stage B   RB-point DFT over jB (giving A[kA + RA kB]), times the filter
//             B[k] = DFT_RC(b)[k] / RC, RB-point inverse DFT, times W_RC^{-qB kA};
//   stage A'  RA-point inverse DFT over kA, giving the convolution at q = RB qA + qB.
// y_0 joins every convolution output through the filtered DC term
// (C_0 <- A_0 B_0 + y_0); X[0] = y_0 + A_0 is formed in stage B.
//
// Against the chirp-z transform of the same length (a 1024-point
// convolution for n = 511) a column needs 511 LDS slots instead of 1025 and
// about half the arithmetic, so two FP64 blocks share a CU instead of one.
// Each column's slots hold N1 rows of PR: the Rader inputs a_p at p < RC and
// y_0 at RC; after stage A' row k1 holds X[k1, g^q] at q and X[k1, 0] at RC.
#include <algorithm>

#include "time_common.hpp"

namespace pcop {

// threadIdx.x through an empty asm statement once per tile: the compiler can
// no longer hoist the many per-lane indices and addresses derived from it out
// of the tile loop (held there, they exceed the register budget)
__device__ __forceinline__ int pr_lane() {
  int v = threadIdx.x;
  asm volatile("" : "+v"(v));
  return v;
}

constexpr int pr_inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return m == 1 ? 0 : -1;
}

template <int N1_, int PR_, int G_, int RA_, int RB_>
struct PrPlan {
  static constexpr int N1 = N1_, PR = PR_, G = G_, RA = RA_, RB = RB_, RC = PR_ - 1, N = N1_ * PR_;
  static constexpr int KM1 = PR_ * pr_inv_mod(PR_ % N1_, N1_);  // output map: k = (KM1 k1 + KM2 k2) mod N
  static constexpr int KM2 = N1_ * pr_inv_mod(N1_ % PR_, PR_);
  static_assert(RA * RB == PR_ - 1, "the convolution length splits as RA RB");
};
// 511 = 7 x 73, generator 5 of the group mod 73, 72 = 9 x 8
using Pr511 = PrPlan<7, 73, 5, 9, 8>;

// cos and sin of 2 pi t / R, t = 1 .. (R - 1)/2, to 36 digits
template <int R>
__device__ __forceinline__ double root_cos(int t);
template <int R>
__device__ __forceinline__ double root_sin(int t);
template <>
__device__ __forceinline__ double root_cos<7>(int t) {
  constexpr double c[4] = {1.0, 0.623489801858733530525004884004239811, -0.222520933956314404288902564496794759,
                           -0.900968867902419126236102319507445051};
  return c[t];
}
template <>
__device__ __forceinline__ double root_sin<7>(int t) {
  constexpr double s[4] = {0.0, 0.781831482468029808708444526674057750, 0.974927912181823607018131682993931217,
                           0.433883739117558120475768332848358755};
  return s[t];
}
template <>
__device__ __forceinline__ double root_cos<9>(int t) {
  constexpr double c[5] = {1.0, 0.766044443118978035202392650555416674, 0.173648177666930348851716626769314796,
                           -0.5, -0.939692620785908384054109277324731470};
  return c[t];
}
template <>
__device__ __forceinline__ double root_sin<9>(int t) {
  constexpr double s[5] = {0.0, 0.642787609686539326322643409907263433, 0.984807753012208059366743024589523014,
                           0.866025403784438646763723170752936183, 0.342020143325668733044099614682259581};
  return s[t];
}

// R-point DFT for odd R with literal roots (inputs r and R - r paired, as in
// dft_odd): X_k = a_0 + sum_r s_r cos + SG i sum_r d_r sin, X_{R-k} with the
// sine sum's sign flipped, s_r = a_r + a_{R-r}, d_r = a_r - a_{R-r}
template <class T, int SG, int R>
__device__ __forceinline__ void dft_odd_lit(cx<T>* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 3) {
    dft3<T, SG>(a);
  } else {
    constexpr int H = (R - 1) / 2;
    cx<T> sm[H + 1], df[H + 1];
    cx<T> x0 = a[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      sm[r] = a[r] + a[R - r];
      df[r] = a[r] - a[R - r];
      x0 = x0 + sm[r];
    }
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cx<T> p = a[0], q{0, 0};
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        const int t = (r * k) % R;
        const T ct = (T)(t <= H ? root_cos<R>(t) : root_cos<R>(R - t));
        const T st = (T)(t <= H ? root_sin<R>(t) : -root_sin<R>(R - t));
        p = p + scale(sm[r], ct);
        q = q + scale(df[r], st);
      }
      const cx<T> iq = mul_i<T, SG>(q);
      a[k] = p + iq;
      a[R - k] = p - iq;
    }
    a[0] = x0;
  }
}

// LDS of one block: the [C][N] column tile, then the tables
template <class PL>
constexpr size_t pr_lds_bytes(int C, int csz) {
  return (size_t)C * PL::N * csz + (size_t)2 * PL::RC * csz + (size_t)2 * PL::N * 8 +
         (size_t)(PL::RC + 2 * PL::PR) * 4;
}

template <class T, class PL>
struct PrTables {
  const cx<T>* tw;   // W_RC^t, t < RC
  const cx<T>* bh;   // DFT_RC(b)[k] / RC
  const double* da;  // forward: d_j;      inverse: d_j / n
  const double* db;  // forward: 1 / d_j;  inverse: 1 / (n d_j)
  const int* gpw;    // g^q mod PR, q < RC
  const int* lg;     // q with g^q = k2 (k2 = 1 .. PR - 1)
  const int* slot;   // Rader slot of j2: RC for j2 = 0, else p with g^-p = j2

  __device__ __forceinline__ PrTables(unsigned char* tail, const void* prt, const double* dpow, bool fwd, int NT) {
    constexpr int RC = PL::RC, PR = PL::PR, N = PL::N;
    const cx<T>* src = reinterpret_cast<const cx<T>*>(prt);
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(tail);
    cx<T>* bh_l = tw_l + RC;
    double* da_l = reinterpret_cast<double*>(bh_l + RC);
    double* db_l = da_l + N;
    int* gpw_l = reinterpret_cast<int*>(db_l + N);
    int* lg_l = gpw_l + RC;
    int* slot_l = lg_l + PR;
    for (int t = threadIdx.x; t < 2 * RC; t += NT) tw_l[t] = src[t];
    for (int t = threadIdx.x; t < N; t += NT) {
      const double d = dpow[t];
      da_l[t] = fwd ? d : d / (double)N;
      db_l[t] = fwd ? 1.0 / d : 1.0 / ((double)N * d);
    }
    for (int q = threadIdx.x; q < RC; q += NT) {
      int v = 1;
      for (int s = 0; s < q; ++s) v = (v * PL::G) % PR;
      gpw_l[q] = v;
      lg_l[v] = q;
      slot_l[v] = (RC - q) % RC;  // g^-p = g^q for p = -q mod RC
    }
    if (threadIdx.x == 0) {
      lg_l[0] = RC;
      slot_l[0] = RC;
    }
    tw = tw_l;
    bh = bh_l;
    da = da_l;
    db = db_l;
    gpw = gpw_l;
    lg = lg_l;
    slot = slot_l;
  }
};

// a[r] *= W_RC^{SG base r}, r = 1..R-1 (SG = +1 conjugates)
template <class T, class PL, int SG, int R>
__device__ __forceinline__ void pr_twiddle(cx<T>* a, int base, const PrTables<T, PL>& tb) {
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
      cx<T> w = tb.tw[(r * base) % PL::RC];
      if (SG > 0) w.y = -w.y;
      a[r] = a[r] * w;
    }
  }
}

// stages A and B of the Rader convolutions of every (column, k1) row of the
// tile, with a barrier after each
template <class T, class PL, int C, int NT>
__device__ __forceinline__ void pr_stages_ab(cx<T>* buf, const PrTables<T, PL>& tb, int lane) {
  constexpr int N1 = PL::N1, PR = PL::PR, RA = PL::RA, RB = PL::RB, RC = PL::RC, LDC = PL::N;
  constexpr int IA = C * N1 * RB, QA = (IA + NT - 1) / NT;
  constexpr int IB = C * N1 * RA, QB = (IB + NT - 1) / NT;
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int e = lane + q * NT;
    if (e < IA) {
      const int c = e % C, r = e / C;
      const int k1 = r / RB, jb = r - k1 * RB;
      cx<T>* row = buf + c * LDC + k1 * PR + jb;
      cx<T> a[RA];
#pragma unroll
      for (int ja = 0; ja < RA; ++ja) a[ja] = row[ja * RB];
      dft_odd_lit<T, -1, RA>(a);
      pr_twiddle<T, PL, -1, RA>(a, jb, tb);
#pragma unroll
      for (int ka = 0; ka < RA; ++ka) row[ka * RB] = a[ka];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int e = lane + q * NT;
    if (e < IB) {
      const int c = e % C, r = e / C;
      const int k1 = r / RA, ka = r - k1 * RA;
      cx<T>* rowk = buf + c * LDC + k1 * PR;
      cx<T> cc[RB];
#pragma unroll
      for (int jb = 0; jb < RB; ++jb) cc[jb] = rowk[ka * RB + jb];
      dftR<T, -1, RB>(cc);  // A[ka + RA kb] = cc[kb]
      if (ka == 0) {
        const cx<T> y0 = rowk[RC];
        rowk[RC] = y0 + cc[0];  // X[k1, 0]
        cc[0] = cc[0] * tb.bh[0] + y0;
#pragma unroll
        for (int kb = 1; kb < RB; ++kb) cc[kb] = cc[kb] * tb.bh[RA * kb];
      } else {
#pragma unroll
        for (int kb = 0; kb < RB; ++kb) cc[kb] = cc[kb] * tb.bh[ka + RA * kb];
      }
      dftR<T, 1, RB>(cc);
      pr_twiddle<T, PL, 1, RB>(cc, ka, tb);
#pragma unroll
      for (int qb = 0; qb < RB; ++qb) rowk[ka * RB + qb] = cc[qb];
    }
  }
  __syncthreads();
}

// FP32 with 512 threads: at least 4 waves per SIMD, so that two blocks share
// a CU (their tiles fit LDS twice); the forward kernel then spills 4 registers
// and still runs 1.2x faster than with one block (measured at n = 511)
template <class T, int NT>
constexpr int pr_min_waves() {
  return NT == 512 && sizeof(T) == 4 ? 4 : 1;
}

template <class T, class PL, int C, int NT>
__global__ void __launch_bounds__(NT, (pr_min_waves<T, NT>())) time_fwd_pr(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const void* __restrict__ prt,
                                                   const double* __restrict__ vscale, int vs_stride, TileWalk tw) {
  constexpr int N = PL::N, N1 = PL::N1, PR = PL::PR, RA = PL::RA, RB = PL::RB, LDC = N;
  constexpr int I0 = C * PR, Q0 = (I0 + NT - 1) / NT;
  constexpr int IA = C * N1 * RB, QA = (IA + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = g.m, K = g.K;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const PrTables<T, PL> tb(smem + sizeof(cx<T>) * C * LDC, prt, dpow, true, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  // v_1, v_2 at the N1 levels j(j1, j2) of this thread's stage-0 items
  double r1[Q0][N1], r2[Q0][N1];
  auto fetch = [&](int t, int lane) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * C;
    const double* v1 = v + (size_t)b * g.vs;
    const double* v2 = v1 + (size_t)N * m;
#pragma unroll
    for (int q = 0; q < Q0; ++q) {
      const int e = lane + q * NT;
      const int c = e % C, j2 = e / C, i = i0 + c;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        // unconditional loads from an in-bounds index: items e >= I0 are
        // not committed and columns i >= m are never stored
        const size_t o = (e < I0 && i < m) ? (size_t)((PR * j1 + N1 * j2) % N) * m + i : 0;
        r1[q][j1] = v1[o];
        r2[q][j1] = v2[o];
      }
    }
  };
  if (tile < tw.ntiles) fetch(tile, pr_lane());
  while (tile < tw.ntiles) {
    const int lane = pr_lane();
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * C;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
    // stage 0: x_j = s (d_j v2_j + i v1_j / d_j), N1-point DFTs over j1, into the Rader slots
#pragma unroll
    for (int q = 0; q < Q0; ++q) {
      const int e = lane + q * NT;
      if (e < I0) {
        const int c = e % C, j2 = e / C;
        cx<T> a[N1];
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) {
          const int j = (PR * j1 + N1 * j2) % N;
          a[j1] = cx<T>{(T)(s * tb.da[j] * r2[q][j1]), (T)(s * tb.db[j] * r1[q][j1])};
        }
        dft_odd_lit<T, -1, N1>(a);
        cx<T>* col = buf + c * LDC + tb.slot[j2];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) col[k1 * PR] = a[k1];
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    pr_stages_ab<T, PL, C, NT>(buf, tb, lane);
    // stage A', in place: row k1 then holds X[k1, g^q] at slot q
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = lane + q * NT;
      if (e < IA) {
        const int c = e % C, r = e / C;
        const int k1 = r / RB, qb = r - k1 * RB;
        cx<T>* row = buf + c * LDC + k1 * PR + qb;
        cx<T> a[RA];
#pragma unroll
        for (int ka = 0; ka < RA; ++ka) a[ka] = row[ka * RB];
        dft_odd_lit<T, 1, RA>(a);
#pragma unroll
        for (int qa = 0; qa < RA; ++qa) row[qa * RB] = a[qa];
      }
    }
    __syncthreads();
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    unpack_store<T>(out, N, K, C, i0, m, [&](int k, int p) {
      const int k1 = k % N1, k2 = k % PR;
      return buf[p * LDC + k1 * PR + tb.lg[k2]];
    });
    __syncthreads();
    tile = nxt;
  }
}

// Inverse DFT through the forward transform, e = conj(DFT(conj(E))), with
// the index maps exchanged (the DFT matrix is symmetric): input k = (KM1 k1 +
// KM2 k2) mod n, output j = (PR j1 + N1 j2) mod n, so that
//   R[j] = sum_{k1} W_N1^{k1 j1} sum_{k2} W_PR^{k2 j2} x[k]
// with the Rader transforms first (row k1 = k mod N1 holds the inputs of
// k2 = k mod PR in their Rader slots, scattered there straight from the
// spectrum) and the N1-point DFTs last, writing HBM directly.
template <class T, class PL, int C, int NT>
__global__ void __launch_bounds__(NT, (pr_min_waves<T, NT>())) time_inv_pr(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const void* __restrict__ prt,
                                                   int accum, TileWalk tw) {
  constexpr int N = PL::N, N1 = PL::N1, PR = PL::PR, RA = PL::RA, RB = PL::RB, RC = PL::RC, LDC = N;
  constexpr int I0 = C * PR, Q0 = (I0 + NT - 1) / NT;
  constexpr int IA = C * N1 * RB, QA = (IA + NT - 1) / NT;
  constexpr int KS = N / 2 + 1;  // spectrum rows
  constexpr int QI = (KS * C + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = g.m;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const PrTables<T, PL> tb(smem + sizeof(cx<T>) * C * LDC, prt, dpow, false, NT);
  __syncthreads();
  const int stride = gridDim.x;
  int tile = tw.next(xcd_remap(blockIdx.x, gridDim.x), stride);
  cx<T> r2[QI], r1[QI];  // Z_2, Z_1 at element e = k C + p
  auto fetch = [&](int t, int lane) {
    const int b = t / tw.tpm;
    const int i0 = (t - b * tw.tpm) * C;
    const cx<T>* in = spec + (size_t)b * (size_t)(2 * KS) * m;
#pragma unroll
    for (int q = 0; q < QI; ++q) {
      const int e = lane + q * NT;
      const int k = e / C, i = i0 + e % C;
      const size_t o = (e < KS * C && i < m) ? (size_t)(2 * k) * m + i : 0;
      r2[q] = in[o];
      r1[q] = in[o + m];
    }
  };
  // LDS slot of input k: row k mod N1, Rader slot of k mod PR
  auto kslot = [&](int k) { return (k % N1) * PR + tb.slot[k % PR]; };
  if (tile < tw.ntiles) fetch(tile, pr_lane());
  while (tile < tw.ntiles) {
    const int lane = pr_lane();
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * C;
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1)
#pragma unroll
    for (int q = 0; q < QI; ++q) {
      const int e = lane + q * NT;
      if (e < KS * C) {
        const int k = e / C, p = e - k * C;
        const cx<T> z2 = r2[q], z1 = r1[q];
        buf[p * LDC + kslot(k)] = cx<T>{z2.x - z1.y, -(z2.y + z1.x)};
        if (k != 0 && 2 * k != N) buf[p * LDC + kslot(N - k)] = cx<T>{z2.x + z1.y, -(z1.x - z2.y)};
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    pr_stages_ab<T, PL, C, NT>(buf, tb, lane);
    // stage A', in place: row k1 then holds its PR-point DFT at j2 = g^q in slot q, j2 = 0 in slot RC
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = lane + q * NT;
      if (e < IA) {
        const int c = e % C, r = e / C;
        const int k1 = r / RB, qb = r - k1 * RB;
        cx<T>* row = buf + c * LDC + k1 * PR + qb;
        cx<T> a[RA];
#pragma unroll
        for (int ka = 0; ka < RA; ++ka) a[ka] = row[ka * RB];
        dft_odd_lit<T, 1, RA>(a);
#pragma unroll
        for (int qa = 0; qa < RA; ++qa) row[qa * RB] = a[qa];
      }
    }
    __syncthreads();
    // N1-point DFTs over the rows and the output: R_j at j = (PR j1 + N1 j2) mod n;
    // e_j = conj(R_j); z_2 = Re(e)/(n d_j), z_1 = Im(e) d_j/n; w_1 = z_1 - z_2, w_2 = z_1 + z_2
    double* w1 = w + (size_t)b * g.vs;
    double* w2 = w1 + (size_t)N * m;
#pragma unroll
    for (int q = 0; q < Q0; ++q) {
      const int e = lane + q * NT;
      if (e < I0) {
        const int c = e % C, sl = e / C;
        const int i = i0 + c;
        cx<T> a[N1];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) a[k1] = buf[c * LDC + k1 * PR + sl];
        dft_odd_lit<T, -1, N1>(a);
        if (i < m) {
          const int j2 = sl == RC ? 0 : tb.gpw[sl];
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) {
            const int j = (PR * j1 + N1 * j2) % N;
            const double z2 = (double)a[j1].x * tb.db[j];
            const double z1 = -(double)a[j1].y * tb.da[j];
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
    }
    __syncthreads();
    tile = nxt;
  }
}

template <class T, class PL, int C, int NT>
static bool pr_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const double* vscale, int vs_stride, int accum, hipStream_t st) {
  constexpr size_t lds = pr_lds_bytes<PL>(C, (int)sizeof(cx<T>));
  static_assert(lds <= kLdsMax, "tile and tables fit LDS");
  if (g.n != PL::N) return false;
  const void* prt = sizeof(T) == 8 ? (const void*)tb.pr64 : (const void*)tb.pr32;
  if (!prt) return false;
  auto kf = time_fwd_pr<T, PL, C, NT>;
  auto ki = time_inv_pr<T, PL, C, NT>;
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
  TileWalk twk{(g.m + C - 1) / C, 0, tb.active};
  twk.ntiles = twk.tpm * g.B;
  // persistent grid: as many blocks as stay resident on every CU
  if (fwd) {
    const int grid = std::min(twk.ntiles, resident_blocks(kf, NT, lds) * std::max(1, tb.ncu));
    kf<<<std::max(grid, 1), NT, lds, st>>>(g, v, spec, tb.dpow, prt, vscale, vs_stride, twk);
  } else {
    const int grid = std::min(twk.ntiles, resident_blocks(ki, NT, lds) * std::max(1, tb.ncu));
    ki<<<std::max(grid, 1), NT, lds, st>>>(g, spec, w, tb.dpow, prt, accum, twk);
  }
  return true;
}

bool pr_params(int n, int* pr, int* gen) {
  if (n == Pr511::N) {
    *pr = Pr511::PR;
    *gen = Pr511::G;
    return true;
  }
  return false;
}

// c = 64: 8 columns per block, 256 threads; c = -64: 16 columns, 512
// threads (output rows of whole 128-byte lines in FP64, one block per CU)
bool pr_exists(int n, int csz, int c) {
  (void)csz;
  return (c == 64 || c == -64) && n == Pr511::N;
}

template <class T>
bool launch_time_pr(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (!pr_exists(g.n, (int)sizeof(cx<T>), c)) return false;
  if (c == -64) return pr_launch<T, Pr511, 16, 512>(fwd, g, v, spec, w, tb, vscale, vs_stride, accum, st);
  return pr_launch<T, Pr511, 8, 256>(fwd, g, v, spec, w, tb, vscale, vs_stride, accum, st);
}

template bool launch_time_pr<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const double*, int, int, hipStream_t);
template bool launch_time_pr<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const double*, int, int, hipStream_t);

}  // namespace pcop
