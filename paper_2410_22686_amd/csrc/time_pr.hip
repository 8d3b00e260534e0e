// Time passes for lengths n = N1 PR (N1 and PR coprime, PR prime) by the
// prime-factor (Good-Thomas) split and Rader's algorithm for the PR-point
// transforms: built for n = 511 = 7 x 73, n = 255 = 15 x 17 and n = 127
// (N1 = 1).  A plan without a Rader stage (RA = 0) would take the PR-point
// DFTs directly in registers instead (for 17 points that needs more
// registers than the Rader stages: 253 VGPRs in FP64).
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

// N1 x PR with a Rader stage of RC = PR - 1 = RA RB (generator G), or, with
// RA = RB = 0, the PR-point DFTs directly in registers; CP / CN spatial
// points per tile for the 256- / 512-thread kernels (time_cols 64 / -64)
template <int N1_, int PR_, int G_, int RA_, int RB_, int CP_, int CN_>
struct PrPlan {
  static constexpr int N1 = N1_, PR = PR_, G = G_, RA = RA_, RB = RB_, RC = PR_ - 1, N = N1_ * PR_;
  static constexpr bool DIRECT = RA_ == 0;
  static constexpr int CP = CP_, CN = CN_;
  static constexpr int KM1 = PR_ * pr_inv_mod(PR_ % N1_, N1_);  // output map: k = (KM1 k1 + KM2 k2) mod N
  static constexpr int KM2 = N1_ * pr_inv_mod(N1_ % PR_, PR_);
  static_assert(DIRECT || RA * RB == PR_ - 1, "the convolution length splits as RA RB");
};
// 511 = 7 x 73, generator 5 of the group mod 73, 72 = 9 x 8.  Wide tiles
// of 16 points (FP64, 512 threads: one block per CU); in FP32 the wide
// kernels take 1024 threads with 28 points forward and 32 inverse (the
// launcher below: stage-0 items in two rounds, longer row segments)
using Pr511 = PrPlan<7, 73, 5, 9, 8, 8, 16>;
// 127 prime, generator 3, 126 = 9 x 14
using Pr127 = PrPlan<1, 127, 3, 9, 14, 16, 32>;
// 255 = 15 x 17, generator 3 of the group mod 17, 16 = 4 x 4; tiles of 15
// and 30 points make the 17 stage-0 items per point fill 255 of 256 and 510
// of 512 threads in one round (with 16 and 32 points a second round of 15
// prefetch slots per thread costs 209 VGPRs in FP64 and spills in FP32)
using Pr255 = PrPlan<15, 17, 3, 4, 4, 15, 30>;

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
__device__ __forceinline__ double root_cos<17>(int t) {
  constexpr double c[9] = {1.0, 0.932472229404355804573115891821563386, 0.739008917220659115924534309872648106,
                           0.445738355776538267396457549379486855, 0.092268359463301995239651107154506480,
                           -0.273662990072082863539077935436813432, -0.602634636379256389178588154986840622,
                           -0.850217135729614152134143922949352058, -0.982973099683901778281948844855198716};
  return c[t];
}
template <>
__device__ __forceinline__ double root_sin<17>(int t) {
  constexpr double s[9] = {0.0, 0.361241666187152948744714596183700164, 0.673695643646557211712691912425694616,
                           0.895163291355062322067016499753785457, 0.995734176295034521871191178905481784,
                           0.961825643172819070408796290731518550, 0.798017227280239503332805112796261369,
                           0.526432162877355800244607799140699566, 0.183749517816570331574408839620727582};
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

template <class T, int SG, int R>
__device__ __forceinline__ void dft_small(cx<T>* a);

// R1 R2-point DFT for coprime R1, R2 by the prime-factor index maps (input
// j = (R2 j1 + R1 j2) mod R, output k = (R2 u1 k1 + R1 u2 k2) mod R with
// u1 = R2^-1 mod R1, u2 = R1^-1 mod R2): R2 DFTs of R1 points, then R1 of R2
// points, no twiddles; every index is a constant after unrolling
template <class T, int SG, int R1, int R2>
__device__ __forceinline__ void dft_pfa2(cx<T>* a) {
  constexpr int R = R1 * R2;
  constexpr int U1 = R2 * pr_inv_mod(R2 % R1, R1), U2 = R1 * pr_inv_mod(R1 % R2, R2);
  cx<T> y[R];
#pragma unroll
  for (int j2 = 0; j2 < R2; ++j2) {
    cx<T> t[R1];
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) t[j1] = a[(R2 * j1 + R1 * j2) % R];
    dft_small<T, SG, R1>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) y[k1 * R2 + j2] = t[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> t[R2];
#pragma unroll
    for (int j2 = 0; j2 < R2; ++j2) t[j2] = y[k1 * R2 + j2];
    dft_small<T, SG, R2>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) a[(U1 * k1 + U2 * k2) % R] = t[k2];
  }
}

// R-point DFT in registers, natural order, for the lengths the plans use
template <class T, int SG, int R>
__device__ __forceinline__ void dft_small(cx<T>* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2 || R == 4 || R == 8) {
    dftR<T, SG, R>(a);
  } else if constexpr (R == 3) {
    dft3<T, SG>(a);
  } else if constexpr (R == 5) {
    dft5<T, SG>(a);
  } else if constexpr (R == 7 || R == 9 || R == 17) {
    dft_odd_lit<T, SG, R>(a);
  } else if constexpr (R == 6) {
    dft_pfa2<T, SG, 2, 3>(a);
  } else if constexpr (R == 14) {
    dft_pfa2<T, SG, 2, 7>(a);
  } else if constexpr (R == 15) {
    dft_pfa2<T, SG, 3, 5>(a);
  } else {
    static_assert(R == 1, "no register DFT of this length");
  }
}

// LDS of one block: the [C][N] column tile, then the tables (the Rader
// twiddles, filter and index tables only for Rader plans)
template <class PL>
constexpr size_t pr_lds_bytes(int C, int csz) {
  return (size_t)C * PL::N * csz + (size_t)2 * PL::N * 8 +
         (PL::DIRECT ? 0 : (size_t)2 * PL::RC * csz + (size_t)(PL::RC + 2 * PL::PR) * 4);
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
    double* da_l = reinterpret_cast<double*>(tail);
    double* db_l = da_l + N;
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(db_l + N);
    cx<T>* bh_l = tw_l + RC;
    int* gpw_l = reinterpret_cast<int*>(bh_l + RC);
    int* lg_l = gpw_l + RC;
    int* slot_l = lg_l + PR;
    for (int t = threadIdx.x; t < N; t += NT) {
      const double d = dpow[t];
      da_l[t] = fwd ? d : d / (double)N;
      db_l[t] = fwd ? 1.0 / d : 1.0 / ((double)N * d);
    }
    if constexpr (!PL::DIRECT) {
      const cx<T>* src = reinterpret_cast<const cx<T>*>(prt);
      for (int t = threadIdx.x; t < 2 * RC; t += NT) tw_l[t] = src[t];
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
    }
    tw = tw_l;
    bh = bh_l;
    da = da_l;
    db = db_l;
    gpw = gpw_l;
    lg = lg_l;
    slot = slot_l;
  }
  // slot of the transform input j2 (k2 in the inverse pass), of the output
  // k2, and the output index held in slot s
  __device__ __forceinline__ int in_slot(int j2) const { return PL::DIRECT ? j2 : slot[j2]; }
  __device__ __forceinline__ int out_slot(int k2) const { return PL::DIRECT ? k2 : lg[k2]; }
  __device__ __forceinline__ int slot_index(int s) const {
    return PL::DIRECT ? s : (s == PL::RC ? 0 : gpw[s]);
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
    // FP32: every twiddle from the correctly rounded table, at r base mod RC
    // kept reduced by a conditional subtraction (base < RC)
    int e = base;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cx<T> w = tb.tw[e];
      if (SG > 0) w.y = -w.y;
      a[r] = a[r] * w;
      e += base;
      if (e >= PL::RC) e -= PL::RC;
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
      dft_small<T, -1, RA>(a);
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
      dft_small<T, -1, RB>(cc);  // A[ka + RA kb] = cc[kb]
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
      dft_small<T, 1, RB>(cc);
      pr_twiddle<T, PL, 1, RB>(cc, ka, tb);
#pragma unroll
      for (int qb = 0; qb < RB; ++qb) rowk[ka * RB + qb] = cc[qb];
    }
  }
  __syncthreads();
}

// The PR-point DFT of every (column, k1) row of the tile, in place, ending
// with a barrier: Rader stages A, B and A' (row k1 then holds X[k1, g^q] at
// slot q and X[k1, 0] at slot RC), or one register DFT per row (direct plans,
// X[k1, k2] at slot k2)
template <class T, class PL, int C, int NT>
__device__ __forceinline__ void pr_rows(cx<T>* buf, const PrTables<T, PL>& tb, int lane) {
  constexpr int N1 = PL::N1, PR = PL::PR, LDC = PL::N;
  if constexpr (PL::DIRECT) {
    constexpr int ID = C * N1, QD = (ID + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < QD; ++q) {
      const int e = lane + q * NT;
      if (e < ID) {
        const int c = e % C, k1 = e / C;
        cx<T>* row = buf + c * LDC + k1 * PR;
        cx<T> a[PR];
#pragma unroll
        for (int j2 = 0; j2 < PR; ++j2) a[j2] = row[j2];
        dft_small<T, -1, PR>(a);
#pragma unroll
        for (int k2 = 0; k2 < PR; ++k2) row[k2] = a[k2];
      }
    }
    __syncthreads();
  } else {
    constexpr int RA = PL::RA, RB = PL::RB;
    constexpr int IA = C * N1 * RB, QA = (IA + NT - 1) / NT;
    pr_stages_ab<T, PL, C, NT>(buf, tb, lane);
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
        dft_small<T, 1, RA>(a);
#pragma unroll
        for (int qa = 0; qa < RA; ++qa) row[qa * RB] = a[qa];
      }
    }
    __syncthreads();
  }
}

// FP32 with 512 threads: at least 4 waves per SIMD, so that two blocks share
// a CU (their tiles fit LDS twice); measured at n = 511 (before its FP32
// kernels took 1024-thread tiles), the forward kernel then spilled 4
// registers and still ran 1.2x faster than with one block
template <class T, int NT>
constexpr int pr_min_waves() {
  return NT == 512 && sizeof(T) == 4 ? 4 : 1;
}

template <class T, class PL, int C, int NT>
__global__ void __launch_bounds__(NT, (pr_min_waves<T, NT>())) time_fwd_pr(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const void* __restrict__ prt,
                                                   const double* __restrict__ vscale, int vs_stride, TileWalk tw) {
  constexpr int N = PL::N, N1 = PL::N1, PR = PL::PR, LDC = N;
  constexpr int I0 = C * PR, Q0 = (I0 + NT - 1) / NT;
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
      // a wave past the last item skips the round (a uniform branch)
      if (I0 % NT != 0 && q == Q0 - 1 && __builtin_amdgcn_readfirstlane(e) >= I0) continue;
      // loads from a clamped in-bounds index: items e >= I0 are not
      // committed and columns i >= m are never stored
      const int c = e % C, j2 = min(e / C, PR - 1), i = min(i0 + c, m - 1);
      // level j = (PR j1 + N1 j2) mod N: N1 j2 < N, and each step of j1 adds
      // PR < N, so one conditional subtraction reduces it
      int j = N1 * j2;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const size_t o = (size_t)j * m + i;
        r1[q][j1] = v1[o];
        r2[q][j1] = v2[o];
        j += PR;
        if (j >= N) j -= N;
      }
    }
  };
  // stage 0 of a tile: x_j = s (d_j v2_j + i v1_j / d_j) from the prefetch
  // registers, N1-point DFTs over j1, into the Rader slots
  auto stage0 = [&](int t, int lane) {
    const int b = t / tw.tpm;
    const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
#pragma unroll
    for (int q = 0; q < Q0; ++q) {
      const int e = lane + q * NT;
      if (e < I0) {
        const int c = e % C, j2 = e / C;
        cx<T> a[N1];
        int j = N1 * j2;  // (PR j1 + N1 j2) mod N, as in the fetch
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) {
          a[j1] = cx<T>{(T)(s * tb.da[j] * r2[q][j1]), (T)(s * tb.db[j] * r1[q][j1])};
          j += PR;
          if (j >= N) j -= N;
        }
        dft_small<T, -1, N1>(a);
        cx<T>* col = buf + c * LDC + tb.in_slot(j2);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) col[k1 * PR] = a[k1];
      }
    }
  };
  // The first tile's stage 0 is peeled off the loop, so that inside it stage
  // 0 always follows the previous tile's (unconditional) stores and the wait
  // for its prefetched inputs leaves those stores in flight.
  if (tile < tw.ntiles) {
    fetch(tile, pr_lane());
    stage0(tile, pr_lane());
  }
  while (tile < tw.ntiles) {
    const int lane = pr_lane();
    const int b = tile / tw.tpm;
    const int i0 = (tile - b * tw.tpm) * C;
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    pr_rows<T, PL, C, NT>(buf, tb, lane);
    cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
    unpack_store_u<T, NT, N / 2 + 1, C>(out, N, i0, m, lane, [&](int k, int p) {
      const int k1 = k % N1, k2 = k % PR;
      return buf[p * LDC + k1 * PR + tb.out_slot(k2)];
    });
    __syncthreads();
    tile = nxt;
    if (tile < tw.ntiles) stage0(tile, lane);
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
  constexpr int N = PL::N, N1 = PL::N1, PR = PL::PR, LDC = N;
  constexpr int I0 = C * PR, Q0 = (I0 + NT - 1) / NT;
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
  // LDS slot of input k: row k mod N1, the transform slot of k mod PR
  auto kslot = [&](int k1, int k2) { return k1 * PR + tb.in_slot(k2); };
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
        // residues of n - k from those of k (N1 and PR divide n)
        const int k1 = k % N1, k2 = k % PR;
        buf[p * LDC + kslot(k1, k2)] = cx<T>{z2.x - z1.y, -(z2.y + z1.x)};
        if (k != 0 && 2 * k != N)
          buf[p * LDC + kslot(k1 ? N1 - k1 : 0, k2 ? PR - k2 : 0)] = cx<T>{z2.x + z1.y, -(z1.x - z2.y)};
      }
    }
    __syncthreads();
    const int nxt = tw.next(tile + stride, stride);
    if (nxt < tw.ntiles) fetch(nxt, lane);
    pr_rows<T, PL, C, NT>(buf, tb, lane);
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
        dft_small<T, -1, N1>(a);
        if (i < m) {
          const int j2 = tb.slot_index(sl);
          int jn = N1 * j2;  // (PR j1 + N1 j2) mod N, one conditional subtraction per step
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) {
            const int j = jn;
            jn += PR;
            if (jn >= N) jn -= N;
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

template <class T, class PL, int C, int NT, bool FWD>
static bool pr_launch(const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const double* vscale, int vs_stride, int accum, hipStream_t st) {
  constexpr size_t lds = pr_lds_bytes<PL>(C, (int)sizeof(cx<T>));
  static_assert(lds <= kLdsMax, "tile and tables fit LDS");
  if (g.n != PL::N) return false;
  const void* prt = sizeof(T) == 8 ? (const void*)tb.pr64 : (const void*)tb.pr32;
  if (!PL::DIRECT && !prt) return false;
  TileWalk twk{(g.m + C - 1) / C, 0, tb.active};
  twk.ntiles = twk.tpm * g.B;
  auto launch = [&](auto kern, auto... args) {
    if constexpr (lds > 65536) {
      // above 64 KiB of dynamic LDS the kernel must opt in (once)
      static bool attr_set = false;
      if (!attr_set) {
        attr_set = true;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLdsMax);
        (void)hipGetLastError();
      }
    }
    // persistent grid: as many blocks as stay resident on every CU
    const int grid = std::min(twk.ntiles, resident_blocks(kern, NT, lds) * std::max(1, tb.ncu));
    kern<<<std::max(grid, 1), NT, lds, st>>>(args...);
  };
  if constexpr (FWD) launch(time_fwd_pr<T, PL, C, NT>, g, v, spec, tb.dpow, prt, vscale, vs_stride, twk);
  else launch(time_inv_pr<T, PL, C, NT>, g, spec, w, tb.dpow, prt, accum, twk);
  return true;
}

// the Rader plans need the twiddle and filter tables of pcop_setup
bool pr_params(int n, int* pr, int* gen) {
  if (n == Pr511::N) {
    *pr = Pr511::PR;
    *gen = Pr511::G;
    return true;
  }
  if (n == Pr127::N) {
    *pr = Pr127::PR;
    *gen = Pr127::G;
    return true;
  }
  if (n == Pr255::N) {
    *pr = Pr255::PR;
    *gen = Pr255::G;
    return true;
  }
  return false;
}

// the automatic choice: the wide-tile kernels where they were measured faster
// than the alternatives (n = 511, both precisions); other lengths are left to
// the tuner
int pr_auto(int n, int csz) { return n == Pr511::N && pr_exists(n, csz, -64) ? -64 : 0; }

// c = 64: the plan's narrower tile with 256 threads; c = -64: the wider tile
// with 512 threads (for n = 511 FP64 output rows of whole 128-byte lines)
bool pr_exists(int n, int csz, int c) {
  (void)csz;
  return (c == 64 || c == -64) && (n == Pr511::N || n == Pr127::N || n == Pr255::N);
}

template <class T, class PL>
static bool pr_launch_c(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w,
                        const PrecondTables& tb, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (c == -64) {
    if constexpr (sizeof(T) == 4 && PL::N == Pr511::N) {
      // n = 511 in FP32: one 1024-thread block per CU with twice the points
      // of the FP64 tile (114 / 131 KiB of LDS), so that each time level's
      // row segment spans 224 / 256 bytes.  A level's row of m doubles starts
      // 8 bytes further into a cache line than the previous one (m odd), so
      // each segment shares a partly written line with the neighbouring
      // tile at both ends; wider segments halve those shared lines.  The
      // forward pass takes 28 points (2044 stage-0 items, two rounds of 1024
      // threads; 32 points would take three and spill), the inverse 32.
      if (fwd) return pr_launch<T, PL, 28, 1024, true>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
      return pr_launch<T, PL, 32, 1024, false>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
    } else {
      if (fwd) return pr_launch<T, PL, PL::CN, 512, true>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
      return pr_launch<T, PL, PL::CN, 512, false>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
    }
  }
  if (fwd) return pr_launch<T, PL, PL::CP, 256, true>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
  return pr_launch<T, PL, PL::CP, 256, false>(g, v, spec, w, tb, vscale, vs_stride, accum, st);
}

template <class T>
bool launch_time_pr(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const double* vscale, int vs_stride, int accum, hipStream_t st) {
  if (!pr_exists(g.n, (int)sizeof(cx<T>), c)) return false;
  switch (g.n) {
    case Pr511::N: return pr_launch_c<T, Pr511>(fwd, c, g, v, spec, w, tb, vscale, vs_stride, accum, st);
    case Pr127::N: return pr_launch_c<T, Pr127>(fwd, c, g, v, spec, w, tb, vscale, vs_stride, accum, st);
    case Pr255::N: return pr_launch_c<T, Pr255>(fwd, c, g, v, spec, w, tb, vscale, vs_stride, accum, st);
    default: return false;
  }
}

template bool launch_time_pr<double>(bool, int, const Geo&, const double*, cx<double>*, double*, const PrecondTables&,
                                     const double*, int, int, hipStream_t);
template bool launch_time_pr<float>(bool, int, const Geo&, const double*, cx<float>*, double*, const PrecondTables&,
                                    const double*, int, int, hipStream_t);

}  // namespace pcop
