// FFT building blocks that run on data staged in LDS.
//
// 1. Mixed-radix Stockham stages for any length n = prod(radices): each
//    thread produces whole outputs, so every radix (including large primes)
//    uses the same code.  Stage with radix R after Ns = prod(previous radices):
//       out[(jb/Ns) Ns R + jb%Ns + r2 Ns] =
//           sum_r in[jb + r n/R] * W_n^{ r (jb%Ns + r2 Ns) n/(Ns R) },
//    W_n = exp(-2 pi i/n) forward, its conjugate inverse.  Data are laid out
//    [n][P] (P independent columns, column index fastest); stages ping-pong
//    between two LDS buffers.
// 2. In-place power-of-two FFTs (radix 8/4/2 butterflies held in registers)
//    used by the sine transforms; layout [LINES][ld].
#pragma once

#include "common.hpp"

namespace pcop {

// Time-axis FFT plan: Stockham radices (each <= 17) or, when n has a larger
// prime factor or no Stockham tile of it fits LDS, Bluestein's chirp-z
// transform with a power-of-two length M.
struct FftPlan {
  int nrad;
  int rad[16];
  int bluestein;
  int M;
};

// ---------------------------------------------------------------------------
// small DFTs, sign SG = -1 (forward) or +1 (inverse)
// ---------------------------------------------------------------------------
template <class T, int SG>
__device__ __forceinline__ void dft2(cx<T>& a0, cx<T>& a1) {
  cx<T> t = a0;
  a0 = t + a1;
  a1 = t - a1;
}

template <class T, int SG>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_i<T, SG>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <class T, int SG>
__device__ __forceinline__ void dft8(cx<T>* a) {
  // even / odd split: E = DFT4(a0,a2,a4,a6), O = DFT4(a1,a3,a5,a7)
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<T, SG>(e0, e1, e2, e3);
  dft4<T, SG>(o0, o1, o2, o3);
  const T r = (T)0.70710678118654752440L;
  // W8^1 = r (1 + SG i), W8^2 = SG i, W8^3 = r (-1 + SG i)
  cx<T> w1o1 = scale(o1 + mul_i<T, SG>(o1), r);
  cx<T> w2o2 = mul_i<T, SG>(o2);
  cx<T> w3o3 = scale(mul_i<T, SG>(o3) - o3, r);
  a[0] = e0 + o0;
  a[4] = e0 - o0;
  a[1] = e1 + w1o1;
  a[5] = e1 - w1o1;
  a[2] = e2 + w2o2;
  a[6] = e2 - w2o2;
  a[3] = e3 + w3o3;
  a[7] = e3 - w3o3;
}

template <class T, int SG>
__device__ __forceinline__ void dft3(cx<T>* a) {
  const T h = (T)0.86602540378443864676L;  // sin(2 pi/3)
  const cx<T> t1 = a[1] + a[2];
  const cx<T> t2 = a[0] - scale(t1, (T)0.5);
  const cx<T> t3 = scale(mul_i<T, SG>(a[1] - a[2]), h);
  a[0] = a[0] + t1;
  a[1] = t2 + t3;
  a[2] = t2 - t3;
}

template <class T, int SG>
__device__ __forceinline__ void dft5(cx<T>* a) {
  const T c1 = (T)0.30901699437494742410L, c2 = (T)-0.80901699437494742410L;
  const T s1 = (T)0.95105651629515357212L, s2 = (T)0.58778525229247312917L;
  const cx<T> t1 = a[1] + a[4], t2 = a[2] + a[3], t3 = a[1] - a[4], t4 = a[2] - a[3];
  const cx<T> u1 = a[0] + scale(t1, c1) + scale(t2, c2);
  const cx<T> u2 = a[0] + scale(t1, c2) + scale(t2, c1);
  const cx<T> v1 = mul_i<T, SG>(scale(t3, s1) + scale(t4, s2));
  const cx<T> v2 = mul_i<T, SG>(scale(t3, s2) - scale(t4, s1));
  a[0] = a[0] + t1 + t2;
  a[1] = u1 + v1;
  a[4] = u1 - v1;
  a[2] = u2 + v2;
  a[3] = u2 - v2;
}

// R-point DFT for odd R; W_R^t = twn[t * stride] (twn: exp(-2 pi i t/n),
// n = R stride).  Inputs r and R - r are paired: with s_r = a_r + a_{R-r},
// d_r = a_r - a_{R-r} and theta = 2 pi r k/R,
//   X_k     = a_0 + sum_{r=1}^{H} s_r cos(theta) + SG i sum_{r=1}^{H} d_r sin(theta),
//   X_{R-k} = the same with the sign of the sine sum flipped,  H = (R-1)/2,
// so only H twiddles are loaded and 4 H^2 real FMAs replace 4 R (R-1).
template <class T, int SG, int R>
__device__ __forceinline__ void dft_odd(cx<T>* a, const cx<T>* __restrict__ twn, int stride) {
  constexpr int H = (R - 1) / 2;
  T c[H + 1], sn[H + 1];  // cos, sin of 2 pi t/R, t = 1..H
#pragma unroll
  for (int t = 1; t <= H; ++t) {
    const cx<T> w = twn[t * stride];
    c[t] = w.x;
    sn[t] = -w.y;
  }
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
      const int t = (r * k) % R;  // cos is even and sin odd in t about R/2
      const T ct = (t <= H) ? c[t] : c[R - t];
      const T st = (t <= H) ? sn[t] : -sn[R - t];
      p = p + scale(sm[r], ct);
      q = q + scale(df[r], st);
    }
    const cx<T> iq = mul_i<T, SG>(q);  // SG i q
    a[k] = p + iq;
    a[R - k] = p - iq;
  }
  a[0] = x0;
}

// dft_odd with each output handed to out(r, X_r) as soon as it is formed
// (same operations in the same order), so the outputs never occupy
// registers together with the pair sums and differences
template <class T, int SG, int R, class OUT>
__device__ __forceinline__ void dft_odd_out(const cx<T>* a, const cx<T>* __restrict__ twn, int stride, OUT out) {
  constexpr int H = (R - 1) / 2;
  T c[H + 1], sn[H + 1];
#pragma unroll
  for (int t = 1; t <= H; ++t) {
    const cx<T> w = twn[t * stride];
    c[t] = w.x;
    sn[t] = -w.y;
  }
  cx<T> sm[H + 1], df[H + 1];
  cx<T> x0 = a[0];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    sm[r] = a[r] + a[R - r];
    df[r] = a[r] - a[R - r];
    x0 = x0 + sm[r];
  }
  out(0, x0);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> p = a[0], q{0, 0};
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      const int t = (r * k) % R;
      const T ct = (t <= H) ? c[t] : c[R - t];
      const T st = (t <= H) ? sn[t] : -sn[R - t];
      p = p + scale(sm[r], ct);
      q = q + scale(df[r], st);
    }
    const cx<T> iq = mul_i<T, SG>(q);
    out(k, p + iq);
    out(R - k, p - iq);
  }
}

template <class T, int SG, int R>
__device__ __forceinline__ void dftR(cx<T>* a) {
  if constexpr (R == 2) dft2<T, SG>(a[0], a[1]);
  else if constexpr (R == 4) dft4<T, SG>(a[0], a[1], a[2], a[3]);
  else dft8<T, SG>(a);
}

template <class T, int SG, int R>
__device__ __forceinline__ void dft_any(cx<T>* a, const cx<T>* __restrict__ twn, int stride) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2 || R == 4 || R == 8) {
    dftR<T, SG, R>(a);
  } else if constexpr (R == 3) {
    dft3<T, SG>(a);
  } else if constexpr (R == 5) {
    dft5<T, SG>(a);
  } else {
    static_assert(R % 2 == 1, "radices other than 2, 4, 8 must be odd");
    dft_odd<T, SG, R>(a, twn, stride);
  }
}

// One Stockham stage with radix R after Ns = prod(previous radices) on a
// length-n transform of P columns; each thread owns whole butterflies.
// load(j, p) / store(j, p, v) read the stage input and write its output, so
// the same code serves global->LDS, LDS->LDS and LDS->global stages.
// twn[t] = exp(-2 pi i t/n); the inter-stage twiddles W_{Ns R}^{r jl} are
// formed by powering W_{Ns R}^{jl}.
template <class T, int R, int P, int SG, class LD, class ST>
__device__ __forceinline__ void sk_stage(int n, int Ns, const cx<T>* __restrict__ twn, LD load, ST store) {
  const int nR = n / R;
  const int tstep = n / (Ns * R);
  for (int bf = threadIdx.x; bf < nR * P; bf += blockDim.x) {
    const int p = bf % P;
    const int jb = bf / P;
    const int jl = jb % Ns;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = load(jb + r * nR, p);
    if (R > 1 && jl != 0) {
      if constexpr (sizeof(T) == 8) {
        // FP64: powers of one looked-up twiddle
        cx<T> w1 = twn[jl * tstep];
        if (SG > 0) w1.y = -w1.y;
        cx<T> w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[r] = v[r] * w;
          w = w * w1;
        }
      } else {
        // FP32: every twiddle from the correctly rounded table
        const int e1 = jl * tstep;
        int e = e1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = twn[e];
          if (SG > 0) w.y = -w.y;
          v[r] = v[r] * w;
          e += e1;
          if (e >= n) e -= n;
        }
      }
    }
    const int base = (jb - jl) * R + jl;
    if constexpr (R >= 7 && R % 2 == 1) {
      // long odd radices: outputs stored as they are formed
      dft_odd_out<T, SG, R>(v, twn, nR, [&](int r, cx<T> val) { store(base + r * Ns, p, val); });
    } else {
      dft_any<T, SG, R>(v, twn, nR);
#pragma unroll
      for (int r = 0; r < R; ++r) store(base + r * Ns, p, v[r]);
    }
  }
}

// runtime radix dispatch (radices produced by the host planner)
template <class T, int P, int SG, class LD, class ST>
__device__ __forceinline__ void sk_stage_rt(int R, int n, int Ns, const cx<T>* __restrict__ twn, LD load,
                                            ST store) {
  switch (R) {
    case 1: sk_stage<T, 1, P, SG>(n, Ns, twn, load, store); break;
    case 2: sk_stage<T, 2, P, SG>(n, Ns, twn, load, store); break;
    case 3: sk_stage<T, 3, P, SG>(n, Ns, twn, load, store); break;
    case 4: sk_stage<T, 4, P, SG>(n, Ns, twn, load, store); break;
    case 5: sk_stage<T, 5, P, SG>(n, Ns, twn, load, store); break;
    case 7: sk_stage<T, 7, P, SG>(n, Ns, twn, load, store); break;
    case 8: sk_stage<T, 8, P, SG>(n, Ns, twn, load, store); break;
    case 11: sk_stage<T, 11, P, SG>(n, Ns, twn, load, store); break;
    case 13: sk_stage<T, 13, P, SG>(n, Ns, twn, load, store); break;
    case 17: sk_stage<T, 17, P, SG>(n, Ns, twn, load, store); break;
    default: break;
  }
}

// In-place Stockham stage over P columns ([n][P] in LDS): each thread loads
// all of its (at most MB) butterflies into registers, the block waits, and the
// outputs are written over the inputs.  load/store as in sk_stage; the caller
// puts a barrier between consecutive LDS stages.
template <class T, int R, int P, int SG, int MB, class LD, class ST>
__device__ __forceinline__ void ip_stage(int n, int Ns, const cx<T>* __restrict__ twn, bool sync_between, LD load,
                                         ST store) {
  const int nR = n / R;
  const int tstep = n / (Ns * R);
  const int nb = nR * P;
  cx<T> v[MB][R];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int bf = threadIdx.x + q * blockDim.x;
    if (bf < nb) {
      const int p = bf % P;
      const int jb = bf / P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = load(jb + r * nR, p);
    }
  }
  if (sync_between) __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int bf = threadIdx.x + q * blockDim.x;
    if (bf < nb) {
      const int p = bf % P;
      const int jb = bf / P;
      const int jl = jb % Ns;
      if (R > 1 && jl != 0) {
        if constexpr (sizeof(T) == 8) {
          cx<T> w1 = twn[jl * tstep];
          if (SG > 0) w1.y = -w1.y;
          cx<T> w = w1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            v[q][r] = v[q][r] * w;
            w = w * w1;
          }
        } else {
          const int e1 = jl * tstep;
          int e = e1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = twn[e];
            if (SG > 0) w.y = -w.y;
            v[q][r] = v[q][r] * w;
            e += e1;
            if (e >= n) e -= n;
          }
        }
      }
      dft_any<T, SG, R>(v[q], twn, nR);
      const int base = (jb - jl) * R + jl;
#pragma unroll
      for (int r = 0; r < R; ++r) store(base + r * Ns, p, v[q][r]);
    }
  }
}

// butterflies per thread a stage needs, rounded up to a supported bound
__host__ __device__ inline int ip_mb(int n, int R, int P, int nt) {
  const int need = (n / R * P + nt - 1) / nt;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
}

template <class T, int R, int P, int SG, class LD, class ST>
__device__ __forceinline__ bool ip_stage_mb(int mb, int n, int Ns, const cx<T>* __restrict__ twn, bool sync_between,
                                            LD load, ST store) {
  if constexpr (R >= 11) {
    if (mb == 1) ip_stage<T, R, P, SG, 1>(n, Ns, twn, sync_between, load, store);
    else if (mb == 2) ip_stage<T, R, P, SG, 2>(n, Ns, twn, sync_between, load, store);
    else return false;
  } else {
    if (mb == 1) ip_stage<T, R, P, SG, 1>(n, Ns, twn, sync_between, load, store);
    else if (mb == 2) ip_stage<T, R, P, SG, 2>(n, Ns, twn, sync_between, load, store);
    else if (mb == 4) ip_stage<T, R, P, SG, 4>(n, Ns, twn, sync_between, load, store);
    else if (mb == 8) ip_stage<T, R, P, SG, 8>(n, Ns, twn, sync_between, load, store);
    else return false;
  }
  return true;
}

template <class T, int P, int SG, class LD, class ST>
__device__ __forceinline__ void ip_stage_rt(int R, int n, int Ns, const cx<T>* __restrict__ twn, bool sync_between,
                                            LD load, ST store) {
  const int mb = ip_mb(n, R, P, blockDim.x);
  switch (R) {
    case 1: ip_stage_mb<T, 1, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 2: ip_stage_mb<T, 2, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 3: ip_stage_mb<T, 3, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 4: ip_stage_mb<T, 4, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 5: ip_stage_mb<T, 5, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 7: ip_stage_mb<T, 7, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 8: ip_stage_mb<T, 8, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 11: ip_stage_mb<T, 11, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 13: ip_stage_mb<T, 13, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    case 17: ip_stage_mb<T, 17, P, SG>(mb, n, Ns, twn, sync_between, load, store); break;
    default: break;
  }
}

// identity output map of the FFT stages
struct P2Keep {
  template <class V>
  __device__ __forceinline__ V operator()(int, V v) const { return v; }
};

// One in-place Stockham stage with radix R over LINES lines of length L held
// in LDS ([LINES][ld]).  Each thread keeps its butterflies in registers
// between the two barriers, which makes the stage safe in place.
// twL[t] = exp(-2 pi i t / L) (FP64 reads t < L/2 only).
// HALF_IN (first stage): the inputs at L/2 and above are zero and not read.
// HALF_OUT (last stage): only the outputs below L/2 are written.
// post(k, value) maps each output k before it is written.
template <class T, int SG, int L, int R, int LINES, int NT, bool HALF_IN, bool HALF_OUT, class POST>
__device__ __forceinline__ void p2_stage_x(cx<T>* buf, int ld, int Ns, const cx<T>* __restrict__ twL, POST post) {
  constexpr int NB = LINES * (L / R);
  constexpr int PER = (NB + NT - 1) / NT;
  constexpr int RIN = HALF_IN ? R / 2 : R;
  constexpr int ROUT = HALF_OUT ? R / 2 : R;
  cx<T> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bf = threadIdx.x + q * NT;
    if (bf < NB) {
      const int line = bf / (L / R);
      const int jb = bf - line * (L / R);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = r < RIN ? buf[line * ld + jb + r * (L / R)] : cx<T>{0, 0};
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bf = threadIdx.x + q * NT;
    if (bf < NB) {
      const int line = bf / (L / R);
      const int jb = bf - line * (L / R);
      const int jl = jb % Ns;
      const int tstep = L / (Ns * R);
      if (jl != 0) {
        if constexpr (sizeof(T) == 8) {
          cx<T> w1 = twL[jl * tstep];
          if (SG > 0) w1.y = -w1.y;
          cx<T> w = w1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            v[q][r] = v[q][r] * w;
            w = w * w1;
          }
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = twL[(r * jl * tstep) & (L - 1)];
            if (SG > 0) w.y = -w.y;
            v[q][r] = v[q][r] * w;
          }
        }
      }
      dftR<T, SG, R>(v[q]);
      const int base = (jb / Ns) * Ns * R + jl;
#pragma unroll
      for (int r = 0; r < ROUT; ++r) buf[line * ld + base + r * Ns] = post(base + r * Ns, v[q][r]);
    }
  }
  __syncthreads();
}

template <class T, int SG, int L, int R, int LINES, int NT>
__device__ __forceinline__ void p2_stage(cx<T>* buf, int ld, int Ns, const cx<T>* __restrict__ twL) {
  p2_stage_x<T, SG, L, R, LINES, NT, false, false>(buf, ld, Ns, twL, P2Keep{});
}

// the stages from size NS on; HALF_IN applies to the first stage, HALF_OUT
// and post to the last
template <class T, int SG, int L, int LINES, int NT, int NS, bool HALF_IN, bool HALF_OUT>
struct P2Stages {
  template <class POST>
  static __device__ __forceinline__ void run(cx<T>* buf, int ld, const cx<T>* __restrict__ twL, POST post) {
    constexpr int R = (L / NS >= 8) ? 8 : (L / NS);
    constexpr bool first = NS == 1;
    if constexpr (NS * R == L) {
      p2_stage_x<T, SG, L, R, LINES, NT, HALF_IN && first, HALF_OUT>(buf, ld, NS, twL, post);
    } else {
      p2_stage_x<T, SG, L, R, LINES, NT, HALF_IN && first, false>(buf, ld, NS, twL, P2Keep{});
      P2Stages<T, SG, L, LINES, NT, NS * R, HALF_IN, HALF_OUT>::run(buf, ld, twL, post);
    }
  }
};

// In-place FFT of LINES lines of power-of-two length L; call with all
// threads of the block after a barrier that publishes the data.
template <class T, int SG, int L, int LINES, int NT>
__device__ __forceinline__ void p2_fft(cx<T>* buf, int ld, const cx<T>* __restrict__ twL) {
  P2Stages<T, SG, L, LINES, NT, 1, false, false>::run(buf, ld, twL, P2Keep{});
}

// The same FFT for zero-padded convolutions: with HALF_IN the inputs at L/2
// and above are zero (and need not be in LDS), with HALF_OUT only outputs
// below L/2 are produced; post(k, X_k) maps the outputs (a pointwise filter).
template <class T, int SG, int L, int LINES, int NT, bool HALF_IN, bool HALF_OUT, class POST>
__device__ __forceinline__ void p2_fft_x(cx<T>* buf, int ld, const cx<T>* __restrict__ twL, POST post) {
  P2Stages<T, SG, L, LINES, NT, 1, HALF_IN, HALF_OUT>::run(buf, ld, twL, post);
}

}  // namespace pcop
