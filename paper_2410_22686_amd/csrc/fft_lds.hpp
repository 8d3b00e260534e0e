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

struct FftPlan {
  int nrad;
  int rad[16];
};

template <class T, bool INV>
__device__ __forceinline__ void tpo_stage(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int n,
                                          int P, int R, int Ns, const cx<T>* __restrict__ tw) {
  const int nR = n / R;
  const int NsR = Ns * R;
  const int tstep = n / NsR;
  const int total = n * P;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int o = t / P;
    const int p = t - o * P;
    const int blk = o / NsR;
    const int rem = o - blk * NsR;
    const int r2 = rem / Ns;
    const int jl = rem - r2 * Ns;
    const int jb = blk * Ns + jl;
    const int E = (jl + r2 * Ns) * tstep;  // < n
    cx<T> acc = in[jb * P + p];
    int e = E;
    for (int r = 1; r < R; ++r) {
      cx<T> w = tw[e];
      if (INV) w.y = -w.y;
      acc = acc + in[(jb + r * nR) * P + p] * w;
      e += E;
      if (e >= n) e -= n;
    }
    out[t] = acc;
  }
}

// Runs all stages; returns the buffer holding the result (a or b).
template <class T, bool INV>
__device__ cx<T>* tpo_fft(cx<T>* a, cx<T>* b, int n, int P, const FftPlan& plan,
                          const cx<T>* __restrict__ tw) {
  int Ns = 1;
  cx<T>* src = a;
  cx<T>* dst = b;
  for (int s = 0; s < plan.nrad; ++s) {
    const int R = plan.rad[s];
    tpo_stage<T, INV>(src, dst, n, P, R, Ns, tw);
    __syncthreads();
    Ns *= R;
    cx<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

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

template <class T, int SG, int R>
__device__ __forceinline__ void dftR(cx<T>* a) {
  if constexpr (R == 2) dft2<T, SG>(a[0], a[1]);
  else if constexpr (R == 4) dft4<T, SG>(a[0], a[1], a[2], a[3]);
  else dft8<T, SG>(a);
}

// One in-place Stockham stage with radix R over LINES lines of length L held
// in LDS ([LINES][ld]).  Each thread keeps its butterflies in registers
// between the two barriers, which makes the stage safe in place.
// twL[t] = exp(-2 pi i t / L).
template <class T, int SG, int L, int R, int LINES, int NT>
__device__ __forceinline__ void p2_stage(cx<T>* buf, int ld, int Ns, const cx<T>* __restrict__ twL) {
  constexpr int NB = LINES * (L / R);
  constexpr int PER = (NB + NT - 1) / NT;
  cx<T> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bf = threadIdx.x + q * NT;
    if (bf < NB) {
      const int line = bf / (L / R);
      const int jb = bf - line * (L / R);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[line * ld + jb + r * (L / R)];
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
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = twL[(r * jl * tstep) & (L - 1)];
        if (SG > 0) w.y = -w.y;
        v[q][r] = v[q][r] * w;
      }
      dftR<T, SG, R>(v[q]);
      const int base = (jb / Ns) * Ns * R + jl;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[line * ld + base + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

template <class T, int SG, int L, int LINES, int NT, int NS>
struct P2Stages {
  static __device__ __forceinline__ void run(cx<T>* buf, int ld, const cx<T>* __restrict__ twL) {
    constexpr int R = (L / NS >= 8) ? 8 : (L / NS);
    p2_stage<T, SG, L, R, LINES, NT>(buf, ld, NS, twL);
    P2Stages<T, SG, L, LINES, NT, NS * R>::run(buf, ld, twL);
  }
};
template <class T, int SG, int L, int LINES, int NT>
struct P2Stages<T, SG, L, LINES, NT, L> {
  static __device__ __forceinline__ void run(cx<T>*, int, const cx<T>* __restrict__) {}
};

// In-place FFT of LINES lines of power-of-two length L; call with all
// threads of the block after a barrier that publishes the data.
template <class T, int SG, int L, int LINES, int NT>
__device__ __forceinline__ void p2_fft(cx<T>* buf, int ld, const cx<T>* __restrict__ twL) {
  P2Stages<T, SG, L, LINES, NT, 1>::run(buf, ld, twL);
}

}  // namespace pcop
