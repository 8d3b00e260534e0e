// The epsilon-circulant RBD preconditioner w = P_eps^{-1} v (Section 2.1):
//   step 1  time pass: scale by D_eps, FFT along time, split the packed
//           spectrum into the two Hermitian block spectra          (a2)
//   step 2  shifted spatial solves by sine transforms (a = 1)     (a3)
//           -- the multigrid alternative lives in multigrid.hip
//   step 3+4 inverse time pass: inverse FFT, undo D_eps, combine
//           w_1 = z_1 - z_2, w_2 = z_1 + z_2                        (a4)
//
// Both blocks ride in one complex FFT per spatial point:
//   c_j = eps^{j/n} v_2^j + i eps^{-j/n} v_1^j,   c_hat = FFT_n(c),
//   V2_k = (c_hat_k + conj c_hat_{-k})/2,  V1_k = (c_hat_k - conj c_hat_{-k})/(2i),
// and only k = 0..n/2 is kept (the spectra are Hermitian).  Block 2 is solved
// with the shift lambda_k + alpha, block 1 with conj(lambda_k) + alpha
// (eq. decomposition_eps; C_eps^T = D F conj(Lambda) F^* D^{-1}).  The
// spectrum buffer is laid out [batch][2K][m], slice q = 2k + s with s = 0
// for V2 and s = 1 for V1, K = n/2 + 1.
#include "common.hpp"
#include "fft_lds.hpp"
#include "launch.hpp"

namespace pcop {

// ---------------------------------------------------------------------------
// time passes
//
// A block owns P consecutive spatial points and all n time levels.
// Stockham mode: LDS holds two [n][P] buffers; the first stage of the forward
// pass reads HBM directly and the last stage of the inverse pass writes HBM
// directly.  Bluestein mode (n has a prime factor > 17): a length-M
// power-of-two convolution in one in-place [P][M+1] LDS buffer,
//   X_k = w_k sum_j (x_j w_j) conj(w_{k-j}),  w_j = exp(-i pi j^2/n),
// with the FFT of the chirp filter precomputed (bhat).
// ---------------------------------------------------------------------------
struct TimeTables {
  const void* twn;    // [n]   exp(-2 pi i t/n)
  const void* twM;    // [M]   exp(-2 pi i t/M)
  const void* chirp;  // [n]   exp(-i pi (t^2 mod 2n)/n)
  const void* bhat;   // [M]   FFT_M of the chirp filter
};

// c_j = s (d_j v2_j + i v1_j / d_j) at time level j, spatial point i
template <class T>
__device__ __forceinline__ cx<T> pack_input(const double* v1, const double* v2, const double* dpow, double s,
                                            int j, int i, int m) {
  if (i >= m) return cx<T>{0, 0};
  const double d = dpow[j];
  const size_t o = (size_t)j * m + i;
  return cx<T>{(T)(s * d * v2[o]), (T)(s * v1[o] / d)};
}

// split the packed spectrum X into the two block spectra and store slices 2k, 2k+1
template <class T, class GET>
__device__ __forceinline__ void unpack_store(cx<T>* out, int n, int K, int P, int i0, int m, GET get) {
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    if (i >= m) continue;
    const int kn = (k == 0) ? 0 : n - k;
    const cx<T> X = get(k, p);
    const cx<T> Y = conj(get(kn, p));
    const cx<T> sum = X + Y, dif = X - Y;
    out[(size_t)(2 * k) * m + i] = cx<T>{sum.x * (T)0.5, sum.y * (T)0.5};
    out[(size_t)(2 * k + 1) * m + i] = cx<T>{dif.y * (T)0.5, -dif.x * (T)0.5};  // dif / (2i)
  }
}

// w_1 = z_1 - z_2, w_2 = z_1 + z_2 with z_2 = Re(e)/(n d_j), z_1 = Im(e) d_j/n
__device__ __forceinline__ void combine_store(double* w1, double* w2, const double* dpow, int n, int m, int j,
                                              int i, double ex, double ey, int accum) {
  const double d = dpow[j];
  const double inv_n = 1.0 / (double)n;
  const double z2 = ex * inv_n / d;
  const double z1 = ey * inv_n * d;
  const size_t o = (size_t)j * m + i;
  if (accum) {
    w1[o] += z1 - z2;
    w2[o] += z1 + z2;
  } else {
    w1[o] = z1 - z2;
    w2[o] = z1 + z2;
  }
}

template <class T, int P>
__global__ void __launch_bounds__(256) time_fwd_sk(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, const double* __restrict__ vscale, int vs_stride,
                                                   const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  const int i0 = bx * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vl;
  const double* v2 = v1 + (size_t)n * m;
  auto ld0 = [&](int j, int p) { return pack_input<T>(v1, v2, dpow, s, j, i0 + p, m); };
  auto stA = [&](int j, int p, cx<T> val) { bufA[j * P + p] = val; };
  sk_stage_rt<T, P, -1>(plan.rad[0], n, 1, twn, ld0, stA);
  __syncthreads();
  cx<T>* src = bufA;
  cx<T>* dst = bufB;
  int Ns = plan.rad[0];
  for (int st = 1; st < plan.nrad; ++st) {
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
}

template <class T, int P>
__global__ void __launch_bounds__(256) time_inv_sk(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, const cx<T>* __restrict__ twn,
                                                   FftPlan plan, int accum, const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* bufA = reinterpret_cast<cx<T>*>(smem);
  cx<T>* bufB = bufA + n * P;
  const int i0 = bx * P;
  const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    cx<T> z2{0, 0}, z1{0, 0};
    if (i < m) {
      z2 = in[(size_t)(2 * k) * m + i];
      z1 = in[(size_t)(2 * k + 1) * m + i];
    }
    // e_k = Z2 + i Z1 and, for the mirrored frequency, e_{n-k} = conj Z2 + i conj Z1
    bufA[k * P + p] = cx<T>{z2.x - z1.y, z2.y + z1.x};
    if (k != 0 && 2 * k != n) bufA[(n - k) * P + p] = cx<T>{z2.x + z1.y, z1.x - z2.y};
  }
  __syncthreads();
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
}

template <class T, int P, int M>
__global__ void __launch_bounds__(256) time_fwd_bl(Geo g, const double* __restrict__ v, cx<T>* __restrict__ spec,
                                                   const double* __restrict__ dpow, TimeTables tt,
                                                   const double* __restrict__ vscale, int vs_stride,
                                                   const int* __restrict__ active) {
  constexpr int LD = M + 1;
  __shared__ cx<T> buf[P * LD];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  const cx<T>* twM = reinterpret_cast<const cx<T>*>(tt.twM);
  const cx<T>* chirp = reinterpret_cast<const cx<T>*>(tt.chirp);
  const cx<T>* bhat = reinterpret_cast<const cx<T>*>(tt.bhat);
  const int i0 = bx * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vl;
  const double* v2 = v1 + (size_t)n * m;
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    cx<T> a{0, 0};
    if (j < n) a = pack_input<T>(v1, v2, dpow, s, j, i0 + p, m) * chirp[j];
    buf[p * LD + j] = a;
  }
  __syncthreads();
  p2_fft<T, -1, M, P, 256>(buf, LD, twM);
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int p = t / M, k = t - p * M;
    buf[p * LD + k] = buf[p * LD + k] * bhat[k];
  }
  __syncthreads();
  p2_fft<T, 1, M, P, 256>(buf, LD, twM);
  const T invM = (T)1 / (T)M;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int p = t / n, k = t - p * n;
    buf[p * LD + k] = scale(buf[p * LD + k] * chirp[k], invM);
  }
  __syncthreads();
  cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
  unpack_store<T>(out, n, K, P, i0, m, [&](int k, int p) { return buf[p * LD + k]; });
}

// inverse DFT through the forward chirp transform: e = conj(DFT(conj(E)))
template <class T, int P, int M>
__global__ void __launch_bounds__(256) time_inv_bl(Geo g, const cx<T>* __restrict__ spec, double* __restrict__ w,
                                                   const double* __restrict__ dpow, TimeTables tt, int accum,
                                                   const int* __restrict__ active) {
  constexpr int LD = M + 1;
  __shared__ cx<T> buf[P * LD];
  // neighbouring column tiles share 128-byte lines: keep them on one XCD
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = lg % gridDim.x;
  const int b = lg / gridDim.x;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  const cx<T>* twM = reinterpret_cast<const cx<T>*>(tt.twM);
  const cx<T>* chirp = reinterpret_cast<const cx<T>*>(tt.chirp);
  const cx<T>* bhat = reinterpret_cast<const cx<T>*>(tt.bhat);
  const int i0 = bx * P;
  const cx<T>* in = spec + (size_t)b * (size_t)(2 * K) * m;
  for (int t = threadIdx.x; t < (M - n) * P; t += blockDim.x) {
    const int j = n + t / P, p = t - (t / P) * P;
    buf[p * LD + j] = cx<T>{0, 0};
  }
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    cx<T> z2{0, 0}, z1{0, 0};
    if (i < m) {
      z2 = in[(size_t)(2 * k) * m + i];
      z1 = in[(size_t)(2 * k + 1) * m + i];
    }
    // conj(e_k) = conj(Z2 + i Z1), conj(e_{n-k}) = conj(conj Z2 + i conj Z1)
    const cx<T> ek{z2.x - z1.y, -(z2.y + z1.x)};
    buf[p * LD + k] = ek * chirp[k];
    if (k != 0 && 2 * k != n) {
      const cx<T> enk{z2.x + z1.y, -(z1.x - z2.y)};
      buf[p * LD + (n - k)] = enk * chirp[n - k];
    }
  }
  __syncthreads();
  p2_fft<T, -1, M, P, 256>(buf, LD, twM);
  for (int t = threadIdx.x; t < M * P; t += blockDim.x) {
    const int p = t / M, k = t - p * M;
    buf[p * LD + k] = buf[p * LD + k] * bhat[k];
  }
  __syncthreads();
  p2_fft<T, 1, M, P, 256>(buf, LD, twM);
  double* w1 = w + (size_t)b * g.vl;
  double* w2 = w1 + (size_t)n * m;
  const double invM = 1.0 / (double)M;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    const int i = i0 + p;
    if (i >= m) continue;
    const cx<T> e = buf[p * LD + j] * chirp[j];
    // e_j = conj(chirp_j c_j / M)
    combine_store(w1, w2, dpow, n, m, j, i, (double)e.x * invM, -(double)e.y * invM, accum);
  }
}

// ---------------------------------------------------------------------------
// sine-transform passes (a = 1)
//
// Y = FFT_L of the odd extension [0, z_1..z_N, 0, -z_N..-z_1], L = 2(N+1),
// gives Y_k = -2i sum_j z_j sin(pi j k/(N+1)); every pass stores Y_1..Y_N.
// The constant (-2i)^{2d} and the orthonormalisation (2/(N+1))^d are folded
// into the division of the last-axis pass:
//     Z = c / (sigma_q + tau mu),  c = (-1/(2(N+1)))^d,
//     mu = (4/h^2) sum_d sin^2(pi k_d h/2).
// Lines: element e of line l of plane p sits at
//     p * plane_stride + l * line_stride + e * elem_stride   (complex units).
// ---------------------------------------------------------------------------
struct LineGeom {
  long long nplanes;
  long long plane_stride;
  int lines;  // lines per plane
  int line_stride;
  int elem_stride;
};

struct DivideParams {
  const double* mu1;     // [nx] 1-D eigenvalues (4/h^2) sin^2(pi k h/2)
  const double* lam;     // [2K] (re, im) of lambda_k
  const double* alpha;   // [B]
  const int* active;     // [B] or null
  double cnorm;
};

template <class T, int L, int LINES, int NT, bool ROWS, bool DIVIDE>
__global__ void __launch_bounds__(NT) dst_lines_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                       const cx<T>* __restrict__ twL, DivideParams dp) {
  constexpr int N = L / 2 - 1;
  constexpr int LD = L + 1;  // odd stride for complex entries
  __shared__ cx<T> buf[LINES * LD];
  const int tiles = (lg.lines + LINES - 1) / LINES;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const long long plane = blk / tiles;
  const int l0 = (int)(blk - plane * tiles) * LINES;
  const long long pbase = plane * lg.plane_stride;
  if (DIVIDE && dp.active) {
    if (!dp.active[(int)(plane / (2 * g.K))]) return;
  }
  for (int t = threadIdx.x; t < LINES * N; t += NT) {
    int l, e;
    if (ROWS) {
      l = t / N;
      e = t - l * N;
    } else {
      e = t / LINES;
      l = t - e * LINES;
    }
    cx<T> val{0, 0};
    if (l0 + l < lg.lines)
      val = data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride];
    buf[l * LD + e + 1] = val;
    buf[l * LD + L - 1 - e] = cx<T>{-val.x, -val.y};
  }
  for (int l = threadIdx.x; l < LINES; l += NT) {
    buf[l * LD] = cx<T>{0, 0};
    buf[l * LD + N + 1] = cx<T>{0, 0};
  }
  __syncthreads();
  p2_fft<T, -1, L, LINES, NT>(buf, LD, twL);
  if (DIVIDE) {
    // the last-axis pass has one plane per slice q of member b; the shift
    // sigma_q = lambda_k + alpha_b (q even) or conj(lambda_k) + alpha_b (q odd)
    // is uniform over the block
    const int b = (int)(plane / (2 * g.K));
    const int q = (int)(plane - (long long)b * 2 * g.K);
    const int k = q >> 1;
    const double sre = dp.lam[2 * k] + dp.alpha[b];
    const double sim = (q & 1) ? -dp.lam[2 * k + 1] : dp.lam[2 * k + 1];
    for (int t = threadIdx.x; t < LINES * N; t += NT) {
      const int e = t / LINES;
      const int l = t - e * LINES;
      cx<T> y = buf[l * LD + e + 1];
      const int line = l0 + l;
      if (line < lg.lines) {
        // in-plane coordinates: line = x1 (+ nx x2 in 3-D), element = last axis
        double mu = dp.mu1[e] + dp.mu1[line % g.nx];
        if (g.dim == 3) mu += dp.mu1[line / g.nx];
        const double dre = sre + g.tau * mu;
        const double den = dre * dre + sim * sim;
        // cnorm / (dre + i sim) = cnorm (dre - i sim) / den
        const double fre = dp.cnorm * dre / den;
        const double fim = -dp.cnorm * sim / den;
        y = y * cx<T>{(T)fre, (T)fim};
      }
      buf[l * LD + e + 1] = y;
      buf[l * LD + L - 1 - e] = cx<T>{-y.x, -y.y};
    }
    for (int l = threadIdx.x; l < LINES; l += NT) {
      buf[l * LD] = cx<T>{0, 0};
      buf[l * LD + N + 1] = cx<T>{0, 0};
    }
    __syncthreads();
    p2_fft<T, -1, L, LINES, NT>(buf, LD, twL);
  }
  for (int t = threadIdx.x; t < LINES * N; t += NT) {
    int l, e;
    if (ROWS) {
      l = t / N;
      e = t - l * N;
    } else {
      e = t / LINES;
      l = t - e * LINES;
    }
    if (l0 + l < lg.lines)
      data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride] = buf[l * LD + e + 1];
  }
}

// lines per block: as many as fit 48 KiB of LDS (three blocks per CU); the
// XCD-aware block order lets neighbouring tiles share partially used lines
// ---------------------------------------------------------------------------
// Register variant of the sine-transform pass.  A line of length L = 2(N+1)
// is owned by TL = L/8 threads; thread t always holds the 8 values at the
// positions t + TL s (s = 0..7).  In a Stockham stage with radix R the inputs
// of the thread's butterflies jb = t + TL q (q < 8/R) sit exactly at those
// positions (element s = q + r 8/R), so the first stage reads the odd
// extension straight from the input and the last stage (Ns R = L) leaves the
// transform in natural order in registers; between stages one LDS exchange.
// LDS index is padded by one complex per 8 to spread the stage writes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pidx(int pos) { return pos + (pos >> 3); }

template <class T, int L, int TL, int SG, int NS>
struct RegStages {
  static __device__ __forceinline__ void run(cx<T> (&v)[8], int t, cx<T>* lbuf, const cx<T>* __restrict__ twL) {
    constexpr int R = (L / NS >= 8) ? 8 : (L / NS);
    constexpr int Q = 8 / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int jb = t + TL * q;
      const int jl = jb % NS;
      cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[q + r * Q];
      if (NS > 1 && jl != 0) {
        constexpr int tstep = L / (NS * R);
        if constexpr (sizeof(T) == 8) {
          cx<T> w1 = twL[jl * tstep];
          if (SG > 0) w1.y = -w1.y;
          cx<T> w = w1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            a[r] = a[r] * w;
            w = w * w1;
          }
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = twL[(r * jl * tstep) & (L - 1)];
            if (SG > 0) w.y = -w.y;
            a[r] = a[r] * w;
          }
        }
      }
      dftR<T, SG, R>(a);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * Q] = a[r];
    }
    if constexpr (NS * R < L) {
      // exchange: outputs to LDS, next stage's inputs back
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int jb = t + TL * q;
        const int jl = jb % NS;
        const int base = (jb - jl) * R + jl;
#pragma unroll
        for (int r = 0; r < R; ++r) lbuf[pidx(base + r * NS)] = v[q + r * Q];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 8; ++s) v[s] = lbuf[pidx(t + TL * s)];
      RegStages<T, L, TL, SG, NS * R>::run(v, t, lbuf, twL);
    }
  }
};

template <class T, int L, int ROWS_, int DIVIDE_>
__global__ void __launch_bounds__(256) dst_reg_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                      const cx<T>* __restrict__ twL, DivideParams dp) {
  constexpr bool ROWS = ROWS_ != 0;
  constexpr bool DIVIDE = DIVIDE_ != 0;
  constexpr int N = L / 2 - 1;
  constexpr int TL = L / 8;
  constexpr int LPB = 256 / TL;
  constexpr int LD = L + L / 8 + 1;
  __shared__ cx<T> buf[LPB * LD];
  const int tiles = (lg.lines + LPB - 1) / LPB;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const long long plane = blk / tiles;
  const int l0 = (int)(blk - plane * tiles) * LPB;
  const long long pbase = plane * lg.plane_stride;
  if (DIVIDE && dp.active) {
    if (!dp.active[(int)(plane / (2 * g.K))]) return;
  }
  const int lid = threadIdx.x / TL;
  const int t = threadIdx.x - lid * TL;
  const int line = l0 + lid;
  const bool valid = line < lg.lines;
  cx<T>* lbuf = buf + lid * LD;
  // column passes stage the [N][LPB] tile through LDS with coalesced loads
  if (!ROWS) {
    for (int idx = threadIdx.x; idx < N * LPB; idx += 256) {
      const int e = idx / LPB;
      const int l = idx - e * LPB;
      cx<T> val{0, 0};
      if (l0 + l < lg.lines)
        val = data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride];
      buf[l * LD + pidx(e)] = val;
    }
    __syncthreads();
  }
  auto zval = [&](int e) -> cx<T> {
    if (ROWS) {
      if (!valid) return cx<T>{0, 0};
      return data[pbase + (long long)line * lg.line_stride + (long long)e * lg.elem_stride];
    }
    return lbuf[pidx(e)];
  };
  cx<T> v[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int pos = t + TL * s;
    if (pos >= 1 && pos <= N) {
      v[s] = zval(pos - 1);
    } else if (pos >= N + 2) {
      const cx<T> z = zval(L - 1 - pos);
      v[s] = cx<T>{-z.x, -z.y};
    } else {
      v[s] = cx<T>{0, 0};
    }
  }
  RegStages<T, L, TL, -1, 1>::run(v, t, lbuf, twL);
  if (DIVIDE) {
    const int b = (int)(plane / (2 * g.K));
    const int q = (int)(plane - (long long)b * 2 * g.K);
    const int k = q >> 1;
    const double sre = dp.lam[2 * k] + dp.alpha[b];
    const double sim = (q & 1) ? -dp.lam[2 * k + 1] : dp.lam[2 * k + 1];
    double mul = dp.mu1[line % g.nx];
    if (g.dim == 3) mul += dp.mu1[(line / g.nx) % g.nx];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N && valid) {
        const double dre = sre + g.tau * (mul + dp.mu1[pos - 1]);
        const double den = dre * dre + sim * sim;
        v[s] = v[s] * cx<T>{(T)(dp.cnorm * dre / den), (T)(-dp.cnorm * sim / den)};
      }
    }
    // odd extension of the divided values: the mirrored half comes from LDS
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N) lbuf[pidx(pos)] = v[s];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= N + 2) {
        const cx<T> z = lbuf[pidx(L - pos)];
        v[s] = cx<T>{-z.x, -z.y};
      } else if (pos == 0 || pos == N + 1) {
        v[s] = cx<T>{0, 0};
      }
    }
    RegStages<T, L, TL, -1, 1>::run(v, t, lbuf, twL);
  }
  if (ROWS) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N && valid)
        data[pbase + (long long)line * lg.line_stride + (long long)(pos - 1) * lg.elem_stride] = v[s];
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N) lbuf[pidx(pos - 1)] = v[s];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * LPB; idx += 256) {
      const int e = idx / LPB;
      const int l = idx - e * LPB;
      if (l0 + l < lg.lines)
        data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride] = buf[l * LD + pidx(e)];
    }
  }
}

template <class T, int L>
constexpr int dst_lines_per_block() {
  constexpr int bytes = (L + 1) * (int)sizeof(cx<T>);
  constexpr int fit = 49152 / bytes;
  return fit < 1 ? 1 : (fit > 64 ? 64 : fit);
}

template <class T, int L>
static void dst_pass_L(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                       const cx<T>* twL, const DivideParams& dp, int variant, hipStream_t st) {
  if (variant == 1) {
    // all stages staged through LDS ([LINES][L+1] tiles)
    constexpr int LINES = dst_lines_per_block<T, L>();
    constexpr int NT = 256;
    const long long tiles = (lg.lines + LINES - 1) / LINES;
    dim3 grid((unsigned)(tiles * lg.nplanes));
    if (rows) {
      if (divide) dst_lines_kernel<T, L, LINES, NT, true, true><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
      else dst_lines_kernel<T, L, LINES, NT, true, false><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
    } else {
      if (divide) dst_lines_kernel<T, L, LINES, NT, false, true><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
      else dst_lines_kernel<T, L, LINES, NT, false, false><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
    }
    return;
  }
  // register variant: L/8 threads per line
  constexpr int LPB = 256 / (L / 8);
  const long long tiles = (lg.lines + LPB - 1) / LPB;
  dim3 grid((unsigned)(tiles * lg.nplanes));
  if (rows) {
    if (divide) dst_reg_kernel<T, L, 1, 1><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
    else dst_reg_kernel<T, L, 1, 0><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
  } else {
    if (divide) dst_reg_kernel<T, L, 0, 1><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
    else dst_reg_kernel<T, L, 0, 0><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
  }
}

template <class T>
static bool dst_pass(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                     const cx<T>* twL, const DivideParams& dp, int variant, hipStream_t st) {
  switch (2 * (g.nx + 1)) {
    case 8: dst_pass_L<T, 8>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 16: dst_pass_L<T, 16>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 32: dst_pass_L<T, 32>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 64: dst_pass_L<T, 64>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 128: dst_pass_L<T, 128>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 256: dst_pass_L<T, 256>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 512: dst_pass_L<T, 512>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    case 1024: dst_pass_L<T, 1024>(g, data, lg, rows, divide, twL, dp, variant, st); return true;
    default: return false;
  }
}

// Step 2 with sine transforms: axes 1..d-1 forward, last axis forward +
// divide + inverse, axes d-1..1 inverse (the transforms commute).
template <class T>
static bool dst_solve(const Geo& g, cx<T>* spec, const PrecondTables& tb, hipStream_t st) {
  const int nx = g.nx;
  const long long slices = (long long)g.B * 2 * g.K;
  DivideParams dp{tb.mu1, tb.lam, tb.alpha, tb.active, 0.0};
  dp.cnorm = (g.dim == 2) ? 1.0 / (4.0 * (nx + 1.0) * (nx + 1.0))
                          : -1.0 / (8.0 * (nx + 1.0) * (nx + 1.0) * (nx + 1.0));
  const cx<T>* twL = reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? (const void*)tb.twL64 : (const void*)tb.twL32);
  // x1: contiguous rows
  LineGeom rows{1, 0, (int)(slices * (g.dim == 3 ? nx * nx : nx)), nx, 1};
  // x2 (3-D only as an outer axis): planes (b, q, x3), lines x1, stride nx
  LineGeom ax2{slices * nx, (long long)nx * nx, nx, 1, nx};
  // last axis with the division: planes (b, q), lines = nx^{d-1}
  const int lines_last = (g.dim == 3) ? nx * nx : nx;
  const int stride_last = (g.dim == 3) ? nx * nx : nx;
  LineGeom last{slices, (long long)g.m, lines_last, 1, stride_last};
  // every pass reads and writes the spectrum of the counted members once
  const double pass_bytes = 2.0 * sizeof(cx<T>) * 2.0 * g.K * (double)g.m * tb.nact;
  bool ok = true;
  auto run = [&](const LineGeom& lg, bool r, bool dv, int fam) {
    if (!ok) return;
    tbeg(tb.timer, fam, pass_bytes);
    ok = dst_pass<T>(g, spec, lg, r, dv, twL, dp, tb.dst_variant, st);
    tend(tb.timer);
  };
  run(rows, true, false, KF_DST_ROWS);
  if (g.dim == 3) run(ax2, false, false, KF_DST_AX2);
  run(last, false, true, KF_DST_LAST);
  if (g.dim == 3) run(ax2, false, false, KF_DST_AX2);
  run(rows, true, false, KF_DST_ROWS);
  return ok;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// columns per block for the time passes (power of two, 4..16, LDS <= 64 KiB)
static int time_cols_sk(int n, int csz) {
  int P = 16;
  while (P > 4 && (size_t)2 * n * P * csz > 65536) P /= 2;
  return ((size_t)2 * n * P * csz <= 65536) ? P : 0;
}
// the chirp-z tile is static LDS; up to 80 KiB keeps two blocks per CU
constexpr size_t kBlueLds = 81920;
static int time_cols_bl(int M, int csz) {
  int P = 16;
  while (P > 4 && (size_t)(M + 1) * P * csz > kBlueLds) P /= 2;
  return ((size_t)(M + 1) * P * csz <= kBlueLds) ? P : 0;
}

bool time_lds_fits(int n, bool fp32) {
  const FftPlan pl = make_time_plan(n);
  const int csz = fp32 ? 8 : 16;
  return pl.bluestein ? time_cols_bl(pl.M, csz) > 0 : time_cols_sk(n, csz) > 0;
}

FftPlan make_time_plan(int n) {
  FftPlan pl{};
  int r = n;
  int big = 0;
  for (int f = 2; f * f <= r; ++f)
    while (r % f == 0) {
      if (f > 17) big = 1;
      r /= f;
    }
  if (r > 17) big = 1;
  if (big) {
    pl.bluestein = 1;
    pl.M = 1;
    while (pl.M < 2 * n - 1) pl.M *= 2;
    pl.nrad = 0;
    return pl;
  }
  r = n;
  while (r % 8 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 8; r /= 8; }
  while (r % 4 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 4; r /= 4; }
  while (r % 2 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 2; r /= 2; }
  for (int f = 3; f <= 17 && pl.nrad < 16; f += 2)
    while (r % f == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = f; r /= f; }
  if (pl.nrad == 0) pl.rad[pl.nrad++] = 1;  // n = 1
  return pl;
}

template <class T, int P, int M>
static void bl_launch(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st) {
  // only shapes whose LDS tile fits 64 KiB are instantiated (time_cols_bl picks P accordingly)
  if constexpr ((size_t)(M + 1) * P * sizeof(cx<T>) <= kBlueLds) {
    dim3 grid((g.m + P - 1) / P, g.B);
    if (fwd)
      time_fwd_bl<T, P, M><<<grid, 256, 0, st>>>(g, v, spec, tb.dpow, tt, vscale, vs_stride, tb.active);
    else
      time_inv_bl<T, P, M><<<grid, 256, 0, st>>>(g, spec, w, tb.dpow, tt, accum, tb.active);
  }
}

template <class T, int P>
static bool bl_dispatch_M(bool fwd, int M, const Geo& g, const double* v, cx<T>* spec, double* w,
                          const PrecondTables& tb, const TimeTables& tt, const double* vscale, int vs_stride,
                          int accum, hipStream_t st) {
  switch (M) {
    case 8: bl_launch<T, P, 8>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 16: bl_launch<T, P, 16>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 32: bl_launch<T, P, 32>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 64: bl_launch<T, P, 64>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 128: bl_launch<T, P, 128>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 256: bl_launch<T, P, 256>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 512: bl_launch<T, P, 512>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 1024: bl_launch<T, P, 1024>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    case 2048: bl_launch<T, P, 2048>(fwd, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st); return true;
    default: return false;
  }
}

template <class T>
static bool time_pass(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const double* vscale, int vs_stride, int accum, hipStream_t st) {
  const bool f32 = sizeof(T) == 4;
  TimeTables tt{f32 ? (const void*)tb.twn32 : (const void*)tb.twn64, f32 ? (const void*)tb.twM32 : (const void*)tb.twM64,
                f32 ? (const void*)tb.chirp32 : (const void*)tb.chirp64, f32 ? (const void*)tb.bhat32 : (const void*)tb.bhat64};
  const int csz = (int)sizeof(cx<T>);
  if (tb.plan.bluestein) {
    const int P = time_cols_bl(tb.plan.M, csz);
    if (P == 16) return bl_dispatch_M<T, 16>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
    if (P == 8) return bl_dispatch_M<T, 8>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
    if (P == 4) return bl_dispatch_M<T, 4>(fwd, tb.plan.M, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
    return false;
  }
  const int P = time_cols_sk(g.n, csz);
  if (P == 0) return false;
  dim3 grid((g.m + P - 1) / P, g.B);
  const size_t lds = (size_t)2 * g.n * P * csz;
  const cx<T>* twn = reinterpret_cast<const cx<T>*>(tt.twn);
#define PCOP_TIME_SK(PP)                                                                                   \
  if (fwd)                                                                                                 \
    time_fwd_sk<T, PP><<<grid, 256, lds, st>>>(g, v, spec, tb.dpow, twn, tb.plan, vscale, vs_stride, tb.active); \
  else                                                                                                     \
    time_inv_sk<T, PP><<<grid, 256, lds, st>>>(g, spec, w, tb.dpow, twn, tb.plan, accum, tb.active);
  if (P == 16) {
    PCOP_TIME_SK(16)
  } else if (P == 8) {
    PCOP_TIME_SK(8)
  } else {
    PCOP_TIME_SK(4)
  }
#undef PCOP_TIME_SK
  return true;
}

template <class T>
static bool time_fwd(const Geo& g, const double* v, cx<T>* spec, const PrecondTables& tb,
                     const double* vscale, int vs_stride, hipStream_t st) {
  const double bytes = (8.0 * g.vl + sizeof(cx<T>) * 2.0 * g.K * (double)g.m) * tb.nact;
  tbeg(tb.timer, KF_TIME_FWD, bytes);
  const bool ok = time_pass<T>(true, g, v, spec, nullptr, tb, vscale, vs_stride, 0, st);
  tend(tb.timer);
  return ok;
}

template <class T>
static bool time_inv(const Geo& g, const cx<T>* spec, double* w, const PrecondTables& tb, int accum,
                     hipStream_t st) {
  const double bytes = ((accum ? 16.0 : 8.0) * g.vl + sizeof(cx<T>) * 2.0 * g.K * (double)g.m) * tb.nact;
  tbeg(tb.timer, KF_TIME_INV, bytes);
  const bool ok = time_pass<T>(false, g, nullptr, const_cast<cx<T>*>(spec), w, tb, nullptr, 0, accum, st);
  tend(tb.timer);
  return ok;
}

bool launch_precond(const Geo& g, const double* v, double* w, void* spec, bool fp32, int spatial,
                    const PrecondTables& tb, const double* vscale, int vs_stride, int accum,
                    hipStream_t st) {
  if (fp32) {
    cx<float>* s = reinterpret_cast<cx<float>*>(spec);
    if (!time_fwd<float>(g, v, s, tb, vscale, vs_stride, st)) return false;
    bool ok = (spatial == 0) ? dst_solve<float>(g, s, tb, st) : launch_mg_solve(g, spec, true, tb, st);
    if (!ok) return false;
    if (!time_inv<float>(g, s, w, tb, accum, st)) return false;
  } else {
    cx<double>* s = reinterpret_cast<cx<double>*>(spec);
    if (!time_fwd<double>(g, v, s, tb, vscale, vs_stride, st)) return false;
    bool ok = (spatial == 0) ? dst_solve<double>(g, s, tb, st) : launch_mg_solve(g, spec, false, tb, st);
    if (!ok) return false;
    if (!time_inv<double>(g, s, w, tb, accum, st)) return false;
  }
  return true;
}

}  // namespace pcop
