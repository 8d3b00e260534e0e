// Step 2 of the preconditioner for a = 1: shifted spatial solves by sine
// transforms, one launch per axis over every frequency slice of every member.
#include <algorithm>

#include "common.hpp"
#include "fft_lds.hpp"
#include "launch.hpp"

namespace pcop {

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
  int spm;               // slices per member: plane p belongs to member p / spm, slice p mod spm
  const double* im1;     // [nx] 1/m_k of the Q1 mass matrix, or null (M = I): the shifted
                         // operator sigma M + tau K has the sine-basis eigenvalues
                         // prod_d m_{k_d} (sigma + tau sum_d k_{k_d}/m_{k_d}), mu1 holding k/m
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
    if (!dp.active[(int)(plane / dp.spm)]) return;
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
    const int b = (int)(plane / dp.spm);
    const int q = (int)(plane - (long long)b * dp.spm);
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
        double psi = 1.0;
        if (dp.im1) {
          psi = dp.im1[e] * dp.im1[line % g.nx];
          if (g.dim == 3) psi *= dp.im1[line / g.nx];
        }
        // cnorm / (dre + i sim) = cnorm (dre - i sim) / (dre^2 + sim^2)
        const double f = psi * dp.cnorm / (dre * dre + sim * sim);
        y = y * cx<T>{(T)(f * dre), (T)(-f * sim)};
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
// LDS slots are swizzled rather than padded (pidx below).
// ---------------------------------------------------------------------------

// LDS slot of position p of a line.  gfx950's LDS serves a 16-byte read to
// 16 lanes per pass, without conflict when their slots differ modulo 16, a
// 16-byte write to 8 lanes per pass (slots differing modulo 8), and 8-byte
// reads and writes to 16 lanes (8-byte slots differing modulo 16); this was
// measured with single-instruction loops over fixed lane patterns.  The
// accesses of a line are runs of consecutive positions (stage reads, the
// post-pass writes), stride-8 runs (first-stage writes, p = 8t + r) and
// stride-4 runs (the post-pass reads, p = 4t + i).  XOR-ing the low three
// bits of p with a function h of its 8-slot block b = p / 8 keeps all three
// conflict-free: h takes eight distinct values on any eight consecutive
// blocks (stride-8 writes), and distinct low two bits on the four blocks of
// equal parity inside eight (stride-4 reads).  With 8-byte slots a stride-8
// run of 16 lanes covers sixteen blocks, so bit 3 of p is also flipped by
// bit 3 of b.  Every slot stays in the aligned group of 8 (16-byte slots, or
// positions below 64) or 16 of its position, so a line of X positions needs
// X slots when X is a multiple of 16.
template <class T>
__device__ __forceinline__ int pidx(int p) {
  const int b = p >> 3;
  if constexpr (sizeof(T) == 8) return p ^ (((b >> 1) & 3) | ((b & 1) << 2));
  else return p ^ (((b >> 1) & 7) | (b & 8));
}

// Synchronisation of the threads of one line around an exchange through the
// line's own LDS slots.  A line of at most 64 threads lies inside one
// wavefront, whose LDS instructions complete in issue order, so a compiler
// barrier suffices to keep its writes before its reads (and its reads
// before the next writes); longer lines span several wavefronts and take
// the block barrier.
template <int TL>
__device__ __forceinline__ void line_sync() {
  if constexpr (TL <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS row length of a line of X positions: X once a line fills whole lane
// groups (X >= 128); shorter lines share a wave's lane groups, and one pad
// slot per 8 then keeps neighbouring lines on different banks
constexpr int line_ld(int X) { return X <= 64 ? X + X / 8 : X; }

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
      line_sync<TL>();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int jb = t + TL * q;
        const int jl = jb % NS;
        const int base = (jb - jl) * R + jl;
#pragma unroll
        for (int r = 0; r < R; ++r) lbuf[pidx<T>(base + r * NS)] = v[q + r * Q];
      }
      line_sync<TL>();
#pragma unroll
      for (int s = 0; s < 8; ++s) v[s] = lbuf[pidx<T>(t + TL * s)];
      RegStages<T, L, TL, SG, NS * R>::run(v, t, lbuf, twL);
    }
  }
};

// shift division of step 2 for one line held in registers:
// v <- c v / (sigma_q + tau mu), mu = mu1[line axes] + mu1[element]
template <class T, int L, int TL>
__device__ __forceinline__ void divide_line(cx<T> (&v)[8], int t, const Geo& g, const DivideParams& dp,
                                            long long plane, int line, bool valid) {
  constexpr int N = L / 2 - 1;
  const int b = (int)(plane / dp.spm);
  const int q = (int)(plane - (long long)b * dp.spm);
  const int k = q >> 1;
  const double sre = dp.lam[2 * k] + dp.alpha[b];
  const double sim = (q & 1) ? -dp.lam[2 * k + 1] : dp.lam[2 * k + 1];
  double mul = dp.mu1[line % g.nx];
  if (g.dim == 3) mul += dp.mu1[(line / g.nx) % g.nx];
  double psl = 1.0;
  if (dp.im1) {
    psl = dp.im1[line % g.nx];
    if (g.dim == 3) psl *= dp.im1[(line / g.nx) % g.nx];
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int pos = t + TL * s;
    if (pos >= 1 && pos <= N && valid) {
      const double dre = sre + g.tau * (mul + dp.mu1[pos - 1]);
      const double psi = dp.im1 ? psl * dp.im1[pos - 1] : 1.0;
      const double f = psi * dp.cnorm / (dre * dre + sim * sim);
      v[s] = v[s] * cx<T>{(T)(f * dre), (T)(-f * sim)};
    }
  }
}

// odd extension of the values at positions 1..N, the mirrored half through LDS
template <class T, int L, int TL>
__device__ __forceinline__ void odd_extend(cx<T> (&v)[8], int t, cx<T>* lbuf) {
  constexpr int N = L / 2 - 1;
  line_sync<TL>();
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int pos = t + TL * s;
    if (pos >= 1 && pos <= N) lbuf[pidx<T>(pos)] = v[s];
  }
  line_sync<TL>();
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int pos = t + TL * s;
    if (pos >= N + 2) {
      const cx<T> z = lbuf[pidx<T>(L - pos)];
      v[s] = cx<T>{-z.x, -z.y};
    } else if (pos == 0 || pos == N + 1) {
      v[s] = cx<T>{0, 0};
    }
  }
}

// threads per block of the register row kernel: 128 from L = 512 on (two
// lines of 64 threads, or one line of 128 at L = 1024, where the block's
// exchanges then wait on two wavefronts instead of four: measured 5% faster
// than 256-thread blocks at L = 1024 and 2% at L = 512 in FP64), else 256
constexpr int reg_threads(int L) { return L >= 512 ? (L / 8 > 128 ? L / 8 : 128) : 256; }

// contiguous lines (x1): each line's values go straight between HBM and registers
template <class T, int L, int DIVIDE_>
__global__ void __launch_bounds__(reg_threads(L)) dst_reg_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                                 const cx<T>* __restrict__ twL, DivideParams dp) {
  constexpr bool DIVIDE = DIVIDE_ != 0;
  constexpr int N = L / 2 - 1;
  constexpr int TL = L / 8;
  constexpr int LPB = reg_threads(L) / TL;
  constexpr int LD = line_ld(L);
  __shared__ cx<T> buf[LPB * LD];
  const int tiles = (lg.lines + LPB - 1) / LPB;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const long long plane = blk / tiles;
  const int l0 = (int)(blk - plane * tiles) * LPB;
  const long long pbase = plane * lg.plane_stride;
  if (DIVIDE && dp.active) {
    if (!dp.active[(int)(plane / dp.spm)]) return;
  }
  const int lid = threadIdx.x / TL;
  const int t = threadIdx.x - lid * TL;
  const int line = l0 + lid;
  const bool valid = line < lg.lines;
  cx<T>* lbuf = buf + lid * LD;
  auto zval = [&](int e) -> cx<T> {
    if (!valid) return cx<T>{0, 0};
    return data[pbase + (long long)line * lg.line_stride + (long long)e * lg.elem_stride];
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
    divide_line<T, L, TL>(v, t, g, dp, plane, line, valid);
    odd_extend<T, L, TL>(v, t, lbuf);
    RegStages<T, L, TL, -1, 1>::run(v, t, lbuf, twL);
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int pos = t + TL * s;
    if (pos >= 1 && pos <= N && valid)
      data[pbase + (long long)line * lg.line_stride + (long long)(pos - 1) * lg.elem_stride] = v[s];
  }
}

// Strided lines (x2, x3; consecutive lines adjacent in memory): a tile of
// LPB lines x N elements is staged through LDS with coalesced accesses.
// Persistent blocks walk tiles blk, blk + grid, ... and fetch the next tile
// into registers while the current one is transformed.
template <class T, int L, int DIVIDE_, int NT>
__global__ void __launch_bounds__(NT) dst_col_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                      const cx<T>* __restrict__ twL, DivideParams dp) {
  constexpr bool DIVIDE = DIVIDE_ != 0;
  constexpr int N = L / 2 - 1;
  constexpr int TL = L / 8;
  constexpr int LPB = NT / TL;
  constexpr int LD = line_ld(L);
  constexpr int QS = (N * LPB + NT - 1) / NT;  // tile elements per thread
  __shared__ cx<T> buf[LPB * LD];
  // twiddles and 1-D eigenvalues in LDS: inside the loop the only global
  // loads are the prefetch (loads retire in order)
  __shared__ cx<T> twl[L];
  __shared__ double mul[DIVIDE ? N : 1];
  for (int k = threadIdx.x; k < L; k += NT) twl[k] = twL[k];
  if (DIVIDE)
    for (int k = threadIdx.x; k < N; k += NT) mul[k] = dp.mu1[k];
  __syncthreads();
  DivideParams dl = dp;
  dl.mu1 = mul;
  const long long tiles = (lg.lines + LPB - 1) / LPB;
  const long long total = tiles * lg.nplanes;
  const int lid = threadIdx.x / TL;
  const int t = threadIdx.x - lid * TL;
  cx<T>* lbuf = buf + lid * LD;
  // tiles blk, blk + G, ...: consecutive logical blocks sit on one XCD and
  // process neighbouring tiles (which share 128-byte lines) at the same time
  auto next = [&](long long blk) {
    if (DIVIDE && dp.active)
      while (blk < total && !dp.active[(int)((blk / tiles) / dp.spm)]) blk += gridDim.x;
    return blk;
  };
  cx<T> pre[QS];
  auto fetch = [&](long long blk) {
    const long long plane = blk / tiles;
    const int l0 = (int)(blk - plane * tiles) * LPB;
    const long long pbase = plane * lg.plane_stride;
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int idx = threadIdx.x + NT * q;
      const int e = idx / LPB, l = idx - (idx / LPB) * LPB;
      const bool ok = idx < N * LPB && l0 + l < lg.lines;
      pre[q] = ok ? data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride]
                  : cx<T>{0, 0};
    }
  };
  long long blk = next(xcd_remap(blockIdx.x, gridDim.x));
  if (blk < total) fetch(blk);
  while (blk < total) {
    const long long plane = blk / tiles;
    const int l0 = (int)(blk - plane * tiles) * LPB;
    const long long pbase = plane * lg.plane_stride;
    const int line = l0 + lid;
    const bool valid = line < lg.lines;
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int idx = threadIdx.x + NT * q;
      if (idx < N * LPB) {
        const int e = idx / LPB, l = idx - (idx / LPB) * LPB;
        buf[l * LD + pidx<T>(e)] = pre[q];
      }
    }
    __syncthreads();
    const long long nxt = next(blk + gridDim.x);
    if (nxt < total) fetch(nxt);
    cx<T> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N) {
        v[s] = lbuf[pidx<T>(pos - 1)];
      } else if (pos >= N + 2) {
        const cx<T> z = lbuf[pidx<T>(L - 1 - pos)];
        v[s] = cx<T>{-z.x, -z.y};
      } else {
        v[s] = cx<T>{0, 0};
      }
    }
    RegStages<T, L, TL, -1, 1>::run(v, t, lbuf, twl);
    if (DIVIDE) {
      divide_line<T, L, TL>(v, t, g, dl, plane, line, valid);
      odd_extend<T, L, TL>(v, t, lbuf);
      RegStages<T, L, TL, -1, 1>::run(v, t, lbuf, twl);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int pos = t + TL * s;
      if (pos >= 1 && pos <= N) lbuf[pidx<T>(pos - 1)] = v[s];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int idx = threadIdx.x + NT * q;
      const int e = idx / LPB, l = idx - (idx / LPB) * LPB;
      if (idx < N * LPB && l0 + l < lg.lines)
        data[pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride] = buf[l * LD + pidx<T>(e)];
    }
    __syncthreads();
    blk = nxt;
  }
}

// ---------------------------------------------------------------------------
// Half-length variant for strided lines.  With M = L/2 = N + 1 and z_0 = 0,
//   y_j = sin(pi j/M) (z_j + z_{M-j}) + (z_j - z_{M-j})/2,  U = FFT_M(y),
// the stored values Y_k = -2i sum_j z_j sin(pi j k/M) of the odd-extension
// transform follow as
//   Y_{2k} = U_k - U_{M-k}   (k >= 1),
//   Y_{2k+1} = -i P_k,  P_k = U_0 + sum_{q=1..k} (U_q + U_{M-q}),
// (for a real z this is the classic sine transform through a real FFT of
// length M: the symmetric part of y gives the odd outputs by a recurrence,
// the antisymmetric part the even ones; the complex data carry two real
// lines at once).  One length-M FFT per transform instead of length 2M:
// M/8 threads per line, so a 256-thread tile holds twice the lines (whole
// 128-byte rows of the strided axis in FP64 for nx = 255).
// ---------------------------------------------------------------------------
template <class T, int L>
struct HalfDst {
  static constexpr int M = L / 2, N = M - 1, TM = M / 8;
  // y_j (j = t + TM s) from the line's values z_{e+1} at lbuf[pidx(e)]
  static __device__ __forceinline__ void pre(cx<T> (&v)[8], int t, const cx<T>* lbuf, const T* sinl) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int j = t + TM * s;
      if (j == 0) {
        v[s] = cx<T>{0, 0};
      } else {
        const cx<T> a = lbuf[pidx<T>(j - 1)], b = lbuf[pidx<T>(M - j - 1)];
        const T sj = sinl[j];
        const cx<T> sum = a + b, dif = a - b;
        v[s] = cx<T>{sj * sum.x + (T)0.5 * dif.x, sj * sum.y + (T)0.5 * dif.y};
      }
    }
  }
  // from U (natural order in v, positions t + TM s) to Y at positions
  // 8t .. 8t + 7 (o[r] = Y_{8t + r}); the prefix sum runs over the TM
  // threads of the line, which sit in one wavefront
  static __device__ __forceinline__ void post(cx<T> (&v)[8], cx<T> (&o)[8], int t, cx<T>* lbuf) {
    line_sync<TM>();
#pragma unroll
    for (int s = 0; s < 8; ++s) lbuf[pidx<T>(t + TM * s)] = v[s];
    line_sync<TM>();
    cx<T> c[4], e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * t + i;
      const cx<T> uk = lbuf[pidx<T>(k)];
      const cx<T> um = lbuf[pidx<T>(k == 0 ? 0 : M - k)];
      c[i] = (k == 0) ? uk : uk + um;
      e[i] = uk - um;
    }
    // inclusive prefix within the thread, then an exclusive scan of the
    // thread totals over the line
    cx<T> run = c[0];
    c[0] = run;
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      run = run + c[i];
      c[i] = run;
    }
    cx<T> incl = run;
#pragma unroll
    for (int d = 1; d < TM; d *= 2) {
      const T px = __shfl_up(incl.x, d, TM);
      const T py = __shfl_up(incl.y, d, TM);
      if (t >= d) incl = incl + cx<T>{px, py};
    }
    const cx<T> excl = incl - run;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const cx<T> pk = excl + c[i];
      o[2 * i] = e[i];                      // Y_{2k} (Y_0 unused)
      o[2 * i + 1] = cx<T>{pk.y, -pk.x};    // -i P_k
    }
  }
};

template <class T, int L, int DIVIDE_, int NT>
__global__ void __launch_bounds__(NT) dst_half_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                       const cx<T>* __restrict__ twL, DivideParams dp) {
  using H = HalfDst<T, L>;
  constexpr bool DIVIDE = DIVIDE_ != 0;
  constexpr int M = H::M, N = H::N, TM = H::TM;
  constexpr int LPB = NT / TM;
  // tile rows: with four lanes on four elements of one line (QUAD below),
  // a row length of 4 mod 16 slots puts a 16-lane read of 4 lines x 4
  // elements and an 8-lane write of 2 lines x 4 elements on distinct banks
  constexpr bool QUAD = TM >= 4;
  constexpr int LD = M >= 128 ? M + 4 : line_ld(M);
  constexpr int QS = (N * LPB + NT - 1) / NT;  // tile elements per thread
  static_assert(LPB * TM == NT, "a tile is a whole number of lines");
  __shared__ cx<T> buf[LPB * LD];
  // length-M twiddles exp(-2 pi i t/M) = twL[2t], sines sin(pi j/M) = -Im twL[j],
  // 1-D eigenvalues: in LDS, so that the tile's loads are the only global loads in the loop
  __shared__ cx<T> twm[M];
  __shared__ T sinl[M];
  __shared__ T mul[DIVIDE ? N : 1];
  for (int k = threadIdx.x; k < M; k += NT) {
    twm[k] = twL[2 * k];
    sinl[k] = -twL[k].y;
  }
  if (DIVIDE)
    for (int k = threadIdx.x; k < N; k += NT) mul[k] = (T)dp.mu1[k];
  __syncthreads();
  const long long tiles = (lg.lines + LPB - 1) / LPB;
  const long long total = tiles * lg.nplanes;
  const int lid = threadIdx.x / TM;
  const int t = threadIdx.x - lid * TM;
  cx<T>* lbuf = buf + lid * LD;
  auto next = [&](long long blk) {
    if (DIVIDE && dp.active)
      while (blk < total && !dp.active[(int)((blk / tiles) / dp.spm)]) blk += gridDim.x;
    return blk;
  };
  // element e of line l0 + l sits at (l0 + l) line_stride + e elem_stride
  // inside its plane (an in-plane offset, below 2^31).  A thread always
  // handles line tl of the tile, elements te + TM q: with QUAD, thread
  // 4 LPB a + 4 l + c takes line l and te = c + 4a, else line
  // threadIdx.x mod LPB and te = threadIdx.x / LPB (both cover every
  // (line, element) pair once; a wave's loads span the same rows either way)
  const int tl = QUAD ? (threadIdx.x >> 2) % LPB : threadIdx.x % LPB;
  const int te = QUAD ? (threadIdx.x & 3) + 4 * (threadIdx.x / (4 * LPB)) : threadIdx.x / LPB;
  long long blk = next(xcd_remap(blockIdx.x, gridDim.x));
  while (blk < total) {
    const long long plane = blk / tiles;
    const int l0 = (int)(blk - plane * tiles) * LPB;
    const long long pbase = plane * lg.plane_stride;
    const int line = l0 + lid;
    const bool valid = line < lg.lines;
    {
      // the tile's loads, straight into LDS (a register prefetch of the
      // next tile was measured slower: its 32 extra registers per thread
      // cost a wave per SIMD in FP64 and stalled the FP32 kernel)
      const cx<T>* src = data + pbase;
      const bool lok = l0 + tl < lg.lines;
      const int off = (l0 + tl) * lg.line_stride + te * lg.elem_stride;
      cx<T> cur[QS];
#pragma unroll
      for (int q = 0; q < QS; ++q) {
        const bool ok = te + TM * q < N && lok;
        cur[q] = ok ? src[off + q * TM * lg.elem_stride] : cx<T>{0, 0};
      }
#pragma unroll
      for (int q = 0; q < QS; ++q)
        if (te + TM * q < N) buf[tl * LD + pidx<T>(te + TM * q)] = cur[q];
    }
    __syncthreads();
    const long long nxt = next(blk + gridDim.x);
    cx<T> v[8], o[8];
    H::pre(v, t, lbuf, sinl);
    RegStages<T, M, TM, -1, 1>::run(v, t, lbuf, twm);
    H::post(v, o, t, lbuf);
    if (DIVIDE) {
      // the shift of plane p = (b, q): lambda_{q/2} + alpha_b, conjugated for odd q
      const int b = (int)(plane / dp.spm);
      const int q = (int)(plane - (long long)b * dp.spm);
      const int k = q >> 1;
      const double sre = dp.lam[2 * k] + dp.alpha[b];
      const double sim = (q & 1) ? -dp.lam[2 * k + 1] : dp.lam[2 * k + 1];
      double ml = mul[line % g.nx];
      if (g.dim == 3) ml += mul[(line / g.nx) % g.nx];
      double psl = 1.0;
      if (dp.im1) {
        psl = dp.im1[line % g.nx];
        if (g.dim == 3) psl *= dp.im1[(line / g.nx) % g.nx];
      }
      if constexpr (sizeof(T) == 4) {
        // the FP32 preconditioner forms the shift factor in FP32 with the
        // hardware reciprocal (about 1 ulp; the denominator is bounded away
        // from zero and well inside the normal range)
        const float srf = (float)sre, sif = (float)sim, tf = (float)g.tau, mlf = (float)ml;
        const float cn = (float)(psl * dp.cnorm);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int pos = 8 * t + r;
          if (pos >= 1 && pos <= N && valid) {
            const float dre = srf + tf * (mlf + mul[pos - 1]);
            const float psi = dp.im1 ? (float)dp.im1[pos - 1] : 1.0f;
            const float f = psi * cn * recip(dre * dre + sif * sif);
            o[r] = o[r] * cx<T>{f * dre, -f * sif};
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int pos = 8 * t + r;
          if (pos >= 1 && pos <= N && valid) {
            const double dre = sre + g.tau * (ml + mul[pos - 1]);
            const double psi = dp.im1 ? psl * dp.im1[pos - 1] : 1.0;
            const double f = psi * dp.cnorm / (dre * dre + sim * sim);
            o[r] = o[r] * cx<T>{(T)(f * dre), (T)(-f * sim)};
          }
        }
      }
      // the divided values become the input of the inverse transform
      line_sync<TM>();
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int pos = 8 * t + r;
        if (pos >= 1 && pos <= N) lbuf[pidx<T>(pos - 1)] = o[r];
      }
      line_sync<TM>();
      H::pre(v, t, lbuf, sinl);
      RegStages<T, M, TM, -1, 1>::run(v, t, lbuf, twm);
      H::post(v, o, t, lbuf);
    }
    line_sync<TM>();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int pos = 8 * t + r;
      if (pos >= 1 && pos <= N) lbuf[pidx<T>(pos - 1)] = o[r];
    }
    __syncthreads();
    if (l0 + tl < lg.lines) {
      cx<T>* dstp = data + pbase;
      const int off = (l0 + tl) * lg.line_stride + te * lg.elem_stride;
#pragma unroll
      for (int q = 0; q < QS; ++q) {
        const int e = te + TM * q;
        if (e < N) dstp[off + q * TM * lg.elem_stride] = buf[tl * LD + pidx<T>(e)];
      }
    }
    __syncthreads();
    blk = nxt;
  }
}

// Half-length transforms of contiguous lines (x1).  A tile is LPB whole
// lines; its elements are loaded and stored in flattened order (element f
// of the tile is element f mod N of line f / N), so consecutive threads
// touch consecutive addresses when the lines follow each other (line
// stride N), and each line's values are staged in LDS for HalfDst::pre.
// Persistent blocks prefetch the next tile into registers.
template <class T, int L, int NT>
__global__ void __launch_bounds__(NT) dst_half_rows_kernel(Geo g, cx<T>* __restrict__ data, LineGeom lg,
                                                            const cx<T>* __restrict__ twL) {
  using H = HalfDst<T, L>;
  constexpr int M = H::M, N = H::N, TM = H::TM;
  constexpr int LPB = NT / TM;
  constexpr int LD = line_ld(M);
  constexpr int QS = (N * LPB + NT - 1) / NT;
  static_assert(LPB * TM == NT, "a tile is a whole number of lines");
  __shared__ cx<T> buf[LPB * LD];
  __shared__ cx<T> twm[M];
  __shared__ T sinl[M];
  for (int k = threadIdx.x; k < M; k += NT) {
    twm[k] = twL[2 * k];
    sinl[k] = -twL[k].y;
  }
  __syncthreads();
  const long long tiles = (lg.lines + LPB - 1) / LPB;
  const long long total = tiles * lg.nplanes;
  const int lid = threadIdx.x / TM;
  const int t = threadIdx.x - lid * TM;
  cx<T>* lbuf = buf + lid * LD;
  // the (line, element) of each of this thread's tile slots
  int sl[QS], se[QS];
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int f = threadIdx.x + NT * q;
    sl[q] = f / N;
    se[q] = f - sl[q] * N;
  }
  cx<T> pre[QS];
  auto fetch = [&](long long blk) {
    const long long plane = blk / tiles;
    const int l0 = (int)(blk - plane * tiles) * LPB;
    const cx<T>* src = data + plane * lg.plane_stride;
    // unconditional loads from a clamped line: slots past the tile or the
    // last line hold copies of real values, which are never stored
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int ln = min(l0 + sl[q], lg.lines - 1);
      pre[q] = src[ln * lg.line_stride + se[q] * lg.elem_stride];
    }
  };
  long long blk = xcd_remap(blockIdx.x, gridDim.x);
  if (blk < total) fetch(blk);
  while (blk < total) {
    const long long plane = blk / tiles;
    const int l0 = (int)(blk - plane * tiles) * LPB;
#pragma unroll
    for (int q = 0; q < QS; ++q)
      if (threadIdx.x + NT * q < N * LPB) buf[sl[q] * LD + pidx<T>(se[q])] = pre[q];
    __syncthreads();
    const long long nxt = blk + gridDim.x;
    if (nxt < total) fetch(nxt);
    cx<T> v[8], o[8];
    H::pre(v, t, lbuf, sinl);
    RegStages<T, M, TM, -1, 1>::run(v, t, lbuf, twm);
    H::post(v, o, t, lbuf);
    line_sync<TM>();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int pos = 8 * t + r;
      if (pos >= 1 && pos <= N) lbuf[pidx<T>(pos - 1)] = o[r];
    }
    __syncthreads();
    cx<T>* dstp = data + plane * lg.plane_stride;
#pragma unroll
    for (int q = 0; q < QS; ++q)
      if (threadIdx.x + NT * q < N * LPB && l0 + sl[q] < lg.lines)
        dstp[(l0 + sl[q]) * lg.line_stride + se[q] * lg.elem_stride] = buf[sl[q] * LD + pidx<T>(se[q])];
    __syncthreads();
    blk = nxt;
  }
}

template <class T, int L>
constexpr int dst_lines_per_block() {
  constexpr int bytes = (L + 1) * (int)sizeof(cx<T>);
  constexpr int fit = 49152 / bytes;
  return fit < 1 ? 1 : (fit > 64 ? 64 : fit);
}

// persistent grid of half-length strided kernels: as many blocks as stay
// resident on every CU
template <class T, int L, int NT>
static void launch_half_strided(const Geo& g, cx<T>* data, const LineGeom& lg, bool divide, const cx<T>* twL,
                                const DivideParams& dp, int ncu, hipStream_t st) {
  constexpr int LPBH = NT / (L / 16);
  const long long tilesh = (lg.lines + LPBH - 1) / LPBH;
  static const int rh1 = resident_blocks(dst_half_kernel<T, L, 1, NT>, NT, 0);
  static const int rh0 = resident_blocks(dst_half_kernel<T, L, 0, NT>, NT, 0);
  const long long want = (long long)(divide ? rh1 : rh0) * std::max(1, ncu);
  dim3 grid((unsigned)std::min(tilesh * lg.nplanes, want));
  if (divide) dst_half_kernel<T, L, 1, NT><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
  else dst_half_kernel<T, L, 0, NT><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
}

template <class T, int L>
static void dst_pass_L(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                       const cx<T>* twL, const DivideParams& dp, int variant, int ncu, hipStream_t st) {
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
  // register variants: L/8 threads per line
  constexpr int LPB = 256 / (L / 8);
  const long long tiles = (lg.lines + LPB - 1) / LPB;
  if constexpr (L >= 16) {
    if (variant == 4 && rows && !divide) {
      // half-length rows: M/8 threads per line, persistent 256-thread tiles
      constexpr int LPBH = 256 / (L / 16);
      const long long tilesh = (lg.lines + LPBH - 1) / LPBH;
      static const int rr = resident_blocks(dst_half_rows_kernel<T, L, 256>, 256, 0);
      const long long want = (long long)rr * std::max(1, ncu);
      dim3 grid((unsigned)std::min(tilesh * lg.nplanes, want));
      dst_half_rows_kernel<T, L, 256><<<grid, 256, 0, st>>>(g, data, lg, twL);
      return;
    }
  }
  if (rows) {
    constexpr int NTR = reg_threads(L), LPBR = NTR / (L / 8);
    dim3 grid((unsigned)((lg.lines + LPBR - 1) / LPBR * lg.nplanes));
    if (divide) dst_reg_kernel<T, L, 1><<<grid, NTR, 0, st>>>(g, data, lg, twL, dp);
    else dst_reg_kernel<T, L, 0><<<grid, NTR, 0, st>>>(g, data, lg, twL, dp);
  } else {
    // persistent grid: as many blocks as stay resident on every CU.  Variant
    // 2 doubles the lines per tile (512 threads) so that each element row of
    // a tile spans 128 bytes instead of 64
    if constexpr (L >= 16) {
      if (variant == 3 || variant == 4) {
        // half-length transforms: M/8 threads per line, 256-thread tiles
        // (512-thread tiles, whose element rows span twice the bytes, were
        // measured slower: their registers allow one block per CU)
        launch_half_strided<T, L, 256>(g, data, lg, divide, twL, dp, ncu, st);
        return;
      }
    }
    if constexpr (L >= 64) {
      if (variant == 2) {
      constexpr int LPB2 = 512 / (L / 8);
      const long long tiles2 = (lg.lines + LPB2 - 1) / LPB2;
      static const int r1 = resident_blocks(dst_col_kernel<T, L, 1, 512>, 512, 0);
      static const int r0 = resident_blocks(dst_col_kernel<T, L, 0, 512>, 512, 0);
      const long long want = (long long)(divide ? r1 : r0) * std::max(1, ncu);
      dim3 grid((unsigned)std::min(tiles2 * lg.nplanes, want));
      if (divide) dst_col_kernel<T, L, 1, 512><<<grid, 512, 0, st>>>(g, data, lg, twL, dp);
      else dst_col_kernel<T, L, 0, 512><<<grid, 512, 0, st>>>(g, data, lg, twL, dp);
      return;
      }
    }
    static const int res1 = resident_blocks(dst_col_kernel<T, L, 1, 256>, 256, 0);
    static const int res0 = resident_blocks(dst_col_kernel<T, L, 0, 256>, 256, 0);
    const long long want = (long long)(divide ? res1 : res0) * std::max(1, ncu);
    dim3 grid((unsigned)std::min(tiles * lg.nplanes, want));
    if (divide) dst_col_kernel<T, L, 1, 256><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
    else dst_col_kernel<T, L, 0, 256><<<grid, 256, 0, st>>>(g, data, lg, twL, dp);
  }
}

template <class T>
static bool dst_pass(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                     const cx<T>* twL, const DivideParams& dp, int variant, int ncu, hipStream_t st) {
  switch (2 * (g.nx + 1)) {
    case 8: dst_pass_L<T, 8>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 16: dst_pass_L<T, 16>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 32: dst_pass_L<T, 32>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 64: dst_pass_L<T, 64>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 128: dst_pass_L<T, 128>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 256: dst_pass_L<T, 256>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 512: dst_pass_L<T, 512>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    case 1024: dst_pass_L<T, 1024>(g, data, lg, rows, divide, twL, dp, variant, ncu, st); return true;
    default: return false;
  }
}

// Step 2 with sine transforms: axes 1..d-1 forward, last axis forward +
// divide + inverse, axes d-1..1 inverse (the transforms commute).  spm
// slices per member; slice q of member b is divided by
// lam_{q/2} + alpha_b (q even) or its conjugate (q odd).
template <class T>
static bool dst_solve(const Geo& g, cx<T>* spec, const PrecondTables& tb, int spm, const double* lam,
                      hipStream_t st) {
  const int nx = g.nx;
  const long long slices = (long long)g.B * spm;
  DivideParams dp{tb.mu1, lam, tb.alpha, tb.active, 0.0, spm, tb.im1};
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
  // every pass reads and writes the slices of the counted members once
  const double pass_bytes = 2.0 * sizeof(cx<T>) * spm * (double)g.m * tb.nact;
  bool ok = true;
  auto run = [&](const LineGeom& lg, bool r, bool dv, int fam) {
    if (!ok) return;
    tbeg(tb.timer, fam, pass_bytes);
    ok = dst_pass<T>(g, spec, lg, r, dv, twL, dp, tb.dst_variant, tb.ncu, st);
    tend(tb.timer);
  };
  run(rows, true, false, KF_DST_ROWS);
  if (g.dim == 3) run(ax2, false, false, KF_DST_AX2);
  run(last, false, true, KF_DST_LAST);
  if (g.dim == 3) run(ax2, false, false, KF_DST_AX2);
  run(rows, true, false, KF_DST_ROWS);
  return ok;
}

bool launch_dst_solve(const Geo& g, void* spec, bool fp32, const PrecondTables& tb, int spm, const double* lam,
                      hipStream_t st) {
  if (fp32) return dst_solve<float>(g, reinterpret_cast<cx<float>*>(spec), tb, spm, lam, st);
  return dst_solve<double>(g, reinterpret_cast<cx<double>*>(spec), tb, spm, lam, st);
}

}  // namespace pcop
