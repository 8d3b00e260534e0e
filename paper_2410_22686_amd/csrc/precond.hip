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
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) time_fwd_kernel(Geo g, const double* __restrict__ v,
                                                       cx<T>* __restrict__ spec,
                                                       const double* __restrict__ dpow,
                                                       const cx<T>* __restrict__ tw, FftPlan plan,
                                                       int P, const double* __restrict__ vscale, int vs_stride,
                                                       const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf0 = reinterpret_cast<cx<T>*>(smem);
  cx<T>* buf1 = buf0 + n * P;
  const int i0 = blockIdx.x * P;
  const double s = vscale ? vscale[(size_t)b * vs_stride] : 1.0;
  const double* v1 = v + (size_t)b * g.vl;
  const double* v2 = v1 + (size_t)n * m;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    const int i = i0 + p;
    double a1 = 0.0, a2 = 0.0;
    if (i < m) {
      a1 = v1[(size_t)j * m + i];
      a2 = v2[(size_t)j * m + i];
    }
    const double d = dpow[j];
    buf0[t] = cx<T>{(T)(s * d * a2), (T)(s * a1 / d)};
  }
  __syncthreads();
  cx<T>* res = tpo_fft<T, false>(buf0, buf1, n, P, plan, tw);
  cx<T>* out = spec + (size_t)b * (size_t)(2 * K) * m;
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int i = i0 + p;
    if (i >= m) continue;
    const int kn = (k == 0) ? 0 : n - k;
    const cx<T> X = res[k * P + p];
    const cx<T> Y = conj(res[kn * P + p]);
    const cx<T> sum = X + Y, dif = X - Y;
    out[(size_t)(2 * k) * m + i] = cx<T>{sum.x * (T)0.5, sum.y * (T)0.5};
    out[(size_t)(2 * k + 1) * m + i] = cx<T>{dif.y * (T)0.5, -dif.x * (T)0.5};  // dif / (2i)
  }
}

template <class T>
__global__ void __launch_bounds__(256) time_inv_kernel(Geo g, const cx<T>* __restrict__ spec,
                                                       double* __restrict__ w,
                                                       const double* __restrict__ dpow,
                                                       const cx<T>* __restrict__ tw, FftPlan plan,
                                                       int P, int accum,
                                                       const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int n = g.n, m = g.m, K = g.K;
  cx<T>* buf0 = reinterpret_cast<cx<T>*>(smem);
  cx<T>* buf1 = buf0 + n * P;
  const int i0 = blockIdx.x * P;
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
    buf0[k * P + p] = cx<T>{z2.x - z1.y, z2.y + z1.x};
    if (k != 0 && 2 * k != n) buf0[(n - k) * P + p] = cx<T>{z2.x + z1.y, z1.x - z2.y};
  }
  __syncthreads();
  cx<T>* res = tpo_fft<T, true>(buf0, buf1, n, P, plan, tw);
  double* w1 = w + (size_t)b * g.vl;
  double* w2 = w1 + (size_t)n * m;
  const double inv_n = 1.0 / (double)n;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) {
    const int j = t / P, p = t - j * P;
    const int i = i0 + p;
    if (i >= m) continue;
    const cx<T> e = res[t];
    const double d = dpow[j];
    const double z2 = (double)e.x * inv_n / d;
    const double z1 = (double)e.y * inv_n * d;
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
  const long long plane = blockIdx.x / tiles;
  const int l0 = (int)(blockIdx.x - plane * tiles) * LINES;
  const long long pbase = plane * lg.plane_stride;
  if (DIVIDE && dp.active) {
    const long long b = pbase / ((long long)2 * g.K * g.m);
    if (!dp.active[b]) return;
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
    const long long slice_len = (long long)2 * g.K * g.m;
    for (int t = threadIdx.x; t < LINES * N; t += NT) {
      const int e = t / LINES;
      const int l = t - e * LINES;
      cx<T> y = buf[l * LD + e + 1];
      if (l0 + l < lg.lines) {
        const long long off = pbase + (long long)(l0 + l) * lg.line_stride + (long long)e * lg.elem_stride;
        const int b = (int)(off / slice_len);
        const long long r = off - (long long)b * slice_len;
        const int q = (int)(r / g.m);
        const int i = (int)(r - (long long)q * g.m);
        const int c1 = i % g.nx;
        const int c2 = (i / g.nx) % g.nx;
        double mu = dp.mu1[c1] + dp.mu1[c2];
        if (g.dim == 3) mu += dp.mu1[i / (g.nx * g.nx)];
        const int k = q >> 1;
        const double lre = dp.lam[2 * k];
        const double lim = (q & 1) ? -dp.lam[2 * k + 1] : dp.lam[2 * k + 1];
        const double dre = lre + dp.alpha[b] + g.tau * mu;
        const double den = dre * dre + lim * lim;
        // cnorm / (dre + i lim) = cnorm (dre - i lim) / den
        const double fre = dp.cnorm * dre / den;
        const double fim = -dp.cnorm * lim / den;
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

template <class T, int L>
constexpr int dst_lines_per_block() {
  constexpr int bytes = L * (int)sizeof(cx<T>);
  constexpr int v = 49152 / bytes;
  return v < 1 ? 1 : (v > 64 ? 64 : v);
}

template <class T, int L>
static void dst_pass_L(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                       const cx<T>* twL, const DivideParams& dp, hipStream_t st) {
  constexpr int LINES = dst_lines_per_block<T, L>();
  constexpr int NT = 256;
  const long long tiles = (lg.lines + LINES - 1) / LINES;
  const long long blocks = tiles * lg.nplanes;
  dim3 grid((unsigned)blocks);
  (void)g;
  if (rows) {
    if (divide)
      dst_lines_kernel<T, L, LINES, NT, true, true><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
    else
      dst_lines_kernel<T, L, LINES, NT, true, false><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
  } else {
    if (divide)
      dst_lines_kernel<T, L, LINES, NT, false, true><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
    else
      dst_lines_kernel<T, L, LINES, NT, false, false><<<grid, NT, 0, st>>>(g, data, lg, twL, dp);
  }
}

template <class T>
static bool dst_pass(const Geo& g, cx<T>* data, const LineGeom& lg, bool rows, bool divide,
                     const cx<T>* twL, const DivideParams& dp, hipStream_t st) {
  switch (2 * (g.nx + 1)) {
    case 8: dst_pass_L<T, 8>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 16: dst_pass_L<T, 16>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 32: dst_pass_L<T, 32>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 64: dst_pass_L<T, 64>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 128: dst_pass_L<T, 128>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 256: dst_pass_L<T, 256>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 512: dst_pass_L<T, 512>(g, data, lg, rows, divide, twL, dp, st); return true;
    case 1024: dst_pass_L<T, 1024>(g, data, lg, rows, divide, twL, dp, st); return true;
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
    ok = dst_pass<T>(g, spec, lg, r, dv, twL, dp, st);
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
template <class T>
static int time_cols(int n) {
  // two ping-pong buffers of n x P complex in <= 64 KiB of LDS
  int P = 65536 / (2 * n * (int)sizeof(cx<T>));
  int p2 = 1;
  while (p2 * 2 <= P && p2 < 64) p2 *= 2;
  return p2;
}

template <class T>
static void time_fwd(const Geo& g, const double* v, cx<T>* spec, const PrecondTables& tb,
                     const double* vscale, int vs_stride, hipStream_t st) {
  const int P = time_cols<T>(g.n);
  dim3 grid((g.m + P - 1) / P, g.B);
  size_t lds = (size_t)2 * g.n * P * sizeof(cx<T>);
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? (const void*)tb.twn64 : (const void*)tb.twn32);
  const double bytes = (8.0 * g.vl + sizeof(cx<T>) * 2.0 * g.K * (double)g.m) * tb.nact;
  tbeg(tb.timer, KF_TIME_FWD, bytes);
  time_fwd_kernel<T><<<grid, 256, lds, st>>>(g, v, spec, tb.dpow, tw, tb.plan, P, vscale, vs_stride, tb.active);
  tend(tb.timer);
}

template <class T>
static void time_inv(const Geo& g, const cx<T>* spec, double* w, const PrecondTables& tb, int accum,
                     hipStream_t st) {
  const int P = time_cols<T>(g.n);
  dim3 grid((g.m + P - 1) / P, g.B);
  size_t lds = (size_t)2 * g.n * P * sizeof(cx<T>);
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? (const void*)tb.twn64 : (const void*)tb.twn32);
  const double bytes = ((accum ? 16.0 : 8.0) * g.vl + sizeof(cx<T>) * 2.0 * g.K * (double)g.m) * tb.nact;
  tbeg(tb.timer, KF_TIME_INV, bytes);
  time_inv_kernel<T><<<grid, 256, lds, st>>>(g, spec, w, tb.dpow, tw, tb.plan, P, accum, tb.active);
  tend(tb.timer);
}

bool time_lds_fits(int n, bool fp32) {
  const int P = fp32 ? time_cols<float>(n) : time_cols<double>(n);
  const size_t bytes = (size_t)2 * n * P * (fp32 ? 8 : 16);
  return P >= 1 && bytes <= 65536;
}

bool launch_precond(const Geo& g, const double* v, double* w, void* spec, bool fp32, int spatial,
                    const PrecondTables& tb, const double* vscale, int vs_stride, int accum,
                    hipStream_t st) {
  if (fp32) {
    cx<float>* s = reinterpret_cast<cx<float>*>(spec);
    time_fwd<float>(g, v, s, tb, vscale, vs_stride, st);
    bool ok = (spatial == 0) ? dst_solve<float>(g, s, tb, st) : launch_mg_solve(g, spec, true, tb, st);
    if (!ok) return false;
    time_inv<float>(g, s, w, tb, accum, st);
  } else {
    cx<double>* s = reinterpret_cast<cx<double>*>(spec);
    time_fwd<double>(g, v, s, tb, vscale, vs_stride, st);
    bool ok = (spatial == 0) ? dst_solve<double>(g, s, tb, st) : launch_mg_solve(g, spec, false, tb, st);
    if (!ok) return false;
    time_inv<double>(g, s, w, tb, accum, st);
  }
  return true;
}

}  // namespace pcop
