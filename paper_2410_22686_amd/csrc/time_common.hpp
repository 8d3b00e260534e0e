// Shared pieces of the time passes (steps 1 and 3-4 of the preconditioner).
#pragma once

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

// c_j = s (d_j v2_j + i v1_j / d_j) at time level j, spatial point i (the
// factors s d_j and s / d_j are formed first, as in every time kernel)
template <class T>
__device__ __forceinline__ cx<T> pack_input(const double* v1, const double* v2, const double* dpow, double s,
                                            int j, int i, int m) {
  if (i >= m) return cx<T>{0, 0};
  const double d = dpow[j];
  const size_t o = (size_t)j * m + i;
  return cx<T>{(T)(s * d * v2[o]), (T)(s * (1.0 / d) * v1[o])};
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
// (factors 1/(n d_j) and d_j/n formed first, as in every time kernel)
__device__ __forceinline__ void combine_store(double* w1, double* w2, const double* dpow, int n, int m, int j,
                                              int i, double ex, double ey, int accum) {
  const double d = dpow[j];
  const double z2 = ex * (1.0 / ((double)n * d));
  const double z1 = ey * (d / (double)n);
  const size_t o = (size_t)j * m + i;
  if (accum) {
    w1[o] += z1 - z2;
    w2[o] += z1 + z2;
  } else {
    w1[o] = z1 - z2;
    w2[o] = z1 + z2;
  }
}


// per-variant launchers (one translation unit each)
template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st);
template <class T, bool FWD>
void launch_time_ip_dir(int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                        const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st);
template <class T>
bool launch_time_bl(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st);
// chirp-z tiles are static LDS; up to 80 KiB keeps two blocks per CU
constexpr size_t kBlueLds = 81920;
// dynamic LDS of the two-buffer kernels: two [n][P] buffers, the n twiddles
// and two tables of n scale factors (D_eps powers and their inverses)
inline size_t sk_lds_bytes(int n, int P, size_t csz) { return (2 * (size_t)P + 1) * n * csz + 16 * (size_t)n; }

}  // namespace pcop
