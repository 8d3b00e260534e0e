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
// directly.  Bluestein mode (n has a prime factor > 17, or no Stockham tile
// fits LDS): a length-M power-of-two convolution in one in-place [P][M+1]
// LDS buffer,
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

// unpack_store with the tile shape fixed at compile time (KP = K P items over
// NT threads) and every store unconditional: an item past the tile's last
// column (or past KP) is replaced by the tile's last valid one and stores the
// same value to the same place.  With no store behind a branch, the wait for
// the next tile's prefetched loads need not wait for this tile's stores.
template <class T, int NT, int K, int P, class GET>
__device__ __forceinline__ void unpack_store_u(cx<T>* out, int n, int i0, int m, int lane, GET get) {
  constexpr int KP = K * P, Q = (KP + NT - 1) / NT;
  const int pmax = (m - i0 < P ? m - i0 : P) - 1;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int t = lane + q * NT;
    if (KP % NT != 0 && t >= KP) t = KP - 1;
    const int k = t / P;
    int p = t - k * P;
    if (p > pmax) p = pmax;
    const int i = i0 + p;
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


// Column tiles of the persistent time kernels: tile t covers member
// t / tiles_per_member and spatial points i0 .. i0 + P - 1 with
// i0 = (t mod tiles_per_member) P.
struct TileWalk {
  int tpm;     // tiles per member
  int ntiles;  // B * tpm
  const int* active;
  // first tile at or after t (stepping by stride) whose member is active.
  // t is uniform over the block and the flags do not change during a launch,
  // so they are read through the constant address space (scalar loads): a
  // vector load here would make the wave wait for every store it has in flight
  __device__ __forceinline__ int next(int t, int stride) const {
    if (!active) return t;
    const __attribute__((address_space(4))) int* a = (const __attribute__((address_space(4))) int*)active;
    while (t < ntiles && !a[t / tpm]) t += stride;
    return t;
  }
};

// per-variant launchers (one translation unit each)
template <class T>
void launch_time_sk(bool fwd, int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st);
template <class T, bool FWD>
void launch_time_ip_dir(int P, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                        const cx<T>* twn, const double* vscale, int vs_stride, int accum, hipStream_t st);
template <class T>
bool launch_time_bl(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st);
// chirp-z with the convolution in three LDS stages (time_cz.hip), for
// M <= 1024: c = 32 (256 threads) or -32 (512 threads)
template <class T>
bool launch_time_cz(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const TimeTables& tt, const double* vscale, int vs_stride, int accum, hipStream_t st);
bool cz_exists(int M, int csz, int c);
int cz_auto(int M, int csz);
// prime-factor kernels (time_pr.hip) for n = N1 PR with a Rader transform of
// the prime PR (n = 127, 255, 511): c = 64 (the plan's narrow tile, 256
// threads) or -64 (its wide tile, 512 threads); pr_auto is the automatic
// choice among them (0: none)
template <class T>
bool launch_time_pr(bool fwd, int c, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                    const double* vscale, int vs_stride, int accum, hipStream_t st);
bool pr_exists(int n, int csz, int c);
int pr_auto(int n, int csz);
// chirp-z kernels for the request req (pcop_options::time_cols): +-32 the
// three-stage kernels with 256 / 512 threads; +P for P points per block of
// the two-FFT kernels with 256 threads, -P with 512 threads; 0 when no shape
// fits.  0 and -1 pick automatically (the three-stage kernels where they
// exist); an explicit request is honoured with at most that many points,
// else the automatic choice is used.
int bl_choice(int M, int n, int csz, int req);

// Chirp-z tile shapes (M = convolution length, P points per block, NT
// threads) that exist as kernels: one [P][M+1] buffer of at most 160 KiB,
// M P <= 8192 (with n <= M/2 at most 16 prefetch slots per thread, and no
// register spills), fewer than 4 points only for M >= 1024, and 512 threads
// only for large tiles.
constexpr size_t kLdsMax = 160 * 1024;
constexpr bool bl_shape_ok(int M, int P, int NT, int csz) {
  return M >= 64 && M <= 4096 && (NT == 256 || NT == 512) && M * P <= 8192 &&
         (size_t)(M + 1) * P * csz <= kLdsMax && (P >= 4 || M >= 1024) &&
         (NT == 256 || (P >= 4 && M * P >= 4096));
}
// The tables (twiddles, filter spectrum, chirp, D_eps factors) go to LDS too
// when they fit beside the buffer for every n <= M/2: 8M bytes of twiddles
// (FP64 stages read only the first half), the M/2 + 1 distinct filter
// values (the filter is even), n chirp values and two tables of n doubles.
constexpr bool bl_tables_in_lds(int M, int P, int csz) {
  return (size_t)(M + 1) * P * csz + 8 * (size_t)M + (size_t)(M / 2 + 1) * csz + (size_t)(M / 2) * (csz + 16) <=
         kLdsMax;
}
inline size_t bl_lds_bytes(int M, int P, int n, int csz) {
  size_t b = (size_t)(M + 1) * P * csz;
  if (bl_tables_in_lds(M, P, csz)) b += 8 * (size_t)M + (size_t)(M / 2 + 1) * csz + (size_t)n * (csz + 16);
  return b;
}
// dynamic LDS of the two-buffer kernels: two [n][P] buffers, the n twiddles
// and two tables of n scale factors (D_eps powers and their inverses)
inline size_t sk_lds_bytes(int n, int P, size_t csz) { return (2 * (size_t)P + 1) * n * csz + 16 * (size_t)n; }

}  // namespace pcop
