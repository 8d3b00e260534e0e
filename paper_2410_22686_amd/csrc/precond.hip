// The epsilon-circulant RBD preconditioner w = P_eps^{-1} v (Section 2.1):
//   step 1  time pass: scale by D_eps, FFT along time, split the packed
//           spectrum into the two Hermitian block spectra
//   step 2  shifted spatial solves: sine transforms for a = 1 (dst.hip) or
//           one multigrid V-cycle (multigrid.hip)
//   step 3+4 inverse time pass: inverse FFT, undo D_eps, combine
//           w_1 = z_1 - z_2, w_2 = z_1 + z_2
//
// Both blocks ride in one complex FFT per spatial point:
//   c_j = eps^{j/n} v_2^j + i eps^{-j/n} v_1^j,   c_hat = FFT_n(c),
//   V2_k = (c_hat_k + conj c_hat_{-k})/2,  V1_k = (c_hat_k - conj c_hat_{-k})/(2i),
// and only k = 0..n/2 is kept (the spectra are Hermitian).  Block 2 is solved
// with the shift lambda_k + alpha, block 1 with conj(lambda_k) + alpha
// (eq. decomposition_eps; C_eps^T = D F conj(Lambda) F^* D^{-1}).  The
// spectrum buffer is laid out [batch][2K][m], slice q = 2k + s with s = 0
// for V2 and s = 1 for V1, K = n/2 + 1.
#include <algorithm>

#include "common.hpp"
#include "fft_lds.hpp"
#include "launch.hpp"
#include "time_common.hpp"

namespace pcop {

// ---------------------------------------------------------------------------
// launchers; the time-pass kernels are in time_sk.hip (two LDS buffers),
// time_ip_*.hip (one in-place buffer), time_cz.hip (chirp-z in three LDS
// stages) and time_bl.hip (chirp-z with two LDS FFTs)
// ---------------------------------------------------------------------------
// points per block of the two-buffer time kernels: the largest power of two
// in 4..want whose two [n][P] buffers fit 64 KiB and whose whole LDS (with
// the tables) fits 80 KiB (two blocks per CU), else 0.  With wide = true,
// 16 points may also use the wide kernels (512 threads, buffers up to
// 128 KiB, one block per CU).
static int time_cols_sk(int n, int csz, int want, bool wide = false) {
  if (wide && want >= 16 && (size_t)2 * n * 16 * csz <= 131072 && sk_lds_bytes(n, 16, csz) <= 160 * 1024 - 1024)
    return 16;
  for (int P = want; P >= 4; P /= 2)
    if ((size_t)2 * n * P * csz <= 65536 && sk_lds_bytes(n, P, csz) <= 81920) return P;
  return 0;
}


// points per block of the in-place time kernels: the largest power of two in
// 4..want that fits 64 KiB with every stage within the supported butterflies
// per thread, else 0
static int time_cols_ip(const FftPlan& pl, int n, int csz, int want) {
  for (int P = want; P >= 4; P /= 2) {
    if ((size_t)n * P * csz > 65536) continue;
    bool ok = true;
    for (int s = 0; s < pl.nrad; ++s) {
      const int mb = ip_mb(n, pl.rad[s], P, 256);
      if (mb == 0 || (pl.rad[s] >= 11 && mb > 2)) ok = false;
    }
    if (ok) return P;
  }
  return 0;
}

// Stockham time kernels for the request req (pcop_options::time_cols):
// -P two buffers with P points per block, +P in place, 0 when none fits.
// Automatic (0) and two-buffer requests fall back to in place when the two
// buffers do not fit, and in-place requests fall back to two buffers.
static int time_block(const FftPlan& pl, int n, int csz, int req) {
  // the Stockham kernels exist for 4, 8 and 16 points: +-32 asks for +-16
  req = std::max(-16, std::min(16, req));
  if (req <= 0) {
    // an explicit -16 admits the wide kernels
    const int P = time_cols_sk(n, csz, req < -1 ? -req : 16, req == -16);
    if (P > 0) return -P;
    return time_cols_ip(pl, n, csz, 16);
  }
  const int P = time_cols_ip(pl, n, csz, req);
  if (P > 0) return P;
  return -time_cols_sk(n, csz, 16);
}

static FftPlan chirp_plan(int n) {
  FftPlan pl{};
  pl.bluestein = 1;
  pl.M = 1;
  while (pl.M < 2 * n - 1) pl.M *= 2;
  pl.nrad = 0;
  return pl;
}

// radix plan of length n (radices 2..17), or the chirp-z plan when n has a
// prime factor above 17
static FftPlan radix_plan(int n) {
  FftPlan pl{};
  int r = n;
  int big = 0;
  for (int f = 2; f * f <= r; ++f)
    while (r % f == 0) {
      if (f > 17) big = 1;
      r /= f;
    }
  if (r > 17) big = 1;
  if (big) return chirp_plan(n);
  r = n;
  while (r % 8 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 8; r /= 8; }
  while (r % 4 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 4; r /= 4; }
  while (r % 2 == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = 2; r /= 2; }
  for (int f = 3; f <= 17 && pl.nrad < 16; f += 2)
    while (r % f == 0 && pl.nrad < 16) { pl.rad[pl.nrad++] = f; r /= f; }
  if (pl.nrad == 0) pl.rad[pl.nrad++] = 1;  // n = 1
  return pl;
}

// The time plan: the radix plan when a Stockham kernel holds its tiles in
// LDS, else the chirp-z transform (lengths with a prime factor above 17, and
// long smooth lengths whose tiles exceed LDS: FP64 n > 1024 among others)
FftPlan make_time_plan(int n, bool fp32) {
  const FftPlan pl = radix_plan(n);
  if (pl.bluestein || time_block(pl, n, fp32 ? 8 : 16, 0) != 0) return pl;
  return chirp_plan(n);
}

bool time_lds_fits(int n, bool fp32) {
  const FftPlan pl = make_time_plan(n, fp32);
  const int csz = fp32 ? 8 : 16;
  return pl.bluestein ? bl_choice(pl.M, n, csz, 0) != 0 : time_block(pl, n, csz, 0) != 0;
}

int time_choice(const Geo& g, const PrecondTables& tb, bool fp32) {
  // the prime-factor kernels, requested explicitly, for any length that has a plan
  if ((tb.time_cols == 64 || tb.time_cols == -64) && pr_exists(g.n, fp32 ? 8 : 16, tb.time_cols))
    return tb.time_cols;
  if (tb.plan.bluestein) return bl_choice(tb.plan.M, g.n, fp32 ? 8 : 16, tb.time_cols);
  return time_block(tb.plan, g.n, fp32 ? 8 : 16, tb.time_cols);
}

template <class T>
static bool time_pass(bool fwd, const Geo& g, const double* v, cx<T>* spec, double* w, const PrecondTables& tb,
                      const double* vscale, int vs_stride, int accum, hipStream_t st) {
  const bool f32 = sizeof(T) == 4;
  TimeTables tt{f32 ? (const void*)tb.twn32 : (const void*)tb.twn64, f32 ? (const void*)tb.twM32 : (const void*)tb.twM64,
                f32 ? (const void*)tb.chirp32 : (const void*)tb.chirp64, f32 ? (const void*)tb.bhat32 : (const void*)tb.bhat64};
  const int csz = (int)sizeof(cx<T>);
  if ((tb.time_cols == 64 || tb.time_cols == -64) && pr_exists(g.n, csz, tb.time_cols))
    return launch_time_pr<T>(fwd, tb.time_cols, g, v, spec, w, tb, vscale, vs_stride, accum, st);
  if (tb.plan.bluestein) {
    const int c = bl_choice(tb.plan.M, g.n, csz, tb.time_cols);
    if (c == 64 || c == -64) return launch_time_pr<T>(fwd, c, g, v, spec, w, tb, vscale, vs_stride, accum, st);
    if (c == 32 || c == -32) return launch_time_cz<T>(fwd, c, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
    return c != 0 && launch_time_bl<T>(fwd, c, g, v, spec, w, tb, tt, vscale, vs_stride, accum, st);
  }
  const cx<T>* twn = reinterpret_cast<const cx<T>*>(tt.twn);
  const int c = time_block(tb.plan, g.n, csz, tb.time_cols);
  if (c > 0) {
    if (fwd) launch_time_ip_dir<T, true>(c, g, v, spec, w, tb, twn, vscale, vs_stride, accum, st);
    else launch_time_ip_dir<T, false>(c, g, v, spec, w, tb, twn, vscale, vs_stride, accum, st);
    return true;
  }
  if (c == 0) return false;
  launch_time_sk<T>(fwd, -c, g, v, spec, w, tb, twn, vscale, vs_stride, accum, st);
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
    bool ok = (spatial == 0) ? launch_dst_solve(g, spec, true, tb, 2 * g.K, tb.lam, st)
                              : launch_mg_solve(g, spec, true, tb, 2 * g.K, tb.lam, st);
    if (!ok) return false;
    if (!time_inv<float>(g, s, w, tb, accum, st)) return false;
  } else {
    cx<double>* s = reinterpret_cast<cx<double>*>(spec);
    if (!time_fwd<double>(g, v, s, tb, vscale, vs_stride, st)) return false;
    bool ok = (spatial == 0) ? launch_dst_solve(g, spec, false, tb, 2 * g.K, tb.lam, st)
                              : launch_mg_solve(g, spec, false, tb, 2 * g.K, tb.lam, st);
    if (!ok) return false;
    if (!time_inv<double>(g, s, w, tb, accum, st)) return false;
  }
  return true;
}

}  // namespace pcop
