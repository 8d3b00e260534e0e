// Arnoldi kernels for GMRES in FP64: fused multi-dot, fused multi-AXPY that
// also measures the updated vector, linear combinations of basis vectors, and
// the per-member Gram-Schmidt bookkeeping.  Reductions are two-level
// (wavefront butterfly + fixed-order block/partial sums), so results are
// bitwise reproducible for a fixed launch shape.
//
// Basis vectors are stored unnormalised: the Arnoldi vector v_i equals
// sc[b][i] * basis_i, which lets the normalisation ride along in the
// coefficients instead of costing a pass over the vector.
#include <array>
#include <utility>

#include "common.hpp"
#include "launch.hpp"

namespace pcop {

constexpr int kNT = 256;
constexpr int kNWave = kNT / kWave;

int krylov_blocks(long long vl) {
  long long want = (vl / 2 + kNT * 4 - 1) / (kNT * 4);
  if (want < 1) want = 1;
  if (want > 1024) want = 1024;
  return (int)want;
}

// Basis vectors are streamed once per pass: their loads are nontemporal, so
// they do not displace the vector being updated (or other live data) from
// the caches.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  return double2{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}

// block-level reduction of NACC accumulators; thread c < ncols writes column c
template <int NACC>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NACC], int ncols, double* out) {
  __shared__ double red[kNWave][NACC];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < NACC; ++c) {
    if (c < ncols) {
      double s = wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = s;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += kNT) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kNWave; ++k) s += red[k][c];
    out[c] = s;
  }
}

// Vectors are read as double2 (the length 2 n m of a member vector is even
// and every base address is 16-byte aligned).  NV (the number of basis
// vectors) is a compile-time constant: every load is issued without a guard.
template <int NV>
__global__ void __launch_bounds__(kNT) mdot_kernel(KrylovArgs ka, const double* __restrict__ w,
                                                   double* __restrict__ partial, int nblk) {
  const int b = blockIdx.y;
  if (ka.active && !ka.active[b]) return;
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  const double2* wb = reinterpret_cast<const double2*>(w + (size_t)b * ka.ms);
  const double2* vb = reinterpret_cast<const double2*>(ka.basis + (size_t)b * ka.ms);
  const long long n2 = ka.vl / 2;
  const long long ss = ka.slot_stride / 2;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < n2; e += (long long)nblk * kNT) {
    const double2 wv = wb[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 v = ld_stream(&vb[(size_t)i * ss + e]);
      acc[i] += v.x * wv.x + v.y * wv.y;
    }
    acc[NV] += wv.x * wv.x + wv.y * wv.y;
  }
  // columns 0..NV-1: dots, column NV: the squared norm
  block_reduce_store<NV + 1>(acc, NV + 1, partial + ((size_t)b * nblk + blockIdx.x) * kRedStride);
}

// the update keeps the basis values of its element in registers for the
// second product, so it works on one double per thread and iteration
template <int NV>
__global__ void __launch_bounds__(kNT) update_kernel(KrylovArgs ka, double* __restrict__ w,
                                                     const double* __restrict__ coef, int coef_ld,
                                                     double* __restrict__ partial, int nblk,
                                                     const int* __restrict__ skip) {
  const int b = blockIdx.y;
  if (ka.active && !ka.active[b]) return;
  if (skip && skip[b]) return;
  __shared__ double c[NV > 0 ? NV : 1];
  for (int i = threadIdx.x; i < NV; i += kNT) c[i] = coef[(size_t)b * coef_ld + i];
  __syncthreads();
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  double* wb = w + (size_t)b * ka.ms;
  const double* vb = ka.basis + (size_t)b * ka.ms;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < ka.vl; e += (long long)nblk * kNT) {
    double v[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = ld_stream(&vb[(size_t)i * ka.slot_stride + e]);
    double wv = wb[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) wv -= c[i] * v[i];
    wb[e] = wv;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += v[i] * wv;
    acc[NV] += wv * wv;
  }
  block_reduce_store<NV + 1>(acc, NV + 1, partial + ((size_t)b * nblk + blockIdx.x) * kRedStride);
}

// the same update on double2 pairs (two elements per thread and step)
template <int MAXNV>
__global__ void __launch_bounds__(kNT) update2_kernel(KrylovArgs ka, int nv, double* __restrict__ w,
                                                      const double* __restrict__ coef, int coef_ld,
                                                      double* __restrict__ partial, int nblk,
                                                      const int* __restrict__ skip) {
  const int b = blockIdx.y;
  if (ka.active && !ka.active[b]) return;
  if (skip && skip[b]) return;
  __shared__ double c[MAXNV];
  for (int i = threadIdx.x; i < MAXNV; i += kNT) c[i] = (i < nv) ? coef[(size_t)b * coef_ld + i] : 0.0;
  __syncthreads();
  double acc[MAXNV + 1];
#pragma unroll
  for (int i = 0; i <= MAXNV; ++i) acc[i] = 0.0;
  double2* wb = reinterpret_cast<double2*>(w + (size_t)b * ka.ms);
  const double2* vb = reinterpret_cast<const double2*>(ka.basis + (size_t)b * ka.ms);
  const long long n2 = ka.vl / 2;
  const long long ss = ka.slot_stride / 2;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < n2; e += (long long)nblk * kNT) {
    double2 v[MAXNV];
#pragma unroll
    for (int i = 0; i < MAXNV; ++i) v[i] = (i < nv) ? ld_stream(&vb[(size_t)i * ss + e]) : double2{0.0, 0.0};
    double2 wv = wb[e];
#pragma unroll
    for (int i = 0; i < MAXNV; ++i)
      if (i < nv) {
        wv.x -= c[i] * v[i].x;
        wv.y -= c[i] * v[i].y;
      }
    wb[e] = wv;
#pragma unroll
    for (int i = 0; i < MAXNV; ++i)
      if (i < nv) acc[i] += v[i].x * wv.x + v[i].y * wv.y;
    acc[MAXNV] += wv.x * wv.x + wv.y * wv.y;
  }
  double out[MAXNV + 1];
#pragma unroll
  for (int i = 0; i <= MAXNV; ++i) out[i] = (i < nv) ? acc[i] : ((i == nv) ? acc[MAXNV] : 0.0);
  block_reduce_store<MAXNV + 1>(out, nv + 1, partial + ((size_t)b * nblk + blockIdx.x) * kRedStride);
}

template <int MAXNV>
__global__ void __launch_bounds__(kNT) combine_kernel(KrylovArgs ka, int nv, const double* __restrict__ coef,
                                                      int coef_ld, double* __restrict__ out, int accum) {
  const int b = blockIdx.y;
  if (ka.active && !ka.active[b]) return;
  __shared__ double c[MAXNV];
  for (int i = threadIdx.x; i < MAXNV; i += kNT) c[i] = (i < nv) ? coef[(size_t)b * coef_ld + i] : 0.0;
  __syncthreads();
  double2* ob = reinterpret_cast<double2*>(out + (size_t)b * ka.ms);
  const double2* vb = reinterpret_cast<const double2*>(ka.basis + (size_t)b * ka.ms);
  const long long n2 = ka.vl / 2;
  const long long ss = ka.slot_stride / 2;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < n2; e += (long long)gridDim.x * kNT) {
    double2 acc = accum ? ob[e] : double2{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < MAXNV; ++i)
      if (i < nv && c[i] != 0.0) {
        const double2 v = ld_stream(&vb[(size_t)i * ss + e]);
        acc.x += c[i] * v.x;
        acc.y += c[i] * v.y;
      }
    ob[e] = acc;
  }
}

// out[b][c] = sum over blocks of partial[b][blk][c]: wave w of the block owns
// the columns c = w, w + 4, ...; lane l adds blocks l, l + 64, ... in order and
// the wave butterfly finishes, so the order is fixed.
__global__ void __launch_bounds__(kNT) reduce_partials_kernel(const double* __restrict__ partial, int nblk,
                                                              int ncols, double* __restrict__ out) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const double* pb = partial + (size_t)b * nblk * kRedStride;
  for (int c = wv; c < ncols; c += kNWave) {
    double s = 0.0;
    for (int k = lane; k < nblk; k += kWave) s += pb[(size_t)k * kRedStride + c];
    s = wave_sum(s);
    if (lane == 0) out[(size_t)b * kRedStride + c] = s;
  }
}

// First Gram-Schmidt pass bookkeeping for Arnoldi step j:
//   h_i = sc_i <basis_i, w>,  H[b][j][i] = h_i,  coef_i = h_i sc_i,  wnorm2 = <w, w>.
__global__ void gs_step1_kernel(const double* __restrict__ red, int j, int B, const double* __restrict__ sc,
                                double* __restrict__ H, int H_ld, double* __restrict__ coef, int coef_ld,
                                double* __restrict__ wnorm2, const int* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (active && !active[b]) return;
  const double* r = red + (size_t)b * kRedStride;
  double* Hc = H + ((size_t)b * (kMaxBasis - 1) + j) * H_ld;
  for (int i = 0; i <= j; ++i) {
    const double s = sc[(size_t)b * kMaxBasis + i];
    const double h = s * r[i];
    Hc[i] = h;
    coef[(size_t)b * coef_ld + i] = h * s;
  }
  wnorm2[b] = r[j + 1];
}

// After an update pass: red holds <basis_i, w'> and <w', w'>.
// final_pass = 0: decide on a second pass (skip[b] = 0 means "run it"); the
//   coefficients of the correction are added to column j of H.
// final_pass = 1: for members that ran the second pass, record the norm.
// In both cases the sub-diagonal entry and the scale of the new basis vector
// are set from the measured norm.
__global__ void gs_step2_kernel(const double* __restrict__ red, int j, int B, const double* __restrict__ sc,
                                double* __restrict__ H, int H_ld, double* __restrict__ coef, int coef_ld,
                                const double* __restrict__ wnorm2, double reorth_tol, int* __restrict__ skip,
                                double* __restrict__ sc_out, const int* __restrict__ active, int final_pass) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (active && !active[b]) return;
  if (final_pass && skip[b]) return;
  const double* r = red + (size_t)b * kRedStride;
  double* Hc = H + ((size_t)b * (kMaxBasis - 1) + j) * H_ld;
  const double nrm2 = r[j + 1];
  if (!final_pass) {
    double c2 = 0.0;
    for (int i = 0; i <= j; ++i) {
      const double h2 = sc[(size_t)b * kMaxBasis + i] * r[i];
      c2 += h2 * h2;
    }
    const bool again = reorth_tol >= 0.0 && c2 > reorth_tol * reorth_tol * nrm2;
    skip[b] = again ? 0 : 1;
    if (again) {
      for (int i = 0; i <= j; ++i) {
        const double s = sc[(size_t)b * kMaxBasis + i];
        const double h2 = s * r[i];
        Hc[i] += h2;
        coef[(size_t)b * coef_ld + i] = h2 * s;
      }
    }
  }
  const double nrm = sqrt(nrm2 > 0.0 ? nrm2 : 0.0);
  Hc[j + 1] = nrm;
  sc_out[(size_t)b * kMaxBasis + j + 1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  (void)wnorm2;
}

// out[b][i] = H[b][j][i] for i <= j + 1 (the column the host reads back) and
// out[b][kMaxBasis] = skip[b] (1: no second Gram-Schmidt pass needed)
__global__ void pack_hcol_kernel(const double* __restrict__ H, int H_ld, int j, int B, const int* __restrict__ skip,
                                 double* __restrict__ out) {
  const int b = blockIdx.x;
  const double* Hc = H + ((size_t)b * (kMaxBasis - 1) + j) * H_ld;
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) out[(size_t)b * (kMaxBasis + 1) + i] = Hc[i];
  if (threadIdx.x == 0) out[(size_t)b * (kMaxBasis + 1) + kMaxBasis] = skip ? (double)skip[b] : 1.0;
  (void)B;
}

// sc[b][col] = 1/sqrt(red[b][0]),  norm[b] = sqrt(red[b][0])
__global__ void set_scale_kernel(const double* __restrict__ red, int col, int B, double* __restrict__ sc,
                                 double* __restrict__ norm, const int* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (active && !active[b]) return;
  const double n2 = red[(size_t)b * kRedStride];
  const double nr = sqrt(n2 > 0.0 ? n2 : 0.0);
  norm[b] = nr;
  sc[(size_t)b * kMaxBasis + col] = nr > 0.0 ? 1.0 / nr : 0.0;
}

// ---------------------------------------------------------------------------
#define PCOP_DISPATCH_NV(KERNEL, NV, GRID, ST, ...)                                   \
  do {                                                                                \
    if ((NV) <= 4) KERNEL<4><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);                      \
    else if ((NV) <= 8) KERNEL<8><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);                 \
    else if ((NV) <= 16) KERNEL<16><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);               \
    else if ((NV) <= 24) KERNEL<24><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);               \
    else if ((NV) <= 32) KERNEL<32><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);               \
    else KERNEL<kMaxBasis><<<GRID, kNT, 0, ST>>>(__VA_ARGS__);                        \
  } while (0)

// exact-size kernels for nv = 0 .. kMaxBasis - 1
using MdotFn = void (*)(KrylovArgs, const double*, double*, int);
using UpdateFn = void (*)(KrylovArgs, double*, const double*, int, double*, int, const int*);
template <int... I>
constexpr std::array<MdotFn, sizeof...(I)> mdot_table(std::integer_sequence<int, I...>) {
  return {&mdot_kernel<I>...};
}
template <int... I>
constexpr std::array<UpdateFn, sizeof...(I)> update_table(std::integer_sequence<int, I...>) {
  return {&update_kernel<I>...};
}
static const auto kMdot = mdot_table(std::make_integer_sequence<int, kMaxBasis>{});
static const auto kUpdate = update_table(std::make_integer_sequence<int, kMaxBasis>{});

void launch_mdot(const KrylovArgs& ka, int nv, const double* w, double* partial, int nblk, hipStream_t st) {
  dim3 grid(nblk, ka.B);
  if (nv < 0 || nv >= kMaxBasis) return;
  kMdot[nv]<<<grid, kNT, 0, st>>>(ka, w, partial, nblk);
}

void launch_update(const KrylovArgs& ka, int nv, double* w, const double* coef, int coef_ld, double* partial,
                   int nblk, const int* skip, hipStream_t st) {
  dim3 grid(nblk, ka.B);
  if (ka.pairs) {
    PCOP_DISPATCH_NV(update2_kernel, nv, grid, st, ka, nv, w, coef, coef_ld, partial, nblk, skip);
  } else if (nv >= 0 && nv < kMaxBasis) {
    kUpdate[nv]<<<grid, kNT, 0, st>>>(ka, w, coef, coef_ld, partial, nblk, skip);
  }
}

void launch_combine(const KrylovArgs& ka, int nv, const double* coef, int coef_ld, double* out, int accum,
                    hipStream_t st) {
  dim3 grid(krylov_blocks(ka.vl), ka.B);
  PCOP_DISPATCH_NV(combine_kernel, nv, grid, st, ka, nv, coef, coef_ld, out, accum);
}

void launch_reduce_partials(const double* partial, int nblk, int ncols, int B, double* out, hipStream_t st) {
  reduce_partials_kernel<<<B, kNT, 0, st>>>(partial, nblk, ncols, out);
}

void launch_gs_step1(const double* red, int j, int B, const double* sc, double* H, int H_ld, double* coef,
                     int coef_ld, double* wnorm2, const int* active, hipStream_t st) {
  gs_step1_kernel<<<(B + 63) / 64, 64, 0, st>>>(red, j, B, sc, H, H_ld, coef, coef_ld, wnorm2, active);
}

void launch_gs_step2(const double* red, int j, int B, const double* sc, double* H, int H_ld, double* coef,
                     int coef_ld, const double* wnorm2, double reorth_tol, int* skip, double* sc_out,
                     const int* active, int final_pass, hipStream_t st) {
  gs_step2_kernel<<<(B + 63) / 64, 64, 0, st>>>(red, j, B, sc, H, H_ld, coef, coef_ld, wnorm2, reorth_tol, skip,
                                                sc_out, active, final_pass);
}

void launch_pack_hcol(const double* H, int H_ld, int j, int B, const int* skip, double* out, hipStream_t st) {
  pack_hcol_kernel<<<B, 64, 0, st>>>(H, H_ld, j, B, skip, out);
}

void launch_set_scale(const double* red, int col, int B, double* sc, double* norm, const int* active,
                      hipStream_t st) {
  set_scale_kernel<<<(B + 63) / 64, 64, 0, st>>>(red, col, B, sc, norm, active);
}

}  // namespace pcop
