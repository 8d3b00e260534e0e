// Step 2 with a variable coefficient: one geometric-multigrid V-cycle per
// frequency slice for (sigma_q I + tau K_a) z = r (Section 2.1 step 2;
// Section 3, Example 2: one V-cycle, Gauss-Seidel pre-smoother, no
// post-smoother).  All slices of all members go through one launch per level.
//
// Cycle (from z = 0; the lexicographic smoothers of mg_smoother = 1, 2 are
// described at their kernels):
//   smooth    one red-black Gauss-Seidel sweep, red = even index sum first.
//             Red points: z = r / d; black points use the red values
//             z_nb = r_nb / d_nb, recomputed on the fly, so the sweep is one
//             pass.  d = sigma_q + tau diag(K_a).
//   restrict  residual r - A z (zero at black points after the sweep, equal
//             to -sum_nb off z_nb at red points), written over the consumed
//             right-hand side, then full weighting to the coarse grid
//             (tensor product of [1/4, 1/2, 1/4]).
//   coarsest  one point: z = r / d.
//   prolong   z += P z_coarse (multilinear interpolation); the finest level
//             writes the result into the spectrum.
// Coarse operators are re-discretised: tau K_a on each level comes from the
// host with a at the level's face midpoints.  Coefficients per level:
// coef[0][i] = tau diag, coef[1 + 2a][i] / coef[2 + 2a][i] = tau times the
// minus / plus neighbour along axis a (zero where the neighbour is outside).
#include "common.hpp"
#include "launch.hpp"

namespace pcop {

struct MgShift {
  const double* lam;    // [K] (re, im)
  const double* alpha;  // [B]
  const int* active;    // [B] or null
  int twoK;             // slices per member
};

template <class T>
__device__ __forceinline__ cx<T> slice_sigma(const MgShift& sh, int slice) {
  const int b = slice / sh.twoK;
  const int q = slice - b * sh.twoK;
  const int k = q >> 1;
  const double re = sh.lam[2 * k] + sh.alpha[b];
  const double im = (q & 1) ? -sh.lam[2 * k + 1] : sh.lam[2 * k + 1];
  return cx<T>{(T)re, (T)im};
}

// (point chunk, slice group) of this block in XCD-friendly order: the blocks
// one XCD runs take consecutive point chunks of a slice group, so the
// neighbour planes a block reads were brought into that XCD's L2 by the
// blocks next to it
__device__ __forceinline__ int2 mg_block() {
  const int lg = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  return make_int2(lg % gridDim.x, lg / gridDim.x);
}

__device__ __forceinline__ void coords(int i, int nx, int dim, int* c) {
  c[0] = i % nx;
  c[1] = (i / nx) % nx;
  c[2] = (dim == 3) ? i / (nx * nx) : 0;
}

// one red-black sweep from z = 0.  A thread owns one point for SB
// consecutive slices: the point's stencil coefficients (and its neighbours'
// diagonals) are loaded once for all of them, since the coefficient arrays
// are shared by every slice and do not stay in the L2.
template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_smooth_kernel(int nx, int m, int slices, const T* __restrict__ coef,
                                                        const cx<T>* __restrict__ r, cx<T>* __restrict__ z,
                                                        MgShift sh) {
  const int2 bk = mg_block();
  const int i = bk.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int c[3];
  coords(i, nx, DIM, c);
  const bool red = ((c[0] + c[1] + c[2]) & 1) == 0;
  const T cdg = coef[i];
  // neighbour n = 2a (minus) / 2a + 1 (plus): offset, its diagonal, the
  // coupling weight; absent neighbours are skipped
  int nbo[2 * DIM];
  bool has[2 * DIM];
  T nbd[2 * DIM], off[2 * DIM];
  {
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      has[2 * a] = !red && c[a] > 0;
      has[2 * a + 1] = !red && c[a] < nx - 1;
      nbo[2 * a] = -stride;
      nbo[2 * a + 1] = stride;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int n = 2 * a + u;
        nbd[n] = has[n] ? coef[i + nbo[n]] : (T)0;
        off[n] = has[n] ? coef[(size_t)(1 + n) * m + i] : (T)0;
      }
      stride *= nx;
    }
  }
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T> sig = slice_sigma<T>(sh, s);
    const cx<T>* rs = r + (size_t)s * m;
    const cx<T> di = cx<T>{sig.x + cdg, sig.y};
    cx<T> acc = rs[i];
#pragma unroll
    for (int n = 0; n < 2 * DIM; ++n) {
      if (has[n]) {
        const cx<T> dn = cx<T>{sig.x + nbd[n], sig.y};
        acc = acc - scale(cdiv(rs[i + nbo[n]], dn), off[n]);
      }
    }
    z[(size_t)s * m + i] = cdiv(acc, di);
  }
}

// fine residual after the sweep, written at red points only (it is zero at
// black points); res may alias the level's right-hand side, which the sweep
// has consumed.  SB slices per thread, the coupling weights loaded once.
template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_residual_kernel(int nx, int m, int slices, const T* __restrict__ coef,
                                                          const cx<T>* __restrict__ z, cx<T>* res, MgShift sh) {
  const int2 bk = mg_block();
  const int i = bk.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int f[3];
  coords(i, nx, DIM, f);
  if (((f[0] + f[1] + f[2]) & 1) != 0) return;
  int nbo[2 * DIM];
  bool has[2 * DIM];
  T off[2 * DIM];
  {
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      has[2 * a] = f[a] > 0;
      has[2 * a + 1] = f[a] < nx - 1;
      nbo[2 * a] = -stride;
      nbo[2 * a + 1] = stride;
      off[2 * a] = has[2 * a] ? coef[(size_t)(1 + 2 * a) * m + i] : (T)0;
      off[2 * a + 1] = has[2 * a + 1] ? coef[(size_t)(2 + 2 * a) * m + i] : (T)0;
      stride *= nx;
    }
  }
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T>* zs = z + (size_t)s * m;
    // r - A z at a red point after the sweep: -sum over the neighbours of off z_nb
    // (minus then plus neighbour, axis by axis)
    cx<T> acc{0, 0};
#pragma unroll
    for (int n = 0; n < 2 * DIM; ++n)
      if (has[n]) acc = acc - scale(zs[i + nbo[n]], off[n]);
    res[(size_t)s * m + i] = acc;
  }
}

// The same sweep with a thread on a pair of neighbouring points of one
// x-row, x = 2u and 2u + 1 (the last pair of a row of odd length holds one
// point): one red and one black point, so every lane does the same work
// (with one point per thread the red half of each wave idles while the
// black half divides by its neighbours' diagonals).  The pairs of a row
// share the row's colour order.  Taken in FP32, where it was measured
// faster (3-D nx = 63, 128 slices, per V-cycle over all levels: smoother
// 0.295 -> 0.281 ms, residual and restriction 0.312 -> 0.279 ms); in FP64
// the per-point kernels above were faster (smoother 0.46 against 0.52 ms),
// the pair kernels' loads then touching every other 16-byte slot.
__device__ __forceinline__ int mg_pairs(int nx, int m) { return m / nx * ((nx + 1) >> 1); }

struct MgPair {
  int ir, ib;        // the pair's red and black point
  bool hr, hb;       // whether the pair holds them
};

template <int DIM>
__device__ __forceinline__ MgPair mg_pair(int u, int nx, int* cb) {
  const int P = (nx + 1) >> 1;
  const int row = u / P, pu = u - row * P;
  const int y = row % nx, zz = DIM == 3 ? row / nx : 0;
  const int x0 = 2 * pu;
  const bool two = x0 + 1 < nx;
  const bool first_red = ((x0 + y + zz) & 1) == 0;
  MgPair p;
  p.ir = row * nx + x0 + (first_red ? 0 : 1);
  p.ib = row * nx + x0 + (first_red ? 1 : 0);
  p.hr = first_red || two;
  p.hb = !first_red || two;
  // coordinates of the black point
  cb[0] = x0 + (first_red ? 1 : 0);
  cb[1] = y;
  cb[2] = zz;
  return p;
}

template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_smooth_pair_kernel(int nx, int m, int slices, const T* __restrict__ coef,
                                                        const cx<T>* __restrict__ r, cx<T>* __restrict__ z,
                                                        MgShift sh) {
  const int2 bk = mg_block();
  const int u = bk.x * blockDim.x + threadIdx.x;
  if (u >= mg_pairs(nx, m)) return;
  int c[3];
  const MgPair pp = mg_pair<DIM>(u, nx, c);
  // red: z = r / d; black: the neighbours (all red) at their z = r / d
  const int ir = pp.hr ? pp.ir : pp.ib, ib = pp.hb ? pp.ib : pp.ir;  // in-range stand-ins
  const T cdr = coef[ir], cdb = coef[ib];
  // neighbour n = 2a (minus) / 2a + 1 (plus) of the black point: offset,
  // its diagonal, the coupling weight; absent neighbours are skipped
  int nbo[2 * DIM];
  bool has[2 * DIM];
  T nbd[2 * DIM], off[2 * DIM];
  {
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      has[2 * a] = pp.hb && c[a] > 0;
      has[2 * a + 1] = pp.hb && c[a] < nx - 1;
      nbo[2 * a] = -stride;
      nbo[2 * a + 1] = stride;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int n = 2 * a + v;
        nbd[n] = has[n] ? coef[ib + nbo[n]] : (T)0;
        off[n] = has[n] ? coef[(size_t)(1 + n) * m + ib] : (T)0;
      }
      stride *= nx;
    }
  }
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T> sig = slice_sigma<T>(sh, s);
    const cx<T>* rs = r + (size_t)s * m;
    cx<T>* zs = z + (size_t)s * m;
    if (pp.hr) zs[ir] = cdiv(rs[ir], cx<T>{sig.x + cdr, sig.y});
    if (pp.hb) {
      cx<T> acc = rs[ib];
#pragma unroll
      for (int n = 0; n < 2 * DIM; ++n) {
        if (has[n]) {
          const cx<T> dn = cx<T>{sig.x + nbd[n], sig.y};
          acc = acc - scale(cdiv(rs[ib + nbo[n]], dn), off[n]);
        }
      }
      zs[ib] = cdiv(acc, cx<T>{sig.x + cdb, sig.y});
    }
  }
}

// the residual at the red point of one pair (mg_pair) per thread, so that no
// lane idles at a black point (FP32; see the pair smoother)
template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_residual_pair_kernel(int nx, int m, int slices, const T* __restrict__ coef,
                                                          const cx<T>* __restrict__ z, cx<T>* res, MgShift sh) {
  const int2 bk = mg_block();
  const int u = bk.x * blockDim.x + threadIdx.x;
  if (u >= mg_pairs(nx, m)) return;
  int cbk[3];
  const MgPair pp = mg_pair<DIM>(u, nx, cbk);
  if (!pp.hr) return;
  const int i = pp.ir;
  int f[3];
  coords(i, nx, DIM, f);
  int nbo[2 * DIM];
  bool has[2 * DIM];
  T off[2 * DIM];
  {
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      has[2 * a] = f[a] > 0;
      has[2 * a + 1] = f[a] < nx - 1;
      nbo[2 * a] = -stride;
      nbo[2 * a + 1] = stride;
      off[2 * a] = has[2 * a] ? coef[(size_t)(1 + 2 * a) * m + i] : (T)0;
      off[2 * a + 1] = has[2 * a + 1] ? coef[(size_t)(2 + 2 * a) * m + i] : (T)0;
      stride *= nx;
    }
  }
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T>* zs = z + (size_t)s * m;
    // r - A z at a red point after the sweep: -sum over the neighbours of off z_nb
    // (minus then plus neighbour, axis by axis)
    cx<T> acc{0, 0};
#pragma unroll
    for (int n = 0; n < 2 * DIM; ++n)
      if (has[n]) acc = acc - scale(zs[i + nbo[n]], off[n]);
    res[(size_t)s * m + i] = acc;
  }
}

// coarse right-hand side by full weighting of the fine residual (red points
// only after a red-black sweep, where the black ones are zero; ALL: every
// point, after the lexicographic sweeps)
template <class T, int DIM, bool ALL>
__global__ void __launch_bounds__(256) mg_restrict_kernel(int nxf, int mf, int nxc, int mc,
                                                          const cx<T>* __restrict__ res, cx<T>* __restrict__ rc,
                                                          MgShift sh) {
  const int2 bk = mg_block();
  const int s = bk.y;
  if (sh.active && !sh.active[s / sh.twoK]) return;
  const int I = bk.x * blockDim.x + threadIdx.x;
  if (I >= mc) return;
  int C[3];
  coords(I, nxc, DIM, C);
  const cx<T>* rs = res + (size_t)s * mf;
  cx<T> acc{0, 0};
  const int o2 = (DIM == 3) ? 1 : 0;
  for (int d2 = -o2; d2 <= o2; ++d2)
    for (int d1 = -1; d1 <= 1; ++d1)
      for (int d0 = -1; d0 <= 1; ++d0) {
        const int f0 = 2 * C[0] + 1 + d0, f1 = 2 * C[1] + 1 + d1, f2 = (DIM == 3) ? 2 * C[2] + 1 + d2 : 0;
        if (!ALL && ((f0 + f1 + f2) & 1) != 0) continue;
        const T w = (d0 == 0 ? (T)1 : (T)0.5) * (d1 == 0 ? (T)1 : (T)0.5) * (d2 == 0 ? (T)1 : (T)0.5);
        acc = acc + scale(rs[f0 + nxf * (f1 + nxf * f2)], w);
      }
  const T inv = (DIM == 3) ? (T)0.125 : (T)0.25;
  rc[(size_t)s * mc + I] = scale(acc, inv);
}

// out = z_fine + P z_coarse (out may alias z_fine).  A thread owns one fine
// point for SB consecutive slices: its coarse indices and weights are formed
// once for all of them.
template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_prolong_kernel(int nxf, int mf, int nxc, int mc, int slices,
                                                         const cx<T>* __restrict__ zf, const cx<T>* __restrict__ zc,
                                                         cx<T>* out, MgShift sh) {
  const int2 bk = mg_block();
  const int i = bk.x * blockDim.x + threadIdx.x;
  if (i >= mf) return;
  int f[3];
  coords(i, nxf, DIM, f);
  // per axis two coarse candidates, clamped in bounds, with weights that are
  // zero where a candidate does not contribute: fine 2I + 1 sits on coarse I
  // (weights 1, 0); fine 2I lies between coarse I - 1 and I (1/2 each, 0 for
  // a candidate outside the grid).  Every thread then issues the same
  // 2^DIM unconditional loads per slice (no divergent loop over 1..8
  // contributions), and indices and weights are formed once for SB slices.
  int ci[DIM][2];
  T cw[DIM][2];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int I = f[a] >> 1;
    if (f[a] & 1) {
      ci[a][0] = I;
      ci[a][1] = I;
      cw[a][0] = (T)1;
      cw[a][1] = (T)0;
    } else {
      // (nxc = 0 on a one-point grid, where the launch only copies: every
      // weight is then zero and every index 0, still a valid address)
      ci[a][0] = I >= 1 ? I - 1 : 0;
      ci[a][1] = I < nxc ? I : (nxc > 0 ? nxc - 1 : 0);
      cw[a][0] = I >= 1 ? (T)0.5 : (T)0;
      cw[a][1] = I < nxc ? (T)0.5 : (T)0;
    }
  }
  constexpr int NC = 1 << DIM;
  int cidx[NC];
  T cwt[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    int I = 0, stride = 1;
    T wt = (T)1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int b = (u >> a) & 1;
      I += ci[a][b] * stride;
      wt *= cw[a][b];
      stride *= nxc;
    }
    cidx[u] = I;
    cwt[u] = wt;
  }
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T>* zcs = zc + (size_t)s * mc;
    cx<T> acc = zf[(size_t)s * mf + i];
#pragma unroll
    for (int u = 0; u < NC; ++u) acc = acc + scale(zcs[cidx[u]], cwt[u]);
    out[(size_t)s * mf + i] = acc;
  }
}

// ---------------------------------------------------------------------------
// Lexicographic Gauss-Seidel (mg_smoother = 1, and = 2 followed by the
// reverse sweep): the natural order (x1 fastest) makes point x depend on its
// minus neighbours, which lie on the hyperplane x1 + x2 (+ x3) one below.
// One block per slice walks the hyperplanes in order (reverse order for the
// backward sweep) with a block barrier between them; the points of one
// hyperplane are independent.  z lives in global memory (a slice does not fit
// LDS); within a block the barrier orders the stores and the later loads.
//   forward   z_x = (r_x - sum_{minus nb} off z_nb) / d_x          (z = 0 before)
//   backward  z_x = (r_x - sum_{all nb} off z_nb) / d_x             (in place)
// ---------------------------------------------------------------------------
template <class T, int DIM, bool BACK>
__global__ void __launch_bounds__(256) mg_sweep_lex_kernel(int nx, int m, const T* __restrict__ coef,
                                                           const cx<T>* __restrict__ r, cx<T>* z, MgShift sh) {
  const int s = blockIdx.x;
  if (sh.active && !sh.active[s / sh.twoK]) return;
  const cx<T> sig = slice_sigma<T>(sh, s);
  const cx<T>* rs = r + (size_t)s * m;
  cx<T>* zs = z + (size_t)s * m;
  const int top = DIM * (nx - 1);
  for (int step = 0; step <= top; ++step) {
    const int w = BACK ? top - step : step;
    // points with x1 + x2 (+ x3) = w: x3 (3-D) and x1 over a box, x2 from w
    const int x3lo = DIM == 3 ? max(0, w - 2 * (nx - 1)) : 0;
    const int x3hi = DIM == 3 ? min(w, nx - 1) : 0;
    const int box = (x3hi - x3lo + 1) * nx;
    for (int t = threadIdx.x; t < box; t += blockDim.x) {
      const int x3 = x3lo + t / nx, x1 = t - (t / nx) * nx;
      const int x2 = w - x3 - x1;
      if (x2 < 0 || x2 >= nx) continue;
      const int c[3] = {x1, x2, x3};
      const int i = x1 + nx * (x2 + nx * x3);
      cx<T> acc = rs[i];
      int stride = 1;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        if (c[a] > 0) acc = acc - scale(zs[i - stride], coef[(size_t)(1 + 2 * a) * m + i]);
        if (BACK && c[a] < nx - 1) acc = acc - scale(zs[i + stride], coef[(size_t)(2 + 2 * a) * m + i]);
        stride *= nx;
      }
      zs[i] = cdiv(acc, cx<T>{sig.x + coef[i], sig.y});
    }
    __syncthreads();
  }
}

// r <- r - A z at every point (in place: each point reads only its own r),
// for the lexicographic sweeps, after which the residual is nonzero everywhere
template <class T, int DIM, int SB>
__global__ void __launch_bounds__(256) mg_residual_full_kernel(int nx, int m, int slices, const T* __restrict__ coef,
                                                               const cx<T>* __restrict__ z, cx<T>* res, MgShift sh) {
  const int2 bk = mg_block();
  const int i = bk.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int f[3];
  coords(i, nx, DIM, f);
  int nbo[2 * DIM];
  bool has[2 * DIM];
  T off[2 * DIM];
  {
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      has[2 * a] = f[a] > 0;
      has[2 * a + 1] = f[a] < nx - 1;
      nbo[2 * a] = -stride;
      nbo[2 * a + 1] = stride;
      off[2 * a] = has[2 * a] ? coef[(size_t)(1 + 2 * a) * m + i] : (T)0;
      off[2 * a + 1] = has[2 * a + 1] ? coef[(size_t)(2 + 2 * a) * m + i] : (T)0;
      stride *= nx;
    }
  }
  const T cdg = coef[i];
  const int s0 = bk.y * SB;
#pragma unroll
  for (int k = 0; k < SB; ++k) {
    const int s = s0 + k;
    if (s >= slices) break;
    if (sh.active && !sh.active[s / sh.twoK]) continue;
    const cx<T> sig = slice_sigma<T>(sh, s);
    const cx<T>* zs = z + (size_t)s * m;
    const cx<T> zi = zs[i];
    // (sigma + cdg) z_i
    cx<T> acc = res[(size_t)s * m + i] - cx<T>{(sig.x + cdg) * zi.x - sig.y * zi.y, (sig.x + cdg) * zi.y + sig.y * zi.x};
#pragma unroll
    for (int n = 0; n < 2 * DIM; ++n)
      if (has[n]) acc = acc - scale(zs[i + nbo[n]], off[n]);
    res[(size_t)s * m + i] = acc;
  }
}

// slices per thread of the smoother, the residual and the prolongation on
// levels where that still gives at least kMgMinBlocks blocks (one slice per
// thread below)
constexpr int kMgSB = 8;
constexpr long long kMgMinBlocks = 1024;

template <class T, int DIM>
static void mg_cycle(const Geo& g, cx<T>* spec, const PrecondTables& tb, int spm, const double* lam,
                     hipStream_t st) {
  const int NL = tb.mg_levels;
  const int slices = g.B * spm;
  MgShift sh{lam, tb.alpha, tb.active, spm};
  // the smoother: red-black (0), lexicographic (1), symmetric lexicographic (2)
  const bool lex = tb.mg_smoother != 0;
  auto coefp = [&](int l) -> const T* {
    return reinterpret_cast<const T*>(sizeof(T) == 4 ? (const void*)tb.mg[l].coef : (const void*)tb.mg[l].coef64);
  };
  auto zbuf = [&](int l) -> cx<T>* {
    return reinterpret_cast<cx<T>*>(l == 0 ? tb.mg[0].r : tb.mg[l].z);
  };
  auto rbuf = [&](int l) -> cx<T>* { return l == 0 ? spec : reinterpret_cast<cx<T>*>(tb.mg[l].r); };
  // pass bytes (algorithmic): complex data in and out of every kernel
  const double cs = sizeof(cx<T>) * (double)slices * tb.nact / g.B;
  // kMgSB slices per thread where that still leaves kMgMinBlocks blocks to
  // fill the chip, one slice per thread on the small (coarse) levels
  auto wide = [&](int m) { return (long long)((m + 255) / 256) * ((slices + kMgSB - 1) / kMgSB) >= kMgMinBlocks; };
  auto grid_sb = [&](int m) {
    const int sb = wide(m) ? kMgSB : 1;
    return dim3((m + 255) / 256, (slices + sb - 1) / sb);
  };
  // the red-black smoother and residual in FP32: one thread per pair of
  // points, with the slice grouping of the level (wide(m))
  constexpr bool pair = sizeof(T) == 4;
  auto grid_pair = [&](int nx, int m) {
    const int sb = wide(m) ? kMgSB : 1;
    const int np = m / nx * ((nx + 1) / 2);
    return dim3((np + 255) / 256, (slices + sb - 1) / sb);
  };
  for (int l = 0; l < NL; ++l) {
    const int nx = tb.mg[l].nx;
    const int m = (int)tb.mg[l].m;
    const dim3 gridb = grid_sb(m);
    tbeg(tb.timer, KF_MG_SMOOTH, 2.0 * cs * m);
    if (lex) {
      mg_sweep_lex_kernel<T, DIM, false><<<slices, 256, 0, st>>>(nx, m, coefp(l), rbuf(l), zbuf(l), sh);
      if (tb.mg_smoother == 2)
        mg_sweep_lex_kernel<T, DIM, true><<<slices, 256, 0, st>>>(nx, m, coefp(l), rbuf(l), zbuf(l), sh);
    } else if (pair) {
      if (wide(m))
        mg_smooth_pair_kernel<T, DIM, kMgSB><<<grid_pair(nx, m), 256, 0, st>>>(nx, m, slices, coefp(l), rbuf(l), zbuf(l), sh);
      else
        mg_smooth_pair_kernel<T, DIM, 1><<<grid_pair(nx, m), 256, 0, st>>>(nx, m, slices, coefp(l), rbuf(l), zbuf(l), sh);
    } else if (wide(m)) {
      mg_smooth_kernel<T, DIM, kMgSB><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), rbuf(l), zbuf(l), sh);
    } else {
      mg_smooth_kernel<T, DIM, 1><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), rbuf(l), zbuf(l), sh);
    }
    tend(tb.timer);
    if (l + 1 < NL) {
      const int nxc = tb.mg[l + 1].nx;
      const int mc = (int)tb.mg[l + 1].m;
      dim3 gc((mc + 255) / 256, slices);
      // residual into the consumed right-hand side (half the points), then
      // full weighting
      if (lex) {
        // r - A z at every point, in place, then full weighting of all points
        tbeg(tb.timer, KF_MG_RESTRICT, cs * (3.0 * m + m + mc));
        if (wide(m))
          mg_residual_full_kernel<T, DIM, kMgSB><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        else
          mg_residual_full_kernel<T, DIM, 1><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        mg_restrict_kernel<T, DIM, true><<<gc, 256, 0, st>>>(nx, m, nxc, mc, rbuf(l), rbuf(l + 1), sh);
      } else {
        tbeg(tb.timer, KF_MG_RESTRICT, cs * (m + 0.5 * m + 0.5 * m + mc));
        if (pair && wide(m))
          mg_residual_pair_kernel<T, DIM, kMgSB><<<grid_pair(nx, m), 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        else if (pair)
          mg_residual_pair_kernel<T, DIM, 1><<<grid_pair(nx, m), 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        else if (wide(m))
          mg_residual_kernel<T, DIM, kMgSB><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        else
          mg_residual_kernel<T, DIM, 1><<<gridb, 256, 0, st>>>(nx, m, slices, coefp(l), zbuf(l), rbuf(l), sh);
        mg_restrict_kernel<T, DIM, false><<<gc, 256, 0, st>>>(nx, m, nxc, mc, rbuf(l), rbuf(l + 1), sh);
      }
      tend(tb.timer);
    }
  }
  for (int l = NL - 2; l >= 0; --l) {
    const int nx = tb.mg[l].nx;
    const int m = (int)tb.mg[l].m;
    const int nxc = tb.mg[l + 1].nx;
    const int mc = (int)tb.mg[l + 1].m;
    const dim3 gridb = grid_sb(m);
    cx<T>* out = (l == 0) ? spec : zbuf(l);
    tbeg(tb.timer, KF_MG_PROLONG, cs * (2.0 * m + mc));
    if (wide(m))
      mg_prolong_kernel<T, DIM, kMgSB><<<gridb, 256, 0, st>>>(nx, m, nxc, mc, slices, zbuf(l), zbuf(l + 1), out, sh);
    else
      mg_prolong_kernel<T, DIM, 1><<<gridb, 256, 0, st>>>(nx, m, nxc, mc, slices, zbuf(l), zbuf(l + 1), out, sh);
    tend(tb.timer);
  }
  if (NL == 1) {
    // single-point grid: the smoothed value is the exact solve; copy it back
    const int m = (int)tb.mg[0].m;
    dim3 grid1((m + 255) / 256, slices);
    mg_prolong_kernel<T, DIM, 1><<<grid1, 256, 0, st>>>(1, m, 0, 0, slices, zbuf(0), zbuf(0), spec, sh);
  }
}

bool launch_mg_solve(const Geo& g, void* spec, bool fp32, const PrecondTables& tb, int spm, const double* lam,
                     hipStream_t st) {
  if (tb.mg_levels < 1) return false;
  if (fp32) {
    if (g.dim == 2) mg_cycle<float, 2>(g, reinterpret_cast<cx<float>*>(spec), tb, spm, lam, st);
    else mg_cycle<float, 3>(g, reinterpret_cast<cx<float>*>(spec), tb, spm, lam, st);
  } else {
    if (g.dim == 2) mg_cycle<double, 2>(g, reinterpret_cast<cx<double>*>(spec), tb, spm, lam, st);
    else mg_cycle<double, 3>(g, reinterpret_cast<cx<double>*>(spec), tb, spm, lam, st);
  }
  return true;
}

}  // namespace pcop
