// Power-of-two DFTs of length R <= 32 held entirely in one thread's
// registers (natural order in and out), for FFT stages that keep a whole
// butterfly group per thread.  Every twiddle inside them is a multiple of
// 2 pi / 32, taken from a table of cos(pi k / 16), so after unrolling each is
// a literal; multiplications by 1, +-i and (1 +- i)/sqrt 2 are written out.
#pragma once

#include "common.hpp"
#include "fft_lds.hpp"

namespace pcop {

// cos(pi k / 16), k = 0..8
__device__ __forceinline__ double cos_pi16(int k) {
  constexpr double c[9] = {1.0,
                           0.98078528040323044912618223613424L,
                           0.92387953251128675612818318939679L,
                           0.83146961230254523707878837761791L,
                           0.70710678118654752440084436210485L,
                           0.55557023301960222474283081394853L,
                           0.38268343236508977172845998403040L,
                           0.19509032201612826784828486847702L,
                           0.0};
  return c[k];
}

// x * exp(SG 2 pi i e / N) for N a power of two dividing 32 (e, N constants
// after unrolling)
template <class T, int SG>
__device__ __forceinline__ cx<T> rot_root(cx<T> x, int e, int N) {
  const int k = ((e * (32 / N)) % 32 + 32) % 32;  // angle pi k / 16
  if (k == 0) return x;
  if (k == 8) return mul_i<T, SG>(x);
  if (k == 16) return cx<T>{-x.x, -x.y};
  if (k == 24) return mul_i<T, -SG>(x);
  // cos and sin of pi k / 16 by quadrant
  const int q = k / 8, r = k % 8;
  double c, s;
  if (q == 0) { c = cos_pi16(r); s = cos_pi16(8 - r); }
  else if (q == 1) { c = -cos_pi16(8 - r); s = cos_pi16(r); }
  else if (q == 2) { c = -cos_pi16(r); s = -cos_pi16(8 - r); }
  else { c = cos_pi16(8 - r); s = -cos_pi16(r); }
  const T ct = (T)c, st = (T)(SG * s);
  if (r == 4) {  // odd multiples of pi/4: |c| = |s| = sqrt(1/2), one product per part
    return (ct == st) ? cx<T>{ct * (x.x - x.y), ct * (x.y + x.x)} : cx<T>{ct * (x.x + x.y), ct * (x.y - x.x)};
  }
  return cx<T>{ct * x.x - st * x.y, ct * x.y + st * x.x};
}

// R-point DFT (R = 1, 2, 4, 8, 16, 32) in registers, natural order; for
// R > 8 a 4 x (R/4) Cooley-Tukey split:
//   X[k1 + 4 k2] = sum_{n2} W_{R/4}^{n2 k2} W_R^{n2 k1} sum_{n1} x[(R/4) n1 + n2] W_4^{n1 k1}
template <class T, int SG, int R>
__device__ __forceinline__ void dft_reg(cx<T>* a) {
  if constexpr (R == 1) {
  } else if constexpr (R <= 8) {
    dftR<T, SG, R>(a);
  } else {
    constexpr int R1 = 4, R2 = R / 4;
    cx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      cx<T> t0 = a[n2], t1 = a[R2 + n2], t2 = a[2 * R2 + n2], t3 = a[3 * R2 + n2];
      dft4<T, SG>(t0, t1, t2, t3);
      y[0 * R2 + n2] = t0;
      y[1 * R2 + n2] = rot_root<T, SG>(t1, n2, R);
      y[2 * R2 + n2] = rot_root<T, SG>(t2, 2 * n2, R);
      y[3 * R2 + n2] = rot_root<T, SG>(t3, 3 * n2, R);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      dft_reg<T, SG, R2>(&y[k1 * R2]);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = y[k1 * R2 + k2];
    }
  }
}

// The same DFT when the inputs a[R/2 .. R-1] are zero (not read): the even
// outputs are the (R/2)-point DFT of a[0..R/2-1], the odd ones that of
// a_j W_R^j.  Writes all R outputs.
template <class T, int SG, int R>
__device__ __forceinline__ void dft_reg_half_in(cx<T>* a) {
  constexpr int H = R / 2;
  cx<T> e[H], o[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    e[j] = a[j];
    o[j] = rot_root<T, SG>(a[j], j, R);
  }
  dft_reg<T, SG, H>(e);
  dft_reg<T, SG, H>(o);
#pragma unroll
  for (int k = 0; k < H; ++k) {
    a[2 * k] = e[k];
    a[2 * k + 1] = o[k];
  }
}

}  // namespace pcop
