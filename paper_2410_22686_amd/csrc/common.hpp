// Shared device helpers: a minimal complex type, reductions and the geometry
// record every kernel receives.  Written for gfx950 (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcop {

constexpr int kWave = 64;

template <class T>
struct cx {
  T x, y;
};

template <class T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <class T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// multiply by +i (sgn = +1) or -i (sgn = -1)
template <class T, int SGN>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return SGN > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}
// a / b = a conj(b) / |b|^2 with one reciprocal of |b|^2 (|b| is bounded
// away from zero, and |b|^2 well inside the normal range, for every shift the
// preconditioner uses): in FP32 the hardware reciprocal (about 1 ulp; two
// correctly rounded divisions cost several times more instructions), in FP64
// one division
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }
template <class T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  const T rd = recip(b.x * b.x + b.y * b.y);
  return {(a.x * b.x + a.y * b.y) * rd, (a.y * b.x - a.x * b.y) * rd};
}

// geometry of one context, passed by value to kernels
struct Geo {
  int dim;       // 2 or 3
  int nx;        // interior points per dimension
  int n;         // time blocks (nt - 1)
  int m;         // nx^dim
  int B;         // batch members
  int K;         // frequencies kept, n/2 + 1
  long long vl;  // doubles per member vector: 2 n m
  long long vs;  // doubles between consecutive members' vectors (>= vl; padded to 256 bytes inside the solver)
  double tau;
  double h2inv;  // 1/h^2
  int fem;       // 1: Q1 finite-element mass and stiffness matrices (M != I), 0: finite differences (M = I)
};

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// For kernels whose neighbouring blocks share data, remap the hardware block
// order so that every XCD walks one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int hw, int total) {
  const int per = total / 8;
  if (hw >= per * 8) return hw;
  return (hw % 8) * per + hw / 8;
}

// fixed-order wavefront sum (xor butterfly over 64 lanes)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

}  // namespace pcop
