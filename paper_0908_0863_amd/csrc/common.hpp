// Shared device/host definitions of libdda: complex arithmetic, launch
// helpers, error reporting.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace dda {

// Interleaved complex value (re, im); layout-compatible with torch.complex64/128.
template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) {
  cx<R> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return mk(s * a.x, s * a.y); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conjg(cx<R> a) { return mk(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__host__ __device__ __forceinline__ cx<R> rot90(cx<R> a) {
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename R>
__host__ __device__ __forceinline__ R abs2(cx<R> a) { return a.x * a.x + a.y * a.y; }

template <typename A, typename B>
__host__ __device__ __forceinline__ cx<A> cvt(cx<B> v) { return mk((A)v.x, (A)v.y); }

// principal square root
template <typename R>
__device__ __forceinline__ cx<R> csqrt(cx<R> z) {
  R r = sqrt(z.x * z.x + z.y * z.y);
  R a = sqrt((R)0.5 * (r + z.x));
  R b = sqrt((R)0.5 * (r - z.x));
  return mk(a, z.y < 0 ? -b : b);
}

using c64 = cx<double>;
using c32 = cx<float>;

constexpr int kMaxStages = 16;

// Sum of two complex values over a block of any size up to 1024 threads, in
// a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum2_any(cx<double>& v0, cx<double>& v1) {
  __shared__ cx<double> sh[2][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  // lanes of this wavefront that exist (a last, partial wavefront adds no
  // value from the lanes it lacks)
  const int nact = min(64, (int)blockDim.x - (wv << 6));
  double a[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(a[q], off, 64);
      if (lane + off < nact) a[q] += o;
    }
  if (lane == 0) {
    sh[0][wv] = mk(a[0], a[1]);
    sh[1][wv] = mk(a[2], a[3]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cx<double> s0 = sh[0][0], s1 = sh[1][0];
    for (int w = 1; w < nw; ++w) {
      s0 = s0 + sh[0][w];
      s1 = s1 + sh[1][w];
    }
    v0 = s0;
    v1 = s1;
  }
}

// Inner products fused into the last pass of the matrix-vector product y = A x
// (accumulated in FP64 while the compressed result is written):
//   DOT_BIL  x^T y            (QMR_sym, bilinear)
//   DOT_HA   a^H y            (BiCGSTAB rhat^H v)
//   DOT_TS   y^H x, y^H y     (BiCGSTAB t^H s, t^H t)
// Partials per block: part[(rhs * nblk + block) * 2 + q].
enum { DOT_NONE = 0, DOT_BIL = 1, DOT_HA = 2, DOT_TS = 3 };
struct DotArgs {
  int mode = DOT_NONE;
  const void* a = nullptr;
  cx<double>* part = nullptr;
};

// A 1D FFT length and its Stockham radix schedule.
struct FftDesc {
  int n;
  int nst;
  int radix[kMaxStages];
};

}  // namespace dda
