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

// A 1D FFT length and its Stockham radix schedule.
struct FftDesc {
  int n;
  int nst;
  int radix[kMaxStages];
};

}  // namespace dda
