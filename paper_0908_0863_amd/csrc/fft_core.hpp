// Workgroup-level 1D FFTs over many lines held in LDS.
//
// Radix-staged Stockham (self-sorting) transforms: every stage reads r
// elements at stride n/r, applies the stage twiddles, performs an r-point DFT
// and writes the r results at stride p (the product of the radices already
// applied).  Ping-pong between two LDS buffers, one barrier per stage, natural
// order in and out.  Radices 2, 3, 4, 5 and 8 cover every 5-smooth length.
//
// The forward transform uses omega = exp(-2 pi i / n) (the Fourier matrix of
// Eq. circdiagl0 without its 1/sqrt(n)); the inverse is unnormalised; the
// 1/(K''J''P'') factor of step 4 of the standard algorithm is applied once at
// the end of the matrix-vector product.
//
// Element (line l, index e) lives at  buf[l * ls + e * es].  When es == 1
// consecutive threads walk along a line, otherwise across lines, so that the
// LDS accesses of a wavefront are consecutive in both layouts.
#pragma once
#include "common.hpp"

namespace dda {

// exact trigonometric constants of the small DFTs
#define DDA_SQRT1_2 0.70710678118654752440
#define DDA_SIN60 0.86602540378443864676
#define DDA_COS72 0.30901699437494742410
#define DDA_COS144 (-0.80901699437494742410)
#define DDA_SIN72 0.95105651629515357212
#define DDA_SIN144 0.58778525229247312917

template <typename R, bool INV>
__host__ __device__ __forceinline__ void dft2(cx<R>& a, cx<R>& b) {
  cx<R> t = a - b;
  a = a + b;
  b = t;
}

template <typename R, bool INV>
__host__ __device__ __forceinline__ void dft4(cx<R>* v) {
  cx<R> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cx<R> t2 = v[1] + v[3], t3 = rot90<R, INV>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename R, bool INV>
__host__ __device__ __forceinline__ void dft3(cx<R>* v) {
  cx<R> s = v[1] + v[2];
  cx<R> d = v[1] - v[2];
  cx<R> m = v[0] - (R)0.5 * s;
  cx<R> q = rot90<R, INV>((R)DDA_SIN60 * d);  // -i sqrt(3)/2 d (forward)
  v[0] = v[0] + s;
  v[1] = m + q;
  v[2] = m - q;
}

template <typename R, bool INV>
__host__ __device__ __forceinline__ void dft5(cx<R>* v) {
  const R c1 = (R)DDA_COS72, c2 = (R)DDA_COS144, s1 = (R)DDA_SIN72, s2 = (R)DDA_SIN144;
  cx<R> b1 = v[1] + v[4], b2 = v[2] + v[3];
  cx<R> d1 = v[1] - v[4], d2 = v[2] - v[3];
  cx<R> m1 = v[0] + c1 * b1 + c2 * b2;
  cx<R> m2 = v[0] + c2 * b1 + c1 * b2;
  cx<R> q1 = rot90<R, INV>(s1 * d1 + s2 * d2);
  cx<R> q2 = rot90<R, INV>(s2 * d1 - s1 * d2);
  v[0] = v[0] + b1 + b2;
  v[1] = m1 + q1;
  v[4] = m1 - q1;
  v[2] = m2 + q2;
  v[3] = m2 - q2;
}

template <typename R, bool INV>
__host__ __device__ __forceinline__ void dft8(cx<R>* v) {
  cx<R> e[4] = {v[0], v[2], v[4], v[6]};
  cx<R> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<R, INV>(e);
  dft4<R, INV>(o);
  const R h = (R)DDA_SQRT1_2;
  // o[k] *= omega_8^k
  cx<R> w1 = INV ? mk(h, h) : mk(h, -h);
  cx<R> w3 = INV ? mk(-h, h) : mk(-h, -h);
  o[1] = o[1] * w1;
  o[2] = rot90<R, INV>(o[2]);
  o[3] = o[3] * w3;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = e[k] + o[k];
    v[k + 4] = e[k] - o[k];
  }
}

template <int RR, typename R, bool INV>
__host__ __device__ __forceinline__ void dft_small(cx<R>* v) {
  if constexpr (RR == 2) dft2<R, INV>(v[0], v[1]);
  else if constexpr (RR == 3) dft3<R, INV>(v);
  else if constexpr (RR == 4) dft4<R, INV>(v);
  else if constexpr (RR == 5) dft5<R, INV>(v);
  else dft8<R, INV>(v);
}

// One Stockham stage of radix RR over nl lines of length n held in `in`.
template <int RR, typename R, bool INV>
__device__ __forceinline__ void stockham_stage(const cx<R>* __restrict__ in, cx<R>* __restrict__ out, int n,
                                               int nl, int ls, int es, int p, const cx<R>* __restrict__ tw,
                                               int tid, int nthr) {
  const int m = n / RR;
  const int tot = m * nl;
  const int tws = n / (p * RR);
  for (int t = tid; t < tot; t += nthr) {
    int l, q;
    if (es == 1) {
      l = t / m;
      q = t - l * m;
    } else {
      q = t / nl;
      l = t - q * nl;
    }
    const int kk = q % p;
    cx<R> v[RR];
#pragma unroll
    for (int j = 0; j < RR; ++j) v[j] = in[l * ls + (q + j * m) * es];
    if (p > 1) {
#pragma unroll
      for (int j = 1; j < RR; ++j) {
        cx<R> w = tw[j * kk * tws];
        if (INV) w.y = -w.y;
        v[j] = v[j] * w;
      }
    }
    dft_small<RR, R, INV>(v);
    const int base = (q - kk) * RR + kk;
#pragma unroll
    for (int j = 0; j < RR; ++j) out[l * ls + (base + j * p) * es] = v[j];
  }
}

// Transform nl lines in place (logically): returns the buffer (a or b) that
// holds the result.  Ends with a barrier, so the result may be read at once.
template <typename R, bool INV>
__device__ cx<R>* lds_fft(cx<R>* a, cx<R>* b, const FftDesc& d, const cx<R>* __restrict__ tw, int nl, int ls,
                          int es, int tid, int nthr) {
  int p = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int r = d.radix[s];
    switch (r) {
      case 2: stockham_stage<2, R, INV>(a, b, d.n, nl, ls, es, p, tw, tid, nthr); break;
      case 3: stockham_stage<3, R, INV>(a, b, d.n, nl, ls, es, p, tw, tid, nthr); break;
      case 4: stockham_stage<4, R, INV>(a, b, d.n, nl, ls, es, p, tw, tid, nthr); break;
      case 5: stockham_stage<5, R, INV>(a, b, d.n, nl, ls, es, p, tw, tid, nthr); break;
      default: stockham_stage<8, R, INV>(a, b, d.n, nl, ls, es, p, tw, tid, nthr); break;
    }
    __syncthreads();
    cx<R>* t = a;
    a = b;
    b = t;
    p *= r;
  }
  return a;
}

}  // namespace dda
