// Device kernels of the interaction spectrum and of the pruned FFT
// matrix-vector product.
//
// Grid layouts (x fastest, as the linear site index n = k*J*K + j*K + i of
// Appendix A):
//   tensor first column   t  [6][P][J][K]            complex FP64
//   spectrum              Y  [6][P_h][J_h][K_h]      unique octant, n_h = n''/2 + 1
//   y-transformed vector  G1 [rhs][3][P][J''][K]     (Sec. 3: K x J'' x P array)
//   xy-transformed vector G2 [rhs][3][P][J''][K'']   (the x-transformed rows of the
//                                                     xz-planes of Sec. 3)
//   compressed vectors    x, y [rhs][3][N_d]         occupied sites only (Sec. 4)
#pragma once
#include "fft_core.hpp"

namespace dda {

// Table 1 of the paper: parity of each tensor component (xx xy xz yy yz zz)
// under reflection of the x, y and z displacement; the Toeplitz-to-circulant
// mirror multiplies mirrored entries by it.
__constant__ int8_t c_sign[3][6] = {
    {+1, -1, -1, +1, +1, +1},
    {+1, -1, +1, +1, -1, +1},
    {+1, +1, -1, +1, -1, +1},
};

// ---------------------------------------------------------------------------
// Tensor first column (Eq. 1): t(d) = -G(d) for d in [0,K)x[0,J)x[0,P), with
// t(0) = 0 (the diagonal is excluded from the convolution, Sec. 3).
// ---------------------------------------------------------------------------
__global__ void k_tensor_column(c64* __restrict__ t, int K, int J, int P, double k) {
  const long N = (long)K * J * P;
  for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < N; s += (long)gridDim.x * blockDim.x) {
    const int i = (int)(s % K);
    const int j = (int)((s / K) % J);
    const int l = (int)(s / ((long)K * J));
    double g[6] = {0, 0, 0, 0, 0, 0}, gi[6] = {0, 0, 0, 0, 0, 0};
    if (s != 0) {
      const double rx = i, ry = j, rz = l;
      const double r2 = rx * rx + ry * ry + rz * rz;
      const double r = sqrt(r2);
      const double u[3] = {rx / r, ry / r, rz / r};
      double sn, cs;
      sincos(k * r, &sn, &cs);
      const double inv3 = 1.0 / (r2 * r);
      // e^{ikr}/r^3 [k^2 r^2 (I - uu) + (1 - ikr)(3uu - I)]
      const double pr = cs * inv3, pi = sn * inv3;
      const double a = k * k * r2;
      const int pq[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double d = (pq[c][0] == pq[c][1]) ? 1.0 : 0.0;
        const double uu = u[pq[c][0]] * u[pq[c][1]];
        const double br = 3.0 * uu - d;                  // (1 - ikr)(3uu - I): real part br, imag -kr br
        const double mr = a * (d - uu) + br;             // real part of the bracket
        const double mi = -k * r * br;                   // imaginary part of the bracket
        g[c] = -(pr * mr - pi * mi);
        gi[c] = -(pr * mi + pi * mr);
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c * N + s] = mk(g[c], gi[c]);
  }
}

// ---------------------------------------------------------------------------
// Lines along the contiguous axis.  Line `ln` reads in[ln*lin_stride + e] for
// e < Lin and writes out[ln*lout_stride + e] for e < Lout.
// MIRROR: the implicit Toeplitz-to-circulant conversion of a tensor line
// (Sec. 3): entry e > n - Lin holds sign * in[n - e] (Table 1), the rest of the
// padded line is zero.
// ---------------------------------------------------------------------------
struct ContigArgs {
  long nlines;
  long lin_stride, lout_stride;
  int Lin, Lout;
  int rows;           // lines per workgroup
  int ls;             // LDS line stride (>= n)
  long lines_per_comp;  // for the mirror sign: component = (ln / lines_per_comp) % 6
  int axis;           // which row of Table 1
  long lines_per_rhs;   // for masking converged right-hand sides (0: none)
  double scale;
};

template <typename R, bool INV, bool MIRROR>
__global__ void __launch_bounds__(256) k_lines_contig(const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                                      ContigArgs a, FftDesc d, const cx<R>* __restrict__ tw,
                                                      const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* A = reinterpret_cast<cx<R>*>(smem);
  cx<R>* B = A + a.rows * a.ls;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long l0 = (long)blockIdx.x * a.rows;
  const int nl = (int)min((long)a.rows, a.nlines - l0);
  if (active && a.lines_per_rhs) {
    // workgroups never straddle right-hand sides (rows divides lines_per_rhs)
    if (!active[l0 / a.lines_per_rhs]) return;
  }
  const int n = d.n;
  for (int idx = tid; idx < nl * n; idx += nthr) {
    const int l = idx / n, e = idx - l * n;
    const long ln = l0 + l;
    const cx<R>* src = in + ln * a.lin_stride;
    cx<R> v = mk((R)0, (R)0);
    if (e < a.Lin) {
      v = src[e];
    } else if (MIRROR && e > n - a.Lin) {
      v = src[n - e];
      if (c_sign[a.axis][(ln / a.lines_per_comp) % 6] < 0) v = mk(-v.x, -v.y);
    }
    A[l * a.ls + e] = v;
  }
  __syncthreads();
  cx<R>* res = lds_fft<R, INV>(A, B, d, tw, nl, a.ls, 1, tid, nthr);
  const R sc = (R)a.scale;
  for (int idx = tid; idx < nl * a.Lout; idx += nthr) {
    const int l = idx / a.Lout, e = idx - l * a.Lout;
    out[(l0 + l) * a.lout_stride + e] = sc * res[l * a.ls + e];
  }
}

// ---------------------------------------------------------------------------
// Lines along a strided axis, processed in tiles of TX adjacent x positions so
// that every global row access is contiguous.  Element e of line (b, o, x) is
// in[b*sb + o*so + e*se + x]; outputs go to out[b*tb + o*to + e*te + x].
// grid = (ceil(NX/TX), NO, NB).
// ---------------------------------------------------------------------------
struct StridedArgs {
  long sb, so, se, tb, to, te;
  int NX, Lin, Lout, TX;
  int axis;  // row of Table 1 for MIRROR
};

template <typename R, bool INV, bool MIRROR>
__global__ void __launch_bounds__(256) k_lines_strided(const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                                       StridedArgs a, FftDesc d, const cx<R>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* A = reinterpret_cast<cx<R>*>(smem);
  cx<R>* B = A + d.n * a.TX;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x0 = blockIdx.x * a.TX;
  const long o = blockIdx.y, b = blockIdx.z;
  const int n = d.n, TX = a.TX;
  const cx<R>* src = in + b * a.sb + o * a.so + x0;
  const bool neg = MIRROR && c_sign[a.axis][b % 6] < 0;
  for (int idx = tid; idx < n * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX;
    cx<R> v = mk((R)0, (R)0);
    if (x0 + l < a.NX) {
      if (e < a.Lin) {
        v = src[e * a.se + l];
      } else if (MIRROR && e > n - a.Lin) {
        v = src[(n - e) * a.se + l];
        if (neg) v = mk(-v.x, -v.y);
      }
    }
    A[e * TX + l] = v;
  }
  __syncthreads();
  cx<R>* res = lds_fft<R, INV>(A, B, d, tw, TX, 1, TX, tid, nthr);
  cx<R>* dst = out + b * a.tb + o * a.to + x0;
  for (int idx = tid; idx < a.Lout * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX;
    if (x0 + l < a.NX) dst[e * a.te + l] = res[e * TX + l];
  }
}

// ---------------------------------------------------------------------------
// Diagonal alpha^{-1} of right-hand side r at entry c N_d + n (component c of
// dipole n; a diagonal polarisability tensor per dipole, so anisotropic and
// multi-material targets, Sec. 2): a0 + S[r] a1 (the LDR term b3 S eps (kd)^2
// depends on the incident direction and polarisation).  Point-Jacobi in
// symmetric form uses s = (alpha^{-1})^{-1/2}.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx<R> diag_of(const cx<R>* __restrict__ a0, const cx<R>* __restrict__ a1, R S, long n) {
  cx<R> v = a0[n];
  if (a1) v = v + S * a1[n];
  return v;
}
template <typename R>
__device__ __forceinline__ cx<R> jacobi_scale(cx<R> a) {
  cx<R> q = csqrt(a);
  return cdiv(mk((R)1, (R)0), q);
}

// Bit-fielded occupancy (Sec. 2: the occupancy is stored one bit per lattice
// site).  Row r = k J + j of the lattice holds W = ceil(K / 32) words; word w
// is the pair (bits, base): bit b of `bits` marks site (32 w + b, j, k), and
// `base` counts the occupied sites before word w in linear order, so the
// dipole index of an occupied site is base + popcount of the lower bits.  One
// 8-byte load per lookup.
struct OccBits {
  const uint2* __restrict__ words;
  int W;
};

// Dipole index of site (i, row) or -1 if the site is empty.
__device__ __forceinline__ int site_index(const OccBits& o, long row, int i) {
  const uint2 wd = o.words[(int)row * o.W + (i >> 5)];
  const uint32_t b = 1u << (i & 31);
  return (wd.x & b) ? (int)wd.y + __popc(wd.x & (b - 1u)) : -1;
}

struct VecArgs {
  int K, J, P, Jpp, Kpp, Ppp;
  int nrhs = 1;  // right-hand sides of the launch
  long nd;
  long dstride;  // distance between the components' diagonals: N_d, or 0 when isotropic (shared entries)
  int TX;
  int jacobi;  // 0: y = A x;  1: y = D^{-1/2} A D^{-1/2} x with D = diag(alpha^{-1})
  double scale;  // 1/(K''J''P'') for the inverse pass
  // Bit-fielded composition (Sec. 2: a material index per dipole and
  // direction, stored at the minimal bit width): when mbits is set, entry
  // e = c N_d + n holds its material in bits [e 2^mlb, (e + 1) 2^mlb) of the
  // word array, and alpha^{-1} = mt0[q] + S mt1[q] comes from the materials'
  // table (of the pass's precision) instead of per-dipole arrays.
  const uint32_t* mbits = nullptr;
  int mlb = 0;
  const void* mt0 = nullptr;
  const void* mt1 = nullptr;
  // a homogeneous target (one permittivity for every dipole): alpha^{-1} =
  // mt0[0] + S mt1[0] for all of them, no per-dipole gathers
  int uniform = 0;
};

// alpha^{-1} of component c of dipole n for orientation factor S
template <typename R>
__device__ __forceinline__ cx<R> diag_at(const cx<R>* __restrict__ a0, const cx<R>* __restrict__ a1,
                                         const VecArgs& a, int c, long n, R S) {
  if (a.uniform) return diag_of((const cx<R>*)a.mt0, (const cx<R>*)a.mt1, S, 0);
  if (a.mbits) {
    const long bit = ((long)c * a.nd + n) << a.mlb;
    const uint32_t w = a.mbits[bit >> 5];
    const int q = (int)((w >> (bit & 31)) & ((1u << (1 << a.mlb)) - 1u));
    return diag_of((const cx<R>*)a.mt0, (const cx<R>*)a.mt1, S, q);
  }
  return diag_of(a0, a1, S, (long)c * a.dstride + n);
}

// Expansion (Sec. 4) of the compressed vector into the zero-padded
// [K x J'' x P] array fused with the forward DFT along y on the K*P lines that
// hold data (Sec. 3).  grid = (ceil(K/TX), P, nrhs*3).
template <typename R>
__global__ void __launch_bounds__(256) k_vec_yfwd(const cx<R>* __restrict__ x, cx<R>* __restrict__ G1,
                                                  OccBits map, const cx<R>* __restrict__ a0,
                                                  const cx<R>* __restrict__ a1, const double* __restrict__ S,
                                                  const int* __restrict__ active, VecArgs a, FftDesc d,
                                                  const cx<R>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int rc = blockIdx.z, rhs = rc / 3;
  if (active && !active[rhs]) return;
  cx<R>* A = reinterpret_cast<cx<R>*>(smem);
  cx<R>* B = A + d.n * a.TX;
  const int tid = threadIdx.x, nthr = blockDim.x, TX = a.TX;
  const int i0 = blockIdx.x * TX, k = blockIdx.y;
  const R Sr = S ? (R)S[rhs] : (R)0;
  const cx<R>* xv = x + (long)rc * a.nd;
  const int cc = rc % 3;  // this component's diagonal entries
  for (int idx = tid; idx < d.n * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX, i = i0 + l;
    cx<R> v = mk((R)0, (R)0);
    if (e < a.J && i < a.K) {
      const int m = site_index(map, (long)k * a.J + e, i);
      if (m >= 0) {
        v = xv[m];
        if (a.jacobi) v = jacobi_scale(diag_at(a0, a1, a, cc, m, Sr)) * v;
      }
    }
    A[e * TX + l] = v;
  }
  __syncthreads();
  cx<R>* res = lds_fft<R, false>(A, B, d, tw, TX, 1, TX, tid, nthr);
  cx<R>* dst = G1 + ((long)rc * a.P + k) * a.Jpp * a.K + i0;
  for (int idx = tid; idx < a.Jpp * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX;
    if (i0 + l < a.K) dst[(long)e * a.K + l] = res[e * TX + l];
  }
}

// Inverse DFT along y on the K*P lines that contribute, normalisation,
// compression back to occupied sites (Sec. 4) and the diagonal term added back
// (step 5 of the standard algorithm).  grid = (ceil(K/TX), P, nrhs*3).
// Accumulate the fused inner product terms of one written element.
template <typename R>
__device__ __forceinline__ void dot_term(const DotArgs& dt, cx<R> xv, cx<R> yv, long gidx, c64& d0, c64& d1) {
  const c64 xd = mk((double)xv.x, (double)xv.y), yd = mk((double)yv.x, (double)yv.y);
  if (dt.mode == DOT_BIL) {
    d0 = d0 + xd * yd;
  } else if (dt.mode == DOT_HA) {
    const cx<R> av = reinterpret_cast<const cx<R>*>(dt.a)[gidx];
    d0 = d0 + conjg(mk((double)av.x, (double)av.y)) * yd;
  } else if (dt.mode == DOT_TS) {
    d0 = d0 + conjg(yd) * xd;
    d1.x += abs2(yd);
  }
}

// Write the block's fused inner-product partials as block blk of nblk per
// right-hand side (all threads must call).
__device__ __forceinline__ void dot_flush_at(const DotArgs& dt, int rhs, long blk, long nblk, c64 d0, c64 d1) {
  if (dt.mode == DOT_NONE) return;
  block_sum2_any(d0, d1);
  if (threadIdx.x == 0) {
    dt.part[((long)rhs * nblk + blk) * 2] = d0;
    dt.part[((long)rhs * nblk + blk) * 2 + 1] = d1;
  }
}
// ... for a grid (tiles, planes, 3 nrhs): component c of right-hand side rhs
__device__ __forceinline__ void dot_flush(const DotArgs& dt, int rhs, int c, c64 d0, c64 d1) {
  dot_flush_at(dt, rhs, ((long)c * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, 3L * gridDim.y * gridDim.x,
               d0, d1);
}

template <typename R>
__global__ void __launch_bounds__(256) k_vec_yinv(const cx<R>* __restrict__ G1, const cx<R>* __restrict__ x,
                                                  cx<R>* __restrict__ y, OccBits map,
                                                  const cx<R>* __restrict__ a0, const cx<R>* __restrict__ a1,
                                                  const double* __restrict__ S, const int* __restrict__ active,
                                                  VecArgs a, FftDesc d, const cx<R>* __restrict__ tw, DotArgs dt) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int rc = blockIdx.z, rhs = rc / 3;
  if (active && !active[rhs]) return;
  cx<R>* A = reinterpret_cast<cx<R>*>(smem);
  cx<R>* B = A + d.n * a.TX;
  const int tid = threadIdx.x, nthr = blockDim.x, TX = a.TX;
  const int i0 = blockIdx.x * TX, k = blockIdx.y;
  const cx<R>* src = G1 + ((long)rc * a.P + k) * a.Jpp * a.K + i0;
  for (int idx = tid; idx < d.n * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX;
    A[e * TX + l] = (i0 + l < a.K) ? src[(long)e * a.K + l] : mk((R)0, (R)0);
  }
  __syncthreads();
  cx<R>* res = lds_fft<R, true>(A, B, d, tw, TX, 1, TX, tid, nthr);
  const R Sr = S ? (R)S[rhs] : (R)0;
  const R sc = (R)a.scale;
  const cx<R>* xv = x + (long)rc * a.nd;
  const int cc = rc % 3;  // this component's diagonal entries
  cx<R>* yv = y + (long)rc * a.nd;
  c64 d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
  for (int idx = tid; idx < a.J * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX, i = i0 + l;
    if (i >= a.K) continue;
    const int m = site_index(map, (long)k * a.J + e, i);
    if (m < 0) continue;
    const cx<R> conv = sc * res[e * TX + l];
    const cx<R> dg = diag_at(a0, a1, a, cc, m, Sr);
    const cx<R> xm = xv[m];
    const cx<R> ym = a.jacobi ? xm + jacobi_scale(dg) * conv : dg * xm + conv;
    yv[m] = ym;
    dot_term(dt, xm, ym, (long)rc * a.nd + m, d0, d1);
  }
  dot_flush(dt, rhs, rc - 3 * rhs, d0, d1);
}

// z direction: forward DFT of the three components on all K''*J'' lines, the
// element-wise product with the 3x3 symmetric spectrum (Eqs. Q0-Q2) read from
// the unique octant with mirrored indices and Table 1 signs, and the inverse
// DFT keeping the first P entries (Sec. 3).  In place on G2.
// grid = (ceil(K''/TX), J'', nrhs).
struct ZArgs {
  int Kpp, Jpp, P, Ppp, Kh, Jh, Ph, TX;
};

template <typename R>
__global__ void __launch_bounds__(256) k_vec_zmul(cx<R>* __restrict__ G2, const cx<R>* __restrict__ Y,
                                                  const int* __restrict__ active, ZArgs a, FftDesc d,
                                                  const cx<R>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int rhs = blockIdx.z;
  if (active && !active[rhs]) return;
  const int tid = threadIdx.x, nthr = blockDim.x, TX = a.TX, n = d.n;
  cx<R>* buf[4];
  buf[0] = reinterpret_cast<cx<R>*>(smem);
  for (int q = 1; q < 4; ++q) buf[q] = buf[q - 1] + n * TX;
  const int i0 = blockIdx.x * TX, jj = blockIdx.y;
  const long plane = (long)a.Jpp * a.Kpp;
  for (int c = 0; c < 3; ++c) {
    const cx<R>* src = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i0;
    for (int idx = tid; idx < n * TX; idx += nthr) {
      const int e = idx / TX, l = idx - e * TX;
      buf[c][e * TX + l] = (e < a.P && i0 + l < a.Kpp) ? src[e * plane + l] : mk((R)0, (R)0);
    }
  }
  __syncthreads();
  int slot[3] = {0, 1, 2}, fr = 3;
  for (int c = 0; c < 3; ++c) {
    cx<R>* r = lds_fft<R, false>(buf[slot[c]], buf[fr], d, tw, TX, 1, TX, tid, nthr);
    if (r == buf[fr]) {
      const int t = slot[c];
      slot[c] = fr;
      fr = t;
    }
  }
  // spectral product
  const int jm = min(jj, a.Jpp - jj);
  const bool my = jj > a.Jpp - jj;
  for (int idx = tid; idx < n * TX; idx += nthr) {
    const int e = idx / TX, l = idx - e * TX, i = i0 + l;
    if (i >= a.Kpp) continue;
    const int im = min(i, a.Kpp - i), km = min(e, n - e);
    const bool mx = i > a.Kpp - i, mz = e > n - e;
    const cx<R>* ys = Y + ((long)km * a.Jh + jm) * a.Kh + im;
    const long cs = (long)a.Ph * a.Jh * a.Kh;
    cx<R> yv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      int sg = 1;
      if (mx) sg *= c_sign[0][c];
      if (my) sg *= c_sign[1][c];
      if (mz) sg *= c_sign[2][c];
      cx<R> v = ys[c * cs];
      yv[c] = sg < 0 ? mk(-v.x, -v.y) : v;
    }
    const int o = e * TX + l;
    const cx<R> x0 = buf[slot[0]][o], x1 = buf[slot[1]][o], x2 = buf[slot[2]][o];
    buf[slot[0]][o] = yv[0] * x0 + yv[1] * x1 + yv[2] * x2;
    buf[slot[1]][o] = yv[1] * x0 + yv[3] * x1 + yv[4] * x2;
    buf[slot[2]][o] = yv[2] * x0 + yv[4] * x1 + yv[5] * x2;
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) {
    cx<R>* r = lds_fft<R, true>(buf[slot[c]], buf[fr], d, tw, TX, 1, TX, tid, nthr);
    if (r == buf[fr]) {
      const int t = slot[c];
      slot[c] = fr;
      fr = t;
    }
  }
  for (int c = 0; c < 3; ++c) {
    cx<R>* dst = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i0;
    for (int idx = tid; idx < a.P * TX; idx += nthr) {
      const int e = idx / TX, l = idx - e * TX;
      if (i0 + l < a.Kpp) dst[e * plane + l] = buf[slot[c]][e * TX + l];
    }
  }
}

// FP64 -> FP32 copy with round-to-nearest-even (the FP32 spectrum is the FP64
// spectrum rounded).
__global__ void k_round_to_f32(const c64* __restrict__ in, c32* __restrict__ out, long n) {
  for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < n; s += (long)gridDim.x * blockDim.x)
    out[s] = mk((float)in[s].x, (float)in[s].y);
}

}  // namespace dda
