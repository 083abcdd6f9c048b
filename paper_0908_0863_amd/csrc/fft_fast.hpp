// Register-resident Stockham FFTs with compile-time length, and the
// matrix-vector passes built on them.
//
// A line of length N is held by T = N/E threads, E complex values each:
// thread t holds positions t + T*m, m = 0..E-1.  In every Stockham stage of
// radix r the butterflies a thread owns read exactly its own positions
// (q + j N/r = t + T (u + j E/r) for q = t + T u), so data only moves through
// LDS between stages (one write, one barrier, one read of the own positions);
// the first stage reads global memory directly and the last one leaves the
// result in the same positions, ready for a coalesced global store.  Lines
// that are only partly non-zero (the padded vector lines of Sec. 3) are loaded
// with zeros and stored up to their useful length.
//
// Lengths: 2^k with E = 8 (radix-8 stages, then 4 or 2) and 3*2^k with
// E = 12 (radix-4 stages, then 2, then 3).  Other 5-smooth lengths use the
// generic LDS kernels of kernels_fft.hpp.
#pragma once
#include "fft_core.hpp"
#include "kernels_fft.hpp"
#include "kernels_solver.hpp"

namespace dda {

// odd part of n (n with every factor 2 divided out)
constexpr int odd_part(int n) {
  while (n % 2 == 0) n /= 2;
  return n;
}

// Compile-time plan of a register-resident length: E values per thread, T
// threads per line, the radix of every Stockham stage.  Lengths 2^k (radix
// 8, then the remainder), 3 2^k (radix 4, then 2 where needed, then 3) and,
// for the y passes and the transposing x passes only, 5 2^k and 25 2^k with
// 4 | N (radix 4, then 2 where needed, then one or two radix-5 stages; 20
// values per thread, T not always a power of two).
template <int N>
struct FastPlan {
  static constexpr bool pow2 = N >= 16 && (N & (N - 1)) == 0;
  static constexpr bool three = N >= 24 && N % 3 == 0 && ((N / 3) & (N / 3 - 1)) == 0;
  static constexpr bool five = N >= 20 && N % 4 == 0 && (odd_part(N) == 5 || odd_part(N) == 25);
  static constexpr bool ok = pow2 || three || five;
  static constexpr int E = pow2 ? 8 : three ? 12 : 20;
  static constexpr int T = N / E;
  static constexpr int nst_calc() {
    int n = N, s = 0;
    if (pow2) {
      while (n >= E) { n /= E; ++s; }
      if (n > 1) ++s;
    } else if (three) {
      n /= 3;
      while (n >= 4) { n /= 4; ++s; }
      if (n > 1) ++s;
      ++s;
    } else {
      n /= odd_part(N);
      while (n >= 4) { n /= 4; ++s; }
      if (n > 1) ++s;
      s += odd_part(N) == 25 ? 2 : 1;
    }
    return s;
  }
  static constexpr int S = nst_calc();
  static constexpr int radix(int s) {
    int n = N, i = 0;
    if (pow2) {
      while (n >= E) {
        if (i == s) return E;
        n /= E;
        ++i;
      }
      return n;
    }
    n /= three ? 3 : odd_part(N);
    while (n >= 4) {
      if (i == s) return 4;
      n /= 4;
      ++i;
    }
    if (n > 1) {
      if (i == s) return n;
      ++i;
    }
    return three ? 3 : 5;
  }
  static constexpr int pbefore(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i);
    return p;
  }
};

// One stage of radix RR at Stockham offset P (product of previous radices).
// lds(e) addresses element e of this thread's line.
template <int PS>
__device__ __forceinline__ int padpos(int e) {
  if constexpr (PS > 0) return e + (e >> PS);
  else return e;
}

template <typename R, bool INV, int N, int E, int RR, int P, bool LAST, int PS, int TWM = 1>
__device__ __forceinline__ void fast_stage(cx<R> (&v)[E], int t, cx<R>* __restrict__ lds, int es, int off,
                                           const cx<R>* __restrict__ tw) {
  constexpr int T = N / E, B = E / RR, TWS = TWM * (N / (P * RR));
  static_assert(E % RR == 0, "radix must divide the per-thread count");
  // butterfly u reads and (in the last stage) writes the slots u + j B: the
  // slot sets of different u are disjoint, so the last stage works in place
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int q = t + T * u;
    const int k = q % P;
    cx<R> a[RR];
#pragma unroll
    for (int j = 0; j < RR; ++j) a[j] = v[u + j * B];
    if constexpr (P > 1) {
#pragma unroll
      for (int j = 1; j < RR; ++j) {
        cx<R> w = tw[j * k * TWS];
        if (INV) w.y = -w.y;
        a[j] = a[j] * w;
      }
    }
    dft_small<RR, R, INV>(a);
    if constexpr (LAST) {
#pragma unroll
      for (int j = 0; j < RR; ++j) v[u + j * B] = a[j];
    } else {
      const int base = (q - k) * RR + k;
#pragma unroll
      for (int j = 0; j < RR; ++j) lds[padpos<PS>(base + j * P) * es + off] = a[j];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[padpos<PS>(t + T * m) * es + off];
    __syncthreads();
  }
}

template <typename R, bool INV, int N, int S, int PS, int TWM>
struct FastStages {
  template <int s>
  __device__ __forceinline__ static void run(cx<R> (&v)[FastPlan<N>::E], int t, cx<R>* lds, int es, int off,
                                             const cx<R>* tw) {
    if constexpr (s < S) {
      constexpr int RR = FastPlan<N>::radix(s);
      constexpr int P = FastPlan<N>::pbefore(s);
      fast_stage<R, INV, N, FastPlan<N>::E, RR, P, s == S - 1, PS, TWM>(v, t, lds, es, off, tw);
      run<s + 1>(v, t, lds, es, off, tw);
    }
  }
};

// In: v[m] = x[t + T m].  Out: v[m] = X[t + T m].  Every thread of the block
// must call it (it contains barriers).  PS > 0 inserts one padding slot every
// 2^PS elements of a line in LDS (spreads the strided Stockham writes over
// the LDS banks).
// TWM: the twiddle table has TWM * N entries (a longer length's table used
// with stride TWM).
template <typename R, bool INV, int N, int PS = 0, int TWM = 1>
__device__ __forceinline__ void fast_fft(cx<R> (&v)[FastPlan<N>::E], int t, cx<R>* lds, int es, int off,
                                         const cx<R>* tw) {
  FastStages<R, INV, N, FastPlan<N>::S, PS, TWM>::template run<0>(v, t, lds, es, off, tw);
}

// Three interleaved transforms (the three vector components) sharing the
// barriers: lds holds three [N][es] planes at offsets 0, cs, 2 cs.
template <typename R, bool INV, int N, int E, int RR, int P, bool LAST, int PS = 0>
__device__ __forceinline__ void fast_stage3(cx<R> (&v)[3][E], int t, cx<R>* __restrict__ lds, int es, int off,
                                            int cs, const cx<R>* __restrict__ tw) {
  constexpr int T = N / E, B = E / RR, TWS = N / (P * RR);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int q = t + T * u;
      const int k = q % P;
      cx<R> a[RR];
#pragma unroll
      for (int j = 0; j < RR; ++j) a[j] = v[c][u + j * B];
      if constexpr (P > 1) {
#pragma unroll
        for (int j = 1; j < RR; ++j) {
          cx<R> w = tw[j * k * TWS];
          if (INV) w.y = -w.y;
          a[j] = a[j] * w;
        }
      }
      dft_small<RR, R, INV>(a);
      if constexpr (LAST) {
#pragma unroll
        for (int j = 0; j < RR; ++j) v[c][u + j * B] = a[j];
      } else {
        const int base = (q - k) * RR + k;
#pragma unroll
        for (int j = 0; j < RR; ++j) lds[c * cs + padpos<PS>(base + j * P) * es + off] = a[j];
      }
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) v[c][m] = lds[c * cs + padpos<PS>(t + T * m) * es + off];
    __syncthreads();
  }
}

template <typename R, bool INV, int N, int S, int PS = 0>
struct FastStages3 {
  template <int s>
  __device__ __forceinline__ static void run(cx<R> (&v)[3][FastPlan<N>::E], int t, cx<R>* lds, int es, int off,
                                             int cs, const cx<R>* tw) {
    if constexpr (s < S) {
      constexpr int RR = FastPlan<N>::radix(s);
      constexpr int P = FastPlan<N>::pbefore(s);
      fast_stage3<R, INV, N, FastPlan<N>::E, RR, P, s == S - 1, PS>(v, t, lds, es, off, cs, tw);
      run<s + 1>(v, t, lds, es, off, cs, tw);
    }
  }
};

// ---------------------------------------------------------------------------
// y forward with expansion (Sec. 3 and 4): one block per (x tile of TX
// columns, z plane, right-hand side, component), block T*TX threads; lane =
// t*TX + l (l fastest: coalesced rows).
// ---------------------------------------------------------------------------
// The y passes' 1D grid: blocks are dealt to the 8 XCDs round-robin, and the
// three component blocks of one (tile, plane, right-hand side) group take
// consecutive slots of one XCD, so the dipoles' occupancy words and diagonal
// entries that all three read come from that XCD's L2 after the first
// (measured at the 128^3 sphere with the components as a grid dimension:
// the y-forward pass fetched 177 MB for 45 MB of such reads).
struct YTile {
  int tile, k, c, rhs;
  bool ok;
};
__device__ __forceinline__ YTile ytile_of(int b, int ntile, int P, int nrhs) {
  const int xcd = b & 7, slot = b >> 3;
  const int g = (slot / 3) * 8 + xcd;
  YTile y;
  y.c = slot - (slot / 3) * 3;
  y.ok = g < ntile * P * nrhs;
  y.tile = g % ntile;
  const int r = g / ntile;
  y.k = r % P;
  y.rhs = r / P;
  return y;
}
// blocks of that grid for ngroups = tiles x planes x right-hand sides
__host__ __device__ constexpr long ytile_blocks(long ngroups) { return 24 * ((ngroups + 7) / 8); }

// QF: a whole QMR_sym step runs here (QmrFuse): the block reduces the
// previous partials and runs the scalar recurrence (as every block of
// k_qmr_step does), then forms vt_{n+1} for the dipoles it expands, which
// are its input values instead of loads of x.
template <typename R, int N, int TX, bool QF>
__global__ void __launch_bounds__(FastPlan<N>::T * TX) k_fast_yfwd(
    const cx<R>* __restrict__ x, cx<R>* __restrict__ G1, OccBits map, const cx<R>* __restrict__ a0,
    const cx<R>* __restrict__ a1, const double* __restrict__ S, const int* __restrict__ active, VecArgs a,
    const cx<R>* __restrict__ tw, QmrFuse<R> qf) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T;
  __shared__ cx<R> lds[N * TX];
  const int ntile = (a.K + TX - 1) / TX;
  const YTile yt = ytile_of(blockIdx.x, ntile, a.P, a.nrhs);
  if (!yt.ok) return;
  const int rhs = yt.rhs, cc = yt.c, rc = 3 * rhs + cc;  // cc: this component's diagonal entries
  if (active && !active[rhs]) return;
  const int l = threadIdx.x % TX, t = threadIdx.x / TX;
  const int i = yt.tile * TX + l, k = yt.k;
  const R Sr = S ? (R)S[rhs] : (R)0;
  const cx<R>* xv = x + (long)rc * a.nd;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  cx<R> v[E];
  QmrCoef qd{};
  if constexpr (QF) {
    __shared__ QmrCoef cq;
    QmrState s0;
    if (threadIdx.x == 0) s0 = qf.sin[rhs];
    c64 r4[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int b = threadIdx.x; b < qf.nblk_in; b += blockDim.x) {
      const c64* p = qf.pnorm_in + ((long)rhs * qf.nblk_in + b) * 2;
      r4[0] = r4[0] + p[0];
      r4[1] = r4[1] + p[1];
    }
    for (int b = threadIdx.x; b < qf.nblk_mv; b += blockDim.x) {
      const c64* p = qf.pdot + ((long)rhs * qf.nblk_mv + b) * 2;
      r4[2] = r4[2] + p[0];
      r4[3] = r4[3] + p[1];
    }
    block_sum_n<4>(r4);
    if (threadIdx.x == 0) {
      const c64 rn[2] = {r4[0], r4[1]}, rd[2] = {r4[2], r4[3]};
      QmrCoef q;
      qmr_scalars(rn, rd, s0, q);
      if (s0.breakdown == 2 && !(s0.rnorm2 < stall_level2<R>() * s0.bnorm2)) {
        s0.breakdown = 0;
        q.stop = s0.converged;
      }
      cq = q;
      if (yt.tile == 0 && k == 0 && cc == 0) {
        s0.ver += 1;
        qf.sout[rhs] = s0;
        if (q.stop) qf.active[rhs] = 0;
      }
    }
    __syncthreads();
    qd = cq;
    if (qd.stop) return;
  }
  {
    const QmrCoefR<R> q(qd);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      cx<R> val = mk((R)0, (R)0);
      if (e < a.J && i < a.K) {
        const int n = site_index(map, (long)k * a.J + e, i);
        if (n >= 0) {
          if constexpr (QF) val = qmr_elem<R>(q, qf, (long)rc * a.nd + n, acc);
          else val = xv[n];
          if (a.jacobi) val = jacobi_scale(diag_at(a0, a1, a, cc, n, Sr)) * val;
        }
      }
      v[m] = val;
    }
  }
  fast_fft<R, false, N>(v, t, lds, TX, l, tw);
  if (i < a.K) {
    cx<R>* dst = G1 + ((long)rc * a.P + k) * N * a.K + i;
#pragma unroll
    for (int m = 0; m < E; ++m) dst[(long)(t + T * m) * a.K] = v[m];
  }
  if constexpr (QF) {
    block_sum2_any(acc[0], acc[1]);
    if (threadIdx.x == 0) {
      const long bid = ((long)cc * a.P + k) * ntile + yt.tile;
      c64* po = qf.pnorm_out + ((long)rhs * qf.nblk_out + bid) * 2;
      po[0] = acc[0];
      po[1] = acc[1];
    }
  }
}

// y inverse, normalisation, compression and diagonal (Sec. 3, 4; step 5 of the
// standard algorithm), with the solver's inner products fused (DotArgs).
template <typename R, int N, int TX>
__global__ void __launch_bounds__(FastPlan<N>::T * TX) k_fast_yinv(
    const cx<R>* __restrict__ G1, const cx<R>* __restrict__ x, cx<R>* __restrict__ y, OccBits map,
    const cx<R>* __restrict__ a0, const cx<R>* __restrict__ a1, const double* __restrict__ S,
    const int* __restrict__ active, VecArgs a, const cx<R>* __restrict__ tw, DotArgs dt) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T;
  __shared__ cx<R> lds[N * TX];
  const int ntile = (a.K + TX - 1) / TX;
  const YTile yt = ytile_of(blockIdx.x, ntile, a.P, a.nrhs);
  if (!yt.ok) return;
  const int rhs = yt.rhs, cc = yt.c, rc = 3 * rhs + cc;  // cc: this component's diagonal entries
  if (active && !active[rhs]) return;
  const int l = threadIdx.x % TX, t = threadIdx.x / TX;
  const int i = yt.tile * TX + l, k = yt.k;
  const cx<R>* src = G1 + ((long)rc * a.P + k) * N * a.K + i;
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = (i < a.K) ? src[(long)(t + T * m) * a.K] : mk((R)0, (R)0);
  fast_fft<R, true, N>(v, t, lds, TX, l, tw);
  const R Sr = S ? (R)S[rhs] : (R)0;
  const R sc = (R)a.scale;
  const cx<R>* xv = x + (long)rc * a.nd;
  cx<R>* yv = y + (long)rc * a.nd;
  c64 d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
  if (i < a.K) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      if (e >= a.J) continue;
      const int n = site_index(map, (long)k * a.J + e, i);
      if (n < 0) continue;
      const cx<R> conv = sc * v[m];
      const cx<R> dg = diag_at(a0, a1, a, cc, n, Sr);
      const cx<R> xn = xv[n];
      const cx<R> yn = a.jacobi ? xn + jacobi_scale(dg) * conv : dg * xn + conv;
      yv[n] = yn;
      dot_term(dt, xn, yn, (long)rc * a.nd + n, d0, d1);
    }
  }
  dot_flush_at(dt, rhs, ((long)cc * a.P + k) * ntile + yt.tile, 3L * a.P * ntile, d0, d1);
}

// x direction on rows: RW rows per block, lane = row*T + t (t fastest).
// Forward: rows of length Lin (K) -> N; inverse: N -> Lout (K).
template <typename R, bool INV, int N, int RW>
__global__ void __launch_bounds__(FastPlan<N>::T * RW) k_fast_x(const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                                                 long nrows, int lin_stride, int lout_stride, int Lin,
                                                                 int Lout, long rows_per_rhs,
                                                                 const int* __restrict__ active,
                                                                 const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T;
  constexpr int ES = 1, LS = N + N / 8 + 1;  // padded row stride in LDS
  __shared__ cx<R> lds[RW * LS];
  const int t = threadIdx.x % T, rw = threadIdx.x / T;
  const long row = (long)blockIdx.x * RW + rw;
  if (active) {  // skip the block when none of the right-hand sides its rows belong to is active
    const long r0 = (long)blockIdx.x * RW, r1 = min(r0 + RW, nrows) - 1;
    bool any = false;
    for (long q = r0 / rows_per_rhs; q <= r1 / rows_per_rhs && !any; ++q) any = active[q] != 0;
    if (!any) return;
  }
  const bool valid = row < nrows && (!active || active[row / rows_per_rhs]);
  const cx<R>* src = in + row * lin_stride;
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    v[m] = (valid && e < Lin) ? src[e] : mk((R)0, (R)0);
  }
  fast_fft<R, INV, N, 3>(v, t, lds, ES, rw * LS, tw);
  if (!valid) return;
  cx<R>* dst = out + row * lout_stride;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    if (e < Lout) dst[e] = v[m];
  }
}

// z direction with the spectral product (Eqs. Q0-Q2, mirrored octant access
// with Table 1 signs), in place on G2.
//
// The spectrum entry of column (i, j) is shared by the mirror columns
// (K''-i, j), (i, J''-j) and (K''-i, J''-j).  Blocks are therefore grouped by
// mirror quadruple {x tile, mirrored x tile} x {j, J''-j}, and the four
// members of a group get consecutive dispatch slots on the same XCD (blocks
// are dealt round-robin to the 8 XCDs: block b runs on XCD b mod 8), so the
// spectrum tile is fetched from HBM once and served to the other three from
// that XCD's L2.  1D grid of 32 * ceil(groups / 8) blocks.
struct ZMap {
  int NX;      // x tiles covering [0, K'')
  int ngx;     // x tile pairs (t, NX-1-t)
  int ngy;     // y pairs (j, J''-j), j in [0, J_h)
  int ngroups; // nrhs * ngx * ngy
};

template <typename R, int N, int TX>
__global__ void __launch_bounds__(FastPlan<N>::T * TX) k_fast_zmul(cx<R>* __restrict__ G2, const cx<R>* __restrict__ Y,
                                                                    const int* __restrict__ active, ZArgs a, ZMap zm,
                                                                    const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T;
  __shared__ cx<R> lds[3 * N * TX];
  const int b = blockIdx.x;
  const int group = (b >> 5) * 8 + (b & 7);
  const int member = (b >> 3) & 3;
  if (group >= zm.ngroups) return;
  const int per_rhs = zm.ngx * zm.ngy;
  const int rhs = group / per_rhs;
  const int rem = group - rhs * per_rhs;
  const int gx = rem / zm.ngy, gy = rem - (rem / zm.ngy) * zm.ngy;
  const int mxm = member & 1, mym = member >> 1;
  const int xt = mxm ? zm.NX - 1 - gx : gx;
  if (mxm && xt == gx) return;
  const int jj = mym ? a.Jpp - gy : gy;
  if (mym && (gy == 0 || jj == gy)) return;
  if (active && !active[rhs]) return;
  // the twiddle table in LDS: the stages read it right after their barriers,
  // where a global-memory round trip would sit on the dependent chain (the
  // first stage has no twiddles, and its barrier publishes the copy)
  __shared__ cx<R> twl[N];
  for (int e = threadIdx.x; e < N; e += blockDim.x) twl[e] = tw[e];
  const int l = threadIdx.x % TX, t = threadIdx.x / TX;
  const int i = xt * TX + l;
  const long plane = (long)a.Jpp * a.Kpp;
  const bool ok = i < a.Kpp;
  cx<R> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R>* src = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      v[c][m] = (ok && e < a.P) ? src[e * plane] : mk((R)0, (R)0);
    }
  }
  FastStages3<R, false, N, FastPlan<N>::S>::template run<0>(v, t, lds, TX, l, N * TX, twl);
  if (ok) {
    const int jm = min(jj, a.Jpp - jj);
    const bool my = jj > a.Jpp - jj;
    const int im = min(i, a.Kpp - i);
    const bool mx = i > a.Kpp - i;
    int sxy[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sxy[c] = (mx ? c_sign[0][c] : 1) * (my ? c_sign[1][c] : 1);
    const long cs = (long)a.Ph * a.Jh * a.Kh;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      const int km = min(e, N - e);
      const bool mz = e > N - e;
      const cx<R>* ys = Y + ((long)km * a.Jh + jm) * a.Kh + im;
      cx<R> yv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int sg = sxy[c] * (mz ? c_sign[2][c] : 1);
        const cx<R> w = ys[c * cs];
        yv[c] = sg < 0 ? mk(-w.x, -w.y) : w;
      }
      const cx<R> x0 = v[0][m], x1 = v[1][m], x2 = v[2][m];
      v[0][m] = yv[0] * x0 + yv[1] * x1 + yv[2] * x2;
      v[1][m] = yv[1] * x0 + yv[3] * x1 + yv[4] * x2;
      v[2][m] = yv[2] * x0 + yv[4] * x1 + yv[5] * x2;
    }
  }
  FastStages3<R, true, N, FastPlan<N>::S>::template run<0>(v, t, lds, TX, l, N * TX, twl);
  if (!ok) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R>* dst = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      if (e < a.P) dst[e * plane] = v[c][m];
    }
  }
}

// z pass with the three components on separate thread groups: a block holds
// TX columns (i'', j'') and 3 T TX threads; group c transforms component c
// (E values per thread instead of 3 E), the groups then exchange their
// spectra through LDS so that group c forms Q_c = sum_b Y_cb X_b (Eqs. Q0-Q2)
// with the three spectrum components of its row, and transforms back.  Same
// tiles and XCD mirror grouping as k_fast_zmul.  More spectrum loads (9 per
// point against 6) and an LDS exchange buy three times the threads per
// column: measured faster for FP64 at 3 * 2^k lengths (the 96^3 ellipsoid),
// slower in FP32; the autotuner decides per lattice and precision.
template <typename R, int N, int TX>
__global__ void __launch_bounds__(3 * FastPlan<N>::T * TX) k_fast_zsplit(
    cx<R>* __restrict__ G2, const cx<R>* __restrict__ Y, const int* __restrict__ active, ZArgs a, ZMap zm,
    const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T;
  __shared__ cx<R> lds[3 * N * TX];
  const int b = blockIdx.x;
  const int group = (b >> 5) * 8 + (b & 7);
  const int member = (b >> 3) & 3;
  if (group >= zm.ngroups) return;
  const int per_rhs = zm.ngx * zm.ngy;
  const int rhs = group / per_rhs;
  const int rem = group - rhs * per_rhs;
  const int gx = rem / zm.ngy, gy = rem - (rem / zm.ngy) * zm.ngy;
  const int mxm = member & 1, mym = member >> 1;
  const int xt = mxm ? zm.NX - 1 - gx : gx;
  if (mxm && xt == gx) return;
  const int jj = mym ? a.Jpp - gy : gy;
  if (mym && (gy == 0 || jj == gy)) return;
  if (active && !active[rhs]) return;
  const int c = threadIdx.x / (T * TX);
  const int rr = threadIdx.x - c * (T * TX);
  const int l = rr % TX, t = rr / TX;
  const int i = xt * TX + l;
  const long plane = (long)a.Jpp * a.Kpp;
  const bool ok = i < a.Kpp;
  cx<R>* pl = lds + c * N * TX;
  cx<R> v[E];
  {
    const cx<R>* src = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      v[m] = (ok && e < a.P) ? src[e * plane] : mk((R)0, (R)0);
    }
  }
  fast_fft<R, false, N>(v, t, pl, TX, l, tw);
  // spectra of all three components at this thread's positions
#pragma unroll
  for (int m = 0; m < E; ++m) pl[(t + T * m) * TX + l] = v[m];
  __syncthreads();
  if (ok) {
    const int jm = min(jj, a.Jpp - jj);
    const bool my = jj > a.Jpp - jj;
    const int im = min(i, a.Kpp - i);
    const bool mx = i > a.Kpp - i;
    // row c of the symmetric tensor: components (c,0), (c,1), (c,2)
    const int u0 = c == 0 ? 0 : (c == 1 ? 1 : 2);
    const int u1 = c == 0 ? 1 : (c == 1 ? 3 : 4);
    const int u2 = c == 0 ? 2 : (c == 1 ? 4 : 5);
    const int sx0 = (mx ? c_sign[0][u0] : 1) * (my ? c_sign[1][u0] : 1);
    const int sx1 = (mx ? c_sign[0][u1] : 1) * (my ? c_sign[1][u1] : 1);
    const int sx2 = (mx ? c_sign[0][u2] : 1) * (my ? c_sign[1][u2] : 1);
    const long cs = (long)a.Ph * a.Jh * a.Kh;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      const int km = min(e, N - e);
      const bool mz = e > N - e;
      const cx<R>* ys = Y + ((long)km * a.Jh + jm) * a.Kh + im;
      cx<R> y0 = ys[u0 * cs], y1 = ys[u1 * cs], y2 = ys[u2 * cs];
      if (sx0 * (mz ? c_sign[2][u0] : 1) < 0) y0 = mk(-y0.x, -y0.y);
      if (sx1 * (mz ? c_sign[2][u1] : 1) < 0) y1 = mk(-y1.x, -y1.y);
      if (sx2 * (mz ? c_sign[2][u2] : 1) < 0) y2 = mk(-y2.x, -y2.y);
      const int q = e * TX + l;
      v[m] = y0 * lds[q] + y1 * lds[N * TX + q] + y2 * lds[2 * N * TX + q];
    }
  }
  __syncthreads();  // every group has read the spectra before its plane is reused
  fast_fft<R, true, N>(v, t, pl, TX, l, tw);
  if (!ok) return;
  cx<R>* dst = G2 + ((long)(rhs * 3 + c) * a.P) * plane + (long)jj * a.Kpp + i;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    if (e < a.P) dst[e * plane] = v[m];
  }
}

// ===========================================================================
// Fused xy-plane passes (lattices whose padded x and y lengths are equal, NN).
//
// Forward: one z-plane k of one component, restricted to the y frequencies
// j'' = D q + py (q < M = NN/D).  Since
//   Y[D q + py] = sum_{j1<M} w_M^{q j1} sum_{j2} X[j1 + M j2] w_NN^{py (j1 + M j2)},
// the block expands its plane (Sec. 4), folds and pre-twiddles each column,
// runs an M-point DFT along y (Sec. 3: only the K*P lines that hold data),
// transposes through LDS and runs the NN-point DFT along x on its M rows
// (K non-zeros each), writing those rows of G2.  No block depends on
// another; the D blocks of one plane read the same input and are dealt to the
// same XCD in consecutive slots.
//
// Inverse: one plane, restricted to the x outputs i = D q + rx:
//   x[D q + rx] = sum_{k1<M} w_M^{-k1 q} sum_{k2} X[k1 + M k2] w_NN^{-(k1 + M k2) rx},
// so the block folds each G2 row, runs an M-point inverse DFT along x keeping
// the outputs i < K, transposes, runs the NN-point inverse DFT along y keeping
// j < J, normalises, compresses and adds the diagonal (with the fused inner
// products of the solver).
// ===========================================================================
template <int D>
__device__ __forceinline__ void xcd_member(int b, int& group, int& member) {
  const int xcd = b & 7, slot = b >> 3;
  member = slot % D;
  group = (slot / D) * 8 + xcd;
}

template <typename R, int NN, int D>
struct XYPlan {
  static constexpr int M = NN / D;
  static constexpr int TB = 256;
  static constexpr int EA = FastPlan<M>::E, TA = FastPlan<M>::T;  // M-point transforms
  static constexpr int CA = TB / TA;                              // columns per chunk
  static constexpr int EB = FastPlan<NN>::E, TBT = FastPlan<NN>::T;  // NN-point transforms
  static constexpr int RB = TB / TBT;                                // rows per chunk
  static constexpr int LSB = NN + NN / 8 + 1;                        // padded row stride
};

template <typename R, int NN, int D>
__global__ void __launch_bounds__(256) k_xy_fwd(const cx<R>* __restrict__ x, cx<R>* __restrict__ G2,
                                                OccBits map, const cx<R>* __restrict__ a0,
                                                const cx<R>* __restrict__ a1, const double* __restrict__ S,
                                                const int* __restrict__ active, VecArgs a, int ngroups,
                                                const cx<R>* __restrict__ twy, const cx<R>* __restrict__ twx) {
  using PL = XYPlan<R, NN, D>;
  constexpr int M = PL::M, EA = PL::EA, TA = PL::TA, CA = PL::CA, EB = PL::EB, TBT = PL::TBT, RB = PL::RB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int KP = ((a.K + CA - 1) / CA) * CA;          // padded row stride: chunks never overlap
  cx<R>* tr = reinterpret_cast<cx<R>*>(smem);       // [M][KP] transpose buffer
  cx<R>* xb = tr + (long)M * KP;                      // [RB][LSB] x-exchange area
  int group, py;
  xcd_member<D>(blockIdx.x, group, py);
  if (group >= ngroups) return;
  const int k = group % a.P, rc = group / a.P, rhs = rc / 3;
  if (active && !active[rhs]) return;
  const R Sr = S ? (R)S[rhs] : (R)0;
  const cx<R>* xv = x + (long)rc * a.nd;
  const int cc = rc % 3;  // this component's diagonal entries
  // phase A: columns i in chunks of CA, M-point DFT along y
  for (int c0 = 0; c0 < a.K; c0 += CA) {
    const int l = threadIdx.x % CA, t = threadIdx.x / CA;
    const int i = c0 + l;
    cx<R> v[EA];
#pragma unroll
    for (int m = 0; m < EA; ++m) {
      const int j1 = t + TA * m;
      cx<R> acc = mk((R)0, (R)0);
      if (i < a.K) {
        for (int j = j1; j < a.J; j += M) {
          const int n = site_index(map, (long)k * a.J + j, i);
          if (n >= 0) {
            cx<R> val = xv[n];
            if (a.jacobi) val = jacobi_scale(diag_at(a0, a1, a, cc, n, Sr)) * val;
            acc = acc + val * twy[(py * j) % NN];
          }
        }
      }
      v[m] = acc;
    }
    // exchange inside this chunk's own columns of the transpose buffer
    fast_fft<R, false, M, 0, D>(v, t, tr + c0, KP, l, twy);
#pragma unroll
    for (int m = 0; m < EA; ++m) tr[(long)(t + TA * m) * KP + i] = v[m];
  }
  __syncthreads();
  // phase B: rows q in chunks of RB, NN-point DFT along x (K non-zeros)
  const int plane_row = a.Kpp;
  cx<R>* g2 = G2 + ((long)rc * a.P + k) * a.Jpp * plane_row;
  for (int r0 = 0; r0 < M; r0 += RB) {
    const int rw = threadIdx.x / TBT, t = threadIdx.x % TBT;
    const int q = r0 + rw;
    cx<R> v[EB];
#pragma unroll
    for (int m = 0; m < EB; ++m) {
      const int e = t + TBT * m;
      v[m] = (q < M && e < a.K) ? tr[(long)q * KP + e] : mk((R)0, (R)0);
    }
    fast_fft<R, false, NN, 3>(v, t, xb, 1, rw * PL::LSB, twx);
    if (q < M) {
      cx<R>* dst = g2 + (long)(D * q + py) * plane_row;
#pragma unroll
      for (int m = 0; m < EB; ++m) dst[t + TBT * m] = v[m];
    }
  }
}

template <typename R, int NN, int D>
__global__ void __launch_bounds__(256) k_xy_inv(const cx<R>* __restrict__ G2, const cx<R>* __restrict__ x,
                                                cx<R>* __restrict__ y, OccBits map,
                                                const cx<R>* __restrict__ a0, const cx<R>* __restrict__ a1,
                                                const double* __restrict__ S, const int* __restrict__ active,
                                                VecArgs a, int ngroups, const cx<R>* __restrict__ twy,
                                                const cx<R>* __restrict__ twx, DotArgs dt) {
  using PL = XYPlan<R, NN, D>;
  constexpr int M = PL::M;
  // x inverse: M-point transforms on rows; y inverse: NN-point on columns
  constexpr int EX = FastPlan<M>::E, TXT = FastPlan<M>::T, RX = 256 / TXT, LSX = M + M / 8 + 1;
  constexpr int EY = FastPlan<NN>::E, TY = FastPlan<NN>::T, CY = 256 / TY;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Q = (a.K + D - 1) / D;                    // x outputs per residue (upper bound)
  const int QP = ((Q + CY - 1) / CY) * CY;            // padded row stride: chunks never overlap
  cx<R>* tr = reinterpret_cast<cx<R>*>(smem);       // [NN][QP] transpose buffer
  cx<R>* xb = tr + (long)NN * QP;                     // [RX][LSX] x-exchange area
  int group, rx;
  xcd_member<D>(blockIdx.x, group, rx);
  c64 d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
  if (group >= ngroups) return;
  const int k = group % a.P, rc = group / a.P, rhs = rc / 3;
  if (active && !active[rhs]) return;
  const cx<R>* g2 = G2 + ((long)rc * a.P + k) * a.Jpp * a.Kpp;
  // phase B': rows j'' in chunks of RX; fold, M-point inverse DFT along x
  for (int r0 = 0; r0 < NN; r0 += RX) {
    const int rw = threadIdx.x / TXT, t = threadIdx.x % TXT;
    const int jr = r0 + rw;
    cx<R> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int k1 = t + TXT * m;
      cx<R> acc = mk((R)0, (R)0);
      if (jr < NN) {
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) {
          const int kk = k1 + M * k2;
          cx<R> w = twx[(kk * rx) % NN];
          w.y = -w.y;
          acc = acc + g2[(long)jr * a.Kpp + kk] * w;
        }
      }
      v[m] = acc;
    }
    fast_fft<R, true, M, 3, D>(v, t, xb, 1, rw * LSX, twx);
    if (jr < NN) {
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        const int q = t + TXT * m;
        if (q < QP) tr[(long)jr * QP + q] = v[m];
      }
    }
  }
  __syncthreads();
  // phase A': columns q in chunks of CY; NN-point inverse DFT along y
  const R Sr = S ? (R)S[rhs] : (R)0;
  const R sc = (R)a.scale;
  const cx<R>* xv = x + (long)rc * a.nd;
  const int cc = rc % 3;  // this component's diagonal entries
  cx<R>* yv = y + (long)rc * a.nd;
  for (int c0 = 0; c0 < Q; c0 += CY) {
    const int l = threadIdx.x % CY, t = threadIdx.x / CY;
    const int q = c0 + l;
    cx<R> v[EY];
#pragma unroll
    for (int m = 0; m < EY; ++m) v[m] = (q < Q) ? tr[(long)(t + TY * m) * QP + q] : mk((R)0, (R)0);
    // the transform exchanges through these same columns: every load first
    __syncthreads();
    fast_fft<R, true, NN>(v, t, tr + c0, QP, l, twy);
    const int i = D * q + rx;
    if (q < Q && i < a.K) {
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const int j = t + TY * m;
        if (j >= a.J) continue;
        const int n = site_index(map, (long)k * a.J + j, i);
        if (n < 0) continue;
        const cx<R> conv = sc * v[m];
        const cx<R> dg = diag_at(a0, a1, a, cc, n, Sr);
        const cx<R> xn = xv[n];
        const cx<R> yn = a.jacobi ? xn + jacobi_scale(dg) * conv : dg * xn + conv;
        yv[n] = yn;
        dot_term(dt, xn, yn, (long)rc * a.nd + n, d0, d1);
      }
    }
  }
  if (dt.mode != DOT_NONE) {
    block_sum2_any(d0, d1);
    if (threadIdx.x == 0) {
      const long nblk = 3L * a.P * D;
      const long blk = ((long)(rc - 3 * rhs) * a.P + k) * D + rx;
      dt.part[((long)rhs * nblk + blk) * 2] = d0;
      dt.part[((long)rhs * nblk + blk) * 2 + 1] = d1;
    }
  }
}

// ===========================================================================
// Five-pass schedule with z-contiguous lines.
//
// The x-forward pass writes its output transposed, G2t[rhs][c][j''][i''][k]
// (k = z fastest), through an LDS transpose, so that every z line of the
// middle pass is one contiguous run of P values and the inverse x pass reads
// it back the same way.  The z pass reads the spectrum in the matching
// z-fastest copy Yz[c][j_h][i_h][k_h].
// ===========================================================================
template <typename R, int N>
constexpr int xt_rows() {
  constexpr int T = FastPlan<N>::T;
  constexpr int want = sizeof(R) == 4 ? 16 : 8;  // 128-byte runs of k
  return (T * want <= 512) ? want : (512 / T > 0 ? 512 / T : 1);
}

// x forward: G1 rows (k0..k0+RK, j'') of K values -> N-point DFT -> G2t.
// grid = (ceil(P/RK), J'', nrhs*3); block RK*T, lane = row*T + t.
template <typename R, int N, int RK>
__global__ void __launch_bounds__(FastPlan<N>::T * RK) k_xT_fwd(const cx<R>* __restrict__ G1, cx<R>* __restrict__ G2t,
                                                               int K, int P, int Jpp, const int* __restrict__ active,
                                                               const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T, LS = N + N / 8 + 1, RKP = RK + 1;
  static_assert(N * RKP <= RK * LS, "transpose stage must fit in the exchange area");
  __shared__ cx<R> lds[RK * LS];
  const int rc = blockIdx.z, jj = blockIdx.y, k0 = blockIdx.x * RK;
  if (active && !active[rc / 3]) return;
  const int rw = threadIdx.x / T, t = threadIdx.x % T;
  const int k = k0 + rw;
  const cx<R>* src = G1 + (((long)rc * P + k) * Jpp + jj) * K;
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    v[m] = (k < P && e < K) ? src[e] : mk((R)0, (R)0);
  }
  fast_fft<R, false, N, 3>(v, t, lds, 1, rw * LS, tw);
  // registers -> [i''][row] in LDS -> coalesced runs of k
#pragma unroll
  for (int m = 0; m < E; ++m) lds[(t + T * m) * RKP + rw] = v[m];
  __syncthreads();
  cx<R>* dst = G2t + (((long)rc * Jpp + jj) * N) * P + k0;
  // E values per thread: every LDS read first, then the E stores
  cx<R> st[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * (T * RK);
    st[q] = lds[(idx / RK) * RKP + idx % RK];
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * (T * RK);
    const int r = idx % RK, i = idx / RK;
    if (k0 + r < P) dst[(long)i * P + r] = st[q];
  }
}

// x inverse: G2t (N values per (j'', k) line, read as runs of k) -> N-point
// inverse DFT -> first K values of G1 rows.
template <typename R, int N, int RK>
__global__ void __launch_bounds__(FastPlan<N>::T * RK) k_xT_inv(const cx<R>* __restrict__ G2t, cx<R>* __restrict__ G1,
                                                               int K, int P, int Jpp, const int* __restrict__ active,
                                                               const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T, LS = N + N / 8 + 1, RKP = RK + 1;
  static_assert(N * RKP <= RK * LS, "transpose stage must fit in the exchange area");
  __shared__ cx<R> lds[RK * LS];
  const int rc = blockIdx.z, jj = blockIdx.y, k0 = blockIdx.x * RK;
  if (active && !active[rc / 3]) return;
  const cx<R>* src = G2t + (((long)rc * Jpp + jj) * N) * P + k0;
  // the block's N x RK values are E per thread: all E loads are issued
  // before the first LDS store, so they are in flight together
  cx<R> ld[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * (T * RK);
    const int r = idx % RK, i = idx / RK;
    ld[q] = (k0 + r < P) ? src[(long)i * P + r] : mk((R)0, (R)0);
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * (T * RK);
    lds[(idx / RK) * RKP + idx % RK] = ld[q];
  }
  __syncthreads();
  const int rw = threadIdx.x / T, t = threadIdx.x % T;
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = lds[(t + T * m) * RKP + rw];
  __syncthreads();  // the transform exchanges through the same LDS
  fast_fft<R, true, N, 3>(v, t, lds, 1, rw * LS, tw);
  const int k = k0 + rw;
  if (k >= P) return;
  cx<R>* dst = G1 + (((long)rc * P + k) * Jpp + jj) * K;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    if (e < K) dst[e] = v[m];
  }
}

template <typename R, int N>
constexpr int zline_rows() {
  constexpr int T = FastPlan<N>::T, LS = N + N / 8 + 1;
  int rl = 512 / T;
  if (rl > 16) rl = 16;
  while (rl > 1 && 3 * rl * LS * (int)sizeof(cx<R>) > 56 * 1024) rl /= 2;
  return rl < 1 ? 1 : rl;
}

// z lines with the spectral product (Eqs. Q0-Q2; mirrored octant of the
// z-fastest spectrum with Table 1 signs), in place on G2t.  Blocks take RL
// consecutive lines i'' at one j''; mirror quadruples of line tiles share
// spectrum rows and are dealt to one XCD in consecutive slots.
// components per 16-byte record of the z-fastest spectrum copy (k_spec_zfast)
template <typename R>
__host__ __device__ constexpr int yz_group() {
  return 16 / (int)sizeof(cx<R>);
}

template <typename R, int N, int RL>
__global__ void __launch_bounds__(FastPlan<N>::T * RL) k_zline(cx<R>* __restrict__ G2t, const cx<R>* __restrict__ Yz,
                                                              const int* __restrict__ active, ZArgs a, ZMap zm,
                                                              const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T, LS = N + N / 8 + 1;
  __shared__ cx<R> lds[3 * RL * LS];
  const int b = blockIdx.x;
  const int group = (b >> 5) * 8 + (b & 7);
  const int member = (b >> 3) & 3;
  if (group >= zm.ngroups) return;
  const int per_rhs = zm.ngx * zm.ngy;
  const int rhs = group / per_rhs;
  const int rem = group - rhs * per_rhs;
  const int gx = rem / zm.ngy, gy = rem - (rem / zm.ngy) * zm.ngy;
  const int mxm = member & 1, mym = member >> 1;
  const int xt = mxm ? zm.NX - 1 - gx : gx;
  if (mxm && xt == gx) return;
  const int jj = mym ? a.Jpp - gy : gy;
  if (mym && (gy == 0 || jj == gy)) return;
  if (active && !active[rhs]) return;
  const int ln = threadIdx.x / T, t = threadIdx.x % T;
  const int i = xt * RL + ln;
  const bool ok = i < a.Kpp;
  const long cstride = (long)a.Jpp * a.Kpp * a.P;  // one component of one right-hand side
  const long line = ((long)jj * a.Kpp + i) * a.P;
  cx<R> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R>* src = G2t + (long)(rhs * 3 + c) * cstride + line;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      v[c][m] = (ok && e < a.P) ? src[e] : mk((R)0, (R)0);
    }
  }
  FastStages3<R, false, N, FastPlan<N>::S, 3>::template run<0>(v, t, lds, 1, ln * LS, RL * LS, tw);
  if (ok) {
    const int jm = min(jj, a.Jpp - jj);
    const bool my = jj > a.Jpp - jj;
    const int im = min(i, a.Kpp - i);
    const bool mx = i > a.Kpp - i;
    int sxy[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sxy[c] = (mx ? c_sign[0][c] : 1) * (my ? c_sign[1][c] : 1);
    constexpr int V = yz_group<R>();
    const cx<R>* yrow = Yz + ((long)jm * a.Kh + im) * a.Ph * 6;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      const int km = min(e, N - e);
      const bool mz = e > N - e;
      cx<R> yv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int sg = sxy[c] * (mz ? c_sign[2][c] : 1);
        const cx<R> w = yrow[((c / V) * a.Ph + km) * V + c % V];
        yv[c] = sg < 0 ? mk(-w.x, -w.y) : w;
      }
      const cx<R> x0 = v[0][m], x1 = v[1][m], x2 = v[2][m];
      v[0][m] = yv[0] * x0 + yv[1] * x1 + yv[2] * x2;
      v[1][m] = yv[1] * x0 + yv[3] * x1 + yv[4] * x2;
      v[2][m] = yv[2] * x0 + yv[4] * x1 + yv[5] * x2;
    }
  }
  FastStages3<R, true, N, FastPlan<N>::S, 3>::template run<0>(v, t, lds, 1, ln * LS, RL * LS, tw);
  if (!ok) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R>* dst = G2t + (long)(rhs * 3 + c) * cstride + line;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + T * m;
      if (e < a.P) dst[e] = v[c][m];
    }
  }
}

// z-fastest copy of the spectrum: per (j, i) column the six components in
// groups of V = 16 / sizeof(cx<R>) (two FP32, one FP64), each group's z
// frequencies consecutive with the group's V values together:
// Yz[j][i][c / V][k][c % V] = Y[c][k][j][i].  One 16-byte load of the T
// lanes of a z line then reads T consecutive records.
template <typename R>
__global__ void k_spec_zfast(const cx<R>* __restrict__ Y, cx<R>* __restrict__ Yz, int Kh, int Jh, int Ph) {
  constexpr int V = yz_group<R>(), G = 6 / V;
  const long n = 6L * Ph * Jh * Kh;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < n; g += (long)gridDim.x * blockDim.x) {
    const int v = (int)(g % V);
    long r = g / V;
    const int k = (int)(r % Ph);
    r /= Ph;
    const int grp = (int)(r % G);
    r /= G;
    const int i = (int)(r % Kh);
    const int j = (int)(r / Kh);
    const int c = grp * V + v;
    Yz[g] = Y[(((long)c * Ph + k) * Jh + j) * Kh + i];
  }
}

}  // namespace dda
