// Register-resident DFTs of compile-time length and the two-level column
// transform built on them.
//
// RDft<R, INV, L, NZ>: an L-point DFT of values held in registers, natural
// order in and out, whose inputs beyond the first NZ are known to be zero
// (the zero-padded halves of the lines of Sec. 3 are never loaded or added).
// Lengths 2, 3, 4, 5, 8 are the butterflies of fft_core.hpp; longer lengths
// split as L = A B (input m = m1 + A m2, output k = k2 + B k1):
//   X[k2 + B k1] = sum_{m1} w_A^{m1 k1} w_L^{m1 k2} sum_{m2} x[m1 + A m2] w_B^{m2 k2},
// all twiddles compile-time constants.  Outputs a caller never reads are
// removed by the compiler, so a transform that only needs its first outputs
// (the inverse lines of Sec. 3 keep k < P) costs less automatically.
//
// Two-level column transform of length N = T E (T threads per column, E
// values each; thread t holds x[t + T m]):
//   X[k1 + E k2] = sum_t w_T^{t k2} [ w_N^{t k1} sum_m x[t + T m] w_E^{m k1} ]
// = an E-point DFT in each thread, a twiddle, one exchange through LDS, and
// T-point DFTs in registers.  Thread t' then holds the E frequencies
// k1 + E k2 with k1 = t' + T q (q < E/T, so E must be a multiple of T), in
// this scrambled order: the spectral product is pointwise, and the inverse
// runs the same steps backwards from there, so neither direction reorders.
#pragma once
#include <utility>

#include "fft_core.hpp"
#include "fft_fast.hpp"
#include "kernels_fft.hpp"

namespace dda {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------
template <typename F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0..N-1, each i a constant expression
template <int N, typename F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;
// Taylor series on [0, pi/4]: the terms after x^27 are below 1e-22
constexpr double sin_q(double x) {
  double t = x, s = x;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    s += t;
  }
  return s;
}
constexpr double cos_q(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    s += t;
  }
  return s;
}
// cos and sin of 2 pi j / L, reduced to an octant so that the series argument
// stays in [0, pi/4]; quarter turns are exact
constexpr void cis(int j, int L, double& c, double& s) {
  j %= L;
  if (j < 0) j += L;
  const long e = 8L * j;
  const int o = (int)(e / L);
  const long r = e - (long)o * L;  // 0 <= r < L
  const double f = kPi / 4.0 * ((double)r / (double)L);
  const double g = kPi / 4.0 * ((double)(L - r) / (double)L);
  switch (o) {
    case 0: c = cos_q(f); s = sin_q(f); break;
    case 1: c = sin_q(g); s = cos_q(g); break;
    case 2: c = -sin_q(f); s = cos_q(f); break;
    case 3: c = -cos_q(g); s = sin_q(g); break;
    case 4: c = -cos_q(f); s = -sin_q(f); break;
    case 5: c = -sin_q(g); s = -cos_q(g); break;
    case 6: c = sin_q(f); s = -cos_q(f); break;
    default: c = cos_q(g); s = -sin_q(g); break;
  }
  if (r == 0) {  // exact multiples of pi/4 with zero or unit parts
    if (o == 0) { c = 1.0; s = 0.0; }
    if (o == 2) { c = 0.0; s = 1.0; }
    if (o == 4) { c = -1.0; s = 0.0; }
    if (o == 6) { c = 0.0; s = -1.0; }
  }
}
constexpr double cosv(int j, int L) { double c = 0, s = 0; cis(j, L, c, s); return c; }
constexpr double sinv(int j, int L) { double c = 0, s = 0; cis(j, L, c, s); return s; }
}  // namespace ct

// v * w_L^J with w_L = exp(-2 pi i / L) (forward) or its conjugate (inverse)
template <typename R, bool INV, int J, int L>
__host__ __device__ __forceinline__ cx<R> twc(cx<R> v) {
  constexpr int j = ((J % L) + L) % L;
  if constexpr (j == 0) {
    return v;
  } else if constexpr (4 * j == L) {
    return rot90<R, INV>(v);  // -i forward, +i inverse
  } else if constexpr (2 * j == L) {
    return mk(-v.x, -v.y);
  } else if constexpr (4 * j == 3 * L) {
    return rot90<R, !INV>(v);
  } else if constexpr (8 * j == L || 8 * j == 3 * L || 8 * j == 5 * L || 8 * j == 7 * L) {
    // odd eighths: (+-h, +-h) with h = 1/sqrt(2)
    constexpr R h = (R)DDA_SQRT1_2;
    constexpr int o = 8 * j / L;
    constexpr R c = (o == 1 || o == 7) ? h : -h;
    constexpr R s0 = (o == 1 || o == 3) ? h : -h;  // sin(2 pi j / L)
    constexpr R s = INV ? s0 : -s0;                  // imaginary part of the twiddle
    return mk(c * v.x - s * v.y, c * v.y + s * v.x);
  } else {
    constexpr R c = (R)ct::cosv(j, L);
    constexpr R s = INV ? (R)ct::sinv(j, L) : (R)(-ct::sinv(j, L));
    return mk(c * v.x - s * v.y, c * v.y + s * v.x);
  }
}

// factor of a composite length: B = 2 when at least the upper half of the
// inputs is zero (the inner transforms are then copies), else a fixed split
template <int L, int NZ>
struct RSplit {
  static constexpr int B = (L % 2 == 0 && 2 * NZ <= L) ? 2
                           : L == 16 ? 4 : L == 12 ? 3 : L == 24 ? 3 : L == 32 ? 4 : L == 6 ? 3 : L == 64 ? 8
                           : L == 48 ? 3 : L == 8 ? 2 : L == 4 ? 2 : 0;
  static_assert(B > 0, "no register DFT for this length");
  static constexpr int A = L / B;
};

template <typename R, bool INV, int L, int NZ>
struct RDft {
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    static_assert(NZ >= 1 && NZ <= L, "non-zero inputs");
    if constexpr (L == 1) {
    } else if constexpr (NZ == 1) {
#pragma unroll
      for (int k = 1; k < L; ++k) v[k] = v[0];
    } else if constexpr ((L == 2 || L == 3 || L == 4 || L == 5 || L == 8) && !(L % 2 == 0 && 2 * NZ <= L)) {
#pragma unroll
      for (int m = NZ; m < L; ++m) v[m] = mk((R)0, (R)0);  // a few zeros: the plain butterfly
      dft_small<L, R, INV>(v);
    } else {
      constexpr int B = RSplit<L, NZ>::B, A = L / B;
      constexpr int NO = NZ < A ? NZ : A;  // outer inputs m1 < NO are the non-zero ones
      cx<R> w[A * B];
      sfor<NO>([&](auto m1c) {
        constexpr int m1 = decltype(m1c)::value;
        constexpr int nzi0 = (NZ - m1 + A - 1) / A;
        constexpr int nzi = nzi0 < B ? nzi0 : B;
        cx<R> u[B];
#pragma unroll
        for (int m2 = 0; m2 < nzi; ++m2) u[m2] = v[m1 + A * m2];
        RDft<R, INV, B, nzi>::run(u);
        sfor<B>([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          w[m1 * B + k2] = twc<R, INV, m1 * k2, L>(u[k2]);
        });
      });
      sfor<B>([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        cx<R> s[A];
#pragma unroll
        for (int m1 = 0; m1 < NO; ++m1) s[m1] = w[m1 * B + k2];
        RDft<R, INV, A, NO>::run(s);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) v[k2 + B * k1] = s[k1];
      });
    }
  }
};

// Buffer accesses of complex values: a resource (uniform base and byte
// range, in SGPRs) and a 32-bit per-lane byte offset.  An offset at or past
// the range loads zero and drops the store (the hardware's range check), which
// serves the padded rows and the ragged column tiles without branches.
constexpr int kBufDword3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9 family)
using brsrc = __amdgpu_buffer_rsrc_t;
template <typename R>
__device__ __forceinline__ brsrc make_rsrc(const cx<R>* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<R>*>(base), (short)0, (int)bytes, kBufDword3);
}
template <typename R>
__device__ __forceinline__ cx<R> bload(brsrc r, unsigned off) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_bit_cast(cx<R>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  } else {
    return __builtin_bit_cast(cx<R>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  }
}
template <typename R>
__device__ __forceinline__ void bstore(brsrc r, unsigned off, cx<R> v) {
  if constexpr (sizeof(R) == 4) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)off, 0, 0);
  } else {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, (int)off, 0, 0);
  }
}
constexpr unsigned kOutOfRange = 0x80000000u;  // byte offset past every range used here

// the six spectrum components of one frequency from the z-fastest copy
// (k_spec_zfast): 16-byte records (two FP32 components, one FP64) at
// off + g gstride, g = 0 .. 6/V - 1 (the uniform part g gstride goes in the
// load's scalar offset, so the six loads share one address register)
template <typename R>
__device__ __forceinline__ void bload6(brsrc r, unsigned off, unsigned gstride, cx<R> (&y)[6]) {
  if constexpr (sizeof(R) == 4) {
    // the loaded vector is bit-cast whole (element access on it compiled to
    // a one-dword load broadcast to all four)
    struct Pair {
      cx<float> a, b;
    };
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      const Pair q = __builtin_bit_cast(Pair, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)(h * gstride), 0));
      y[2 * h] = q.a;
      y[2 * h + 1] = q.b;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 6; ++u)
      y[u] = __builtin_bit_cast(cx<R>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)(u * gstride), 0));
  }
}

// ---------------------------------------------------------------------------
// z pass with the spectral product on the two-level transform (Sec. 3 z lines;
// Eqs. Q0-Q2 with the mirrored octant and Table 1 signs), in place on G2.
//
// Every wavefront owns CW = 64/T adjacent columns i'' of one y row j''
// (lane = t CW + c, so each row of its columns is one run of CW values) and
// exchanges only among its own lanes: the LDS accesses of one wavefront are
// performed in order, so the exchanges need no block barrier and the
// wavefronts of a block run independently.  A block's W wavefronts cover a
// tile of W CW columns and run it for RB right-hand sides in turn, so the
// spectrum entries it gathers are reused from the caches.  Per right-hand
// side and component: E-point DFT of the P <= N/2 loaded values (the upper
// half of each thread's inputs is the zero padding), twiddle, exchange,
// T-point DFTs; product; the same steps backwards, storing z < P.  Mirror
// quadruples of column tiles share their spectrum entries and are dealt to
// one XCD in consecutive slots (as in k_fast_zmul).
//
// BLK selects the layout of the x-transformed array.  false: [rhs][3][P][J''][K'']
// (the rows of a column tile lie a whole z plane apart).  true: tile-blocked,
// [rhs][3][J''][NT][P][C] with NT = ceil(K''/C): each tile's P x C values are
// one contiguous run, which the strided plane rows are not (a plain in-place
// pass over 64-512 B runs a plane apart measured 2.5-3.5 TB/s against 5.5
// TB/s for a contiguous copy of the same 201 MB at the 128^3 sphere); the x
// passes k_xb write and read it RW rows at a time, RW x C contiguous values
// per tile.
// ---------------------------------------------------------------------------
struct Z2Map {
  int NX;       // column tiles covering [0, K'')
  int ngx;      // tile pairs (t, NX-1-t)
  int ngy;      // y pairs (j, J''-j), j in [0, J_h)
  int ngroups;  // nrg * ngx * ngy
  int nrhs;     // right-hand sides
  int RB;       // right-hand sides per block
};

// LDS exchange area of one wavefront: element (k1, s, c) at k1 RP + s CW + c.
// The pitch RP = 64 + CW puts the CW-lane groups of a read (one k1 each) on
// consecutive bank ranges, so neither the writes nor the reads conflict.
// WPE wavefronts per SIMD (Z2Shape): two leave up to 256 registers, so more
// of the spectrum gathers stay in flight, which measured faster than three
// at 168 for four-wavefront blocks (FP32 at the 128^3 sphere: 235 against
// 271 us, before the spectrum components were interleaved).
template <typename R, int N, int T, int W, bool BLK, int WPE>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_z2(cx<R>* __restrict__ G2, const cx<R>* __restrict__ Yz,
                                              const int* __restrict__ active, ZArgs a, Z2Map zm,
                                              const cx<R>* __restrict__ tw) {
  constexpr int E = N / T, Q = E / T, HE = E / 2, CW = 64 / T, C = W * CW, RP = 64 + CW;
  constexpr unsigned SZ = sizeof(cx<R>);
  static_assert(E % T == 0 && E % 2 == 0 && 64 % T == 0, "two-level split");
  __shared__ cx<R> xb[W * E * RP];  // one exchange area per wavefront (one component at a time)
  __shared__ cx<R> tws[N];          // tws[k1 T + t] = w_N^{t k1}
  const int b = blockIdx.x;
  const int group = (b >> 5) * 8 + (b & 7);
  const int member = (b >> 3) & 3;
  if (group >= zm.ngroups) return;
  const int per_rg = zm.ngx * zm.ngy;
  const int rg = group / per_rg;
  const int rem = group - rg * per_rg;
  const int gx = rem / zm.ngy, gy = rem - (rem / zm.ngy) * zm.ngy;
  const int mxm = member & 1, mym = member >> 1;
  const int xt = mxm ? zm.NX - 1 - gx : gx;
  if (mxm && xt == gx) return;
  const int jj = mym ? a.Jpp - gy : gy;
  if (mym && (gy == 0 || jj == gy)) return;
  const int r0 = rg * zm.RB, r1 = min(zm.nrhs, r0 + zm.RB);
  if (active) {  // a block none of whose right-hand sides is active leaves at once
    bool any = false;
    for (int q = r0; q < r1 && !any; ++q) any = active[q] != 0;
    if (!any) return;
  }
  for (int e = threadIdx.x; e < N; e += blockDim.x) tws[e] = tw[(e % T) * (e / T)];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane % CW, t = lane / CW;
  const int i = xt * C + wv * CW + c;
  const bool ok = i < a.Kpp;
  const unsigned plane = (unsigned)a.Jpp * (unsigned)a.Kpp;
  // byte offset of row t of this column in a component's slab ([P][J''][K''],
  // or the tile's [P][C] when blocked); rows z >= P fall past the slab's
  // range and read as zero
  const unsigned vo = !ok ? kOutOfRange
                          : BLK ? ((unsigned)t * C + (unsigned)(wv * CW + c)) * SZ
                                : ((unsigned)t * plane + (unsigned)(jj * a.Kpp + i)) * SZ;
  const unsigned mstep = BLK ? (unsigned)T * C * SZ : (unsigned)T * plane * SZ;
  const unsigned slab = BLK ? (unsigned)a.P * C * SZ : (unsigned)a.P * plane * SZ;
  cx<R>* const xwv = xb + wv * (E * RP);
  cx<R>* const xw = xwv + t * CW + c;       // (k1, t): xw[k1 RP]
  cx<R>* const xr = xwv + t * RP + c;       // (t + T q, s): xr[q T RP + s CW]
  const cx<R>* const twp = tws + t;         // w_N^{t k1}: twp[k1 T]
  // mirrored octant of this column and the Table 1 signs of its x, y mirrors
  const int jm = min(jj, a.Jpp - jj), im = min(i, a.Kpp - i);
  const bool my = jj > a.Jpp - jj, mx = i > a.Kpp - i;
  int sxy[6];
#pragma unroll
  for (int u = 0; u < 6; ++u) sxy[u] = (mx ? c_sign[0][u] : 1) * (my ? c_sign[1][u] : 1);
  const unsigned cs = (unsigned)a.Ph * a.Jh * a.Kh;
  // the spectrum's z-fastest copy (k_spec_zfast): the T lanes of a column
  // gather T consecutive z frequencies, one run instead of T rows (measured
  // 185 against 240 us for the FP32 pass at the 128^3 sphere), and FP32
  // takes two components per 16-byte load
  const unsigned yl = (unsigned)(jm * a.Kh + im) * (unsigned)a.Ph * 6 * SZ;
  const unsigned ygs = (unsigned)a.Ph * 16;  // one component group's run
  const brsrc yr = make_rsrc(Yz, 6 * cs * SZ);
  __syncthreads();  // twiddle table ready; from here on the wavefronts are independent
  for (int rhs = r0; rhs < r1; ++rhs) {
    if (active && !active[rhs]) continue;
    brsrc gr[3];
#pragma unroll
    for (int u = 0; u < 3; ++u)
      gr[u] = make_rsrc(BLK ? G2 + ((((size_t)(rhs * 3 + u) * a.Jpp + jj) * zm.NX + xt) * a.P) * C
                            : G2 + (size_t)(rhs * 3 + u) * a.P * plane,
                        slab);
    cx<R> v[3][E];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int m = 0; m < HE; ++m) v[u][m] = bload<R>(gr[u], vo + m * mstep);
    // forward: E-point DFTs (upper half zero), twiddle w_N^{t k1}, exchange,
    // T-point DFTs; afterwards v[u][q T + k2] = X[k1 + E k2], k1 = t + T q
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      RDft<R, false, E, HE>::run(v[u]);
#pragma unroll
      for (int k1 = 1; k1 < E; ++k1) v[u][k1] = v[u][k1] * twp[k1 * T];
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) xw[k1 * RP] = v[u][k1];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T; ++s) v[u][q * T + s] = xr[q * T * RP + s * CW];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < Q; ++q) RDft<R, false, T, T>::run(&v[u][q * T]);
    }
    // Q_a = sum_b Y_ab X_b at every frequency (Eqs. Q0-Q2)
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k2 = 0; k2 < T; ++k2) {
        const int f = t + T * q + E * k2;
        const int km = min(f, N - f);
        const bool mz = f > N - f;
        cx<R> yv[6];
        bload6<R>(yr, yl + (unsigned)km * 16, ygs, yv);
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          const int sg = sxy[u] * (mz ? c_sign[2][u] : 1);
          if (sg < 0) yv[u] = mk(-yv[u].x, -yv[u].y);
        }
        const int p = q * T + k2;
        const cx<R> x0 = v[0][p], x1 = v[1][p], x2 = v[2][p];
        v[0][p] = yv[0] * x0 + yv[1] * x1 + yv[2] * x2;
        v[1][p] = yv[1] * x0 + yv[3] * x1 + yv[4] * x2;
        v[2][p] = yv[2] * x0 + yv[4] * x1 + yv[5] * x2;
      }
    // inverse: T-point inverse DFTs, exchange back, twiddle w_N^{-t k1},
    // E-point inverse DFT keeping z < P (the first half of each thread's rows)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
#pragma unroll
      for (int q = 0; q < Q; ++q) RDft<R, true, T, T>::run(&v[u][q * T]);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T; ++s) xr[q * T * RP + s * CW] = v[u][q * T + s];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) v[u][k1] = xw[k1 * RP];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int k1 = 1; k1 < E; ++k1) v[u][k1] = v[u][k1] * conjg(twp[k1 * T]);
      RDft<R, true, E, E>::run(v[u]);
#pragma unroll
      for (int m = 0; m < HE; ++m) bstore<R>(gr[u], vo + m * mstep, v[u][m]);
    }
  }
}

// x direction to and from the tile-blocked layout (Sec. 3 x lines): a block
// runs RW consecutive z rows k of one (right-hand side, component, y row j'')
// (lane = row T + t).  Forward: G1 rows [rc][k][j''][K] (K non-zero values)
// -> N-point DFT -> blocked rows (i'' in tile i'' >> lc at column i'' & (C-1),
// C = 2^lc).  Inverse: blocked rows -> N-point inverse DFT -> the first K
// values into G1.
template <typename R, bool INV, int N, int RW>
__global__ void __launch_bounds__(FastPlan<N>::T* RW) k_xb(const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                                         int K, int P, int Jpp, int NT, int lc,
                                                         const int* __restrict__ active,
                                                         const cx<R>* __restrict__ tw) {
  constexpr int E = FastPlan<N>::E, T = FastPlan<N>::T, LS = N + N / 8 + 1;
  __shared__ cx<R> lds[RW * LS];
  const int t = threadIdx.x % T, rw = threadIdx.x / T;
  const int rc = blockIdx.z, jj = blockIdx.y, k = blockIdx.x * RW + rw;
  if (active && !active[rc / 3]) return;  // uniform over the block
  const bool valid = k < P;
  const int cm = (1 << lc) - 1;
  const long g1row = (((long)rc * P + k) * Jpp + jj) * K;
  const long brow = ((long)rc * Jpp + jj) * NT * (long)P * (cm + 1) + (long)k * (cm + 1);
  const long tstep = (long)P * (cm + 1);  // one tile
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    if (INV) v[m] = valid ? in[brow + (e >> lc) * tstep + (e & cm)] : mk((R)0, (R)0);
    else v[m] = (valid && e < K) ? in[g1row + e] : mk((R)0, (R)0);
  }
  fast_fft<R, INV, N, 3>(v, t, lds, 1, rw * LS, tw);
  if (!valid) return;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    if (INV) {
      if (e < K) out[g1row + e] = v[m];
    } else {
      out[brow + (e >> lc) * tstep + (e & cm)] = v[m];
    }
  }
}

// (T, W, WPE) of the two-level z pass per length and layout: E = N/T a
// multiple of T; W wavefronts per block, C = W 64/T columns per tile, WPE
// wavefronts per SIMD.  The tile-blocked layout runs one wavefront per
// block: FP32 with E <= 16 at three per SIMD (the 96 data registers and the
// spectrum gathers fit 168; 146 against 168 us for four wavefronts at two per
// SIMD at the 128^3 sphere), FP64 and E = 24 at two (FP64 312 against 322 us
// at the 128^3 sphere; FP32 length 192, 128 right-hand sides of the 96^3
// ellipsoid, 7.5 against 8.0 ms).  The strided layout keeps four (its rows
// are runs of C values: 220 us with two wavefronts, 276 with one).
// (FP64 with E = 24 is left out: its 16-byte values make the exchange areas
// of a block 110 KB at N = 192, one wavefront per SIMD.)
template <typename R, int N, bool BLK>
struct Z2Shape {
  static constexpr int T0 = N == 16 ? 2 : N == 24 ? 2 : N == 32 ? 4 : N == 48 ? 4 : N == 64 ? 8 : N == 96 ? 4
                            : N == 128 ? 8 : N == 192 ? 8 : N == 256 ? 16 : 0;
  static constexpr int T = (sizeof(R) == 8 && T0 > 0 && N / T0 > 16) ? 0 : T0;
  static constexpr bool ok = T > 0;
  static constexpr bool narrow = BLK && ok;
  static constexpr int W = narrow ? 1 : 4;
  static constexpr int WPE = narrow && sizeof(R) == 4 && N / T <= 16 ? 3 : 2;
  static constexpr int C = ok ? W * 64 / T : 1;
};

}  // namespace dda
