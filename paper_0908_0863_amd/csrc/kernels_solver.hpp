// Krylov-solver kernels: fused vector updates with wavefront reductions that
// accumulate in FP64 whatever the vector precision, and one-block-per-RHS
// finalisers that reduce the partial sums in a fixed order (deterministic) and
// update the per-RHS solver scalars on the device, so the host never waits on
// a scalar inside the iteration.
//
// Vectors are [nrhs][3][N_d]; each right-hand side has its own scalars and an
// `active` flag (0 once converged or stopped) that masks every kernel.
#pragma once
#include "common.hpp"

namespace dda {

constexpr int kRedThreads = 1024;

// Sum of ND complex values over a 256-thread block, in a fixed order.
// Result valid in thread 0.
template <int ND>
__device__ __forceinline__ void block_sum(c64 (&v)[ND]) {
  __shared__ c64 sh[ND][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    double a = v[q].x, b = v[q].y;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (lane == 0) sh[q][wv] = mk(a, b);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      c64 s = sh[q][0];
      for (int w = 1; w < kRedThreads / 64; ++w) s = s + sh[q][w];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Reduce nblk partial blocks of ND sums for right-hand side `rhs` (fixed
// order); result valid in thread 0.
template <int ND>
__device__ __forceinline__ void reduce_partials(const c64* __restrict__ part, int nblk, int rhs, c64 (&v)[ND]) {
#pragma unroll
  for (int q = 0; q < ND; ++q) v[q] = mk(0.0, 0.0);
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const c64* p = part + ((long)rhs * nblk + b) * ND;
#pragma unroll
    for (int q = 0; q < ND; ++q) v[q] = v[q] + p[q];
  }
  block_sum<ND>(v);
}

// complex helpers in FP64 for mixed products
template <typename R>
__device__ __forceinline__ c64 up(cx<R> a) { return mk((double)a.x, (double)a.y); }
__device__ __forceinline__ c64 cmulc(c64 a, c64 b) { return conjg(a) * b; }  // a^H b term

struct SolverDims {
  long n3;    // 3 * N_d elements per right-hand side
  int nblk;   // blocks per right-hand side in the vector kernels
};

// Grid-stride range of this block inside one right-hand side's vector.
#define DDA_RANGE(dims, i)                                                        \
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (dims).n3; \
       i += (long)(dims).nblk * blockDim.x)

// ============================================================================
// Shared pieces of the fused iteration kernels.
//
// Every scalar the next vector update needs is reduced from the partial sums
// of the previous kernel by each block redundantly (the same fixed-order
// reduction in every block, so all blocks agree bit for bit); block 0 writes
// the updated scalars to the *other* state buffer, so no block can observe a
// half-updated state.  The iteration therefore needs no single-block
// finalising launches.
// ============================================================================

// Iterations without a 2% improvement of the best residual after which an
// inner solve is declared stagnated; the refinement loop then restarts from
// the FP64 true residual.  FP32 vectors lose the Lanczos/BiCG relations early
// (a restart is cheaper than a long plateau), so an FP32 solve may stall at
// any level; an FP64 solve only near its rounding level, since plateaus above
// it are ordinary Krylov behaviour at large size parameters.
constexpr int kStallWindow = 64;
template <typename R>
__device__ __forceinline__ double stall_level2() {
  return sizeof(R) == 4 ? 2.0 : 1e-22;  // relative |r|^2 below which a stall counts
}

// Reduce the partials of right-hand side `rhs` and broadcast to every thread.
template <int ND>
__device__ __forceinline__ void reduce_all(const c64* __restrict__ part, int nblk, int rhs, c64 (&v)[ND]) {
  __shared__ c64 bc[ND];
  reduce_partials<ND>(part, nblk, rhs, v);
  if (threadIdx.x == 0)
    for (int q = 0; q < ND; ++q) bc[q] = v[q];
  __syncthreads();
  for (int q = 0; q < ND; ++q) v[q] = bc[q];
}

__device__ __forceinline__ bool tiny(c64 a, double scale) { return !(abs2(a) > 1e-300 * scale); }
// a scalar coefficient that the vector precision R can hold (finite, both parts
// at most R's largest value): an FP32 inner solve overflows far above the
// FP64 breakdown thresholds
template <typename R>
__device__ __forceinline__ bool holds(c64 a) {
  constexpr double big = sizeof(R) == 4 ? 3.0e38 : 1.0e300;
  return fabs(a.x) <= big && fabs(a.y) <= big;
}

// ============================================================================
// BiCGSTAB (van der Vorst 1992), complex, Hermitian inner products
//   p = r + beta (p - omega v);  v = A p;  alpha = rho / rhat^H v;  s = r - alpha v;
//   t = A s;  omega = t^H s / t^H t;  u += alpha p + omega s;  r = s - omega t;
//   rho' = rhat^H r;  beta = (rho'/rho)(alpha/omega)
// ============================================================================
struct BcgState {
  c64 rho, rho_old, alpha, omega, beta;
  double bnorm2, rnorm2, tol2, best2;
  int s_conv, converged, breakdown, iters, best_it;
  int ver;  // incremented by every kernel that writes the state
};

// r = b, rhat = b, p = v = u = 0; partials |b|^2 (slot 0) and rhat^H r = |b|^2 (slot 1)
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bcg_init(const cx<R>* __restrict__ b, cx<R>* __restrict__ r,
                                                  cx<R>* __restrict__ rhat, cx<R>* __restrict__ p,
                                                  cx<R>* __restrict__ v, cx<R>* __restrict__ u,
                                                  const int* __restrict__ active, SolverDims dm,
                                                  c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[1] = {mk(0.0, 0.0)};
  if (active[rhs]) {
    const long o = (long)rhs * dm.n3;
    DDA_RANGE(dm, i) {
      const cx<R> bv = b[o + i];
      r[o + i] = bv;
      rhat[o + i] = bv;
      p[o + i] = mk((R)0, (R)0);
      v[o + i] = mk((R)0, (R)0);
      u[o + i] = mk((R)0, (R)0);
      acc[0].x += abs2(up(bv));
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[0];
  }
}

// initial state (one block per right-hand side)
__global__ void k_bcg_fin_init(const c64* __restrict__ part, int nblk, BcgState* __restrict__ st,
                               int* __restrict__ active, const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  c64 v[2];
  reduce_partials<2>(part, nblk, rhs, v);
  if (threadIdx.x == 0) {
    BcgState s;
    s.bnorm2 = v[0].x;
    s.rnorm2 = v[0].x;
    const double tol = tolv[rhs];
    s.tol2 = tol * tol * v[0].x;
    s.best2 = v[0].x;
    s.best_it = 0;
    s.rho = mk(0.0, 0.0);  // the first p kernel moves rho' = |b|^2 into rho
    s.rho_old = mk(1.0, 0.0);
    s.alpha = mk(1.0, 0.0);
    s.omega = mk(1.0, 0.0);
    s.beta = mk(0.0, 0.0);
    s.s_conv = 0;
    s.converged = v[0].x == 0.0;
    s.breakdown = 0;
    s.iters = -1;  // the first p kernel counts iteration 0 as not yet done
    s.ver = 0;
    st[rhs] = s;
    if (s.converged) active[rhs] = 0;
  }
}

// Start of an iteration: from the previous update's partials [|r|^2, rhat^H r]
// decide convergence / stagnation / breakdown, then beta and
// p = r + beta (p - omega v).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bcg_p(const cx<R>* __restrict__ r, cx<R>* __restrict__ p,
                                               const cx<R>* __restrict__ v, const c64* __restrict__ pupd,
                                               const BcgState* __restrict__ sin, BcgState* __restrict__ sout,
                                               int* __restrict__ active, SolverDims dm) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pupd, dm.nblk, rhs, red);
  BcgState s = sin[rhs];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  s.iters += 1;
  int stop = 0;
  if (s.converged || s.s_conv) {
    s.converged = 1;
    stop = 1;
  } else {
    s.rnorm2 = red[0].x;
    s.rho_old = s.rho;
    s.rho = red[1];
    if (!isfinite(red[0].x)) {
      s.breakdown = 1;
      stop = 1;
    } else if (s.rnorm2 <= s.tol2) {
      s.converged = 1;
      stop = 1;
    } else if (s.rnorm2 < 0.98 * s.best2) {
      s.best2 = s.rnorm2;
      s.best_it = s.iters;
    } else if (s.iters - s.best_it > kStallWindow && s.rnorm2 < stall_level2<R>() * s.bnorm2) {
      s.breakdown = 2;  // stagnated
      stop = 1;
    }
    if (!stop && s.iters > 0) {
      if (tiny(s.omega, 1.0) || tiny(s.rho, s.bnorm2 * s.bnorm2 * 1e-32)) {
        s.breakdown = 1;  // restart from the current iterate (refinement loop)
        stop = 1;
      } else {
        s.beta = cdiv(s.rho, s.rho_old) * cdiv(s.alpha, s.omega);
      }
    }
  }
  if (lead) {
    { s.ver += 1; sout[rhs] = s; }
    if (stop) active[rhs] = 0;
  }
  if (stop) return;
  const cx<R> beta = cvt<R>(s.beta), om = cvt<R>(s.omega);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) { p[o + i] = r[o + i] + beta * (p[o + i] - om * v[o + i]); }
}

// alpha = rho / (rhat^H v);  s = r - alpha v (stored in r); partials |s|^2
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bcg_s(cx<R>* __restrict__ r, const cx<R>* __restrict__ v,
                                               const c64* __restrict__ pdot, int nblk_mv,
                                               const BcgState* __restrict__ sin, BcgState* __restrict__ sout,
                                               int* __restrict__ active, SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pdot, nblk_mv, rhs, red);
  BcgState s = sin[rhs];
  const bool bad = tiny(red[0], s.bnorm2 * s.bnorm2) || !isfinite(red[0].x);
  if (bad) {
    s.breakdown = 1;
  } else {
    s.alpha = cdiv(s.rho, red[0]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    { s.ver += 1; sout[rhs] = s; }
    if (bad) active[rhs] = 0;
  }
  if (bad) return;
  const cx<R> al = cvt<R>(s.alpha);
  c64 acc[1] = {mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> sv = r[o + i] - al * v[o + i];
    r[o + i] = sv;
    acc[0].x += abs2(up(sv));
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) part[(long)rhs * dm.nblk + blockIdx.x] = acc[0];
}

// omega = t^H s / t^H t (partials pts = [t^H s, t^H t]); |s|^2 from ps.
// u += alpha p + omega s;  r = s - omega t;  partials [|r|^2, rhat^H r]
// (if |s| already met the tolerance: u += alpha p and stop next iteration).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bcg_update(cx<R>* __restrict__ u, cx<R>* __restrict__ r,
                                                    const cx<R>* __restrict__ p, const cx<R>* __restrict__ t,
                                                    const cx<R>* __restrict__ rhat, const c64* __restrict__ ps,
                                                    const c64* __restrict__ pts, int nblk_mv,
                                                    const BcgState* __restrict__ sin, BcgState* __restrict__ sout,
                                                    const int* __restrict__ active, SolverDims dm,
                                                    c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 rs[1], rt[2];
  reduce_all<1>(ps, dm.nblk, rhs, rs);
  reduce_all<2>(pts, nblk_mv, rhs, rt);
  BcgState s = sin[rhs];
  s.s_conv = rs[0].x <= s.tol2;
  if (s.s_conv) s.rnorm2 = rs[0].x;
  else s.omega = (rt[1].x > 0.0) ? mk(rt[0].x / rt[1].x, rt[0].y / rt[1].x) : mk(0.0, 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) { s.ver += 1; sout[rhs] = s; }
  const cx<R> al = cvt<R>(s.alpha), om = cvt<R>(s.omega);
  const bool sc = s.s_conv;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> sv = r[o + i];
    if (sc) {
      u[o + i] = u[o + i] + al * p[o + i];
    } else {
      u[o + i] = u[o + i] + al * p[o + i] + om * sv;
      const cx<R> rn = sv - om * t[o + i];
      r[o + i] = rn;
      const c64 rd = up(rn);
      acc[0].x += abs2(rd);
      acc[1] = acc[1] + cmulc(up(rhat[o + i]), rd);
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// ============================================================================
// BiCG for complex-symmetric matrices, BiCG_sym (Freund 1992a; also known as
// COCG): the BiCG recurrences with the shadow vectors equal to the conjugate
// iterates, so one matrix-vector product per iteration and the bilinear form
//   p = r + beta p;  q = A p;  alpha = rho / p^T q;  u += alpha p;  r -= alpha q;
//   rho' = r^T r;  beta = rho' / rho.
// Stopping on ||r|| (Hermitian norm of the recursive residual).
// ============================================================================
struct CgState {
  c64 rho, rho_old, alpha, beta;
  double bnorm2, rnorm2, tol2, best2;
  int converged, breakdown, iters, best_it;
  int ver;  // incremented by every kernel that writes the state
};

// r = b, p = u = 0; partials [|b|^2, b^T b]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cg_init(const cx<R>* __restrict__ b, cx<R>* __restrict__ r,
                                                         cx<R>* __restrict__ p, cx<R>* __restrict__ u,
                                                         const int* __restrict__ active, SolverDims dm,
                                                         c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  if (active[rhs]) {
    const long o = (long)rhs * dm.n3;
    DDA_RANGE(dm, i) {
      const cx<R> bv = b[o + i];
      r[o + i] = bv;
      p[o + i] = mk((R)0, (R)0);
      u[o + i] = mk((R)0, (R)0);
      const c64 bd = up(bv);
      acc[0].x += abs2(bd);
      acc[1] = acc[1] + bd * bd;
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

__global__ void k_cg_fin_init(const c64* __restrict__ part, int nblk, CgState* __restrict__ st,
                              int* __restrict__ active, const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  c64 v[2];
  reduce_partials<2>(part, nblk, rhs, v);
  if (threadIdx.x == 0) {
    CgState s;
    s.bnorm2 = v[0].x;
    s.rnorm2 = v[0].x;
    const double tol = tolv[rhs];
    s.tol2 = tol * tol * v[0].x;
    s.best2 = v[0].x;
    s.best_it = 0;
    s.rho = mk(0.0, 0.0);  // the first p kernel moves rho' = b^T b into rho
    s.rho_old = mk(1.0, 0.0);
    s.alpha = mk(0.0, 0.0);
    s.beta = mk(0.0, 0.0);
    s.converged = v[0].x == 0.0;
    s.breakdown = 0;
    s.iters = -1;
    s.ver = 0;
    st[rhs] = s;
    if (s.converged) active[rhs] = 0;
  }
}

// From the previous update's partials [|r|^2, r^T r]: convergence,
// stagnation, breakdown; then beta = rho'/rho and p = r + beta p.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cg_p(const cx<R>* __restrict__ r, cx<R>* __restrict__ p,
                                                      const c64* __restrict__ pupd,
                                                      const CgState* __restrict__ sin, CgState* __restrict__ sout,
                                                      int* __restrict__ active, SolverDims dm) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pupd, dm.nblk, rhs, red);
  CgState s = sin[rhs];
  s.iters += 1;
  s.rnorm2 = red[0].x;
  s.rho_old = s.rho;
  s.rho = red[1];
  int stop = 0;
  if (!isfinite(red[0].x)) {
    s.breakdown = 1;
    stop = 1;
  } else if (s.rnorm2 <= s.tol2) {
    s.converged = 1;
    stop = 1;
  } else if (s.rnorm2 < 0.98 * s.best2) {
    s.best2 = s.rnorm2;
    s.best_it = s.iters;
  } else if (s.iters - s.best_it > kStallWindow && s.rnorm2 < stall_level2<R>() * s.bnorm2) {
    s.breakdown = 2;  // stagnated
    stop = 1;
  }
  if (!stop) {
    if (tiny(s.rho, s.bnorm2 * s.bnorm2 * 1e-32)) {
      s.breakdown = 1;  // r^T r = 0 with r != 0: restart from the current iterate
      stop = 1;
    } else {
      s.beta = s.iters > 0 ? cdiv(s.rho, s.rho_old) : mk(0.0, 0.0);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
    if (stop) active[rhs] = 0;
  }
  if (stop) return;
  const cx<R> beta = cvt<R>(s.beta);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) { p[o + i] = r[o + i] + beta * p[o + i]; }
}

// alpha = rho / p^T q (partials from the matrix-vector product, nblk_mv blocks,
// stride 2); u += alpha p; r -= alpha q; partials [|r|^2, r^T r]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cg_update(cx<R>* __restrict__ u, cx<R>* __restrict__ r,
                                                           const cx<R>* __restrict__ p, const cx<R>* __restrict__ q,
                                                           const c64* __restrict__ pdot, int nblk_mv,
                                                           const CgState* __restrict__ sin,
                                                           CgState* __restrict__ sout, int* __restrict__ active,
                                                           SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pdot, nblk_mv, rhs, red);
  CgState s = sin[rhs];
  const bool bad = tiny(red[0], s.bnorm2 * s.bnorm2 * 1e-32) || !isfinite(red[0].x);
  if (bad) s.breakdown = 1;
  else s.alpha = cdiv(s.rho, red[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
    if (bad) active[rhs] = 0;
  }
  if (bad) return;
  const cx<R> al = cvt<R>(s.alpha);
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    u[o + i] = u[o + i] + al * p[o + i];
    const cx<R> rn = r[o + i] - al * q[o + i];
    r[o + i] = rn;
    const c64 rd = up(rn);
    acc[0].x += abs2(rd);
    acc[1] = acc[1] + rd * rd;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}
// ============================================================================
// CGS, conjugate gradients squared (Sonneveld 1989): transpose-free, two
// products per iteration, Hermitian shadow inner products with rt = r_0
//   rho = rt^H r;  beta = rho / rho_old;  uu = r + beta q;
//   p = uu + beta (q + beta p);  v = A p;  alpha = rho / rt^H v;
//   q = uu - alpha v;  w = uu + q;  u += alpha w;  r -= alpha A w
// ============================================================================
struct CgsState {
  c64 rho, rho_old, alpha, beta;
  double bnorm2, rnorm2, tol2, best2;
  int converged, breakdown, iters, best_it;
  int ver;  // incremented by every kernel that writes the state
};

// r = rt = b, p = q = u = 0; partials [|b|^2, rt^H r = |b|^2]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cgs_init(const cx<R>* __restrict__ b, cx<R>* __restrict__ r,
                                                          cx<R>* __restrict__ rt, cx<R>* __restrict__ p,
                                                          cx<R>* __restrict__ q, cx<R>* __restrict__ u,
                                                          const int* __restrict__ active, SolverDims dm,
                                                          c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[1] = {mk(0.0, 0.0)};
  if (active[rhs]) {
    const long o = (long)rhs * dm.n3;
    const cx<R> z = mk((R)0, (R)0);
    DDA_RANGE(dm, i) {
      const cx<R> bv = b[o + i];
      r[o + i] = bv;
      rt[o + i] = bv;
      p[o + i] = z;
      q[o + i] = z;
      u[o + i] = z;
      acc[0].x += abs2(up(bv));
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[0];
  }
}

__global__ void k_cgs_fin_init(const c64* __restrict__ part, int nblk, CgsState* __restrict__ st,
                               int* __restrict__ active, const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  c64 v[2];
  reduce_partials<2>(part, nblk, rhs, v);
  if (threadIdx.x == 0) {
    CgsState s;
    s.bnorm2 = v[0].x;
    s.rnorm2 = v[0].x;
    const double tol = tolv[rhs];
    s.tol2 = tol * tol * v[0].x;
    s.best2 = v[0].x;
    s.best_it = 0;
    s.rho = mk(0.0, 0.0);
    s.rho_old = mk(1.0, 0.0);
    s.alpha = mk(0.0, 0.0);
    s.beta = mk(0.0, 0.0);
    s.converged = v[0].x == 0.0;
    s.breakdown = 0;
    s.iters = -1;
    s.ver = 0;
    st[rhs] = s;
    if (s.converged) active[rhs] = 0;
  }
}

// From the previous update's partials [|r|^2, rt^H r]: stopping tests, beta,
// uu = r + beta q and p = uu + beta (q + beta p).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cgs_p(const cx<R>* __restrict__ r, const cx<R>* __restrict__ q,
                                                       cx<R>* __restrict__ uu, cx<R>* __restrict__ p,
                                                       const c64* __restrict__ pupd,
                                                       const CgsState* __restrict__ sin,
                                                       CgsState* __restrict__ sout, int* __restrict__ active,
                                                       SolverDims dm) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pupd, dm.nblk, rhs, red);
  CgsState s = sin[rhs];
  s.iters += 1;
  s.rnorm2 = red[0].x;
  s.rho_old = s.rho;
  s.rho = red[1];
  int stop = 0;
  if (!isfinite(red[0].x)) {
    s.breakdown = 1;
    stop = 1;
  } else if (s.rnorm2 <= s.tol2) {
    s.converged = 1;
    stop = 1;
  } else if (s.rnorm2 < 0.98 * s.best2) {
    s.best2 = s.rnorm2;
    s.best_it = s.iters;
  } else if (s.iters - s.best_it > kStallWindow && s.rnorm2 < stall_level2<R>() * s.bnorm2) {
    s.breakdown = 2;  // stagnated
    stop = 1;
  }
  if (!stop) {
    if (tiny(s.rho, s.bnorm2 * s.bnorm2 * 1e-32)) {
      s.breakdown = 1;  // rt^H r = 0: restart from the current iterate
      stop = 1;
    } else {
      s.beta = s.iters > 0 ? cdiv(s.rho, s.rho_old) : mk(0.0, 0.0);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
    if (stop) active[rhs] = 0;
  }
  if (stop) return;
  const cx<R> be = cvt<R>(s.beta);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> qi = q[o + i];
    const cx<R> ui = r[o + i] + be * qi;
    uu[o + i] = ui;
    p[o + i] = ui + be * (qi + be * p[o + i]);
  }
}

// alpha = rho / rt^H v (partials from the product, nblk_mv blocks, stride 2);
// q = uu - alpha v;  w = uu + q;  u += alpha w
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cgs_q(const cx<R>* __restrict__ uu, const cx<R>* __restrict__ v,
                                                       cx<R>* __restrict__ q, cx<R>* __restrict__ w,
                                                       cx<R>* __restrict__ u, const c64* __restrict__ pdot,
                                                       int nblk_mv, const CgsState* __restrict__ sin,
                                                       CgsState* __restrict__ sout, int* __restrict__ active,
                                                       SolverDims dm) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pdot, nblk_mv, rhs, red);
  CgsState s = sin[rhs];
  const bool bad = tiny(red[0], s.bnorm2 * s.bnorm2 * 1e-32) || !isfinite(red[0].x);
  if (bad) s.breakdown = 1;
  else s.alpha = cdiv(s.rho, red[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
    if (bad) active[rhs] = 0;
  }
  if (bad) return;
  const cx<R> al = cvt<R>(s.alpha);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> ui = uu[o + i];
    const cx<R> qi = ui - al * v[o + i];
    q[o + i] = qi;
    const cx<R> wi = ui + qi;
    w[o + i] = wi;
    u[o + i] = u[o + i] + al * wi;
  }
}

// r -= alpha t (t = A w); partials [|r|^2, rt^H r]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cgs_update(cx<R>* __restrict__ r, const cx<R>* __restrict__ t,
                                                            const cx<R>* __restrict__ rt,
                                                            const CgsState* __restrict__ sin,
                                                            const int* __restrict__ active, SolverDims dm,
                                                            c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const cx<R> al = cvt<R>(sin[rhs].alpha);
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> rn = r[o + i] - al * t[o + i];
    r[o + i] = rn;
    const c64 rd = up(rn);
    acc[0].x += abs2(rd);
    acc[1] = acc[1] + conjg(up(rt[o + i])) * rd;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}
// ============================================================================
// TFQMR, transpose-free QMR (Freund 1993): two products per iteration, shadow
// vector rt = r_0 with Hermitian inner products.  Half-steps m = 0, 1, ...
// with u_m = ue (m even) or uo (m odd):
//   m even: alpha = rho / rt^H v;  uo = ue - alpha v
//   w -= alpha A u_m;  d = u_m + (theta^2 / alpha) eta d
//   theta' = |w| / tau;  c = (1 + theta'^2)^{-1/2};  tau' = tau theta' c;
//   eta' = c^2 alpha;  x += eta' d
//   m odd:  rho' = rt^H w;  beta = rho' / rho;  ue = w + beta uo;
//           v = A ue + beta (A uo + beta v)
// rt^H v is carried by the recurrence sigma' = rt^H A ue + beta (rt^H A uo +
// beta sigma), both inner products fused into the products.  Stopping on the
// residual bound |r_m| <= sqrt(m + 1) tau_m.  A right-hand side that meets it
// after its x update only marks the state; the next iteration's first kernel,
// where no block does vector work, clears `active`, so no block of an
// updating kernel can miss its update.
// ============================================================================
struct TfqState {
  c64 rho, sigma, s_uo, alpha, beta, eta;
  double tau, theta, bnorm2, tol2, best2, rnorm2;
  int m, converged, breakdown, iters, best_it;
  int ver;  // incremented by every kernel that writes the state
};

// Close a half-step from |w|^2: theta, c, tau, eta = c^2 alpha; true when the
// residual bound meets the tolerance.
__device__ inline bool tfq_close(TfqState& s, double w2) {
  const double th = sqrt(w2) / s.tau;
  const double c2 = 1.0 / (1.0 + th * th);
  s.tau = s.tau * th * sqrt(c2);
  s.theta = th;
  s.eta = c2 * s.alpha;
  s.m += 1;
  s.rnorm2 = s.tau * s.tau * (double)(s.m + 1);
  s.iters = (s.m + 1) / 2;
  return s.rnorm2 <= s.tol2 || !(w2 > 0.0);
}

// x = 0, ue = w = rt = b, uo = v = d = A uo = 0; partials [|b|^2, 0]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_tfq_init(const cx<R>* __restrict__ b, cx<R>* __restrict__ x,
                                                          cx<R>* __restrict__ rt, cx<R>* __restrict__ w,
                                                          cx<R>* __restrict__ ue, cx<R>* __restrict__ uo,
                                                          cx<R>* __restrict__ v, cx<R>* __restrict__ d,
                                                          cx<R>* __restrict__ auo, const int* __restrict__ active,
                                                          SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[1] = {mk(0.0, 0.0)};
  if (active[rhs]) {
    const long o = (long)rhs * dm.n3;
    const cx<R> z = mk((R)0, (R)0);
    DDA_RANGE(dm, i) {
      const cx<R> bv = b[o + i];
      x[o + i] = z;
      rt[o + i] = bv;
      w[o + i] = bv;
      ue[o + i] = bv;
      uo[o + i] = z;
      v[o + i] = z;
      d[o + i] = z;
      auo[o + i] = z;
      acc[0].x += abs2(up(bv));
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = mk(0.0, 0.0);
  }
}

__global__ void k_tfq_fin_init(const c64* __restrict__ part, int nblk, TfqState* __restrict__ st,
                               int* __restrict__ active, const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  c64 v[2];
  reduce_partials<2>(part, nblk, rhs, v);
  if (threadIdx.x == 0) {
    TfqState s;
    const double nb2 = v[0].x;
    s.bnorm2 = nb2;
    s.rnorm2 = nb2;
    const double tol = tolv[rhs];
    s.tol2 = tol * tol * nb2;
    s.best2 = nb2;
    s.best_it = 0;
    s.rho = mk(nb2, 0.0);  // rt^H r_0
    s.sigma = mk(0.0, 0.0);
    s.s_uo = mk(0.0, 0.0);
    s.alpha = mk(0.0, 0.0);
    s.beta = mk(0.0, 0.0);
    s.eta = mk(0.0, 0.0);
    s.tau = sqrt(nb2);
    s.theta = 0.0;
    s.m = 0;
    s.converged = nb2 == 0.0;
    s.breakdown = 0;
    s.iters = 0;
    s.ver = 0;
    st[rhs] = s;
    if (s.converged) active[rhs] = 0;
  }
}

// First kernel of an iteration (half-step m even opens).  pue: rt^H A ue
// (nblk_mv blocks, stride 2).  sigma, v = A ue + beta (A uo + beta v),
// alpha = rho / sigma, uo = ue - alpha v, w -= alpha A ue,
// d = ue + (theta^2 / alpha) eta d;  partials [|w|^2, 0].
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_tfq_a(const cx<R>* __restrict__ ue, const cx<R>* __restrict__ aue,
                                                       const cx<R>* __restrict__ auo, cx<R>* __restrict__ v,
                                                       cx<R>* __restrict__ uo, cx<R>* __restrict__ w,
                                                       cx<R>* __restrict__ d, const c64* __restrict__ pue,
                                                       int nblk_mv, const TfqState* __restrict__ sin,
                                                       TfqState* __restrict__ sout, int* __restrict__ active,
                                                       SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 red[2];
  reduce_all<2>(pue, nblk_mv, rhs, red);
  TfqState s = sin[rhs];
  int stop = s.converged || s.breakdown;
  c64 dcoef = mk(0.0, 0.0);
  if (!stop) {
    s.sigma = red[0] + s.beta * (s.s_uo + s.beta * s.sigma);
    if (tiny(s.sigma, s.bnorm2 * s.bnorm2 * 1e-32) || !isfinite(s.sigma.x) || !isfinite(s.sigma.y)) {
      s.breakdown = 1;
      stop = 1;
    } else {
      s.alpha = cdiv(s.rho, s.sigma);
      dcoef = (s.theta * s.theta) * cdiv(s.eta, s.alpha);
      // alpha and the d coefficient must be usable in the vectors' precision
      // (a vanishing alpha makes eta / alpha 0/0 and x += eta d NaN)
      if (tiny(s.alpha, 1.0) || !holds<R>(s.alpha) || !holds<R>(dcoef)) {
        s.breakdown = 1;
        stop = 1;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
    if (stop) active[rhs] = 0;
  }
  if (stop) return;
  const cx<R> be = cvt<R>(s.beta), al = cvt<R>(s.alpha), dc = cvt<R>(dcoef);
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> ai = aue[o + i];
    const cx<R> vi = ai + be * (auo[o + i] + be * v[o + i]);
    v[o + i] = vi;
    const cx<R> ui = ue[o + i];
    uo[o + i] = ui - al * vi;
    const cx<R> wi = w[o + i] - al * ai;
    w[o + i] = wi;
    d[o + i] = ui + dc * d[o + i];
    acc[0].x += abs2(up(wi));
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// Half-step m closes (|w|^2 from pw; x += eta d); half-step m + 1 (odd)
// opens: w -= alpha A uo, d = uo + (theta^2 / alpha) eta d; partials
// [|w|^2, rt^H w].  rt^H A uo (puo) is kept for the sigma recurrence.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_tfq_b(cx<R>* __restrict__ x, const cx<R>* __restrict__ uo,
                                                       const cx<R>* __restrict__ auo, const cx<R>* __restrict__ rt,
                                                       cx<R>* __restrict__ w, cx<R>* __restrict__ d,
                                                       const c64* __restrict__ pw, const c64* __restrict__ puo,
                                                       int nblk_mv, const TfqState* __restrict__ sin,
                                                       TfqState* __restrict__ sout, const int* __restrict__ active,
                                                       SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 rw[2], ru[2];
  reduce_all<2>(pw, dm.nblk, rhs, rw);
  reduce_all<2>(puo, nblk_mv, rhs, ru);
  TfqState s = sin[rhs];
  if (s.converged || s.breakdown) {
    // carry a stopped state into this kernel's output buffer: the state
    // buffers swap roles every iteration, so a state left behind here would
    // be read back stale two kernels later
    if (blockIdx.x == 0 && threadIdx.x == 0) sout[rhs] = s;
    return;
  }
  bool conv = tfq_close(s, rw[0].x);
  s.s_uo = ru[0];
  if (conv) s.converged = 1;
  const c64 dcoef = (s.theta * s.theta) * cdiv(s.eta, s.alpha);
  if (!conv && (!holds<R>(s.eta) || !holds<R>(dcoef))) {
    // x is still updated with this half-step's eta when it is usable; the
    // second half-step is not opened
    s.breakdown = 1;
    conv = true;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
  }
  const cx<R> et = holds<R>(s.eta) ? cvt<R>(s.eta) : mk((R)0, (R)0), al = cvt<R>(s.alpha), dc = cvt<R>(dcoef);
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> di = d[o + i];
    x[o + i] = x[o + i] + et * di;
    if (!conv) {
      const cx<R> wi = w[o + i] - al * auo[o + i];
      w[o + i] = wi;
      d[o + i] = uo[o + i] + dc * di;
      const c64 wd = up(wi);
      acc[0].x += abs2(wd);
      acc[1] = acc[1] + conjg(up(rt[o + i])) * wd;
    }
  }
  if (conv) return;
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// Half-step m + 1 closes (x += eta d); then rho' = rt^H w, beta = rho'/rho,
// ue = w + beta uo (the next product's input).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_tfq_c(cx<R>* __restrict__ x, const cx<R>* __restrict__ d,
                                                       const cx<R>* __restrict__ w, const cx<R>* __restrict__ uo,
                                                       cx<R>* __restrict__ ue, const c64* __restrict__ pw,
                                                       const TfqState* __restrict__ sin, TfqState* __restrict__ sout,
                                                       int* __restrict__ active, SolverDims dm) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 rw[2];
  reduce_all<2>(pw, dm.nblk, rhs, rw);
  TfqState s = sin[rhs];
  if (s.converged || s.breakdown) {
    // stopped at the first half-step (k_tfq_b): pass the state on (the next
    // iteration reads this kernel's output buffer) and stop the right-hand side
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sout[rhs] = s;
      active[rhs] = 0;
    }
    return;
  }
  const bool conv = tfq_close(s, rw[0].x);
  bool upd = !conv;
  if (conv) {
    s.converged = 1;
  } else {
    const c64 rho_new = rw[1];
    // rho' = rt^H w vanishing (or not finite) is a breakdown now, before the
    // next half-step divides by alpha = rho' / sigma
    const c64 beta = cdiv(rho_new, s.rho);
    if (tiny(rho_new, s.bnorm2 * s.bnorm2 * 1e-32) || !isfinite(rho_new.x) || !isfinite(rho_new.y) ||
        !holds<R>(beta)) {
      s.breakdown = 1;
      upd = false;
    } else {
      s.beta = beta;
      s.rho = rho_new;
    }
    if (s.rnorm2 < 0.98 * s.best2) {
      s.best2 = s.rnorm2;
      s.best_it = s.iters;
    } else if (s.iters - s.best_it > kStallWindow && s.rnorm2 < stall_level2<R>() * s.bnorm2) {
      s.breakdown = 2;  // stagnated
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.ver += 1;
    sout[rhs] = s;
  }
  const cx<R> et = cvt<R>(s.eta), be = cvt<R>(s.beta);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    x[o + i] = x[o + i] + et * d[o + i];
    if (upd) ue[o + i] = w[o + i] + be * uo[o + i];
  }
}
// ============================================================================
// QMR for complex-symmetric matrices (Freund 1992): Lanczos with the bilinear
// form x^T y and Euclidean-normalised vectors v_n = vt_n / rho_n, the
// tridiagonal matrix reduced by Givens rotations, iterate u_n updated through
// p_n.  The unnormalised vectors vt_n are what is stored (and fed to the
// matrix-vector product); 1/rho_n is applied on the fly.  One fused kernel per
// iteration finishes column n-1 (rotation, p_{n-1}, u) and builds vt_{n+1}.
// Stopping: the quasi-residual |tau_n| <= tol |b| (the QMR residual estimate);
// the FP64 refinement loop checks the true residual.
// ============================================================================
struct QmrState {
  c64 alpha_prev, beta_prev, delta_prev;  // alpha_{n-1}, beta_{n-1}, delta_{n-1}
  double rho_prev;                        // rho_{n-1} = |vt_{n-1}|
  c64 s1, s2;                             // sines of rotations n-2, n-3
  double c1, c2;                          // cosines of rotations n-2, n-3
  c64 tau;                                // quasi-residual tau_{n-1}
  double bnorm2, rnorm2, tol2, best2;
  int n, converged, breakdown, iters, best_it;
  int ver;  // incremented by every kernel that writes the state
};

// u = 0; vt_1 = b; vt_0 = 0; p ring = 0; r = b; partials [(|b|^2, |r|^2), b^T b]
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_qmr_init(const cx<R>* __restrict__ b, cx<R>* __restrict__ u,
                                                  cx<R>* __restrict__ v1, cx<R>* __restrict__ v0,
                                                  cx<R>* __restrict__ pa, cx<R>* __restrict__ pb,
                                                  cx<R>* __restrict__ r, const int* __restrict__ active,
                                                  SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  if (active[rhs]) {
    const long o = (long)rhs * dm.n3;
    const cx<R> z = mk((R)0, (R)0);
    DDA_RANGE(dm, i) {
      const cx<R> bv = b[o + i];
      u[o + i] = z;
      v1[o + i] = bv;
      v0[o + i] = z;
      pa[o + i] = z;
      pb[o + i] = z;
      r[o + i] = bv;
      const c64 bd = up(bv);
      acc[0].x += abs2(bd);
      acc[0].y += abs2(bd);
      acc[1] = acc[1] + bd * bd;
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

__global__ void k_qmr_fin_init(const c64* __restrict__ part, int nblk, QmrState* __restrict__ st,
                               int* __restrict__ active, const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  c64 v[2];
  reduce_partials<2>(part, nblk, rhs, v);
  if (threadIdx.x == 0) {
    QmrState s;
    const double nb2 = v[0].x;
    s.bnorm2 = nb2;
    s.rnorm2 = nb2;
    const double tol = tolv[rhs];
    s.tol2 = tol * tol * nb2;
    s.best2 = nb2;
    s.best_it = 0;
    s.alpha_prev = s.beta_prev = mk(0.0, 0.0);
    s.delta_prev = mk(1.0, 0.0);
    s.rho_prev = 1.0;
    s.s1 = s.s2 = mk(0.0, 0.0);
    s.c1 = s.c2 = 1.0;
    s.tau = mk(0.0, 0.0);
    s.n = 1;
    s.converged = nb2 == 0.0;
    s.breakdown = 0;
    s.iters = 0;
    s.ver = 0;
    st[rhs] = s;
    if (s.converged) active[rhs] = 0;
  }
}

// Iteration n (after w~ = A vt_n).  pnorm_in: partials [(|vt_n|^2, |r_{n-2}|^2),
// vt_n^T vt_n] (dm.nblk blocks); pdot: vt_n^T w~ from the matrix-vector
// product (nblk_mv blocks, stride 2).  vn = vt_n, vp = vt_{n-1} (overwritten
// by vt_{n+1}), p1 = p_{n-2}, p2 = p_{n-3} (overwritten by p_{n-1}).
//
// Stopping uses the QMR residual itself, carried by the recurrence
//   r_{n-1} = |s_{n-1}|^2 r_{n-2} + c_{n-1} tau_n vt_n / |vt_n|
// (the residual is tau_n V_{n+1} Q^H e_{n+1} and the last column of Q^H
// changes by one rotation per step), not the quasi-residual |tau_n|, which can
// sit far below the residual when the Lanczos vectors are far from
// orthogonal.  The norm of r_{n-2} arrives with this step's partials, when u
// still holds u_{n-2}; a right-hand side that stops (converged, stagnated or
// broken down) stops here with u = u_{n-2} and no vector written, so every
// block agrees whether or not it saw the cleared `active` flag.
//
// One wave reduces the partials (fixed order: identical in every block) and
// one lane runs the scalar recurrences; the vector coefficients reach the
// block through LDS.

// Scalar part of a QMR_sym step: from the reduced partials and the state,
// the next state and the coefficients of the vector update.
struct QmrCoef {
  double sgp, sg, rs;
  c64 fpp, ep, rinv, coef, rc, alpha, bs;
  int upd, stop;
};

__device__ inline void qmr_scalars(const c64 (&rn)[2], const c64 (&rd)[2], QmrState& s, QmrCoef& q) {
  const int n = s.n;
  // residual of the current iterate u_{n-2}
  const double r2 = rn[0].y;
  s.rnorm2 = r2;
  q.upd = 0;
  q.stop = 0;
  if (r2 <= s.tol2 || !isfinite(r2)) {
    if (r2 <= s.tol2) s.converged = 1;
    else s.breakdown = 1;
    s.iters = n >= 2 ? n - 2 : 0;
    q.stop = 1;
    return;
  }
  if (r2 < 0.98 * s.best2) {
    s.best2 = r2;
    s.best_it = n;
  } else if (n - s.best_it > kStallWindow) {
    s.breakdown = 2;  // stagnated (kept only where the rule applies, see below)
  }
  const double rho = sqrt(rn[0].x);
  // Lanczos scalars of step n
  c64 alpha = mk(0.0, 0.0), beta = mk(0.0, 0.0), delta = mk(0.0, 0.0);
  double sig = 0.0;
  if (rho > 0.0 && isfinite(rho)) {
    sig = 1.0 / rho;
    delta = (sig * sig) * rn[1];
    if (!(abs2(delta) > 1e-300)) {
      s.breakdown = 1;  // Lanczos breakdown: vt_n^T vt_n = 0
    } else {
      alpha = cdiv((sig * sig) * rd[0], delta);
      beta = (n == 1) ? mk(0.0, 0.0) : rho * cdiv(delta, s.delta_prev);
    }
  }
  if (n == 1) s.tau = mk(rho, 0.0);
  // column n-1 of the tridiagonal matrix: (beta_{n-1}, alpha_{n-1}, rho_n)
  const bool upd = n >= 2;
  c64 ep = mk(0.0, 0.0), fpp = mk(0.0, 0.0), rinv = mk(0.0, 0.0), coef = mk(0.0, 0.0), rc = mk(0.0, 0.0);
  double rs = 1.0;
  if (upd) {
    const double h = rho;
    const c64 f = s.beta_prev, g = s.alpha_prev;
    ep = s.s2 * f;
    const c64 fp = s.c2 * f;
    fpp = s.c1 * fp + s.s1 * g;
    const c64 gp = s.c1 * g - conjg(s.s1) * fp;
    const double ag = sqrt(abs2(gp));
    double c;
    c64 sn, rnn;
    if (ag == 0.0) {
      c = 0.0;
      sn = mk(1.0, 0.0);
      rnn = mk(h, 0.0);
    } else {
      const double nrm = sqrt(ag * ag + h * h);
      c = ag / nrm;
      sn = (c * h) * cdiv(mk(1.0, 0.0), conjg(gp));
      rnn = (nrm / ag) * gp;
    }
    if (abs2(rnn) > 0.0) {
      rinv = cdiv(mk(1.0, 0.0), rnn);
      coef = c * s.tau;
      s.tau = (-1.0) * (conjg(sn) * s.tau);
      rs = abs2(sn);
      rc = (c * sig) * s.tau;
    } else {
      s.breakdown = 1;
    }
    s.c2 = s.c1;
    s.s2 = s.s1;
    s.c1 = c;
    s.s1 = sn;
    s.iters = n - 1;
  }
  if (!(rho > 0.0)) s.converged = 1;  // vt_n = 0: the Krylov space is invariant
  if (!isfinite(rho)) s.breakdown = 1;
  const double sigp = 1.0 / s.rho_prev;
  s.alpha_prev = alpha;
  s.beta_prev = beta;
  s.delta_prev = delta;
  s.rho_prev = rho > 0.0 ? rho : 1.0;
  s.n = n + 1;
  q.stop = s.converged || s.breakdown;
  q.upd = upd;
  q.sgp = sigp;
  q.sg = sig;
  q.rs = rs;
  q.fpp = fpp;
  q.ep = ep;
  q.rinv = rinv;
  q.coef = coef;
  q.rc = rc;
  q.alpha = alpha;
  q.bs = sigp * beta;
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_qmr_step(const cx<R>* __restrict__ w, const cx<R>* __restrict__ vn,
                                                  cx<R>* __restrict__ vp, const cx<R>* __restrict__ p1,
                                                  cx<R>* __restrict__ p2, cx<R>* __restrict__ u,
                                                  cx<R>* __restrict__ r, const c64* __restrict__ pnorm_in,
                                                  const c64* __restrict__ pdot, int nblk_mv,
                                                  const QmrState* __restrict__ sin, QmrState* __restrict__ sout,
                                                  int* __restrict__ active, SolverDims dm,
                                                  c64* __restrict__ pnorm_out) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  __shared__ QmrCoef cq;
  if (threadIdx.x < 64) {
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < dm.nblk; b += 64) {
      const c64* pp = pnorm_in + ((long)rhs * dm.nblk + b) * 2;
      v[0] += pp[0].x;
      v[1] += pp[0].y;
      v[2] += pp[1].x;
      v[3] += pp[1].y;
    }
    for (int b = threadIdx.x; b < nblk_mv; b += 64) {
      const c64* pp = pdot + ((long)rhs * nblk_mv + b) * 2;
      v[4] += pp[0].x;
      v[5] += pp[0].y;
      v[6] += pp[1].x;
      v[7] += pp[1].y;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    if (threadIdx.x == 0) {
      const c64 rn[2] = {mk(v[0], v[1]), mk(v[2], v[3])};
      const c64 rd[2] = {mk(v[4], v[5]), mk(v[6], v[7])};
      QmrState s = sin[rhs];
      QmrCoef q;
      qmr_scalars(rn, rd, s, q);
      // the stagnation rule applies to FP64 vectors only near their rounding level
      if (s.breakdown == 2 && !(s.rnorm2 < stall_level2<R>() * s.bnorm2)) {
        s.breakdown = 0;
        q.stop = s.converged;
      }
      cq = q;
      if (blockIdx.x == 0) {
        s.ver += 1;
        sout[rhs] = s;
        if (q.stop) active[rhs] = 0;
      }
    }
  }
  __syncthreads();
  const QmrCoef q = cq;
  if (q.stop) return;
  const bool upd = q.upd;
  const R sgp = (R)q.sgp, sg = (R)q.sg, rsr = (R)q.rs;
  const cx<R> fppr = cvt<R>(q.fpp), epr = cvt<R>(q.ep), rir = cvt<R>(q.rinv), cf = cvt<R>(q.coef),
              rcr = cvt<R>(q.rc);
  const cx<R> al = cvt<R>(q.alpha), bs = cvt<R>(q.bs);
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const cx<R> vpi = vp[o + i];
    const cx<R> vni = vn[o + i];
    cx<R> ri = r[o + i];
    if (upd) {
      const cx<R> pn = rir * (sgp * vpi - fppr * p1[o + i] - epr * p2[o + i]);
      p2[o + i] = pn;
      u[o + i] = u[o + i] + cf * pn;
      ri = rsr * ri + rcr * vni;
      r[o + i] = ri;
    }
    const cx<R> t = sg * (w[o + i] - al * vni) - bs * vpi;
    vp[o + i] = t;
    const c64 td = up(t);
    acc[0].x += abs2(td);
    acc[0].y += abs2(up(ri));
    acc[1] = acc[1] + td * td;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    pnorm_out[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    pnorm_out[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// Fused form of the same step: the whole step runs inside the y-forward pass
// of the next product, which consumes vt_{n+1} as it is formed, so the
// iteration has no separate step kernel and vt_{n+1} is not read back.  As in
// k_qmr_step, every block reduces the partials in the same fixed order and
// runs the scalar recurrence redundantly (block 0 of each right-hand side
// writes the state); same recurrences and stopping.  The partials of
// |vt_{n+1}|^2, |r|^2 and vt_{n+1}^T vt_{n+1} come from the y-forward blocks
// (nblk_out per RHS).
template <typename R>
struct QmrFuse {
  const cx<R>* w;
  const cx<R>* vn;
  cx<R>* vp;
  const cx<R>* p1;
  cx<R>* p2;
  cx<R>* u;
  cx<R>* r;
  c64* pnorm_out;  // [nrhs][nblk_out][2]
  int nblk_out;
  const c64* pnorm_in;  // the previous step's partials [nrhs][nblk_in][2]
  int nblk_in;
  const c64* pdot;
  int nblk_mv;
  const QmrState* sin;
  QmrState* sout;
  int* active;
};

// Sum of ND complex values over a block of any size up to 1024 threads; fixed
// order, result valid in thread 0.
template <int ND>
__device__ __forceinline__ void block_sum_n(c64 (&v)[ND]) {
  __shared__ c64 shn[ND][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  const int nact = min(64, (int)blockDim.x - (wv << 6));  // lanes of a last, partial wavefront
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    double a = v[q].x, b = v[q].y;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double oa = __shfl_down(a, off, 64), ob = __shfl_down(b, off, 64);
      if (lane + off < nact) {
        a += oa;
        b += ob;
      }
    }
    if (lane == 0) shn[q][wv] = mk(a, b);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      c64 s = shn[q][0];
      for (int w = 1; w < nw; ++w) s = s + shn[q][w];
      v[q] = s;
    }
  }
  __syncthreads();
}

// The step's coefficients in the vector precision.
template <typename R>
struct QmrCoefR {
  bool upd;
  R sgp, sg, rs;
  cx<R> fpp, ep, rinv, coef, rc, alpha, bs;
  __device__ explicit QmrCoefR(const QmrCoef& q)
      : upd(q.upd != 0), sgp((R)q.sgp), sg((R)q.sg), rs((R)q.rs), fpp(cvt<R>(q.fpp)), ep(cvt<R>(q.ep)),
        rinv(cvt<R>(q.rinv)), coef(cvt<R>(q.coef)), rc(cvt<R>(q.rc)), alpha(cvt<R>(q.alpha)), bs(cvt<R>(q.bs)) {}
};

// Vector part of the step for element i of one right-hand side (the body of
// k_qmr_step's loop); returns vt_{n+1}[i].
template <typename R>
__device__ __forceinline__ cx<R> qmr_elem(const QmrCoefR<R>& q, const QmrFuse<R>& f, long i, c64 (&acc)[2]) {
  const cx<R> vpi = f.vp[i];
  const cx<R> vni = f.vn[i];
  cx<R> ri = f.r[i];
  if (q.upd) {
    const cx<R> pn = q.rinv * (q.sgp * vpi - q.fpp * f.p1[i] - q.ep * f.p2[i]);
    f.p2[i] = pn;
    f.u[i] = f.u[i] + q.coef * pn;
    ri = q.rs * ri + q.rc * vni;
    f.r[i] = ri;
  }
  const cx<R> t = q.sg * (f.w[i] - q.alpha * vni) - q.bs * vpi;
  f.vp[i] = t;
  const c64 td = up(t);
  acc[0].x += abs2(td);
  acc[0].y += abs2(up(ri));
  acc[1] = acc[1] + td * td;
  return t;
}

// ============================================================================
// Outer (FP64) refinement, incident field, cross sections, gradient
// ============================================================================

// Incident plane wave E[r][c][n] = ehat_r[c] exp(i k khat_r . r_n) (Sec. 1),
// site coordinates from the linear index n = k*J*K + j*K + i.
__global__ void k_einc(c64* __restrict__ E, const int* __restrict__ sites, long nd, int K, int J, double k,
                       const double* __restrict__ khat, const double* __restrict__ ehat) {
  const int rhs = blockIdx.y;
  const double* kh = khat + 3 * rhs;
  const double* eh = ehat + 6 * rhs;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < nd; n += (long)gridDim.x * blockDim.x) {
    const int s = sites[n];
    const double x = s % K, y = (s / K) % J, z = s / (K * J);
    double sn, cs;
    sincos(k * (kh[0] * x + kh[1] * y + kh[2] * z), &sn, &cs);
    const c64 ph = mk(cs, sn);
    for (int c = 0; c < 3; ++c) E[((long)rhs * 3 + c) * nd + n] = mk(eh[2 * c], eh[2 * c + 1]) * ph;
  }
}

// out[r] = (jacobi ? s_n : 1) * in[r] * scale_r  (FP64 -> precision R), the
// right-hand side of an inner solve
template <typename R>
__global__ void k_scale_rhs(const c64* __restrict__ in, cx<R>* __restrict__ out, const c64* __restrict__ a0,
                            const c64* __restrict__ a1, const double* __restrict__ S,
                            const double* __restrict__ sc, const int* __restrict__ active, long nd,
                            int jacobi) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const long n3 = 3 * nd;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x) {
    c64 v = sc[rhs] * in[(long)rhs * n3 + i];
    if (jacobi) {
      c64 a = a0[i];
      if (a1) a = a + S[rhs] * a1[i];
      v = cdiv(mk(1.0, 0.0), csqrt(a)) * v;
    }
    out[(long)rhs * n3 + i] = cvt<R>(v);
  }
}

// P += (jacobi ? s_n : 1) * d * scale_r   (d in precision R)
template <typename R>
__global__ void k_accumulate(c64* __restrict__ P, const cx<R>* __restrict__ d, const c64* __restrict__ a0,
                             const c64* __restrict__ a1, const double* __restrict__ S,
                             const double* __restrict__ sc, const int* __restrict__ active, long nd,
                             int jacobi) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const long n3 = 3 * nd;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x) {
    c64 v = sc[rhs] * up(d[(long)rhs * n3 + i]);
    if (jacobi) {
      c64 a = a0[i];
      if (a1) a = a + S[rhs] * a1[i];
      v = cdiv(mk(1.0, 0.0), csqrt(a)) * v;
    }
    P[(long)rhs * n3 + i] = P[(long)rhs * n3 + i] + v;
  }
}

// r = E - y; partials |r|^2 and |E|^2
__global__ void __launch_bounds__(kRedThreads) k_residual(const c64* __restrict__ E, const c64* __restrict__ y,
                                                  c64* __restrict__ r, SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
    const c64 e = E[o + i];
    const c64 rv = e - y[o + i];
    r[o + i] = rv;
    acc[0].x += abs2(rv);
    acc[1].x += abs2(e);
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// Sums for the cross sections (Draine 1988, |E0| = 1):
//   [0] sum Im(E^* . P)              -> C_ext = 4 pi k [0]
//   [1] sum_c,n |P_cn|^2 (-Im a_cn - 2k^3/3)  -> C_abs = 4 pi k [1]
__global__ void __launch_bounds__(kRedThreads) k_cross_sums(const c64* __restrict__ E, const c64* __restrict__ P,
                                                    const c64* __restrict__ a0, const c64* __restrict__ a1,
                                                    const double* __restrict__ S, long nd, double k,
                                                    SolverDims dm, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
  const long o = (long)rhs * dm.n3;
  const double rad = (2.0 / 3.0) * k * k * k;
  DDA_RANGE(dm, i) {
    const c64 pv = P[o + i];
    acc[0].x += (conjg(E[o + i]) * pv).y;
    c64 a = a0[i];
    if (a1) a = a + S[rhs] * a1[i];
    acc[1].x += abs2(pv) * (-a.y - rad);
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    part[((long)rhs * dm.nblk + blockIdx.x) * 2] = acc[0];
    part[((long)rhs * dm.nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// Adjoint right-hand side W conj(P), w_cn = 4 pi k (-Im alpha_cn^{-1} - 2k^3/3)
__global__ void k_adjoint_rhs(const c64* __restrict__ P, c64* __restrict__ out, const c64* __restrict__ a0,
                              const c64* __restrict__ a1, const double* __restrict__ S, long nd, double k,
                              int nrhs) {
  const long n3 = 3 * nd;
  const double rad = (2.0 / 3.0) * k * k * k, fk = 4.0 * M_PI * k;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < n3 * nrhs; g += (long)gridDim.x * blockDim.x) {
    const int rhs = (int)(g / n3);
    const long e = g % n3;
    c64 a = a0[e];
    if (a1) a = a + S[rhs] * a1[e];
    out[g] = (fk * (-a.y - rad)) * conjg(P[g]);
  }
}

// dC_abs/d eps_n from the forward and adjoint solutions (A mu = W conj(P)):
//   dC/dRe = -2 Re[(mu_n . P_n) a'] - 4 pi k Im[a'] |P_n|^2
//   dC/dIm = +2 Im[(mu_n . P_n) a'] - 4 pi k Re[a'] |P_n|^2
// with a' = d alpha_n^{-1} / d eps_n = d0[n] + S_r d1[n]; out = dRe + i dIm.
__global__ void k_gradient(const c64* __restrict__ P, const c64* __restrict__ mu, const c64* __restrict__ d0,
                           const c64* __restrict__ d1, const double* __restrict__ S, long nd, double k,
                           int nrhs, c64* __restrict__ grad) {
  const double fk = 4.0 * M_PI * k;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < nd * nrhs; g += (long)gridDim.x * blockDim.x) {
    const int rhs = (int)(g / nd);
    const long n = g % nd;
    const long o = (long)rhs * 3 * nd + n;
    c64 muP = mk(0.0, 0.0);
    double p2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      muP = muP + mu[o + c * nd] * P[o + c * nd];
      p2 += abs2(P[o + c * nd]);
    }
    c64 da = d0[n];
    if (d1) da = da + S[rhs] * d1[n];
    const c64 m = muP * da;
    grad[g] = mk(-2.0 * m.x - fk * da.y * p2, 2.0 * m.y - fk * da.x * p2);
  }
}

}  // namespace dda
