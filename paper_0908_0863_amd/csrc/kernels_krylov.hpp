// Krylov solvers with longer recurrences: BiCG (Fletcher 1975) and QMR with
// coupled two-term recurrences (Freund & Nachtigal), both with shadow
// products A^H y; BiCGSTAB(l) (Sleijpen & Fokkema 1993, the restarted
// "RBiCGSTAB" of the paper's list of schemes, Sec. 4) and ML(n)BiCGSTAB in
// its IDR(s) form (Sonneveld & van Gijzen 2008, biorthogonal variant).
//
// They are built from three generic kernels driven by a fixed host-side
// program per solver, so the iteration is still a device-only kernel
// sequence that a HIP graph can capture:
//   k_gen_dot     up to kGenDots inner products per right-hand side, FP64
//                 partial sums per block
//   k_gen_scalar  one block per right-hand side: fixed-order reduction of the
//                 partials, then one step of the solver's scalar recurrence in
//                 FP64 (stopping tests included)
//   k_gen_lin     up to kGenOut linear combinations V[out] = sum c_t V[src_t],
//                 applied in order per element (an output may feed a later
//                 one), coefficients read from the per-RHS scalar state.
//
// Shadow products.  A and its Point-Jacobi form D^{-1/2} A D^{-1/2} are
// complex symmetric (A^T = A), so A^H y = conj(A conj(y)).  The shadow
// vectors are stored conjugated: for yh = conj(y) the shadow recurrence
// y' = A^H z - conj(c) y reads yh' = A zh - c yh, and a Hermitian product
// y^H x with a shadow vector becomes the bilinear yh^T x.  One matrix-vector
// kernel therefore serves both Lanczos sequences.
#pragma once
#include "common.hpp"
#include "kernels_solver.hpp"

namespace dda {

constexpr int kGenDots = 16;   // inner products per k_gen_dot launch
constexpr int kGenOut = 8;     // outputs per k_gen_lin launch
constexpr int kGenTerms = 10;  // terms per output
constexpr int kGenScal = 40;   // complex scalars per right-hand side
constexpr int kGenMaxParam = 4;  // l of BiCGSTAB(l), n of ML(n)BiCGSTAB

// Coefficient code of a k_gen_lin term: scalar index (kGenOne = 1.0), with
// flags to negate the coefficient and to conjugate the source vector.
constexpr short kGenOne = kGenScal;
constexpr short kGenNeg = 0x100;
constexpr short kGenConj = 0x200;

struct GenState {
  double bnorm2, rnorm2, tol2, best2;
  int converged, breakdown, iters, mv, best_mv, ver;
  c64 s[kGenScal];
};

struct GenDots {
  int n;
  signed char a[kGenDots], b[kGenDots], herm[kGenDots];  // slots; herm: a^H b, else a^T b
};

struct GenLin {
  int nout;
  signed char out[kGenOut], nt[kGenOut];
  signed char src[kGenOut][kGenTerms];
  short coef[kGenOut][kGenTerms];
};

// solver ids of the generic engine (the C ABI's enum values)
enum { GEN_BICG = 5, GEN_QMR = 6, GEN_BICGSTAB_L = 7, GEN_IDR = 8 };
// steps: 0 initialises every solver; the others are per solver
enum { GS_INIT = 0, GS_A = 1, GS_B = 2, GS_C = 3 };
struct GenStep {
  int solver, step, sub, param, mv_per_iter;
};

// Scalar slots of each solver's state.
enum { BG_RHO, BG_RHO_OLD, BG_BETA, BG_ALPHA };
enum { QM_RHO, QM_XI, QM_DELTA, QM_EPS, QM_BETA, QM_THETA, QM_GAMMA, QM_ETA, QM_INVRHO, QM_INVXI, QM_CP, QM_CQ, QM_CD };
enum { BL_RHO0, BL_ALPHA, BL_OMEGA, BL_BETA, BL_GAM /* gamma_j at BL_GAM + j - 1, j = 1..l */ };
enum { ID_OMEGA, ID_BETA, ID_F = 2, ID_C = ID_F + kGenMaxParam, ID_OC = ID_C + kGenMaxParam,
       ID_AL = ID_OC + kGenMaxParam, ID_M = ID_AL + kGenMaxParam /* M[j][i] at ID_M + j * 4 + i */ };
static_assert(ID_M + kGenMaxParam * kGenMaxParam <= kGenScal, "IDR scalars exceed the state");

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_gen_dot(const cx<R>* __restrict__ V, long vsz, GenDots d,
                                                     const int* __restrict__ active, SolverDims dm,
                                                     c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  c64 acc[kGenDots];
#pragma unroll
  for (int q = 0; q < kGenDots; ++q) acc[q] = mk(0.0, 0.0);
  const long o = (long)rhs * dm.n3;
  DDA_RANGE(dm, i) {
#pragma unroll
    for (int q = 0; q < kGenDots; ++q) {
      if (q < d.n) {
        const c64 x = up(V[d.a[q] * vsz + o + i]);
        const c64 y = up(V[d.b[q] * vsz + o + i]);
        acc[q] = acc[q] + (d.herm[q] ? conjg(x) : x) * y;
      }
    }
  }
  block_sum<kGenDots>(acc);
  if (threadIdx.x == 0) {
    c64* p = part + ((long)rhs * dm.nblk + blockIdx.x) * kGenDots;
#pragma unroll
    for (int q = 0; q < kGenDots; ++q) p[q] = acc[q];  // unused entries hold zeros
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_gen_lin(cx<R>* V, long vsz, GenLin L, const GenState* __restrict__ st,
                                                 const int* __restrict__ active, long n3) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  __shared__ cx<R> cf[kGenOut][kGenTerms];
  for (int e = threadIdx.x; e < kGenOut * kGenTerms; e += blockDim.x) {
    const int oo = e / kGenTerms, tt = e - oo * kGenTerms;
    const short code = L.coef[oo][tt];
    const int idx = code & 0xff;
    c64 v = idx >= kGenScal ? mk(1.0, 0.0) : st[rhs].s[idx];
    if (code & kGenNeg) v = mk(-v.x, -v.y);
    cf[oo][tt] = cvt<R>(v);
  }
  __syncthreads();
  const long o = (long)rhs * n3;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x) {
    for (int q = 0; q < L.nout; ++q) {
      cx<R> acc = mk((R)0, (R)0);
      for (int t = 0; t < L.nt[q]; ++t) {
        cx<R> x = V[L.src[q][t] * vsz + o + i];
        if (L.coef[q][t] & kGenConj) x = conjg(x);
        acc = acc + cf[q][t] * x;
      }
      V[L.out[q] * vsz + o + i] = acc;
    }
  }
}

// SplitMix64 (Steele, Lea & Flood 2014): the counter-based generator of the
// shadow vectors of IDR(s); entry i of vector `slot` of right-hand side `rhs`
// hashes the counter (seed, rhs, slot, i).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// V[slot] = (u1 + i u2) / sqrt(n3) with u1, u2 uniform in [-1, 1).
template <typename R>
__global__ void __launch_bounds__(256) k_gen_random(cx<R>* __restrict__ V, long vsz, int slot, uint64_t seed,
                                                    const int* __restrict__ active, long n3) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const double sc = 1.0 / sqrt((double)n3);
  const long o = (long)rhs * n3;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x) {
    const uint64_t key = seed ^ ((uint64_t)rhs << 48) ^ ((uint64_t)slot << 40);
    const uint64_t h1 = splitmix64(key + 2 * (uint64_t)i), h2 = splitmix64(key + 2 * (uint64_t)i + 1);
    const double u1 = (double)(h1 >> 11) * 0x1.0p-52 - 1.0, u2 = (double)(h2 >> 11) * 0x1.0p-52 - 1.0;
    V[slot * vsz + o + i] = mk((R)(sc * u1), (R)(sc * u2));
  }
}

// ---------------------------------------------------------------------------
// Scalar recurrences (thread 0 of one block per right-hand side)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool gen_tiny(c64 a, double scale2) {
  return !(abs2(a) > 1e-60 * scale2) || !isfinite(a.x) || !isfinite(a.y);
}
__device__ __forceinline__ c64 neg(c64 a) { return mk(-a.x, -a.y); }

// Start of an iteration: count it and test the recursive residual.
template <typename R>
__device__ int gen_check(GenState& s, double r2, int mv_per_iter) {
  s.iters += 1;
  if (s.iters > 0) s.mv += mv_per_iter;
  s.rnorm2 = r2;
  if (!isfinite(r2)) {
    s.breakdown = 1;
    return 1;
  }
  if (r2 <= s.tol2) {
    s.converged = 1;
    return 1;
  }
  if (r2 < 0.98 * s.best2) {
    s.best2 = r2;
    s.best_mv = s.mv;
  } else if (s.mv - s.best_mv > 2 * kStallWindow && r2 < stall_level2<R>() * s.bnorm2) {
    s.breakdown = 2;  // stagnated: the refinement loop restarts from the true residual
    return 1;
  }
  return 0;
}

// Forward substitution M c = f on the lower-triangular block M[k0..n)[k0..n)
// of the IDR(s) matrix (M[j][i] = P_j^H G_i); false if a pivot vanishes.
__device__ __forceinline__ bool idr_lower_solve(const GenState& s, int k0, int n, c64* out) {
  for (int k = k0; k < n; ++k) {
    c64 acc = s.s[ID_F + k];
    for (int i = k0; i < k; ++i) acc = acc - s.s[ID_M + k * kGenMaxParam + i] * out[i];
    const c64 piv = s.s[ID_M + k * kGenMaxParam + k];
    if (gen_tiny(piv, 1e-200)) return false;
    out[k] = cdiv(acc, piv);
  }
  return true;
}

// Returns 1 when the right-hand side stops (converged, breakdown, stagnation).
template <typename R>
__device__ int gen_step(const GenStep& g, GenState& s, const c64* v, double tol) {
  const double b2 = s.bnorm2;
  if (g.step == GS_INIT) {
    s.bnorm2 = s.rnorm2 = s.best2 = v[0].x;
    s.tol2 = tol * tol * v[0].x;
    s.converged = !(v[0].x > 0.0);
    s.breakdown = 0;
    s.iters = -1;
    s.mv = s.best_mv = 0;
    s.ver = 0;
    for (int q = 0; q < kGenScal; ++q) s.s[q] = mk(0.0, 0.0);
    if (g.solver == GEN_QMR) {
      const double nb = sqrt(v[0].x);
      s.s[QM_RHO] = mk(nb, 0.0);
      s.s[QM_GAMMA] = mk(1.0, 0.0);
      s.s[QM_ETA] = mk(-1.0, 0.0);
      s.s[QM_EPS] = mk(1.0, 0.0);
    } else if (g.solver == GEN_BICGSTAB_L) {
      s.s[BL_RHO0] = mk(1.0, 0.0);
      s.s[BL_OMEGA] = mk(1.0, 0.0);
    } else if (g.solver == GEN_IDR) {
      s.s[ID_OMEGA] = mk(1.0, 0.0);
      for (int j = 0; j < kGenMaxParam; ++j) s.s[ID_M + j * kGenMaxParam + j] = mk(1.0, 0.0);
    }
    return s.converged;
  }
  c64* x = s.s;
  switch (g.solver) {
    // ---- BiCG: dots A = [|r|^2, rh^T r], B = [ph^T q]
    case GEN_BICG:
      if (g.step == GS_A) {
        if (gen_check<R>(s, v[0].x, g.mv_per_iter)) return 1;
        x[BG_RHO_OLD] = x[BG_RHO];
        x[BG_RHO] = v[1];
        if (gen_tiny(v[1], b2 * b2)) break;
        x[BG_BETA] = s.iters == 0 ? mk(0.0, 0.0) : cdiv(x[BG_RHO], x[BG_RHO_OLD]);
        return 0;
      } else {
        if (gen_tiny(v[0], b2 * b2)) break;
        x[BG_ALPHA] = cdiv(x[BG_RHO], v[0]);
        return 0;
      }
    // ---- QMR: A = [|r|^2, |wt|^2, wt^T vt], B = [qh^T pt], C = [|vt|^2]
    case GEN_QMR:
      if (g.step == GS_A) {
        if (gen_check<R>(s, v[0].x, g.mv_per_iter)) return 1;
        const double rho = x[QM_RHO].x, xi = sqrt(v[1].x);
        if (!(rho > 1e-30 * sqrt(b2)) || !(xi > 1e-30 * sqrt(b2))) break;
        const c64 delta = (1.0 / (rho * xi)) * v[2];
        if (gen_tiny(delta, 1.0)) break;
        x[QM_XI] = mk(xi, 0.0);
        x[QM_DELTA] = delta;
        x[QM_INVRHO] = mk(1.0 / rho, 0.0);
        x[QM_INVXI] = mk(1.0 / xi, 0.0);
        if (s.iters == 0) {
          x[QM_CP] = x[QM_CQ] = mk(0.0, 0.0);
        } else {
          x[QM_CP] = cdiv(xi * delta, x[QM_EPS]);
          x[QM_CQ] = cdiv(rho * delta, x[QM_EPS]);
        }
        return 0;
      } else if (g.step == GS_B) {
        if (gen_tiny(v[0], 1.0)) break;  // v and w are unit vectors: eps is scale-free
        x[QM_EPS] = v[0];
        x[QM_BETA] = cdiv(v[0], x[QM_DELTA]);
        if (gen_tiny(x[QM_BETA], 1e-200)) break;
        return 0;
      } else {
        const double rho_n = sqrt(v[0].x), rho = x[QM_RHO].x;
        const double g_old = x[QM_GAMMA].x, th_old = x[QM_THETA].x;
        const c64 beta = x[QM_BETA];
        const double theta = rho_n / (g_old * sqrt(abs2(beta)));
        const double gam = 1.0 / sqrt(1.0 + theta * theta);
        if (!(gam > 0.0) || !isfinite(theta)) break;
        // eta_i = -eta_{i-1} rho_i gamma_i^2 / (beta_i gamma_{i-1}^2)
        const c64 eta = cdiv((-rho * gam * gam / (g_old * g_old)) * x[QM_ETA], beta);
        x[QM_CD] = mk((th_old * gam) * (th_old * gam), 0.0);
        x[QM_ETA] = eta;
        x[QM_THETA] = mk(theta, 0.0);
        x[QM_GAMMA] = mk(gam, 0.0);
        x[QM_RHO] = mk(rho_n, 0.0);
        return 0;
      }
    // ---- BiCGSTAB(l): A(j) = [|r_0|^2 (j = 0), rt^H r_j], B(j) = [rt^H u_{j+1}],
    //      C = Gram matrix of r_1..r_l and r_i^H r_0
    case GEN_BICGSTAB_L: {
      const int l = g.param, j = g.sub;
      if (g.step == GS_A) {
        const c64 rho1 = j == 0 ? v[1] : v[0];
        if (j == 0) {
          if (gen_check<R>(s, v[0].x, g.mv_per_iter)) return 1;
          x[BL_RHO0] = neg(x[BL_OMEGA] * x[BL_RHO0]);
        }
        if (gen_tiny(x[BL_RHO0], b2 * b2 * 1e-200)) break;
        x[BL_BETA] = cdiv(x[BL_ALPHA] * rho1, x[BL_RHO0]);
        x[BL_RHO0] = rho1;
        return 0;
      } else if (g.step == GS_B) {
        if (gen_tiny(v[0], b2 * b2)) break;
        x[BL_ALPHA] = cdiv(x[BL_RHO0], v[0]);
        return 0;
      } else {
        // minimise |r_0 - sum_j gamma_j r_j| : Z gamma = y, Z_ik = r_i^H r_k, y_i = r_i^H r_0
        c64 Z[kGenMaxParam][kGenMaxParam + 1];
        int q = 0;
        for (int i = 0; i < l; ++i)
          for (int k = i; k < l; ++k) {
            Z[i][k] = v[q];
            Z[k][i] = conjg(v[q]);
            ++q;
          }
        for (int i = 0; i < l; ++i) Z[i][l] = v[q + i];
        // Gaussian elimination with partial pivoting (Z is Hermitian positive
        // definite unless the r_j are linearly dependent)
        for (int c = 0; c < l; ++c) {
          int pr = c;
          for (int r = c + 1; r < l; ++r)
            if (abs2(Z[r][c]) > abs2(Z[pr][c])) pr = r;
          if (!(abs2(Z[pr][c]) > 1e-300)) {
            s.breakdown = 1;  // r_1..r_l linearly dependent
            return 1;
          }
          if (pr != c)
            for (int k = 0; k <= l; ++k) {
              const c64 tmp = Z[c][k];
              Z[c][k] = Z[pr][k];
              Z[pr][k] = tmp;
            }
          for (int r = c + 1; r < l; ++r) {
            const c64 f = cdiv(Z[r][c], Z[c][c]);
            for (int k = c; k <= l; ++k) Z[r][k] = Z[r][k] - f * Z[c][k];
          }
        }
        for (int c = l - 1; c >= 0; --c) {
          c64 acc = Z[c][l];
          for (int k = c + 1; k < l; ++k) acc = acc - Z[c][k] * x[BL_GAM + k];
          x[BL_GAM + c] = cdiv(acc, Z[c][c]);
        }
        x[BL_OMEGA] = x[BL_GAM + l - 1];
        for (int c = 0; c < l; ++c)
          if (!isfinite(x[BL_GAM + c].x) || !isfinite(x[BL_GAM + c].y)) {
            s.breakdown = 1;
            return 1;
          }
        if (gen_tiny(x[BL_OMEGA], 1e-200)) break;
        return 0;
      }
    }
    // ---- IDR(s): A = [P_j^H r, |r|^2], B(k) = [P_j^H G_k], C = [t^H r, t^H t]
    case GEN_IDR: {
      const int n = g.param;
      if (g.step == GS_A) {
        if (gen_check<R>(s, v[n].x, g.mv_per_iter)) return 1;
        for (int j = 0; j < n; ++j) x[ID_F + j] = v[j];
        c64 c[kGenMaxParam];
        if (!idr_lower_solve(s, 0, n, c)) break;
        for (int j = 0; j < n; ++j) {
          x[ID_C + j] = c[j];
          x[ID_OC + j] = x[ID_OMEGA] * c[j];
        }
        return 0;
      } else if (g.step == GS_B) {
        const int k = g.sub;
        // alpha_i (i < k): M[0..k)[0..k) alpha = P_{0..k}^H G_k, so that G_k
        // loses its components along G_0..G_{k-1} seen by P_0..P_{k-1}
        c64 al[kGenMaxParam];
        for (int i = 0; i < k; ++i) {
          c64 acc = v[i];
          for (int m = 0; m < i; ++m) acc = acc - x[ID_M + i * kGenMaxParam + m] * al[m];
          const c64 piv = x[ID_M + i * kGenMaxParam + i];
          if (gen_tiny(piv, 1e-200)) {
            s.breakdown = 1;
            return 1;
          }
          al[i] = cdiv(acc, piv);
          x[ID_AL + i] = al[i];
        }
        for (int j = k; j < n; ++j) {
          c64 acc = v[j];
          for (int i = 0; i < k; ++i) acc = acc - x[ID_M + j * kGenMaxParam + i] * al[i];
          x[ID_M + j * kGenMaxParam + k] = acc;
        }
        const c64 mkk = x[ID_M + k * kGenMaxParam + k];
        if (gen_tiny(mkk, 1e-200)) break;
        const c64 beta = cdiv(x[ID_F + k], mkk);
        x[ID_BETA] = beta;
        for (int j = k + 1; j < n; ++j) x[ID_F + j] = x[ID_F + j] - beta * x[ID_M + j * kGenMaxParam + k];
        if (k + 1 < n) {
          c64 c[kGenMaxParam];
          if (!idr_lower_solve(s, k + 1, n, c)) break;
          for (int j = k + 1; j < n; ++j) {
            x[ID_C + j] = c[j];
            x[ID_OC + j] = x[ID_OMEGA] * c[j];
          }
        }
        return 0;
      } else {
        if (!(v[1].x > 1e-300)) break;
        x[ID_OMEGA] = (1.0 / v[1].x) * v[0];
        if (gen_tiny(x[ID_OMEGA], 1e-200)) break;
        return 0;
      }
    }
    default:
      break;
  }
  s.breakdown = 1;  // a vanishing denominator: restart from the current iterate
  return 1;
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_gen_scalar(const c64* __restrict__ part, int nblk, GenStep g,
                                                        GenState* __restrict__ st, int* __restrict__ active,
                                                        const double* __restrict__ tolv) {
  const int rhs = blockIdx.x;
  if (!active[rhs]) return;
  __shared__ GenState sh;
  constexpr int W = sizeof(GenState) / sizeof(int);
  static_assert(sizeof(GenState) % sizeof(int) == 0, "state is copied as words");
  for (int e = threadIdx.x; e < W; e += blockDim.x)
    reinterpret_cast<int*>(&sh)[e] = reinterpret_cast<const int*>(st + rhs)[e];
  c64 v[kGenDots];
  reduce_partials<kGenDots>(part, nblk, rhs, v);  // ends with a barrier
  if (threadIdx.x == 0) {
    const int stop = gen_step<R>(g, sh, v, tolv[rhs]);
    sh.ver += 1;
    if (stop) active[rhs] = 0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < W; e += blockDim.x)
    reinterpret_cast<int*>(st + rhs)[e] = reinterpret_cast<const int*>(&sh)[e];
}

}  // namespace dda
