// Far-field outputs of a solved polarisation: the scattering amplitude of the
// dipole array in any direction, C_sca by angular quadrature, and the
// amplitude and Mueller matrices (the quantities the paper's code reports
// after the solve, Sec. 6: Q_sca; formulas of Draine 1988 and Bohren &
// Huffman 1983, Sec. 3.2-3.3).
//
// F(n) = k^2 (I - n n) A(n),  A(n) = sum_m e^{-i k n . r_m} P_m,
// the scattered field being e^{ikr}/r F(n) as r -> infinity (|E0| = 1).
// Lattice sites are integer points, so e^{-i k n . r} = a_x^i a_y^j a_z^l
// with a per-axis table a_x^i = e^{-i k n_x i}: each block builds the tables
// of its directions in LDS once and each dipole then costs two complex
// products per direction instead of a sine and cosine.
#pragma once
#include "common.hpp"
#include "kernels_solver.hpp"

namespace dda {

constexpr int kFarDirs = 4;  // directions per block

// part[((rhs * ntile + tile) * nchunk + chunk) * kFarDirs * 3 + d * 3 + c]:
// partial A_c over the dipoles of `chunk` for direction tile * kFarDirs + d.
__global__ void __launch_bounds__(kRedThreads) k_far_partial(const c64* __restrict__ P, const int* __restrict__ sites,
                                                        long nd, int K, int J, int L, double k,
                                                        const double* __restrict__ dirs, int ndir, int nchunk,
                                                        c64* __restrict__ part) {
  extern __shared__ c64 tab[];  // [kFarDirs][K + J + L]
  const int tile = blockIdx.x, chunk = blockIdx.y, rhs = blockIdx.z;
  const int ntile = gridDim.x;
  const int W = K + J + L;
  for (int e = threadIdx.x; e < kFarDirs * W; e += blockDim.x) {
    const int d = e / W, x = e - d * W;
    const int dir = tile * kFarDirs + d;
    c64 v = mk(0.0, 0.0);
    if (dir < ndir) {
      const int axis = x < K ? 0 : (x < K + J ? 1 : 2);
      const int xv = axis == 0 ? x : (axis == 1 ? x - K : x - K - J);
      double sn, cs;
      sincos(-k * dirs[3 * dir + axis] * (double)xv, &sn, &cs);
      v = mk(cs, sn);
    }
    tab[e] = v;
  }
  __syncthreads();
  c64 acc[kFarDirs * 3];
#pragma unroll
  for (int q = 0; q < kFarDirs * 3; ++q) acc[q] = mk(0.0, 0.0);
  const long per = (nd + nchunk - 1) / nchunk;
  const long n0 = (long)chunk * per, n1 = n0 + per < nd ? n0 + per : nd;
  const c64* Pr = P + (long)rhs * 3 * nd;
  for (long n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    const int s = sites[n];
    const int i = s % K, j = (s / K) % J, l = s / (K * J);
    const c64 p0 = Pr[n], p1 = Pr[nd + n], p2 = Pr[2 * nd + n];
#pragma unroll
    for (int d = 0; d < kFarDirs; ++d) {
      const c64 e = tab[d * W + i] * tab[d * W + K + j] * tab[d * W + K + J + l];
      acc[3 * d] = acc[3 * d] + e * p0;
      acc[3 * d + 1] = acc[3 * d + 1] + e * p1;
      acc[3 * d + 2] = acc[3 * d + 2] + e * p2;
    }
  }
  block_sum<kFarDirs * 3>(acc);
  if (threadIdx.x == 0) {
    c64* out = part + (((long)rhs * ntile + tile) * nchunk + chunk) * kFarDirs * 3;
#pragma unroll
    for (int q = 0; q < kFarDirs * 3; ++q) out[q] = acc[q];
  }
}

// F[rhs][dir][c] = k^2 (A - n (n . A)), A summed over the chunks in order.
__global__ void k_far_finish(const c64* __restrict__ part, int ntile, int nchunk, const double* __restrict__ dirs,
                             int ndir, int nrhs, double k, c64* __restrict__ F) {
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g >= (long)nrhs * ndir) return;
  const int rhs = (int)(g / ndir), dir = (int)(g - (long)rhs * ndir);
  const int tile = dir / kFarDirs, d = dir - tile * kFarDirs;
  c64 A[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int ch = 0; ch < nchunk; ++ch) {
    const c64* p = part + (((long)rhs * ntile + tile) * nchunk + ch) * kFarDirs * 3 + 3 * d;
    for (int c = 0; c < 3; ++c) A[c] = A[c] + p[c];
  }
  const double n[3] = {dirs[3 * dir], dirs[3 * dir + 1], dirs[3 * dir + 2]};
  const c64 nA = n[0] * A[0] + n[1] * A[1] + n[2] * A[2];
  const double k2 = k * k;
  for (int c = 0; c < 3; ++c) F[g * 3 + c] = k2 * (A[c] - n[c] * nA);
}

// Partials of sum_d w_d |F_d|^2 per right-hand side (C_sca quadrature).
__global__ void __launch_bounds__(kRedThreads) k_far_power(const c64* __restrict__ F, const double* __restrict__ w,
                                                      int ndir, c64* __restrict__ part) {
  const int rhs = blockIdx.y;
  c64 acc[1] = {mk(0.0, 0.0)};
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < ndir; d += gridDim.x * blockDim.x) {
    const c64* f = F + ((long)rhs * ndir + d) * 3;
    acc[0].x += w[d] * (abs2(f[0]) + abs2(f[1]) + abs2(f[2]));
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = acc[0];
}

// Amplitude matrix (S1, S2, S3, S4) and Mueller matrix for incidence along +z
// from the far fields Fx, Fy of the x- and y-polarised solves at (theta, phi):
// basis e_par,i = cos(phi) x + sin(phi) y, e_perp,i = sin(phi) x - cos(phi) y,
// e_par,s = theta-hat, e_perp,s = -phi-hat, and
// [E_par,s, E_perp,s] = e^{ikr}/(-ikr) [[S2, S3], [S4, S1]] [E_par,i, E_perp,i].
// Mueller elements in the closed form of Bohren & Huffman (Eq. 3.16).
__global__ void k_mueller(const c64* __restrict__ Fx, const c64* __restrict__ Fy, const double* __restrict__ tp,
                          int ndir, double k, c64* __restrict__ Sout, double* __restrict__ M) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndir) return;
  const double th = tp[2 * d], ph = tp[2 * d + 1];
  double st, ct, sp, cp;
  sincos(th, &st, &ct);
  sincos(ph, &sp, &cp);
  const double that[3] = {ct * cp, ct * sp, -st};
  const double phat[3] = {-sp, cp, 0.0};
  c64 fpar[3], fperp[3];
  for (int c = 0; c < 3; ++c) {
    fpar[c] = cp * Fx[3 * d + c] + sp * Fy[3 * d + c];
    fperp[c] = sp * Fx[3 * d + c] - cp * Fy[3 * d + c];
  }
  auto dotr = [](const double* a, const c64* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  const c64 mik = mk(0.0, -k);
  const c64 S2 = mik * dotr(that, fpar);
  const c64 S3 = mik * dotr(that, fperp);
  const c64 S4 = (-1.0) * (mik * dotr(phat, fpar));
  const c64 S1 = (-1.0) * (mik * dotr(phat, fperp));
  if (Sout) {
    Sout[4 * d] = S1;
    Sout[4 * d + 1] = S2;
    Sout[4 * d + 2] = S3;
    Sout[4 * d + 3] = S4;
  }
  if (!M) return;
  const double a1 = abs2(S1), a2 = abs2(S2), a3 = abs2(S3), a4 = abs2(S4);
  const c64 s23 = S2 * conjg(S3), s14 = S1 * conjg(S4), s24 = S2 * conjg(S4), s13 = S1 * conjg(S3);
  const c64 s12 = S1 * conjg(S2), s34 = S3 * conjg(S4);
  double* m = M + 16 * d;
  m[0] = 0.5 * (a1 + a2 + a3 + a4);
  m[1] = 0.5 * (a2 - a1 + a4 - a3);
  m[2] = s23.x + s14.x;
  m[3] = s23.y - s14.y;
  m[4] = 0.5 * (a2 - a1 - a4 + a3);
  m[5] = 0.5 * (a2 + a1 - a4 - a3);
  m[6] = s23.x - s14.x;
  m[7] = s23.y + s14.y;
  m[8] = s24.x + s13.x;
  m[9] = s24.x - s13.x;
  m[10] = s12.x + s34.x;
  m[11] = -s12.y - s34.y;  // Im(S2 S1^* + S4 S3^*)
  m[12] = -s24.y + s13.y;  // Im(S2^* S4 + S3^* S1)
  m[13] = -s24.y - s13.y;  // Im(S4 S2^* - S1 S3^*)
  m[14] = s12.y - s34.y;
  m[15] = s12.x - s34.x;
}

}  // namespace dda
