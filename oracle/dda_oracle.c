/*
 * Plain FP64 CPU oracle for the discrete dipole approximation (DDA).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * path.
 *
 * What it computes is the plain definition of the DDA system (Eq. 1 of the
 * paper, written in Gaussian units with lattice spacing d = 1):
 *
 *     A_nn = alpha_n^{-1} I3,      A_nm = -G(r_n - r_m)   (n != m)
 *     G(r) = e^{ikr}/r^3 [ k^2 r^2 (I - rr) + (1 - ikr)(3 rr - I) ],  rr = r^ r^
 *
 * The paper's own normalisation, A^paper (k^2/eps0) = -G/(4 pi eps0), differs
 * from this by a global constant only; cross sections are identical.
 *
 * Vectors are stored component-major: v[c * nd + n], c = 0,1,2 (x,y,z), which
 * is the split into three component vectors of the paper's Sec. 3.
 * Sites are integer lattice coordinates (i,j,k), listed in increasing linear
 * index n = k*J*K + j*K + i (Appendix A).
 *
 * Everything is O(N_d^2) direct summation: no FFT, no Toeplitz structure.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Tensor t(r) = -G(r) for one displacement r != 0, as the six independent
 * components xx, xy, xz, yy, yz, zz (the ordering T0..T5 of Sec. 3).
 * Eq. 1 of the paper; the rr-dyadic is Eq. 2. */
void ora_neg_green(double k, double rx, double ry, double rz, double *out /* 12 doubles */)
{
    double r2 = rx * rx + ry * ry + rz * rz;
    double r = sqrt(r2);
    double u[3] = {rx / r, ry / r, rz / r};
    cplx ph = cexp(I * k * r) / (r2 * r);
    cplx a = k * k * r2;          /* coefficient of (I - rr)   */
    cplx b = 1.0 - I * k * r;     /* coefficient of (3rr - I)  */
    int comp[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int c = 0; c < 6; ++c) {
        int p = comp[c][0], q = comp[c][1];
        double d = (p == q) ? 1.0 : 0.0;
        double uu = u[p] * u[q];
        cplx g = ph * (a * (d - uu) + b * (3.0 * uu - d));
        out[2 * c] = -creal(g);
        out[2 * c + 1] = -cimag(g);
    }
}

/* -G at many displacements: r*: [n], out: [6][n] complex (interleaved re,im).
 * A zero displacement yields 0 (the self term is not part of the convolution,
 * Sec. 3 and step 5 of the standard algorithm). */
void ora_neg_green_many(double k, int64_t n, const double *rx, const double *ry, const double *rz,
                        double *out)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t q = 0; q < n; ++q) {
        double o[12] = {0};
        if (rx[q] != 0.0 || ry[q] != 0.0 || rz[q] != 0.0) ora_neg_green(k, rx[q], ry[q], rz[q], o);
        for (int c = 0; c < 6; ++c) {
            out[2 * (c * n + q)] = o[2 * c];
            out[2 * (c * n + q) + 1] = o[2 * c + 1];
        }
    }
}

/* full 3x3 of -G, row-major */
static void neg_green_3x3(double k, double rx, double ry, double rz, cplx t[3][3])
{
    double o[12];
    ora_neg_green(k, rx, ry, rz, o);
    cplx c[6];
    for (int i = 0; i < 6; ++i) c[i] = o[2 * i] + I * o[2 * i + 1];
    t[0][0] = c[0]; t[0][1] = c[1]; t[0][2] = c[2];
    t[1][0] = c[1]; t[1][1] = c[3]; t[1][2] = c[4];
    t[2][0] = c[2]; t[2][1] = c[4]; t[2][2] = c[5];
}

/* Blocked (two-level) summation accumulator: terms are summed in blocks of
 * BLK, block sums are then added; keeps the rounding error ~ (BLK + N/BLK) eps
 * instead of N eps for long rows. */
#define BLK 256

/*
 * y = A x on a subset of rows (dipoles `rows[0..nrows)`, or all dipoles when
 * rows == NULL).  sites: int32 [nd][3]; ainv: complex [3][nd] (alpha^{-1} of
 * each component of each dipole: a diagonal polarisability tensor, Sec. 2);
 * x: complex [3][nd]; y: complex [3][nrows].  Direct double summation.
 */
void ora_dense_matvec(int64_t nd, const int32_t *sites, double k, const double *ainv,
                      int64_t nrows, const int64_t *rows, const double *x, double *y,
                      int nthreads)
{
    const cplx *xc = (const cplx *)x;
    const cplx *ai = (const cplx *)ainv;
    cplx *yc = (cplx *)y;
    if (nrows < 0 || rows == NULL) nrows = nd;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t n = rows ? rows[q] : q;
        cplx tot[3] = {0, 0, 0}, blk[3] = {0, 0, 0};
        int cnt = 0;
        for (int64_t m = 0; m < nd; ++m) {
            if (m == n) continue;
            double rx = sites[3 * n] - sites[3 * m];
            double ry = sites[3 * n + 1] - sites[3 * m + 1];
            double rz = sites[3 * n + 2] - sites[3 * m + 2];
            cplx t[3][3];
            neg_green_3x3(k, rx, ry, rz, t);
            for (int a = 0; a < 3; ++a)
                blk[a] += t[a][0] * xc[m] + t[a][1] * xc[nd + m] + t[a][2] * xc[2 * nd + m];
            if (++cnt == BLK) {
                for (int a = 0; a < 3; ++a) { tot[a] += blk[a]; blk[a] = 0; }
                cnt = 0;
            }
        }
        for (int a = 0; a < 3; ++a) {
            tot[a] += blk[a];
            yc[a * nrows + q] = ai[a * nd + n] * xc[a * nd + n] + tot[a];
        }
    }
}

/* Explicit 3nd x 3nd matrix, row-major, index (c*nd + n, c'*nd + m). */
void ora_dense_matrix(int64_t nd, const int32_t *sites, double k, const double *ainv, double *Aout)
{
    cplx *A = (cplx *)Aout;
    const cplx *ai = (const cplx *)ainv;
    int64_t N3 = 3 * nd;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (int64_t n = 0; n < nd; ++n) {
        for (int64_t m = 0; m < nd; ++m) {
            cplx t[3][3];
            if (m == n) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) t[a][b] = (a == b) ? ai[a * nd + n] : 0;
            } else {
                neg_green_3x3(k, (double)(sites[3 * n] - sites[3 * m]),
                              (double)(sites[3 * n + 1] - sites[3 * m + 1]),
                              (double)(sites[3 * n + 2] - sites[3 * m + 2]), t);
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) A[(a * nd + n) * N3 + b * nd + m] = t[a][b];
        }
    }
}

/*
 * Dense LU with partial pivoting (Doolittle, row interchanges), then forward
 * and back substitution for nrhs right-hand sides.  A: n x n row-major
 * (overwritten by its factors), B: n x nrhs row-major (overwritten by X).
 * Returns 0, or the 1-based index of a zero pivot.
 */
int ora_lu_solve(int64_t n, double *Aio, int64_t nrhs, double *Bio)
{
    cplx *A = (cplx *)Aio, *B = (cplx *)Bio;
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = c;
        double best = cabs(A[c * n + c]);
        for (int64_t r = c + 1; r < n; ++r) {
            double v = cabs(A[r * n + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return (int)(c + 1);
        if (piv != c) {
            for (int64_t j = 0; j < n; ++j) {
                cplx t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t;
            }
            for (int64_t j = 0; j < nrhs; ++j) {
                cplx t = B[c * nrhs + j]; B[c * nrhs + j] = B[piv * nrhs + j]; B[piv * nrhs + j] = t;
            }
        }
        cplx inv = 1.0 / A[c * n + c];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t r = c + 1; r < n; ++r) {
            cplx f = A[r * n + c] * inv;
            A[r * n + c] = f;
            for (int64_t j = c + 1; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            for (int64_t j = 0; j < nrhs; ++j) B[r * nrhs + j] -= f * B[c * nrhs + j];
        }
    }
    for (int64_t c = n - 1; c >= 0; --c) {
        cplx inv = 1.0 / A[c * n + c];
        for (int64_t j = 0; j < nrhs; ++j) {
            cplx s = B[c * nrhs + j];
            for (int64_t r = c + 1; r < n; ++r) s -= A[c * n + r] * B[r * nrhs + j];
            B[c * nrhs + j] = s * inv;
        }
    }
    return 0;
}

/*
 * Scattering cross section by angular quadrature of the far field:
 *   C_sca = k^4 \int |sum_n e^{-ik n.r_n} (P_n - n (n.P_n))|^2 dOmega
 * over the unit sphere (Draine 1988, |E0| = 1).  The caller supplies the
 * quadrature nodes: ncos Gauss-Legendre nodes/weights in cos(theta) and nphi
 * equally spaced azimuths with equal weights 2pi/nphi.
 */
double ora_csca_quadrature(int64_t nd, const int32_t *sites, double k, const double *P,
                           int ncos, const double *cosn, const double *wcos, int nphi)
{
    const cplx *Pc = (const cplx *)P;
    double total = 0.0;
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : total) schedule(dynamic, 1) collapse(2)
#endif
    for (int a = 0; a < ncos; ++a) {
        for (int b = 0; b < nphi; ++b) {
            double ct = cosn[a], st = sqrt(fmax(0.0, 1.0 - ct * ct));
            double ph = 2.0 * M_PI * b / nphi;
            double nv[3] = {st * cos(ph), st * sin(ph), ct};
            cplx F[3] = {0, 0, 0};
            for (int64_t n = 0; n < nd; ++n) {
                double dot = nv[0] * sites[3 * n] + nv[1] * sites[3 * n + 1] + nv[2] * sites[3 * n + 2];
                cplx e = cexp(-I * k * dot);
                cplx p[3] = {Pc[n], Pc[nd + n], Pc[2 * nd + n]};
                cplx np = nv[0] * p[0] + nv[1] * p[1] + nv[2] * p[2];
                for (int c = 0; c < 3; ++c) F[c] += e * (p[c] - nv[c] * np);
            }
            double f2 = 0.0;
            for (int c = 0; c < 3; ++c) f2 += creal(F[c]) * creal(F[c]) + cimag(F[c]) * cimag(F[c]);
            total += wcos[a] * (2.0 * M_PI / nphi) * f2;
        }
    }
    return pow(k, 4) * total;
}

/*
 * The same C_sca as an exact double sum (the plane-wave integral of the
 * transverse projector is (4 pi / k^3) Im G(R) for R != 0 and 8 pi / 3 at
 * R = 0):
 *   C_sca = 4 pi k [ (2/3) k^3 sum_n |P_n|^2 + sum_{n != m} P_n^H Im G(r_n - r_m) P_m ].
 * Here Im G is the element-wise imaginary part of G (= -t).
 */
double ora_csca_double_sum(int64_t nd, const int32_t *sites, double k, const double *P)
{
    const cplx *Pc = (const cplx *)P;
    double self = 0.0, cross = 0.0;
    for (int64_t n = 0; n < nd; ++n)
        for (int c = 0; c < 3; ++c) {
            cplx v = Pc[c * nd + n];
            self += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : cross) schedule(dynamic, 16)
#endif
    for (int64_t n = 0; n < nd; ++n) {
        for (int64_t m = 0; m < nd; ++m) {
            if (m == n) continue;
            cplx t[3][3];
            neg_green_3x3(k, (double)(sites[3 * n] - sites[3 * m]),
                          (double)(sites[3 * n + 1] - sites[3 * m + 1]),
                          (double)(sites[3 * n + 2] - sites[3 * m + 2]), t);
            cplx acc = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    acc += conj(Pc[a * nd + n]) * (-cimag(t[a][b])) * Pc[b * nd + m];
            cross += creal(acc);
        }
    }
    return 4.0 * M_PI * k * ((2.0 / 3.0) * k * k * k * self + cross);
}
