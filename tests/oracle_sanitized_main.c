/* Test harness (CPU, test infrastructure): runs the plain-C oracle built
 * with AddressSanitizer and UndefinedBehaviorSanitizer on inputs written by
 * tests/test_oracle_sanitized.py and writes its results back.
 *
 * Input file:  int64 nd, nrows, ncos, nphi; double k;
 *              int32 sites[nd][3]; complex ainv[3][nd]; complex x[3][nd];
 *              int64 rows[nrows]; double cosn[ncos], wcos[ncos].
 * Output file: complex y[3][nd] (all rows), complex yr[3][nrows] (rows),
 *              complex z[3][nd] (dense LU solution of A z = x),
 *              double csca (far-field quadrature of P = z), int32 info. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ora_dense_matvec(int64_t nd, const int32_t *sites, double k, const double *ainv, int64_t nrows,
                      const int64_t *rows, const double *x, double *y, int nthreads);
void ora_dense_matrix(int64_t nd, const int32_t *sites, double k, const double *ainv, double *Aout);
int ora_lu_solve(int64_t n, double *Aio, int64_t nrhs, double *Bio);
double ora_csca_quadrature(int64_t nd, const int32_t *sites, double k, const double *P, int ncos,
                           const double *cosn, const double *wcos, int nphi);

static void *read_n(FILE *f, size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t *hdr = read_n(f, 4 * sizeof(int64_t));
  const int64_t nd = hdr[0], nrows = hdr[1], ncos = hdr[2], nphi = hdr[3];
  double *kp = read_n(f, sizeof(double));
  int32_t *sites = read_n(f, (size_t)nd * 3 * sizeof(int32_t));
  double *ainv = read_n(f, (size_t)3 * nd * 2 * sizeof(double));
  double *x = read_n(f, (size_t)3 * nd * 2 * sizeof(double));
  int64_t *rows = read_n(f, (size_t)nrows * sizeof(int64_t));
  double *cosn = read_n(f, (size_t)ncos * sizeof(double));
  double *wcos = read_n(f, (size_t)ncos * sizeof(double));
  fclose(f);

  const int64_t n = 3 * nd;
  double *y = malloc((size_t)n * 2 * sizeof(double));
  double *yr = malloc((size_t)3 * nrows * 2 * sizeof(double));
  double *A = malloc((size_t)n * n * 2 * sizeof(double));
  double *z = malloc((size_t)n * 2 * sizeof(double));
  ora_dense_matvec(nd, sites, *kp, ainv, -1, NULL, x, y, 1);
  ora_dense_matvec(nd, sites, *kp, ainv, nrows, rows, x, yr, 1);
  ora_dense_matrix(nd, sites, *kp, ainv, A);
  for (int64_t i = 0; i < 2 * n; ++i) z[i] = x[i];
  int32_t info = ora_lu_solve(n, A, 1, z);
  double csca = ora_csca_quadrature(nd, sites, *kp, z, (int)ncos, cosn, wcos, (int)nphi);

  FILE *o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(y, sizeof(double), (size_t)n * 2, o);
  fwrite(yr, sizeof(double), (size_t)3 * nrows * 2, o);
  fwrite(z, sizeof(double), (size_t)n * 2, o);
  fwrite(&csca, sizeof(double), 1, o);
  fwrite(&info, sizeof(int32_t), 1, o);
  fclose(o);
  free(hdr); free(kp); free(sites); free(ainv); free(x); free(rows); free(cosn); free(wcos);
  free(y); free(yr); free(A); free(z);
  return 0;
}
