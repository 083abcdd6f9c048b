/*
 * libdda — the CG-FFT discrete dipole approximation on one MI355X (gfx950).
 *
 * The library solves the DDA system of the paper's Eq. 1,
 *
 *     alpha_n^{-1} P_n - sum_{m != n} G(r_n - r_m) P_m = E_inc,n ,
 *
 * written in Gaussian units with lattice spacing d = 1 (the paper's
 * normalisation k^2/eps0 * A differs by a global constant; cross sections are
 * identical), for dipoles on the occupied sites of a K x J x P cubic lattice.
 * The off-diagonal part is applied as a convolution: the block-Toeplitz tensor
 * is embedded in a zero-padded level-three circulant (Sec. 3, Appendix A) and
 * every 3D DFT runs as ensembles of 1D transforms that skip the all-zero lines
 * and planes (Sec. 3, Table 2).
 *
 * Conventions
 *  - Lattice index: site (i, j, k) has linear index n = k*J*K + j*K + i
 *    (Appendix A).  Dipoles are the occupied sites in increasing n.
 *  - Vectors are component-major [nrhs][3][N_d] of interleaved complex
 *    (re, im): complex128 for DDA_FP64, complex64 for DDA_FP32 (the x0/x1/x2
 *    split of Sec. 3).  Compatible with torch.complex128/complex64.
 *  - Pointers named *_dev are device pointers on the library's device; all
 *    other pointers are host pointers.  The caller owns every buffer passed in;
 *    the library owns the handles' internal storage and frees it in
 *    *_destroy / dda_close.
 *  - Device work is enqueued on the caller's HIP stream (NULL = the default
 *    stream).  Calls that return host results synchronise that stream.
 *  - Errors: every int-returning call returns DDA_OK or a negative code and
 *    sets a thread-local message readable with dda_last_error().  No call
 *    throws.  One target must not be used from two threads at once.
 */
#ifndef DDA_H
#define DDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DDA_OK = 0,
  DDA_EINVAL = -1,   /* invalid argument (sizes, poles of alpha, NULL buffers) */
  DDA_ENOMEM = -2,   /* device allocation failed                               */
  DDA_EDEVICE = -3,  /* HIP runtime error                                      */
  DDA_ENOTCONV = -4, /* a right-hand side missed the tolerance                 */
  DDA_ESTATE = -5    /* call out of order (e.g. matvec before the spectrum)    */
};

enum { DDA_FP64 = 0, DDA_FP32 = 1 };                       /* vector precision   */
enum { DDA_POL_CM = 0, DDA_POL_RR = 1, DDA_POL_LDR = 2 };  /* polarisability     */
/* Krylov solvers (schemes of Sec. 4): BiCGSTAB (van der Vorst 1992), CGS
 * (Sonneveld 1989) and TFQMR (Freund 1993), two products per iteration;
 * QMR_sym and BiCG_sym (Freund 1992a; complex-symmetric, one product per
 * iteration, bilinear form x^T y); BiCG (Fletcher 1975) and QMR with coupled
 * two-term recurrences (Freund & Nachtigal), whose shadow products A^H y are
 * computed as conj(A conj(y)) since A is complex symmetric, two products per
 * iteration; RBiCGSTAB = BiCGSTAB(l) (Sleijpen & Fokkema 1993), one iteration
 * = l BiCG steps and a degree-l minimal-residual polynomial, 2l products;
 * ML(n)BiCGSTAB (Yeung & Chan 1999) in the IDR(s) form with s = n
 * (Sonneveld & van Gijzen 2008), one iteration = n + 1 products.  The l and
 * n of the last two come from dda_solve_opts.solver_param. */
enum {
  DDA_BICGSTAB = 0,
  DDA_QMR_SYM = 1,
  DDA_BICG_SYM = 2,
  DDA_CGS = 3,
  DDA_TFQMR = 4,
  DDA_BICG = 5,
  DDA_QMR = 6,
  DDA_RBICGSTAB = 7,
  DDA_MLBICGSTAB = 8
};
enum { DDA_SOLVE_FP64 = 0, DDA_SOLVE_MIXED = 1 };          /* solve precision    */

typedef struct dda_lib dda_lib;
typedef struct dda_target dda_target;

/* Open the library on HIP device `hip_device`.  `tune_cache_path` (nullable)
 * names a text file where the FFT-schedule autotuner keeps its choices. */
int dda_open(int hip_device, const char *tune_cache_path, dda_lib **out);
void dda_close(dda_lib *lib);

/* A target on a K x J x P lattice (K, J, P >= 1) with wavenumber kd > 0 in
 * units of the lattice spacing.  Chooses the padded FFT sizes
 * K'' >= 2K-1, J'' >= 2J-1, P'' >= 2P-1 (Sec. 3: any size >= 2n-1 embeds the
 * Toeplitz matrix in a circulant; the smallest 2^a 3^b 5^c length is used,
 * or a length with register-resident kernels when it is at most 30% longer).
 * The target uses its library until dda_target_destroy, which frees the
 * target's device memory and may run after dda_close of the library; every
 * other call on a target needs its library open. */
int dda_target_create(dda_lib *lib, int K, int J, int P, double kd, dda_target **out);
void dda_target_destroy(dda_target *t);

/* Occupancy: occ[K*J*P] (0/1, linear index order).  Returns N_d >= 1 in
 * *nd_out.  Invalidates polarisabilities. */
int dda_set_occupancy(dda_target *t, const uint8_t *occ, int64_t *nd_out);

/* Per-dipole permittivity eps[2*N_d] (re, im) and a polarisability
 * prescription.  The paper names the radiative-reaction correction and the
 * lattice dispersion relation (Sec. 1) without formulas; the published ones are
 * used (d = 1):
 *   CM : alpha^{-1} = (4 pi / 3)(eps + 2)/(eps - 1)
 *   RR : CM - (2/3) i kd^3
 *   LDR: CM + (b1 + b2 eps + b3 S eps) kd^2 - (2/3) i kd^3,  S = sum_a (khat_a ehat_a)^2
 * (S is per right-hand side and passed with each call).  DDA_EINVAL for
 * eps = 1 or a non-finite alpha^{-1}.  Enables dda_grad_cabs_eps. */
int dda_set_permittivity(dda_target *t, const double *eps, int prescription);

/* Per-dipole polarisability alpha[2*N_d] (re, im), used as given. */
int dda_set_polarizability(dda_target *t, const double *alpha);

/* Multi-material, anisotropic composition (Sec. 2: every dipole carries a
 * material index for each of the directions x, y, z).  eps[2*nmat] (re, im)
 * the materials' permittivities (nmat <= 256); flags[3*N_d] the material
 * index of component c of dipole n at c*N_d + n.  The polarisability tensor is
 * diagonal in the lattice axes, component c taking the prescription (as for
 * dda_set_permittivity) at its own material.  The library keeps the flags
 * bit-fielded at the smallest power-of-two width that holds nmat - 1 (1, 2, 4
 * or 8 bits) with an nmat-entry table of alpha^{-1} per precision, which is
 * what the matrix-vector passes read.  DDA_EINVAL for a flag >= nmat
 * or a material without finite alpha^{-1}.  dda_grad_cabs_eps needs an
 * isotropic dda_set_permittivity instead (DDA_ESTATE after this call). */
int dda_set_composition(dda_target *t, int nmat, const double *eps, const uint8_t *flags, int prescription);

/* Interaction spectrum (Sec. 3): the six tensor components' first columns
 * t = -G on [0,K)x[0,J)x[0,P), implicit Toeplitz-to-circulant conversion with
 * the Table 1 signs, 1D DFTs along x (J*P lines), y (K_h*P) and z (K_h*J_h),
 * keeping the unique octant of n_h = n''/2 + 1 entries per axis.  Built in
 * FP64; the FP32 copy is the FP64 one rounded to nearest even. */
int dda_build_spectrum(dda_target *t, void *hip_stream);

/* y = A x (Eq. 1) for nrhs right-hand sides, FP64 or FP32 vectors.
 * S: host [nrhs] LDR orientation factors (NULL = 0).
 * jacobi != 0 applies the symmetric Point-Jacobi form D^{-1/2} A D^{-1/2},
 * D = diag(alpha^{-1}). */
int dda_matvec(dda_target *t, int precision, int nrhs, const double *S, int jacobi, const void *x_dev,
               void *y_dev, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of dda_matvec with every device buffer it needs beyond x_dev and y_dev (the
 * nrhs orientation factors and the two FFT workspaces, K'' padded to whole
 * z tiles) placed in a device scratch array that the library holds on each
 * device until the process ends, at most 64 MiB (e.g. the 64^3 cube with one
 * FP32 right-hand side needs 38 MB).  A call that needs more returns
 * DDA_EINVAL and does nothing.  The call allocates nothing, does not autotune
 * (it runs the schedule the library has tuned for this lattice and
 * right-hand-side count, else the five plain passes; DDA_OPT_SCHEDULE
 * applies), records no profiling events, and synchronises the stream before
 * returning (S may be reused at once).  All calls on one device share its
 * scratch: calls that overlap in time on one device, from any target or
 * library, race.  Arguments, layout and results as for dda_matvec. */
int dda_matvec_noalloc(dda_target *t, int precision, int nrhs, const double *S, int jacobi, const void *x_dev,
                       void *y_dev, void *hip_stream);

typedef struct {
  int solver;        /* one of the DDA_* solver values above                      */
  int precision;     /* DDA_SOLVE_FP64, or DDA_SOLVE_MIXED (FP32 inner, FP64 outer) */
  int max_iter;      /* total inner iterations per right-hand side (<= 0: 10000)  */
  int max_outer;     /* refinement steps (<= 0: 20)                               */
  double tol;        /* ||E - A P|| / ||E|| target, true FP64 residual             */
  double inner_tol;  /* relative tolerance of each FP32 inner solve (<= 0: 1e-3)   */
  int jacobi;        /* Point-Jacobi preconditioning (symmetric form)             */
  int check_every;   /* iterations between convergence read-backs (<= 0: 8)        */
  int use_graph;     /* capture the inner iteration in a HIP graph                */
  int solver_param;  /* l of DDA_RBICGSTAB, n of DDA_MLBICGSTAB: 1..4 (<= 0: 2);
                        ignored by the other solvers                             */
} dda_solve_opts;

typedef struct {
  int converged;        /* true FP64 residual <= tol                      */
  int iterations;       /* inner Krylov iterations (all refinement steps) */
  int outer_iterations; /* refinement steps                               */
  int matvecs;          /* matrix-vector products (both precisions)       */
  double rel_residual;  /* ||E - A P|| / ||E|| in FP64 at exit             */
} dda_solve_info;

/* Solve A P = E_inc for nrhs right-hand sides with a zero initial guess.
 * E_inc is einc_dev ([nrhs][3][N_d] complex128) or, if NULL, plane waves
 * ehat exp(i kd khat . r) built from khat[3*nrhs] and ehat[6*nrhs] (re, im).
 * S (nullable) as for dda_matvec; when NULL and the prescription is LDR, S is
 * computed from khat/ehat (S = sum_a Re[(khat_a ehat_a)^2]), and an LDR
 * target given neither S nor khat/ehat is DDA_EINVAL.  The S values used are
 * kept with the target (dda_solve_orientation_factors) for the calls that
 * follow the solve.  p_dev: out [nrhs][3][N_d] complex128.
 * info: host [nrhs].  DDA_ENOTCONV if a right-hand side missed tol;
 * DDA_EINVAL for an unknown solver, a solver_param above 4, tol outside
 * (0, 1) or an unknown precision. */
int dda_solve(dda_target *t, const dda_solve_opts *opts, int nrhs, const double *khat, const double *ehat,
              const double *S, const void *einc_dev, void *p_dev, dda_solve_info *info, void *hip_stream);

/* The LDR orientation factors S[nrhs] (host out) that the last dda_solve on
 * the target used: the S it was given, or those it derived from khat/ehat (0
 * for CM/RR targets).  DDA_ESTATE if no solve ran since the occupancy was set
 * or it had another right-hand-side count. */
int dda_solve_orientation_factors(const dda_target *t, int nrhs, double *S);

/* One target's share of a batch: the arguments dda_solve takes for it. */
typedef struct {
  dda_target *target;       /* distinct per item, opened on the batch's library */
  int nrhs;                 /* >= 1                                            */
  const double *khat;       /* host [3*nrhs] or NULL (then einc_dev is used)    */
  const double *ehat;       /* host [6*nrhs] (re, im) or NULL                   */
  const double *S;          /* host [nrhs] or NULL, as for dda_solve            */
  const void *einc_dev;     /* [nrhs][3][N_d] complex128 or NULL                */
  void *p_dev;              /* out [nrhs][3][N_d] complex128                    */
  dda_solve_info *info;     /* host out [nrhs] (nullable)                       */
} dda_batch_item;

/* Solve many targets (uneven lattices and right-hand-side counts, e.g. an
 * ensemble of aggregates or orientations) as one call: the items are ordered
 * longest first (FFT grid volume x nrhs) and drawn from a shared queue by
 * nworkers host workers (<= 0: 4, the HIP hardware queues per process), each
 * enqueueing on its own library-owned stream of default priority, so that
 * the solves of small targets overlap on the device.  Work starts after what
 * is already enqueued on hip_stream; the call returns when every item is
 * solved.  Each item behaves as dda_solve on it.  DDA_EINVAL for a repeated
 * target or an item of another library; DDA_ENOTCONV if some right-hand side
 * missed tol (all items are still solved); any other error stops the queue and
 * is returned with the failing item's message. */
int dda_batch_solve(dda_lib *lib, const dda_solve_opts *opts, int nitems, const dda_batch_item *items,
                    int nworkers, void *hip_stream);

/* Incident plane waves at the dipoles, E[r][c][n] = ehat_r[c] exp(i kd khat_r . r_n)
 * (Sec. 1; |E0| = 1): khat[3*nrhs] real unit vectors, ehat[6*nrhs] (re, im).
 * e_dev: out [nrhs][3][N_d] complex128. */
int dda_incident_field(dda_target *t, int nrhs, const double *khat, const double *ehat, void *e_dev,
                       void *hip_stream);

/* C_ext = 4 pi k sum Im(E^* . P), C_abs = 4 pi k sum |P|^2 (-Im alpha^{-1} - 2k^3/3)
 * (Draine 1988, |E0| = 1) and C_sca = C_ext - C_abs, per right-hand side
 * (host outputs, nrhs each; any may be NULL).  S (host [nrhs], nullable):
 * the LDR orientation factors of alpha^{-1}; when NULL, an LDR target takes
 * those of the last dda_solve if it had nrhs right-hand sides and is
 * DDA_EINVAL otherwise (CM/RR targets have no S term). */
int dda_cross_sections(dda_target *t, int nrhs, const double *S, const void *einc_dev, const void *p_dev,
                       double *cext, double *cabs, double *csca, void *hip_stream);

/* Far-field amplitude of the solved dipoles (the step after the solve; the
 * paper reports Q_sca from it, Sec. 6): F(n) = kd^2 (I - n n) sum_m
 * exp(-i kd n . r_m) P_m, so that the scattered field is exp(i kd r)/r F(n) as
 * r -> infinity (Gaussian units, |E0| = 1; Draine 1988).  dirs: host
 * [ndir][3] unit vectors (DDA_EINVAL otherwise).  p_dev [nrhs][3][N_d]
 * complex128; f_dev out [nrhs][ndir][3] complex128.  Synchronises the stream. */
int dda_far_field(dda_target *t, int nrhs, const void *p_dev, int ndir, const double *dirs, void *f_dev,
                  void *hip_stream);

/* C_sca = integral of |F|^2 over the sphere by Gauss-Legendre quadrature in
 * cos(theta) (ntheta nodes) times a uniform azimuth grid (nphi nodes); the
 * integrand is band-limited by kd D (D the target's diameter), so the default
 * (ntheta <= 0: ceil(kd (D + 1)) + 16, nphi = 2 ntheta) converges to rounding.
 * Independent of dda_cross_sections' C_ext - C_abs: the two agree to the
 * solve's residual (optical theorem).  csca: host out [nrhs]. */
int dda_csca_quadrature(dda_target *t, int nrhs, const void *p_dev, int ntheta, int nphi, double *csca,
                        void *hip_stream);

/* Amplitude scattering matrix and Mueller matrix for incidence along +z
 * (Bohren & Huffman 1983, Sec. 3.2-3.3).  p_dev holds the two solves
 * [2][3][N_d] complex128 for polarisation x (first) and y (second).
 * theta_phi: host [ndir][2] scattering angles.  Basis: e_par,i =
 * cos(phi) x + sin(phi) y, e_perp,i = sin(phi) x - cos(phi) y, e_par,s =
 * theta-hat, e_perp,s = -phi-hat, [E_par,s, E_perp,s] = exp(i kd r)/(-i kd r)
 * [[S2, S3], [S4, S1]] [E_par,i, E_perp,i].  s_dev out [ndir][4] complex128
 * (S1, S2, S3, S4), m_dev out [ndir][4][4] float64 row-major (either may be
 * NULL, not both).  Synchronises the stream. */
int dda_mueller(dda_target *t, const void *p_dev, int ndir, const double *theta_phi, void *s_dev, void *m_dev,
                void *hip_stream);

/* dC_abs/d eps_n for every dipole and right-hand side by one adjoint solve
 * with the same matrix (A is complex symmetric: A mu = W conj(P)).
 * grad_dev: out [nrhs][N_d] complex128 = dC/dRe eps + i dC/dIm eps.
 * S as for dda_cross_sections.  Requires dda_set_permittivity. */
int dda_grad_cabs_eps(dda_target *t, const dda_solve_opts *opts, int nrhs, const double *S, const void *p_dev,
                      void *grad_dev, void *hip_stream);

/* Options of a target.  DDA_OPT_SCHEDULE selects the matrix-vector schedule:
 * -1 (default) the autotuned choice; 0 five separate passes (y, x, z with
 * product, x inverse, y inverse) with the z lines read as strided tiles;
 * 1 five passes with the x passes transposing so that z lines are contiguous;
 * 3 five passes with the z pass spread over three thread groups, one per
 * vector component (fewer registers per thread, spectra exchanged in LDS);
 * 5 five passes with a two-level z pass (each z line as an E-point DFT per
 * thread and T-point DFTs after one LDS exchange, the product taken in that
 * scrambled frequency order, several right-hand sides per block);
 * 6 as 5 with the x-transformed array stored in z-column tiles (each tile's
 * rows contiguous), written and read by x passes that take several z rows
 * of one y row at a time;
 * D in {2, 4, 8} the fused xy-plane passes with the frequency range split
 * into D residue classes.  DDA_EINVAL if that schedule does not exist for the
 * lattice. */
/* DDA_OPT_INJECT_BREAKDOWN (fault injection for tests of the recovery path):
 * the next `value` BiCGSTAB inner solves start from a zero shadow vector, so
 * their first step breaks down (rhat^H v = 0) and the refinement loop must
 * restart from the true residual.  DDA_EINVAL for a negative value. */
/* DDA_OPT_CANARY (debug, value 0 or 1): dda_matvec fills its FFT workspaces
 * with NaN (hipMemsetAsync, so not for stream capture) before the passes, so
 * that a pruned pass reading data no earlier pass wrote shows as a non-finite
 * or wrong product. */
/* DDA_OPT_FUSE_QMR_STEP (value 1, the default, or 0): QMR_sym runs the vector
 * part of each step inside the y-forward pass of the next product where the
 * schedule's y pass allows it (schedules 0, 1, 3); 0 keeps the separate step
 * kernel.  Same recurrences either way. */
/* DDA_OPT_RHS_PER_BLOCK (0..8): right-hand sides each block of the two-level
 * z pass (schedules 5 and 6) runs in turn, sharing its spectrum tile; 0
 * (default) is one. */
/* DDA_OPT_Y_TILE (-1, the default, or 0..2): the y passes of the five-pass
 * schedules take 2^value times their default number of adjacent x positions
 * per block (longer contiguous runs of the y-transformed array, up to 1024
 * threads and 64 KB of LDS per block; a precision without that variant
 * takes its widest); -1 leaves it to the autotuner, which times the wider
 * variants after choosing the schedule.  DDA_EINVAL if even FP32 has no such
 * variant for the lattice. */
/* DDA_OPT_INJECT_BAD_STEP (fault injection for tests of the recovery path):
 * the next `value` refinement steps of dda_solve add their correction with the
 * wrong sign, so the true residual grows and the step must be taken back (P
 * and the residual of the step's start restored, the right-hand side moved to
 * FP64 inner solves).  DDA_EINVAL for a negative value. */
/* DDA_OPT_X_ROWS (-1, the default, or 0..2): the x passes of the register-
 * resident schedules take their default number of rows per block (0), half
 * of it (1) or twice it (2), within 1024 threads and 64 KB of LDS (a variant
 * that does not fit runs the default); -1 leaves it to the autotuner, which
 * times 1 and 2 after the y tiles.  DDA_EINVAL outside -1..2. */
enum { DDA_OPT_SCHEDULE = 1, DDA_OPT_INJECT_BREAKDOWN = 2, DDA_OPT_CANARY = 3, DDA_OPT_FUSE_QMR_STEP = 4,
       DDA_OPT_RHS_PER_BLOCK = 5, DDA_OPT_Y_TILE = 6, DDA_OPT_INJECT_BAD_STEP = 7, DDA_OPT_X_ROWS = 8 };
int dda_target_set_option(dda_target *t, int option, int value);

/* Sizes of the embedding, for inspection:
 * dims[0..8] = K'', J'', P'', K_h, J_h, P_h, N_d, and the 1D transform counts
 * of one matrix-vector product per right-hand side (forward + inverse) and of
 * the spectrum build (Table 2). */
int dda_target_info(const dda_target *t, int64_t *dims /* 9 */);

/* The padded FFT lengths K'', J'', P'' of the circulant embedding (Sec. 3:
 * every length n'' >= 2n - 1 embeds the Toeplitz blocks, so the product does
 * not depend on the choice, up to rounding).  0 for an axis takes the default
 * rule (the smallest 2^a 3^b 5^c length >= 2n - 1, or the smallest one with
 * register-resident kernels when that is at most 30% longer: 2^k and 3 2^k,
 * and for J'' also 5 2^k and 25 2^k).  Each nonzero
 * length must be >= 2n - 1, of the form 2^a 3^b 5^c and at most
 * max(16, 4 (2n - 1)); DDA_EINVAL otherwise, and when a schedule forced with
 * DDA_OPT_SCHEDULE does not exist at the new lengths (nothing changes then).
 * New lengths drop the spectrum (dda_build_spectrum must run again before a
 * product or solve: DDA_ESTATE until then), the product workspaces and the
 * captured iterations; the lengths already in use change nothing. */
int dda_target_set_padding(dda_target *t, int Kpp, int Jpp, int Ppp);

/* Padded lengths chosen by measurement, the analogue of planning an FFT by
 * measuring (Sec. 3).  Per axis the candidates are the default rule's length,
 * the smallest 2^a 3^b 5^c length >= 2n - 1 and the smallest length >= 2n - 1
 * with register-resident kernels when it is at most twice that; for every
 * combination (those with a forced schedule only) the spectrum is built, the
 * schedule tuned and `nrhs` products in `precision` timed on hip_stream with
 * HIP events (Jacobi form, S = 0, a fixed input pattern).  A combination
 * must beat the default rule's by more than 3%.  The target keeps the
 * fastest lengths with their spectrum built, and lengths[0..2] (may be NULL)
 * receives them.  The choice is kept in the library handle per (lattice,
 * nrhs, precision, forced schedule) and appended to the tune-cache file, so a
 * later call only sets the lengths and builds the spectrum.  Needs the
 * occupancy and the polarisability (DDA_ESTATE otherwise); DDA_EINVAL for
 * nrhs < 1 or an unknown precision.  If a measurement fails, the target
 * is back at the lengths it had, without a spectrum (build it again), and the
 * error is returned.  Allocates and frees two vectors of nrhs x 3 x N_d. */
int dda_tune_padding(dda_target *t, int nrhs, int precision, int *lengths /* 3, or NULL */, void *hip_stream);

/* Copy the spectrum [6][P_h][J_h][K_h] (complex128 or complex64) to out_dev. */
int dda_get_spectrum(dda_target *t, int precision, void *out_dev, void *hip_stream);

/* Kernel timing for measurement: while enabled (enable = 1), every launch of
 * a matrix-vector pass, and every whole product, is bracketed by HIP events on
 * its own stream (and the solver does not capture graphs); enable = 2 records
 * the whole products only, with no events between their passes; 0 turns it
 * off, any other value is DDA_EINVAL.  dda_profile_read
 * fills ms[2*DDA_PROF_SLOTS] (summed milliseconds) and
 * count[2*DDA_PROF_SLOTS] (launches) for the slots y-forward, x-forward,
 * z (forward, product, inverse), x-inverse, y-inverse, fused xy-forward,
 * fused xy-inverse and the whole product (all its passes and the gaps
 * between them), with FP64 vectors (slots 0..DDA_PROF_SLOTS-1) and FP32
 * vectors (the next DDA_PROF_SLOTS); it waits for the recorded events. */
enum { DDA_PROF_SLOTS = 8 };
int dda_profile_enable(dda_lib *lib, int enable);
int dda_profile_read(dda_lib *lib, double *ms, int64_t *count);
int dda_profile_reset(dda_lib *lib);

/* Message of the last failing call on this thread ("" if none). */
const char *dda_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDA_H */
