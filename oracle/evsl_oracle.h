/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously-correct CPU implementation of what the polynomial-
 * filtered spectrum-slicing path computes, written from the EVSL paper (Li, Xi,
 * Erlandson, Saad, "The Eigenvalues Slicing Library (EVSL): Algorithms,
 * Implementation, and Software", arXiv:1802.05215). Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code with the HIP library, and the HIP library never calls it.
 *
 * Everything is FP64. Matrices are CSR (int32 row_ptr[n+1], int32 col[nnz]
 * ascending within a row, double val[nnz]). Blocks of vectors are row-major
 * n x nvec unless a comment says column-major.
 */
#ifndef EVSL_ORACLE_H
#define EVSL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_DAMP_NONE 0
#define OR_DAMP_SIGMA 1   /* Lanczos sigma factors, eq:polPJ */
#define OR_DAMP_JACKSON 2 /* Jackson kernel (Weisse et al., Rev. Mod. Phys. 78, 275, 2006) */

/* SplitMix64 output number i+1 of the generator seeded with `seed`. */
uint64_t or_splitmix64(uint64_t seed, uint64_t i);
double or_uniform01(uint64_t seed, uint64_t i);

/* y = A x, one row at a time, sum in column order. */
void or_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
             const double *x, double *y);

/* Damping factors g[0..k] for a degree-k Chebyshev expansion. Returns 0 or -1. */
int or_damping(int kind, int k, double *g);

/* Evaluate sum_{j=0..k} c[j] T_j(t) with T_j(t) = cos(j acos t) on [-1,1]
 * (cosh(j acosh|t|) with the sign (-1)^j for t < -1 outside). */
double or_cheb_series(int k, const double *c, double t);

/* find_pol (Section 2.2.1, eq:mapping, eq:Cheb0, eq:mu, eq:Neq, eq:polPJ).
 * intv = {t_i, t_{i+1}, lambda_min, lambda_max}. Writes the degree, the centre
 * gamma, the threshold bar = rho(t_i-hat) (= rho(t_{i+1}-hat)), the map
 * constants cc, dd, and coef[0..deg] with rho(t) = sum coef[j] T_j(t).
 * coef must hold max_deg+1 doubles. Returns 0, 1 if max_deg was reached
 * (filter still returned at max_deg), -1 on invalid input. */
int or_find_pol(const double intv[4], int damping, double tau, double tau_ext,
                int max_deg, int *deg, double *gamma, double *bar, double *cc,
                double *dd, double *coef, int *boundary);

/* Y = p(A-hat) V with p = sum_{j=0..k} coef[j] T_j and A-hat = (A - cc I)/dd,
 * by the forward three-term Chebyshev recurrence. V, Y row-major n x nvec. */
void or_filter_apply(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                     double cc, double dd, int k, const double *coef, int nvec,
                     const double *V, double *Y);

/* Rademacher block (row-major n x nvec): sign of output l*n+i of stream `seed`. */
void or_rademacher(uint64_t seed, int64_t n, int nvec, double *V);

/* KPM moments zeta_k = (1/nvec) sum_l v_l^T T_k(A-hat) v_l, k = 0..K, for the
 * probe block V (row-major n x nvec). */
void or_kpm_moments(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                    double lmin, double lmax, int K, int nvec, const double *V,
                    double *mom);

/* Estimated eigenvalue count in [x0, x1] from the damped KPM expansion. */
double or_kpm_count(int K, const double *mom, int damping, double lmin, double lmax,
                    double x0, double x1);

/* Slicer (eq:slice-ti): cut intv[0..1] into nslices pieces of equal estimated
 * count using an npts-point grid. sli has nslices+1 entries. Returns 0 / -1. */
int or_slicer(int K, const double *mom, int damping, const double intv[4], int nslices,
              int npts, double *sli);

/* Cyclic Jacobi eigen-decomposition of the symmetric m x m column-major A
 * (overwritten). w[m] ascending, Vec m x m column-major (column j = vector j). */
int or_jacobi_eig(int m, double *A, double *w, double *Vec);

/* Spectrum bounds by nsteps Lanczos steps with full reorthogonalisation from
 * the start vector of stream `seed` (see or_lanczos_start), widened by the
 * extreme Ritz residual estimates. */
int or_lanczos_bounds(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                      int nsteps, uint64_t seed, double *lmin, double *lmax);

/* Lanczos start vector: x_i = 2 u(seed, restart*n + i) - 1 (not normalised). */
void or_lanczos_start(uint64_t seed, int64_t n, int64_t restart, double *x);

typedef struct {
  int m;          /* Krylov dimension per cycle */
  int max_its;    /* cap on Lanczos steps */
  int ncycle;     /* early-restart test period */
  double tol;     /* residual tolerance relative to ||A|| */
  uint64_t seed;  /* start-vector stream */
  int nev_cap;    /* capacity of lam/res/Y */
} or_lan_opts;

typedef struct {
  int nev;
  int niter;      /* Lanczos steps taken */
  int nmv;        /* products with A */
  int nrestart;
  int status;     /* 0 ok, 1 max_its reached, 2 capacity exceeded */
} or_lan_stats;

/* Filtered thick-restart Lanczos with locking (Algorithm alg:FiltLanTR, Section
 * 2.5) for the slice intv = {t_i, t_{i+1}, lambda_min, lambda_max} with the
 * filter (deg, coef, bar) from or_find_pol. Outputs lam[nev] ascending,
 * res[nev] = ||A u - lam u|| / ||A|| and Y (n x nev_cap column-major). */
int or_filtered_lanczos(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                        const double intv[4], int deg, const double *coef, double bar,
                        const or_lan_opts *opt, double *lam, double *res, double *Y,
                        or_lan_stats *st);

/* Filtered non-restart Lanczos (ChebLanNr, Section 2.3 and the solver list of
 * Section 3): Lanczos on p(A-hat) from one seeded random vector, with full
 * reorthogonalisation, up to opt->m steps; every opt->ncycle steps the sum of
 * the Ritz values >= bar is compared with its value at the previous test, and
 * the run stops when it has settled (relative change < 1e-10). The Ritz
 * vectors of the Ritz values >= bar then give Rayleigh quotients with A; those
 * inside the slice with residual <= tol are returned (lam ascending, res, Y as
 * in or_filtered_lanczos). st->status: 0 settled, 1 stopped at m steps. */
int or_filtered_lanczos_nr(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                           const double intv[4], int deg, const double *coef, double bar,
                           const or_lan_opts *opt, double *lam, double *res, double *Y,
                           or_lan_stats *st);

/* Lanczos DOS (landos; Section 2.1: a Lanczos procedure with the related
 * Gaussian quadrature, and the solver list of Section 3.1). For probe
 * l = 0..nvec-1, m Lanczos steps with full reorthogonalisation from the
 * Lanczos start vector of stream (seed, block l) give T_m; its eigenvalues
 * are the quadrature nodes and the squared first components of its
 * eigenvectors the weights (they sum to 1), so that
 * sum_k w_k f(theta_k) = v^T f(A) v / v^T v exactly for polynomials f of degree
 * < 2m. nodes/weights: nvec x m row-major, row l holding dims[l] <= m entries
 * (fewer at an invariant subspace), the rest 0. */
int or_lanczos_dos(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, int m,
                   int nvec, uint64_t seed, double *nodes, double *weights, int *dims);
/* Estimated count in [x0, x1] from the quadrature: n / nvec times the sum of
 * the weights of the nodes inside, each node spread by a Gaussian of standard
 * deviation sigma (sigma = 0: a point mass). */
double or_lanczos_count(const double *nodes, const double *weights, const int *dims, int nvec,
                        int m, int64_t n, double sigma, double x0, double x1);
/* Slicer on the Lanczos count (spslicer2), the same grid rule as or_slicer. */
int or_lanczos_slicer(const double *nodes, const double *weights, const int *dims, int nvec,
                      int m, int64_t n, double sigma, double xi, double eta, int nslices,
                      int npts, double *sli);

/* ---- generalized problems A x = lambda B x, B SPD (Section 2.4, eq:stdB,
 * Algorithm alg:LanAB; filtering through eq:gen1 and eq:polyapp1) ---- */

/* Least-squares Chebyshev approximation on [lo, hi] (lsPol, Section 3.1: the
 * polynomial approximations of t^(-1) and t^(-1/2) used for solves with B):
 * kind 0: f(t) = 1/t, kind 1: f(t) = 1/sqrt(t); coef[0..deg] are the
 * Chebyshev coefficients in u = (t - c)/d, c = (hi + lo)/2, d = (hi - lo)/2,
 * from the Chebyshev-Gauss quadrature of f with 1024 nodes (the truncated
 * Chebyshev series is the least-squares fit in the Chebyshev weight). */
int or_lspol(int kind, double lo, double hi, int deg, double *coef);
/* x = B^(-1) r by conjugate gradients to ||r - B x|| <= 1e-15 ||r||. */
int or_cg_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *vb,
                const double *r, double *x);
/* Bounds of the pencil's spectrum: nsteps of Algorithm alg:LanAB (full
 * reorthogonalisation, exact solves) from the Lanczos start vector of stream
 * `seed`, widened by the extreme Ritz residual estimates. */
int or_lanczos_bounds_gen(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                          const int32_t *rpb, const int32_t *cib, const double *vb, int nsteps,
                          uint64_t seed, double *lmin, double *lmax);
/* Filtered non-restart Lanczos for (A, B): Algorithm alg:LanAB applied to the
 * pencil (B rho(B^(-1) A-hat), B) of eq:gen1, so that its product step is eq:polyapp1,
 * z = rho(A-hat B^(-1)) z_i - beta_i z_{i-1} with A-hat = (A - cB)/d; the
 * Chebyshev recurrence in A-hat B^(-1) needs one solve with B and one product
 * with A per degree step (exact solves here). Stopping as
 * or_filtered_lanczos_nr; Ritz vectors W_m y (eq:gen1), each checked by its
 * Rayleigh quotient x^T A x / x^T B x and residual
 * ||A x - lambda B x|| / (||B x|| max(|lambda_min|, |lambda_max|)). Y holds
 * B-normalised vectors. */
int or_filtered_lanczos_gen(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                            const int32_t *rpb, const int32_t *cib, const double *vb,
                            const double intv[4], int deg, const double *coef, double bar,
                            const or_lan_opts *opt, double *lam, double *res, double *Y,
                            or_lan_stats *st);

/* The thick-restart form of Algorithm alg:FiltLanTR for the pencil, in the
 * B-inner product with the bases of Algorithm alg:LanAB; locked vectors
 * B-orthonormal (Y), every reading as or_filtered_lanczos. */
int or_filtered_lanczos_gen_tr(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *rpb, const int32_t *cib, const double *vb,
                               const double intv[4], int deg, const double *coef, double bar,
                               const or_lan_opts *opt, double *lam, double *res, double *Y,
                               or_lan_stats *st);

typedef struct {
  int block;      /* subspace dimension b */
  int max_its;    /* cap on iterations */
  double tol;     /* residual tolerance relative to ||A|| */
  uint64_t seed;  /* start-block stream: column j is the Lanczos start vector of block j */
  int nev_cap;    /* capacity of lam/res/Y */
} or_si_opts;

/* Filtered subspace iteration (ChebSI, end of Section 2.5 and Section 3.1): V <- p(A-hat) V,
 * orthonormalised (classical Gram-Schmidt, two passes; a column that vanishes
 * is replaced by the next random vector of the stream), then Rayleigh-Ritz
 * with A. After each filter application mu_j = v_j^T p(A-hat) v_j is known for
 * the current Ritz vectors; the run stops when the number of converged Ritz
 * pairs inside the slice (residual <= tol) is the same as at the previous
 * iteration and no unconverged Ritz value inside the slice has mu_j >= bar
 * (such a pair would be a wanted eigenvector still converging; an unconverged
 * pair with mu_j < bar is a mixture of eigenvectors outside the slice).
 * Outputs as or_filtered_lanczos; st->niter counts iterations (filter
 * applications to the block), st->status: 0 stopped by the rule, 1 max_its,
 * 2 capacity exceeded, 3 the slice filled the subspace (b too small). */
int or_filtered_subspace(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                         const double intv[4], int deg, const double *coef, double bar,
                         const or_si_opts *opt, double *lam, double *res, double *Y,
                         or_lan_stats *st);

#ifdef __cplusplus
}
#endif
#endif
