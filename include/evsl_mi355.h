/*
 * evsl_mi355 -- polynomial-filtered spectrum slicing for large sparse real
 * symmetric matrices on one AMD MI355X (gfx950).
 *
 * Method: EVSL (Li, Xi, Erlandson, Saad, "The Eigenvalues Slicing Library
 * (EVSL): Algorithms, Implementation, and Software", arXiv:1802.05215). All
 * eigenpairs of A in [xi, eta] are found by cutting the interval into slices
 * with a kernel-polynomial (KPM) density-of-states estimate (Section 2.1,
 * eq:DOS0, eq:slice-ti) and running, per slice, a thick-restart Lanczos with
 * locking on a Chebyshev polynomial filter p(A) (Section 2.2.1, Section 2.5,
 * Algorithm alg:FiltLanTR).
 *
 * Conventions for every entry point:
 *  - Return value: EVSL_OK (0) or one of the EVSL_E* codes below; no C++
 *    exception crosses this interface. evsl_strerror() names a code.
 *  - "device" pointers are HIP device memory on the device current when the
 *    context was created; "host" pointers are ordinary host memory.
 *  - Device inputs are owned by the caller, read-only, and must stay valid
 *    until the call returns (or, for asynchronous calls, until the context's
 *    stream has executed the work).
 *  - The spectrum interval convention follows the paper's intv[4]
 *    (Section 3.1): {xi, eta, lambda_min, lambda_max}.
 */
#ifndef EVSL_MI355_H
#define EVSL_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define EVSL_OK 0
#define EVSL_EINVAL 1    /* bad argument: n <= 0, xi >= eta, NULL pointer, interval outside the bounds */
#define EVSL_ENOMEM 2    /* device or host allocation failed */
#define EVSL_EHIP 3      /* HIP runtime error (the hipError_t is kept in the context) */
#define EVSL_EDEGREE 4   /* filter needs more than max_deg; the max_deg filter is returned */
#define EVSL_ENOCONV 5   /* Lanczos step cap reached; the pairs locked so far are returned */
#define EVSL_ESPECTRUM 6 /* filter blow-up: [lambda_min, lambda_max] misses part of the spectrum
                            (a Ritz value of p(A-hat) exceeds sum |coef_j|, the bound of |p| on
                            [-1, 1], or a non-finite value appears) */
#define EVSL_ENOTIMPL 7  /* option not implemented */
#define EVSL_ESCRATCH 8  /* the problem needs more device scratch than the allocation-free
                            entry point holds (EVSL_NOALLOC_SCRATCH_BYTES) */

/* Bytes of the allocation-free entry point's device scratch: one array per
 * device, held from the library's load until the process ends. */
#define EVSL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* ---- value types ---- */
#define EVSL_F64 0
#define EVSL_F32 1

/* ---- Lanczos variant of a slice (evsl_lan_opts_t.method) ---- */
#define EVSL_LAN_TR 0 /* thick restart with locking (ChebLanTr, Algorithm alg:FiltLanTR) */
#define EVSL_LAN_NR 1 /* non-restart (ChebLanNr, Sections 2.3 and 3.1) */

/* ---- damping of the Chebyshev expansion ---- */
#define EVSL_DAMP_NONE 0
#define EVSL_DAMP_SIGMA 1   /* Lanczos sigma factors, eq:polPJ (the paper's default) */
#define EVSL_DAMP_JACKSON 2 /* Jackson kernel (Weisse et al., Rev. Mod. Phys. 78, 275, 2006) */

typedef struct evsl_ctx_s *evsl_ctx_t;

/* CSR matrix (Section 3.1: matrices are stored in CSR). All arrays are
 * device memory: row_ptr[n+1] and col[nnz] int32, col ascending within a row,
 * val[nnz] double (dtype EVSL_F64) or float (EVSL_F32). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  int dtype;
} evsl_csr_t;

/* Polynomial filter (find_pol, Section 2.2.1): rho(t) = sum_j coef[j] T_j(t)
 * on the mapped variable t = (lambda - cc)/dd (eq:mapping). `coef` is a host
 * buffer of `cap` doubles supplied by the caller; deg + 1 entries are used.
 * boundary: 0 interior slice, -1 left end at lambda_min, +1 right end at
 * lambda_max. bar is the filter value at the slice ends: Ritz values of
 * rho(A) at or above bar are the candidates of Algorithm alg:FiltLanTR. */
typedef struct {
  int deg;
  int boundary;
  double gamma;
  double cc;
  double dd;
  double bar;
  double *coef;
  int cap;
} evsl_pol_t;

/* Options of the filtered Lanczos (Algorithm alg:FiltLanTR). Zero fields take
 * the documented defaults. */
typedef struct {
  int m;          /* Krylov dimension per cycle; 0: max(3 nev_est + 30, 60);
                     EVSL_LAN_NR: total step cap; 0: max(5 nev_est + 200, 400) */
  int max_its;    /* cap on Lanczos steps; 0: max(20 m, 2000) (EVSL_LAN_NR: m) */
  int ncycle;     /* early-restart test period; 0: 10 (EVSL_LAN_TR), 30 (EVSL_LAN_NR).
                     Thick restart: a settled test ends a cycle only once it has run 30
                     steps */
  double tol;     /* residual tolerance ||A u - lambda u|| / ||A||; 0: 1e-8 */
  uint64_t seed;  /* start-vector stream (SplitMix64); restarts draw further blocks */
  int nev_est;    /* expected count in the slice (sizing only); 0: 50 */
  int nev_cap;    /* capacity for locked pairs; 0: max(2 nev_est + 40, 100) */
  int prec;       /* filter arithmetic: EVSL_F64, or EVSL_F32 (precision form, below) */
  const void *val32; /* EVSL_F32: device float values of A (NULL: the library converts A) */
  double tol_lo;  /* EVSL_F32: lock tolerance of the FP32 phase;
                     0: max(tol, min(1e-3, 2e-7 deg)) */
  int polish;     /* EVSL_F32: < 0: no FP64 phase (the FP32-phase pairs are returned as they
                     are); otherwise the FP64 phase below runs when needed */
  int polish_div; /* unused; keep 0 */
  int method;     /* EVSL_LAN_TR (0) or EVSL_LAN_NR (FP64 only; else EVSL_ENOTIMPL) */
  int reserved;
} evsl_lan_opts_t;
/* Non-restart form (method = EVSL_LAN_NR): Lanczos on p(A-hat) from one
 * seeded random vector with full reorthogonalisation and no restart; every
 * ncycle steps the sum of the Ritz values >= bar is compared with its value at
 * the previous test and the run ends once it has settled (relative change
 * < 1e-10) or after m steps (then EVSL_ENOCONV). The Ritz vectors of all Ritz
 * values >= bar are then checked against A, in chunks of
 * max(3 nev_est + 30, 60) columns; those inside the slice with residual <= tol
 * are returned (at most nev_cap). Device memory: (nev_cap + m + 1) basis
 * columns plus two chunks. */
/* Precision form (prec = EVSL_F32): the filter recurrence runs in FP32 values,
 * vectors and accumulation; reorthogonalisation, Rayleigh-Ritz, the residual
 * test and the coefficients stay FP64. The FP32 phase locks pairs at tol_lo
 * (residuals computed in FP64) and ends by the usual rule, or when two
 * restarts in a row lock nothing while candidates remain (the FP32 floor).
 * When any pair misses tol, or candidates remain, or the phase hit max_its,
 * an FP64 phase follows. First the polish: Rayleigh-Ritz with A on the span
 * of the FP32 phase's locked pairs and candidates, then, while some Ritz pair
 * inside the slice misses tol, up to two FP64 filter applications to that
 * block, each followed by Rayleigh-Ritz (the filtered subspace iteration,
 * Section 2.5, started from the FP32 block). The polish ends a slice only when
 * the FP32 phase had ended by the stopping rule; pairs still above tol, or a
 * slice whose FP32 phase stopped short (max_its, capacity, candidates left at
 * the FP32 floor), then go to the thick-restart continuation: the same
 * Lanczos with the FP64 filter, deflated against the pairs that meet tol and
 * started from the normalised sum of the others (a random vector when none is
 * left), run to tol by the ordinary stopping rule, so the result is complete
 * at tol. In a batch the polish of all slices shares its block
 * filter launches and the continuations run together. npolish: 0 when no
 * FP64 phase ran, else 1 + the polish's FP64 filter applications, plus 100
 * when the thick-restart continuation ran. */

/* Result of one slice. lam/res are host arrays and Y a device n x nev
 * column-major array, all allocated by the library and released with
 * evsl_eigs_free(). lam ascending; res[j] = ||A y_j - lam_j y_j|| / ||A|| with
 * ||A|| = max(|lambda_min|, |lambda_max|). */
typedef struct {
  int nev;
  double *lam;
  double *res;
  double *Y;
  int niter;      /* Lanczos steps */
  int nmv;        /* products with A (filter steps + Ritz checks) */
  int nrestart;
  int npolish;    /* precision form: 0 without an FP64 phase; else 1 + FP64 filter
                     applications of the polish, + 100 with the thick-restart
                     continuation (see the precision form above) */
  int status;     /* EVSL_OK or EVSL_ENOCONV */
  int north2;     /* Lanczos steps whose reorthogonalisation made a second
                     Gram-Schmidt pass (DGKS test, Section 2.3) */
  double t_mv;    /* seconds in filter products */
  double t_orth;  /* seconds in reorthogonalisation */
  double t_ritz;  /* seconds in Rayleigh-Ritz, locking and restarts */
  double t_tot;   /* wall time of the call; in a batch, when this slice finished */
} evsl_eigs_t;

/* Device memory allocator of a context. alloc returns at least `bytes` bytes
 * of device memory usable on `stream` (the context's hipStream_t), or NULL
 * when it cannot: the call that asked then returns EVSL_ENOMEM with every
 * buffer it had taken handed back to free and the context's ledger
 * (evsl_mem_stats) where it was. free receives exactly the pointers alloc
 * returned, once each, after the work on `stream` that uses them has been
 * ordered before it (the library synchronises the stream before freeing
 * workspace). `user` is passed through unchanged. */
typedef struct {
  void *(*alloc)(void *user, size_t bytes, void *stream);
  void (*free)(void *user, void *ptr, void *stream);
  void *user;
} evsl_alloc_t;

/* ---- context (replaces EVSLStart/EVSLFinish of Section 3.1) ----
 * stream: a hipStream_t (NULL = the null stream). alloc: the device allocator
 * for every buffer the context holds (workspace, slice bases, result
 * vectors), copied into the context; NULL = hipMalloc/hipFree; EVSL_EINVAL
 * when given with a NULL alloc or free. The context holds the stream, a
 * grow-only device workspace, the tuning table and timers. Not thread-safe:
 * one context per host thread and stream. */
int evsl_create(evsl_ctx_t *ctx, void *stream, const evsl_alloc_t *alloc);
int evsl_destroy(evsl_ctx_t ctx);
/* hipError_t of the last EVSL_EHIP returned by this context. */
int evsl_last_hip_error(evsl_ctx_t ctx);
const char *evsl_strerror(int code);

/* ---- spectrum bounds (LanBounds/LanTrbounds, Section 3.1; Section 2.2.1)
 * nsteps Lanczos steps with full reorthogonalisation from the start vector of
 * stream `seed`; the extreme Ritz values are widened by their residual
 * estimates |beta_{m+1} y_{m,j}|. Host outputs; synchronous. */
int evsl_spectrum_bounds(evsl_ctx_t ctx, const evsl_csr_t *A, int nsteps, uint64_t seed,
                         double *lmin, double *lmax);

/* ---- 1. KPM density of states (kpmdos, Section 2.1) ----
 * moments[k] (host, degree+1 doubles) estimates trace T_k(A-hat),
 * A-hat = (A - c I)/d with c, d from intv[2..3], from `nvec` Rademacher probe
 * vectors whose signs come from SplitMix64 stream `seed` (entry (i, l) from
 * output l*n + i). nev_est (host) is the damped estimate of the number of
 * eigenvalues in [intv[0], intv[1]]. Synchronous. */
int evsl_kpm_dos(evsl_ctx_t ctx, const evsl_csr_t *A, const double intv[4], int degree,
                 int nvec, uint64_t seed, int damping, double *moments, double *nev_est);

/* ---- 2. spectrum slicer (spslicer, eq:slice-ti) ----
 * Host-only pure function. Cuts [intv[0], intv[1]] into nslices pieces with
 * equal estimated counts using an npts-point uniform grid; sli (host) gets
 * nslices+1 boundaries, sli[0] = xi, sli[nslices] = eta. */
int evsl_slice_spectrum(const double *moments, int degree, int damping, const double intv[4],
                        int nslices, int npts, double *sli);

/* Estimated count in [x0, x1] from KPM moments (host-only). */
int evsl_kpm_count(const double *moments, int degree, int damping, double lmin, double lmax,
                   double x0, double x1, double *count);

/* ---- 2b. Lanczos DOS and its slicer (landos / spslicer2; Section 2.1: a
 * Lanczos procedure with the related Gaussian quadrature; Section 3.1) ----
 * For probe l = 0..nvec-1: msteps Lanczos steps with full reorthogonalisation
 * (fewer at an invariant subspace, dims[l] < msteps) from the Lanczos start
 * vector of stream (seed, block l); the eigenvalues of T are the quadrature
 * nodes and the squared first components of its eigenvectors the weights
 * (summing to 1 per probe). nodes, weights: host, nvec x msteps row-major,
 * unused entries 0; dims: host, nvec. Synchronous. */
int evsl_lanczos_dos(evsl_ctx_t ctx, const evsl_csr_t *A, int msteps, int nvec, uint64_t seed,
                     double *nodes, double *weights, int *dims);
/* Host-only. Estimated count in [x0, x1]: n / nvec times the quadrature weight
 * inside, each node spread by a Gaussian of standard deviation sigma (0: a
 * point mass). */
int evsl_lanczos_count(const double *nodes, const double *weights, const int *dims, int nvec,
                       int msteps, int64_t n, double sigma, double x0, double x1, double *count);
/* Host-only. Cuts [xi, eta] into nslices pieces of equal estimated count on an
 * npts-point grid (the rule of evsl_slice_spectrum); sli gets nslices+1 points. */
int evsl_slice_spectrum_lanczos(const double *nodes, const double *weights, const int *dims,
                                int nvec, int msteps, int64_t n, double sigma, double xi,
                                double eta, int nslices, int npts, double *sli);

/* ---- 3. filter coefficients (find_pol, Section 2.2.1: eq:mapping, eq:Cheb0,
 * eq:mu, eq:Neq, eq:polPJ) ----
 * Host-only. intv = {t_i, t_{i+1}, lambda_min, lambda_max}. The degree is the
 * smallest k >= 2 at which the balanced filter's end values are <= tau
 * (interior slice) or, for a boundary slice, the inner end value is
 * <= tau_ext. Returns EVSL_EDEGREE when max_deg is reached (the max_deg
 * filter is still returned), EVSL_EINVAL when pol->cap < max_deg + 1. */
int evsl_cheb_coeffs(const double intv[4], int damping, double tau, double tau_ext,
                     int max_deg, evsl_pol_t *pol);

/* ---- 4. filter application Y = p(A-hat) V (eq:Cheb0; Table tab:itercomp:
 * k products with A for a degree-k filter) ----
 * V, Y: device, row-major n x ncols with leading dimension ldv >= ncols, of
 * type prec (double for EVSL_F64, float for EVSL_F32; with EVSL_F32 A must
 * have dtype EVSL_F32). Column c uses filter pols[col_group[c]] (col_group is
 * a host array of ncols indices < npol); all filters must share cc and dd.
 * Columns ordered by non-increasing degree run fastest. A single vector
 * (ncols = ldv = 1) runs the three-term recurrence with its running sum; a
 * block is evaluated by Clenshaw's recurrence for the same polynomial (four
 * passes over the block per degree step instead of five). Asynchronous on the
 * context's stream. */
int evsl_filter_apply(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_pol_t *pols, int npol,
                      const int32_t *col_group, const void *V, void *Y, int64_t ldv,
                      int ncols, int prec);

/* ---- allocation-free filter application ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as evsl_filter_apply, with every device
 * buffer beyond V and Y (the coefficient table, 8 * ncols * (max degree + 1)
 * bytes, and the two recurrence blocks, 2 * n * ldv values, each rounded up to
 * 256 bytes) taken from a static device array of EVSL_NOALLOC_SCRATCH_BYTES
 * per device instead of the context's workspace; it reads the 32-bit column
 * indices (no 16-bit offset table is built). Calls no hipMalloc, hipFree or
 * other allocating routine. Returns EVSL_ESCRATCH, with nothing launched,
 * when the buffers do not fit the array. Every call on a device shares that
 * device's array, which keeps the last call's contents (the recurrence blocks
 * are cleared by a kernel at the start of each call): calls that overlap on
 * one device, on any streams or contexts, race. The array's device address is
 * looked up in evsl_create (hipGetSymbolAddress), once per device.
 * Synchronises the context's stream once, after uploading the coefficient
 * table, as evsl_filter_apply does. */
int evsl_filter_apply_noalloc(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_pol_t *pols,
                              int npol, const int32_t *col_group, const void *V, void *Y,
                              int64_t ldv, int ncols, int prec);

/* ---- 5. filtered thick-restart Lanczos with locking (ChebLanTr,
 * Algorithm alg:FiltLanTR) on one slice ----
 * intv = {t_i, t_{i+1}, lambda_min, lambda_max}; pol from evsl_cheb_coeffs
 * on the same intv. Returns every converged eigenpair whose eigenvalue lies
 * in [t_i, t_{i+1}] (out, allocated by the library). Synchronous. Returns
 * EVSL_ENOCONV (with the pairs found) when max_its is reached. */
int evsl_filtered_lanczos(evsl_ctx_t ctx, const evsl_csr_t *A, const double intv[4],
                          const evsl_pol_t *pol, const evsl_lan_opts_t *opt, evsl_eigs_t *out);

/* Several slices of one matrix solved together: each Lanczos step applies all
 * active slices' filters in one block SpMM launch per degree step (columns
 * are slices, ordered by degree). intv holds 4 doubles per slice; pols and
 * outs one entry per slice; opts one entry per slice. Synchronous. */
int evsl_filtered_lanczos_batch(evsl_ctx_t ctx, const evsl_csr_t *A, int nslices,
                                const double *intv, const evsl_pol_t *pols,
                                const evsl_lan_opts_t *opts, evsl_eigs_t *outs);

/* ---- 6. filtered subspace iteration (ChebSI; end of Section 2.5 and Section
 * 3.1: a projection method beside Lanczos whose block size comes from the DOS
 * count) on one or several slices ----
 * Each iteration filters the slice's block V (n x block) with p(A-hat),
 * orthonormalises the result (two SVQB passes: Gram matrix on FP64 MFMA,
 * eigen-decomposition on the host; directions lost to rank deficiency are
 * replaced by further random vectors of the seed's stream) and runs
 * Rayleigh-Ritz with A. The run ends when the count of converged Ritz pairs in
 * the slice (residual <= tol) repeats and no unconverged Ritz value in the
 * slice has a filter Rayleigh quotient v^T p(A-hat) v >= bar. Returns the
 * converged pairs in the slice. EVSL_ENOCONV (with the pairs found) when
 * max_its is reached or when every Ritz value lies in the slice (block too
 * small for the slice's count). Device memory per slice: 3 n x block FP64
 * plus, for the batch, 3 n x (sum of blocks) for the filter. In a batch all
 * active slices' blocks are filtered together, one block SpMM launch per
 * degree step. Synchronous. out->nrestart counts replaced directions. */
typedef struct {
  int block;      /* subspace dimension; 0: 3 nev_est + 8 (at most n) */
  int max_its;    /* cap on iterations (filter applications); 0: 100 */
  double tol;     /* residual tolerance ||A u - lambda u|| / ||A||; 0: 1e-8 */
  uint64_t seed;  /* start block: column j is restart block j of the Lanczos start stream */
  int nev_est;    /* expected count in the slice (sizes the block); 0: 50 */
  int reserved[3];
} evsl_si_opts_t;
int evsl_filtered_subspace(evsl_ctx_t ctx, const evsl_csr_t *A, const double intv[4],
                           const evsl_pol_t *pol, const evsl_si_opts_t *opt, evsl_eigs_t *out);
int evsl_filtered_subspace_batch(evsl_ctx_t ctx, const evsl_csr_t *A, int nslices,
                                 const double *intv, const evsl_pol_t *pols,
                                 const evsl_si_opts_t *opts, evsl_eigs_t *outs);

/* ---- 7. generalized problems A x = lambda B x, B SPD (Section 2.4; eq:stdB,
 * Algorithm alg:LanAB; filtering through eq:gen1 and eq:polyapp1) ----
 * Solves with B are the least-squares Chebyshev approximation of 1/t on
 * [bbounds[0], bbounds[1]] (a range containing B's spectrum, bbounds[0] > 0,
 * e.g. from evsl_spectrum_bounds on B) of degree bdeg (lsPol, Section 3.1);
 * its error decays like ((sqrt(k) - 1)/(sqrt(k) + 1))^bdeg with
 * k = bbounds[1]/bbounds[0]. */
/* Host-only. Chebyshev coefficients (in u = (t - c)/d on [lo, hi]) of the
 * least-squares approximation of 1/t (kind 0) or 1/sqrt(t) (kind 1). */
int evsl_lspol(int kind, double lo, double hi, int deg, double *coef);
/* Bounds of the pencil's spectrum from nsteps of Algorithm alg:LanAB (full
 * reorthogonalisation) from the Lanczos start vector of stream `seed`, widened
 * by the extreme Ritz residual estimates. Synchronous. */
int evsl_spectrum_bounds_gen(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_csr_t *B,
                             const double bbounds[2], int bdeg, int nsteps, uint64_t seed,
                             double *lmin, double *lmax);
/* Filtered Lanczos for (A, B) on one slice: Algorithm alg:LanAB applied to
 * (B rho(B^-1 A-hat), B), its product step as eq:polyapp1 (per degree step one
 * solve with B and one product with A), full reorthogonalisation. With
 * opt->method = EVSL_LAN_NR (or opt NULL) the non-restart form and its settled
 * sum test; with EVSL_LAN_TR the thick-restart form of Algorithm
 * alg:FiltLanTR in the B-inner product (locked vectors B-orthonormal, the same
 * sizes and readings as evsl_filtered_lanczos). intv = {t_i, t_{i+1},
 * lambda_min, lambda_max} of the pencil and pol from evsl_cheb_coeffs on it;
 * prec EVSL_F32: EVSL_ENOTIMPL. Returns the Ritz pairs in the slice with
 * ||A y - lambda B y|| / (||B y|| max(|lambda_min|, |lambda_max|)) <= tol; Y is
 * B-orthonormal. out->nrestart counts the solves with B. Synchronous. */
int evsl_filtered_lanczos_gen(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_csr_t *B,
                              const double bbounds[2], int bdeg, const double intv[4],
                              const evsl_pol_t *pol, const evsl_lan_opts_t *opt,
                              evsl_eigs_t *out);

/* Copies the result vectors into a caller-owned device array dst (column j
 * of out->Y to dst + j*ldd, ldd >= n). Asynchronous on the context stream. */
int evsl_eigs_get_vectors(evsl_ctx_t ctx, const evsl_eigs_t *out, int64_t n, double *dst,
                          int64_t ldd);

/* Releases lam, res (host) and Y (device) of a result; safe on zeroed structs. */
void evsl_eigs_free(evsl_ctx_t ctx, evsl_eigs_t *out);

/* Block Gram product C = X^T Y (FP64 MFMA): X n x p and Y n x q column-major
 * device arrays with leading dimensions ldx, ldy >= n; C is a device p x q
 * column-major array (ldc >= p). Summation order is fixed. Asynchronous. */
int evsl_gram(evsl_ctx_t ctx, int64_t n, int p, int q, const double *X, int64_t ldx,
              const double *Y, int64_t ldy, double *C, int64_t ldc);

/* ---- tuning ----
 * Autotuner for the batched filter: times Chebyshev steps of A (in the
 * arithmetic `prec`, EVSL_F64 or EVSL_F32; A itself is FP64) over scratch
 * blocks of g = 1, 2, 3, 4, 5, 6, 8, ... <= max_cols columns (and of the
 * remainder widths max_cols mod g) and keeps the group width whose split of
 * max_cols columns (floor(max_cols / g) groups of g and one of the rest) takes
 * the least time per degree step (a narrower group wins unless a wider one is
 * more than 2% faster); us_per_colstep is that time over max_cols. Batches then
 * filter their slices in groups of that width, one launch per group and degree
 * step. Synchronous; the scratch contents are arbitrary. */
int evsl_autotune(evsl_ctx_t ctx, const evsl_csr_t *A, int max_cols, int prec, int *group_width,
                  double *us_per_colstep);
/* Sets the batch group width directly (0: all active slices in one group). */
int evsl_set_group_width(evsl_ctx_t ctx, int g);

/* ---- measurement helpers ----
 * Number of filter-step kernels launched and their total device time (from
 * HIP events on the context stream) since the last reset. */
int evsl_filter_stats(evsl_ctx_t ctx, int64_t *launches, double *seconds, double *bytes);
int evsl_reset_stats(evsl_ctx_t ctx);
/* Device memory the context holds, in bytes: `current` now (workspace kept
 * for reuse, plus result vectors not yet passed to evsl_eigs_free) and `peak`
 * since creation or the last reset (reset_peak != 0 sets peak = current
 * after reading). Host-side bookkeeping of the library's own allocations
 * only; a serving layer uses it to check its admission footprints. */
int evsl_mem_stats(evsl_ctx_t ctx, int64_t *current, int64_t *peak, int reset_peak);
/* Bandwidth reference: `reps` launches of a plain copy kernel reading and
 * writing `bytes` bytes (rounded down to a multiple of 16) of context
 * workspace; returns the average seconds per copy (HIP events). Used to
 * calibrate hardware traffic counters. Synchronous. */
int evsl_copy_probe(evsl_ctx_t ctx, int64_t bytes, int reps, double *seconds_per_copy);
/* Enables (1) or disables (0) HIP-event timing of each filter application. */
int evsl_set_timing(evsl_ctx_t ctx, int on);
/* Enables (1, the default) or disables (0) HIP graphs in evsl_filtered_lanczos_batch:
 * each group's filter (gather, one launch per degree step, scatter) is captured
 * once per active set and replayed every Lanczos step. Results are identical
 * either way (same kernels, same order). */
int evsl_set_graphs(evsl_ctx_t ctx, int on);
/* Selects the kernel for single-vector filter steps: 0 auto, 1 direct
 * row-per-thread, 2 LDS-staged CSR stream, 3 LDS-staged with the nonzero loop
 * unrolled by 8 and XCD-contiguous workgroup order, 4 as 3 without the XCD
 * order. */
int evsl_set_spmv_variant(evsl_ctx_t ctx, int variant);
/* Selects the kernel for block (several columns) filter steps, process-wide:
 * 1 global loads, 2 LDS-staged + unrolled + XCD order with two columns per
 * lane (16-byte loads) when the block allows it (default), 3 as 2 without the
 * XCD order and one column per lane, 4 as 2 with one column per lane. */
int evsl_set_block_variant(int variant);
/* Launch schedule of this context's block filter steps (variant 2), a choice
 * of how workgroups walk an n x nc row-major block and so of what the caches
 * can reuse; results are bit-identical under every schedule (each element is
 * computed by the same arithmetic in the same order):
 *   map 0  row blocks in launch order, all nc columns per row block;
 *   map 1  (default) as 0 with each of the 8 XCDs sweeping a contiguous row
 *          range;
 *   map 2  the columns in chunks of chunk_cols, one chunk after another over
 *          all rows; within a chunk, row blocks are dealt to the XCDs in runs
 *          of `group` consecutive blocks, so all XCDs sweep the same rows
 *          together while each keeps short runs of neighbouring rows.
 * lane_cols: block columns per lane (0: 16-byte lanes, i.e. 2 FP64 or 4 FP32;
 * 1, 2 or 4 when the block's width, leading dimension and alignment allow,
 * else halved until they do). rows_per_wg: rows per workgroup (0: four passes
 * of the workgroup's row group; else rounded down to whole passes, at most 256).
 * lds_staging 0: the kernel that reads the CSR rows from global memory without
 * staging them in LDS (one chunk, launch order, one column per lane; 1: the
 * LDS-staged kernel). A chunk as wide as the block, or not a multiple of the
 * lane width, falls back to map 1; so do the KPM steps. EVSL_EINVAL for a map
 * outside 0-2, a map-2 chunk or group below 1, another lane width, rows_per_wg
 * outside 0-256 or lds_staging other than 0 or 1. */
int evsl_set_block_schedule(evsl_ctx_t ctx, int map, int chunk_cols, int group, int lane_cols,
                            int rows_per_wg, int lds_staging);
int evsl_get_block_schedule(evsl_ctx_t ctx, int *map, int *chunk_cols, int *group,
                            int *lane_cols, int *rows_per_wg, int *lds_staging);
/* Times the Clenshaw degree step of the block filter (eq:Cheb0 evaluated by
 * Clenshaw's recurrence) on A over an n x ncols block of scratch vectors for
 * each candidate schedule (maps 0 and 1; map 2 with chunks of 16-128 columns
 * and runs of 1-64 row blocks; in FP64 each also with 4 columns per lane), then
 * for the fastest one 1, 2 and 8 passes per workgroup and the kernel without
 * LDS staging, keeps the fastest in the context and
 * returns its milliseconds per step. Uses 3 n x ncols blocks of workspace
 * (value size by prec). Synchronous. */
int evsl_autotune_schedule(evsl_ctx_t ctx, const evsl_csr_t *A, int ncols, int prec,
                           double *ms_per_step);

#ifdef __cplusplus
}
#endif
#endif
