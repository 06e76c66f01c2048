// Internal launch interface of the HIP kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace evk {

struct Csr {
  int n;
  int64_t nnz;
  const int *rp;
  const int *ci;
  const void *va;
  int dtype;  // 0 double, 1 float
  // optional: col[k] - row(k) as 16-bit offsets (make_col_offsets); when set,
  // the block filter reads these instead of ci
  const int16_t *cd = nullptr;
};

// cd[k] = col[k] - row(k) for every nonzero; returns false (cd unusable) when
// an offset does not fit 16 bits. `flag` is one device int of scratch.
// Synchronous.
bool make_col_offsets(hipStream_t s, const Csr &A, int16_t *cd, int *flag);

// Step kinds of the three-term Chebyshev recurrence (eq:Cheb0) on
// A-hat = (A - c I)/d:
//   PLAIN: Wn = s1 * A W + s0 * W                      (no Y)
//   FIRST: Wn = s1 * A W + s0 * W, Y = c0 W + c1 Wn    (s1 = 1/d, s0 = -c/d)
//   NEXT : Wn = s1 * A W + s0 * W - Wp, Y += c Wn     (s1 = 2/d, s0 = -2c/d)
// Wn may alias Wp (each element is read, then written, by one thread).
enum StepKind {
  STEP_PLAIN = 0,
  STEP_FIRST = 1,
  STEP_NEXT = 2,
  STEP_KPM_FIRST = 3,
  STEP_KPM_NEXT = 4,
  // Clenshaw step: Wn = coef[col][jnext] Vd + s1 A W + s0 W - Wp (Wn may be Wp)
  STEP_CLEN = 5
};

// Single vectors stored as columns of a column-major array (column stride ld);
// grid.y runs over ncol columns. coef: device table, column c uses
// coef[c * cld + j]. variant: 1 direct (row per thread), 2 LDS-staged.
template <typename T>
void cheb_vec(hipStream_t s, const Csr &A, int variant, int kind, double s1, double s0,
              const T *W, const T *Wp, T *Wn, T *Y, int64_t ld, int ncol, const double *coef,
              int cld, int jnext, const T *Vd = nullptr);

// Launch schedule of the block filter (see k_cheb_blk_lds): map 0 launch
// order, 1 contiguous row ranges per XCD, 2 column chunks of cw columns one
// after another with row blocks dealt to the XCDs in runs of grp; vec: columns
// per lane (0: 16-byte lanes; 1, 2 or 4 when the block's alignment allows);
// rows: rows per workgroup (0: the default, four passes of the workgroup's
// row group; else rounded to whole passes, at most 256 rows); lds = 0: the
// global-load kernel (no LDS staging of the CSR rows, launch order).
struct BlkSched {
  int map = 1;
  int cw = 0;
  int grp = 1;
  int vec = 0;
  int rows = 0;
  int lds = 1;
};

// Row-major block n x ld, first nc columns active. For the KPM kinds, Vd is
// the probe block and partial receives one partial sum of Vd . Wn per
// workgroup (partial must hold blk_partials(n, nc) doubles). sched: null =
// one chunk with contiguous row ranges per XCD (map 1).
template <typename T>
void cheb_blk(hipStream_t s, const Csr &A, int kind, double s1, double s0, const T *W,
              const T *Wp, T *Wn, T *Y, int64_t ld, int nc, const double *coef, int cld, int jnext,
              const T *Vd, double *partial, const BlkSched *sched = nullptr);
int blk_partials(int n, int nc);
// Block kernel choice: 1 global loads, 2 LDS-staged and scheduled (default), 3 LDS-staged,
// one column per lane, launch order, 4 as 2 with one column per lane.
void set_blk_variant(int v);

// Gather / scatter FP64 columns into / out of a row-major block of type TB:
// blk[r * ldb + c] = src[c][r] for c < nc (pointers in a device array).
template <typename TB>
void gather_cols(hipStream_t s, int n, int nc, const double *const *src, TB *blk, int64_t ldb);
template <typename TB>
void scatter_cols(hipStream_t s, int n, int nc, const TB *blk, int64_t ldb, double *const *dst);
// C (p x q, column-major, ldc) = X^T Y with X n x p, Y n x q column-major, on
// FP64 MFMA; `partial` holds gemm_tn_partials(n, p, q) doubles. Deterministic.
int64_t gemm_tn_partials(int n, int p, int q);
int64_t gemm_tn_partials_bound(int n, int p, int q);
void gemm_tn(hipStream_t s, int n, int p, int q, const double *X, int64_t ldx, const double *Y,
             int64_t ldy, double *C, int64_t ldc, double *partial);

// h[j] = B[:, j] . z  for j < nb (B column-major, leading dim ld); uses
// `partial` (gemv_partials(n, nb) doubles). Deterministic order.
int gemv_partials(int n, int nb);
// With `gate` set, the launches do nothing and h = 0 when gate[0] == 0.
void gemv_t(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *z,
            double *partial, double *h, const int *gate = nullptr);
// z -= B h (nothing when gate is set and gate[0] == 0)
void gemv_n_sub(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *h,
                double *z, const int *gate = nullptr);
// z -= B h, and per-workgroup sums of squares of the new z into nrm_partial
// (nrm_partials(n) doubles)
int nrm_partials(int n);
void gemv_n_sub_nrm(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *h,
                    double *z, double *nrm_partial);
// gate[0] = 1 when a second Gram-Schmidt pass is due: ||z||^2 (from the
// partials of gemv_n_sub_nrm) < sum of h[j]^2 over j in [lo, hi), or always
// when force is set
void dgks_gate(hipStream_t s, int n, const double *nrm_partial, const double *h, int lo, int hi,
               int *gate, int force = 0);
// The three-term subtraction of a Lanczos step: z -= alpha[0] q + beta qp
// (alpha a device scalar; qp may be null).
void three_term(hipStream_t s, int n, double *z, const double *q, const double *qp,
                const double *alpha, double beta);
// out[c] = X[:, c] . Y[:, c] for c < ncol (column-major, strides ldx, ldy).
int dot_partials(int n, int ncol);
void col_dots(hipStream_t s, int n, int ncol, const double *X, int64_t ldx, const double *Y,
              int64_t ldy, double *partial, double *out);
// out[c] = || AX[:, c] - lam_c X[:, c] ||^2 with lam_c = xax[c] / xx[c].
void col_resid2(hipStream_t s, int n, int ncol, const double *X, const double *AX, int64_t ld,
                const double *xax, const double *xx, double *partial, double *out);
// dst = src / sqrt(nrm2[0]); beta_out[0] = sqrt(nrm2[0]) when beta_out != nullptr.
void normalize(hipStream_t s, int n, const double *src, double *dst, const double *nrm2,
               double *beta_out);
// X[:, c] *= 1/sqrt(nrm2[c]) for c < ncol.
void normalize_cols(hipStream_t s, int n, int ncol, double *X, int64_t ld, const double *nrm2);
// C = A B: A n x K column-major (lda), B K x N column-major (ldb), C n x N (ldc).
void gemm_nn(hipStream_t s, int n, int K, int N, const double *A, int64_t lda, const double *B,
             int64_t ldb, double *C, int64_t ldc);
// p[0 .. count) = 0 (a kernel, so that it can be captured in a graph)
template <typename T>
void fill_zero(hipStream_t s, int64_t count, T *p);
// Counter-based random numbers (SplitMix64 output index + 1 from state seed).
void rademacher(hipStream_t s, int n, int nvec, uint64_t seed, double *V);
void lanczos_start(hipStream_t s, int n, uint64_t seed, int64_t restart, double *x);
// Final fixed-order reduction of nw partial sums per column:
// out[c] = scale * sum_w partial[c * nw + w].
void reduce_partials(hipStream_t s, int nw, int ncol, const double *partial, double scale,
                     double *out, const int *gate = nullptr);
// y += a x over len doubles.
void axpy(hipStream_t s, int64_t len, double a, const double *x, double *y);
// Plain copy of `bytes` (a multiple of 16) from x to y: the bandwidth reference.
void copy_probe(hipStream_t s, int64_t bytes, const void *x, void *y);
// y = float(x) / x = double(y)
void to_f32(hipStream_t s, int64_t n, const double *x, float *y);
void to_f64(hipStream_t s, int64_t n, const float *x, double *y);

}  // namespace evk
