// Host-side polynomial work: damping, find_pol, KPM count, slicer.
#pragma once
#include <cstdint>
#include <vector>

namespace evh {

struct FilterOut {
  int deg;
  int boundary;
  double gamma, cc, dd, bar;
  double *coef;  // caller buffer of max_deg + 1
};

// kind: 0 none, 1 Lanczos sigma (eq:polPJ), 2 Jackson. g has k+1 entries.
int damping_factors(int kind, int k, double *g);
// 0: found, 1: max_deg reached (max_deg filter returned), -1: invalid.
int find_filter(const double intv[4], int damp, double tau, double tau_ext, int max_deg,
                FilterOut *out);
// g: damping factors for degree K; c, d: spectrum map.
double kpm_count(int K, const double *mom, const double *g, double c, double d, double x0,
                 double x1);
int slice(int K, const double *mom, int damp, const double intv[4], int nslices, int npts,
          double *sli);
// Count in [x0, x1] from a Gaussian quadrature of the spectral density (nvec
// probes, nodes/weights nvec x m row-major, dims[l] valid entries per row):
// n / nvec times the weight inside, each node spread by a Gaussian of standard
// deviation sigma (0: a point mass).
double quad_count(const double *nodes, const double *weights, const int *dims, int nvec, int m,
                  int64_t n, double sigma, double x0, double x1);
// Equal-count slicing of [xi, eta] on that count (npts-point grid).
int quad_slice(const double *nodes, const double *weights, const int *dims, int nvec, int m,
               int64_t n, double sigma, double xi, double eta, int nslices, int npts, double *sli);

// Symmetric eigen-decomposition of the m x m column-major A (overwritten):
// Householder tridiagonalisation, then implicit QR steps with Wilkinson
// shifts (Golub and Van Loan, Sections 8.3.1-8.3.3). w ascending; V (m x m,
// column-major, may be null for eigenvalues only).
int sym_eig(int m, double *A, double *w, double *V);
// The QR phase alone, for a matrix that is already tridiagonal: diagonal d,
// off-diagonal e (both overwritten); V as in sym_eig (identity or a prior
// transformation, m x m) or null. O(m^2) without vectors.
int tridiag_eig(int m, double *d, double *e, double *w, double *V);
// All eigenvalues (ascending, in w) of the tridiagonal (d, e), not
// overwritten, by QR, and the eigenvectors of those >= thr by inverse
// iteration (Vsel, m x nsel, in the order of w[m - nsel .. m - 1]); returns nsel.
int tridiag_eig_sel(int m, const double *d, const double *e, double *w, double thr,
                    double *Vsel);
// The projected matrix after a thick restart (Section 2.3.2, arrowhead form):
// diagonal th[0..l-1], their couplings s[0..l-1] to index l, T(l, l) = al,
// then tridiagonal from index l on. reduce() brings the (l+1) x (l+1) leading
// block to tridiagonal form by reflectors that leave index l fixed, ordered so
// that index l comes last (d: l+1 values, e: l); with T's coupling of l to
// l+1 and the rest of T this is one tridiagonal matrix with T's eigenvalues.
// back() maps rows 0..l of nvec eigenvectors of that tridiagonal (leading
// dimension ldy) to eigenvectors of T; rows l+1.. are unchanged.
struct ArrowForm {
  int l = -1;
  std::vector<double> R, betas;
  void reduce(int nl, const double *th, const double *s, double al, double *d, double *e);
  void back(int nvec, double *Y, int64_t ldy) const;
};
// Eigenvectors of the tridiagonal (d, e) for nsel eigenvalues lam (ascending)
// by inverse iteration; Z is m x nsel column-major.
void tridiag_eigvecs(int m, const double *d, const double *e, int nsel, const double *lam,
                     double *Z);
// Cholesky G = R^T R (R upper triangular); -1 if G is not positive definite.
int chol_upper(int m, const double *G, double *R);
// Inverse of an upper-triangular matrix.
void tri_inv_upper(int m, const double *R, double *Ri);
// Chebyshev-Jackson delta filter of fixed degree k centred at gamma:
// coef_j = g_j mu_j / sum_i g_i mu_i T_i(gamma) (eq:Cheb0, eq:mu with Jackson damping).
void delta_filter(int k, double gamma, int damp, double *coef);

}  // namespace evh
