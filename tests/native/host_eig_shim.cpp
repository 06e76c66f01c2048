// C entry points over the library's host eigensolver, for CPU tests only.
#include <algorithm>
#include <vector>

#include "host_poly.hpp"

extern "C" {
int t_sym_eig(int m, double *A, double *w, double *V) { return evh::sym_eig(m, A, w, V); }
int t_tridiag_eig(int m, double *d, double *e, double *w, double *V) {
  return evh::tridiag_eig(m, d, e, w, V);
}
void t_tridiag_eigvecs(int m, const double *d, const double *e, int nsel, const double *lam,
                       double *Z) {
  evh::tridiag_eigvecs(m, d, e, nsel, lam, Z);
}
}

extern "C" {
// eigenvalues (ascending) of the thick-restart matrix of dimension k (arrowhead
// block th, s, al[0] then tridiagonal al[1..k-l-1], be[0..k-l-2]: be[0] couples
// index l to l+1) through ArrowForm and the tridiagonal QR, and the
// eigenvectors of those >= thr (k x nsel); returns nsel
int t_arrow_eig_sel(int k, int l, const double *th, const double *s, const double *al,
                    const double *be, double *w, double thr, double *V) {
  std::vector<double> d(k), e(std::max(k - 1, 1), 0.0);
  evh::ArrowForm f;
  f.reduce(l, th, s, al[0], d.data(), e.data());
  for (int r = l + 1; r < k; ++r) d[r] = al[r - l];
  for (int r = l; r + 1 < k; ++r) e[r] = be[r - l];
  const int nsel = evh::tridiag_eig_sel(k, d.data(), e.data(), w, thr, V);
  if (nsel > 0) f.back(nsel, V, k);
  return nsel;
}
}
