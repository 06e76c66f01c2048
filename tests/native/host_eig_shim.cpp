// C entry points over the library's host eigensolver, for CPU tests only.
#include "host_poly.hpp"

extern "C" {
int t_sym_eig(int m, double *A, double *w, double *V) { return evh::sym_eig(m, A, w, V); }
int t_tridiag_eig(int m, double *d, double *e, double *w, double *V) {
  return evh::tridiag_eig(m, d, e, w, V);
}
int t_sym_eig_sel(int m, double *A, double *w, double thr, double *V) {
  return evh::sym_eig_sel(m, A, w, thr, V);
}
void t_tridiag_eigvecs(int m, const double *d, const double *e, int nsel, const double *lam,
                       double *Z) {
  evh::tridiag_eigvecs(m, d, e, nsel, lam, Z);
}
}
