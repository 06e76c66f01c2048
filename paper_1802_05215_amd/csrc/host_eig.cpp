// Dense symmetric eigensolver for the small projected matrices of the
// Lanczos process (T_m of eq:Tm, tridiagonal, or arrowhead plus tridiagonal
// after a thick restart). Householder reduction to tridiagonal form, then
// implicit symmetric QR steps with the Wilkinson shift and bulge chasing by
// Givens rotations (Golub and Van Loan, Matrix Computations, 8.3.1-8.3.3).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "host_poly.hpp"

namespace evh {

namespace {

// Householder tridiagonalisation of the symmetric m x m A (column-major,
// overwritten): reflector k = I - beta_k v_k v_k^T zeroes column k below the
// subdiagonal (v_k on rows k+1..m-1). d, e receive the tridiagonal. When R is
// given, v_k goes to column k of R and beta_k to betas[k]; when V is given it
// accumulates V <- V H_k.
void householder(int m, double *A, double *d, double *e, double *R, double *betas, double *V) {
  auto a = [&](int i, int j) -> double & { return A[i + (size_t)j * m]; };
  std::vector<double> v(m), p(m), q(m);
  for (int k = 0; k + 2 < m; ++k) {
    if (betas) betas[k] = 0.0;
    const int len = m - k - 1;
    double sig = 0.0;
    for (int i = 0; i < len; ++i) sig += a(k + 1 + i, k) * a(k + 1 + i, k);
    if (sig == 0.0) continue;
    const double x0 = a(k + 1, k);
    const double alpha = x0 >= 0 ? -std::sqrt(sig) : std::sqrt(sig);
    for (int i = 0; i < len; ++i) v[i] = a(k + 1 + i, k);
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < len; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta * A22 v, column by column (A is column-major)
    std::fill(p.begin(), p.begin() + len, 0.0);
    for (int j = 0; j < len; ++j) {
      const double vj = v[j];
      const double *col = &a(k + 1, k + 1 + j);
      for (int i = 0; i < len; ++i) p[i] += col[i] * vj;
    }
    double pv = 0.0;
    for (int i = 0; i < len; ++i) {
      p[i] *= beta;
      pv += p[i] * v[i];
    }
    const double kk = 0.5 * beta * pv;
    for (int i = 0; i < len; ++i) q[i] = p[i] - kk * v[i];
    // A22 <- A22 - v q^T - q v^T
    for (int j = 0; j < len; ++j) {
      const double vj = v[j], qj = q[j];
      double *col = &a(k + 1, k + 1 + j);
      for (int i = 0; i < len; ++i) col[i] -= v[i] * qj + q[i] * vj;
    }
    a(k + 1, k) = alpha;
    a(k, k + 1) = alpha;
    for (int i = 1; i < len; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
    if (R) {
      for (int i = 0; i < len; ++i) R[(k + 1 + i) + (size_t)k * m] = v[i];
      betas[k] = beta;
    }
    if (V) {  // V <- V (I - beta v v^T) on columns k+1..m-1
      for (int r = 0; r < m; ++r) {
        double t = 0.0;
        for (int i = 0; i < len; ++i) t += V[r + (size_t)(k + 1 + i) * m] * v[i];
        t *= beta;
        for (int i = 0; i < len; ++i) V[r + (size_t)(k + 1 + i) * m] -= t * v[i];
      }
    }
  }
  for (int i = 0; i < m; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < m; ++i) e[i] = a(i + 1, i);
}

// z <- H_0 H_1 ... H_{m-3} z for nvec columns of Z (leading dimension ldz,
// rows 0..m-1): the reflectors from the last to the first.
void apply_reflectors(int m, const double *R, const double *betas, int nvec, double *Z,
                      int64_t ldz) {
  for (int k = m - 3; k >= 0; --k) {
    if (betas[k] == 0.0) continue;
    const double *vk = R + (size_t)k * m;
    for (int c = 0; c < nvec; ++c) {
      double *z = Z + (size_t)c * ldz;
      double t = 0.0;
      for (int i = k + 1; i < m; ++i) t += vk[i] * z[i];
      t *= betas[k];
      for (int i = k + 1; i < m; ++i) z[i] -= t * vk[i];
    }
  }
}

}  // namespace

int sym_eig(int m, double *A, double *w, double *V) {
  if (m <= 0) return -1;
  if (m == 1) {
    w[0] = A[0];
    if (V) V[0] = 1.0;
    return 0;
  }
  if (V) {
    std::fill(V, V + (size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[i + (size_t)i * m] = 1.0;
  }
  std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
  householder(m, A, d.data(), e.data(), nullptr, nullptr, V);
  return tridiag_eig(m, d.data(), e.data(), w, V);
}

// Implicit symmetric QR on the tridiagonal (d, e); V (m x m) accumulates the
// rotations when not null (it must hold the transformation so far).
int tridiag_eig(int m, double *d, double *e, double *w, double *V) {
  if (m <= 0) return -1;
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  for (long iter = 0; hi > 0 && iter < 60L * m + 100; ++iter) {
    // deflate converged trailing entries
    while (hi > 0 && std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi])) * 0.5) {
      e[hi - 1] = 0.0;
      --hi;
    }
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo])) * 0.5)
      --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    // Wilkinson shift from the trailing 2 x 2 block
    const double del = 0.5 * (d[hi - 1] - d[hi]);
    const double e2 = e[hi - 1] * e[hi - 1];
    const double sgn = del >= 0 ? 1.0 : -1.0;
    const double mu = d[hi] - e2 / (del + sgn * std::sqrt(del * del + e2));
    double x = d[lo] - mu, z = e[lo];
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      // |x|, |z| are of the order of ||T||: no scaling needed against overflow
      const double r = std::sqrt(x * x + z * z);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : -z / r;
      if (k > lo) e[k - 1] = r;
      // rotate the 2 x 2 block (k, k+1): G^T B G with G = [[c, s], [-s, c]]
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = dk * c * c - 2.0 * ek * c * s + dk1 * s * s;
      d[k + 1] = dk * s * s + 2.0 * ek * c * s + dk1 * c * c;
      e[k] = (dk - dk1) * c * s + ek * (c * c - s * s);
      if (k + 1 < hi) {
        bulge = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      if (V) {
        double *vk = V + (size_t)k * m, *vk1 = V + (size_t)(k + 1) * m;
        for (int r2 = 0; r2 < m; ++r2) {
          const double t0 = vk[r2], t1 = vk1[r2];
          vk[r2] = c * t0 - s * t1;
          vk1[r2] = s * t0 + c * t1;
        }
      }
      x = e[k];
      z = bulge;
    }
  }
  // --- sort ascending
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return d[i] < d[j]; });
  for (int i = 0; i < m; ++i) w[i] = d[idx[i]];
  if (V) {
    std::vector<double> tmp((size_t)m * m);
    for (int j = 0; j < m; ++j)
      std::copy(V + (size_t)idx[j] * m, V + (size_t)idx[j] * m + m, tmp.begin() + (size_t)j * m);
    std::copy(tmp.begin(), tmp.end(), V);
  }
  return 0;
}

// G = R^T R with R upper triangular (column-major m x m, written into R).
// Returns -1 when G is not numerically positive definite.
int chol_upper(int m, const double *G, double *R) {
  for (int i = 0; i < m * m; ++i) R[i] = 0.0;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = G[i + (size_t)j * m];
      for (int k = 0; k < i; ++k) s -= R[k + (size_t)i * m] * R[k + (size_t)j * m];
      if (i == j) {
        if (!(s > 0.0)) return -1;
        R[j + (size_t)j * m] = std::sqrt(s);
      } else {
        R[i + (size_t)j * m] = s / R[i + (size_t)i * m];
      }
    }
  }
  return 0;
}

// Inverse of an upper-triangular R (column-major), by back substitution.
void tri_inv_upper(int m, const double *R, double *Ri) {
  for (int i = 0; i < m * m; ++i) Ri[i] = 0.0;
  for (int j = 0; j < m; ++j) {
    Ri[j + (size_t)j * m] = 1.0 / R[j + (size_t)j * m];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i + (size_t)k * m] * Ri[k + (size_t)j * m];
      Ri[i + (size_t)j * m] = -s / R[i + (size_t)i * m];
    }
  }
}

// Eigenvectors of the symmetric tridiagonal (d, e) for the eigenvalues lam
// (ascending, nsel of them) by inverse iteration: T - x I is factored by
// Gaussian elimination with partial pivoting (U has two superdiagonals), three
// solves from a fixed start vector, each result orthogonalised (modified
// Gram-Schmidt) against the vectors already computed for eigenvalues of the
// same cluster (gaps below 1e-3 ||T||), whose shifts are pushed apart by
// 10 eps |x| so that the factorisations differ. Z is m x nsel column-major.
void tridiag_eigvecs(int m, const double *d, const double *e, int nsel, const double *lam,
                     double *Z) {
  const double eps = 2.220446049250313e-16;
  double tnorm = 0.0;
  for (int i = 0; i < m; ++i) {
    double r = std::fabs(d[i]);
    if (i > 0) r += std::fabs(e[i - 1]);
    if (i + 1 < m) r += std::fabs(e[i]);
    tnorm = std::max(tnorm, r);
  }
  const double tiny = std::max(eps * tnorm, 1e-300);
  const double clus = 1e-3 * tnorm;
  std::vector<double> a(m), up(m), up2(m), lo(m), y(m);
  std::vector<char> swp(m);
  int cstart = 0;
  double xprev = 0.0;
  for (int j = 0; j < nsel; ++j) {
    double x = lam[j];
    if (j > 0 && lam[j] - lam[j - 1] < clus) {
      const double push = 10.0 * eps * std::fabs(x) + tiny;
      if (x - xprev < push) x = xprev + push;
    } else {
      cstart = j;
    }
    xprev = x;
    // factor T - x I
    for (int i = 0; i < m; ++i) {
      a[i] = d[i] - x;
      up[i] = i + 1 < m ? e[i] : 0.0;
      up2[i] = 0.0;
    }
    for (int i = 0; i + 1 < m; ++i) {
      const double sub = e[i];
      if (std::fabs(a[i]) >= std::fabs(sub)) {
        if (a[i] == 0.0) a[i] = tiny;
        lo[i] = sub / a[i];
        swp[i] = 0;
        a[i + 1] -= lo[i] * up[i];
      } else {
        // rows i and i+1 exchange
        const double f = a[i] / sub;
        lo[i] = f;
        swp[i] = 1;
        a[i] = sub;
        const double t = a[i + 1];
        a[i + 1] = up[i] - f * t;
        if (i + 2 < m) {
          up2[i] = up[i + 1];
          up[i + 1] = -f * up[i + 1];
        }
        up[i] = t;
      }
    }
    if (a[m - 1] == 0.0) a[m - 1] = tiny;
    for (int i = 0; i < m; ++i)
      if (std::fabs(a[i]) < tiny) a[i] = a[i] < 0 ? -tiny : tiny;
    // start vector: a fixed, non-degenerate pattern
    for (int i = 0; i < m; ++i) y[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3 * j);
    double *z = Z + (size_t)j * m;
    for (int it = 0; it < 3; ++it) {
      // forward: L with the row exchanges
      for (int i = 0; i + 1 < m; ++i) {
        if (swp[i]) std::swap(y[i], y[i + 1]);
        y[i + 1] -= lo[i] * y[i];
      }
      // back: U with two superdiagonals
      y[m - 1] /= a[m - 1];
      if (m > 1) y[m - 2] = (y[m - 2] - up[m - 2] * y[m - 1]) / a[m - 2];
      for (int i = m - 3; i >= 0; --i)
        y[i] = (y[i] - up[i] * y[i + 1] - up2[i] * y[i + 2]) / a[i];
      // orthogonalise against the cluster's earlier vectors, then normalise
      for (int k = cstart; k < j; ++k) {
        const double *zk = Z + (size_t)k * m;
        double h = 0.0;
        for (int i = 0; i < m; ++i) h += zk[i] * y[i];
        for (int i = 0; i < m; ++i) y[i] -= h * zk[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < m; ++i) nrm += y[i] * y[i];
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0)) {
        for (int i = 0; i < m; ++i) y[i] = (i == j % m) ? 1.0 : 0.0;
        nrm = 1.0;
      }
      for (int i = 0; i < m; ++i) y[i] /= nrm;
    }
    std::copy(y.begin(), y.end(), z);
  }
}

int tridiag_eig_sel(int m, const double *d, const double *e, double *w, double thr,
                    double *Vsel) {
  if (m <= 0) return -1;
  {
    std::vector<double> d2(d, d + m), e2(std::max(m - 1, 1), 0.0);
    std::copy(e, e + (m - 1), e2.begin());
    tridiag_eig(m, d2.data(), e2.data(), w, nullptr);
  }
  int first = m;
  while (first > 0 && w[first - 1] >= thr) --first;
  const int nsel = m - first;
  if (nsel > 0) tridiag_eigvecs(m, d, e, nsel, w + first, Vsel);
  return nsel;
}

void ArrowForm::reduce(int nl, const double *th, const double *s, double al, double *d,
                       double *e) {
  l = nl;
  const int L = l + 1;
  // the block in the order [l, 0, 1, ..., l-1]: index l first, so that the
  // reflectors (which act on rows 1..L-1) leave it fixed
  std::vector<double> M((size_t)L * L, 0.0);
  M[0] = al;
  for (int j = 0; j < l; ++j) {
    M[(j + 1)] = s[j];
    M[(size_t)(j + 1) * L] = s[j];
    M[(j + 1) + (size_t)(j + 1) * L] = th[j];
  }
  R.assign((size_t)L * L, 0.0);
  betas.assign(std::max(L, 1), 0.0);
  std::vector<double> dm(L), em(std::max(L - 1, 1), 0.0);
  if (L == 1) {
    dm[0] = al;
  } else {
    householder(L, M.data(), dm.data(), em.data(), R.data(), betas.data(), nullptr);
  }
  // reversed, so that index l comes last and couples to index l+1 of T
  for (int p = 0; p < L; ++p) d[p] = dm[L - 1 - p];
  for (int p = 0; p + 1 < L; ++p) e[p] = em[L - 2 - p];
}

void ArrowForm::back(int nvec, double *Y, int64_t ldy) const {
  const int L = l + 1;
  std::vector<double> u((size_t)L * nvec);
  for (int c = 0; c < nvec; ++c)
    for (int p = 0; p < L; ++p) u[(size_t)c * L + (L - 1 - p)] = Y[p + (size_t)c * ldy];
  if (L > 2) apply_reflectors(L, R.data(), betas.data(), nvec, u.data(), L);
  for (int c = 0; c < nvec; ++c) {
    double *y = Y + (size_t)c * ldy;
    const double *uc = u.data() + (size_t)c * L;
    y[l] = uc[0];
    for (int j = 0; j < l; ++j) y[j] = uc[j + 1];
  }
}

}  // namespace evh
