/*
 * ORACLE -- test infrastructure only (see evsl_oracle.h).
 *
 * Plain FP64 CPU code written from the EVSL paper, arXiv:1802.05215. Each
 * function names the passage it follows. Loops are written out; the only
 * optional speed-up is OpenMP on row loops (static schedule), which does not
 * change any result because every row is computed the same way by one thread.
 * Reductions (dot products, norms) run sequentially in index order.
 *
 * Parity status of each function (what pins it) is listed in the test-suite;
 * no function here is "parity unpinned".
 */
#include "evsl_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).
 * Output number i+1 of the generator whose state starts at `seed`. */
uint64_t or_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double or_uniform01(uint64_t seed, uint64_t i) {
  return (double)(or_splitmix64(seed, i) >> 11) * (1.0 / 9007199254740992.0);
}

void or_lanczos_start(uint64_t seed, int64_t n, int64_t restart, double *x) {
  for (int64_t i = 0; i < n; ++i)
    x[i] = 2.0 * or_uniform01(seed, (uint64_t)restart * (uint64_t)n + (uint64_t)i) - 1.0;
}

void or_rademacher(uint64_t seed, int64_t n, int nvec, double *V) {
  for (int64_t i = 0; i < n; ++i)
    for (int l = 0; l < nvec; ++l) {
      uint64_t b = or_splitmix64(seed, (uint64_t)l * (uint64_t)n + (uint64_t)i) >> 63;
      V[i * nvec + l] = b ? -1.0 : 1.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Small dense helpers (sequential). */
static double dot(int64_t n, const double *x, const double *y) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
  return s;
}

static double nrm2(int64_t n, const double *x) { return sqrt(dot(n, x, x)); }

/* ------------------------------------------------------------------------ */
/* CSR product y = A x (Section 3.1: matrices are stored in CSR). */
void or_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
             const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * x[ci[p]];
    y[i] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* Damping multipliers for a degree-k expansion.
 * SIGMA: Lanczos sigma factors of eq:polPJ, sigma_0 = 1,
 *        sigma_j = sin(j theta_k)/(j theta_k), theta_k = pi/(k+1).
 * JACKSON: the paper names damping approaches without formulas; the Jackson
 *        kernel is taken from Weisse, Wellein, Alvermann and Fehske (2006) with
 *        N = k+1 moments: g_j = [(N-j+1) cos(pi j/(N+1)) + sin(pi j/(N+1)) cot(pi/(N+1))]/(N+1). */
int or_damping(int kind, int k, double *g) {
  if (k < 0) return -1;
  if (kind == OR_DAMP_NONE) {
    for (int j = 0; j <= k; ++j) g[j] = 1.0;
    return 0;
  }
  if (kind == OR_DAMP_SIGMA) {
    double th = M_PI / (double)(k + 1);
    g[0] = 1.0;
    for (int j = 1; j <= k; ++j) g[j] = sin(j * th) / (j * th);
    return 0;
  }
  if (kind == OR_DAMP_JACKSON) {
    double N = (double)(k + 1);
    double al = M_PI / (N + 1.0);
    for (int j = 0; j <= k; ++j)
      g[j] = ((N - j + 1.0) * cos(j * al) + sin(j * al) * cos(al) / sin(al)) / (N + 1.0);
    return 0;
  }
  return -1;
}

/* T_j(t) for any real t: cos(j acos t) inside [-1,1], cosh form outside. */
static double cheb_T(int j, double t) {
  if (t >= -1.0 && t <= 1.0) return cos(j * acos(t));
  double v = cosh(j * acosh(fabs(t)));
  return (t < 0 && (j & 1)) ? -v : v;
}

double or_cheb_series(int k, const double *c, double t) {
  double s = 0.0;
  for (int j = 0; j <= k; ++j) s += c[j] * cheb_T(j, t);
  return s;
}

/* ------------------------------------------------------------------------ */
/* find_pol: Section 2.2.1.
 * rho(t) = sum_j g_j mu_j T_j(t) / sum_j g_j mu_j T_j(gamma) (eq:Cheb0 with the
 * damped mu of eq:polPJ), mu_0 = 1/2, mu_j = cos(j acos gamma) (eq:mu).
 * For each degree k = 2, 3, ... the centre gamma = cos(theta) balances the
 * filter, rho(a) = rho(b) (eq:Neq), by Newton's method in theta (bracketed, with
 * a bisection fallback); the first k whose end values do not exceed tau is
 * returned. The balance equation is written without the common positive
 * denominator and the j = 0 term, which cancel:
 *   f(theta) = sum_{j>=1} g_j cos(j theta) (T_j(a) - T_j(b)).
 * Boundary slices (an end at or beyond the spectrum bound) use gamma = -1 or
 * +1 and compare the inner end value with tau_ext. */
static void pol_coefs(int k, const double *g, double theta, double *coef) {
  double den = 0.5 * g[0];
  for (int j = 1; j <= k; ++j) den += g[j] * cos(j * theta) * cos(j * theta);
  coef[0] = 0.5 * g[0] / den;
  for (int j = 1; j <= k; ++j) coef[j] = g[j] * cos(j * theta) / den;
}

static double balance_f(int k, const double *g, const double *dT, double theta, double *fp) {
  double f = 0.0, d = 0.0;
  for (int j = 1; j <= k; ++j) {
    f += g[j] * cos(j * theta) * dT[j];
    d -= j * g[j] * sin(j * theta) * dT[j];
  }
  if (fp) *fp = d;
  return f;
}

int or_find_pol(const double intv[4], int damping, double tau, double tau_ext, int max_deg,
                int *deg, double *gamma, double *bar, double *cc, double *dd, double *coef,
                int *boundary) {
  double lmin = intv[2], lmax = intv[3];
  if (!(lmax > lmin) || !(intv[1] > intv[0]) || max_deg < 2) return -1;
  double c = 0.5 * (lmax + lmin), d = 0.5 * (lmax - lmin);
  double a = (intv[0] - c) / d, b = (intv[1] - c) / d;
  *cc = c;
  *dd = d;
  int bnd = 0;
  if (a <= -1.0) bnd = -1;
  if (b >= 1.0) bnd = (bnd == -1) ? 2 : 1;
  if (bnd == 2) return -1; /* interval covers the whole spectrum */
  if (boundary) *boundary = bnd;
  double *g = (double *)malloc(sizeof(double) * (max_deg + 1));
  double *dT = (double *)malloc(sizeof(double) * (max_deg + 1));
  int status = 1;
  int k;
  double theta = 0.0;
  for (k = 2; k <= max_deg; ++k) {
    or_damping(damping, k, g);
    if (bnd != 0) {
      theta = (bnd == -1) ? M_PI : 0.0;
      pol_coefs(k, g, theta, coef);
      double inner = (bnd == -1) ? b : a;
      *bar = or_cheb_series(k, coef, inner);
      if (*bar <= tau_ext) { status = 0; break; }
      continue;
    }
    for (int j = 0; j <= k; ++j) dT[j] = cheb_T(j, a) - cheb_T(j, b);
    double lo = acos(b), hi = acos(a); /* theta range, lo < hi */
    double flo = balance_f(k, g, dT, lo, NULL), fhi = balance_f(k, g, dT, hi, NULL);
    if (flo == 0.0) theta = lo;
    else if (fhi == 0.0) theta = hi;
    else if ((flo < 0) == (fhi < 0)) continue; /* not balanceable at this degree */
    else {
      theta = 0.5 * (lo + hi);
      for (int it = 0; it < 200; ++it) {
        double fp;
        double f = balance_f(k, g, dT, theta, &fp);
        if (f == 0.0) break;
        if ((f < 0) == (flo < 0)) { lo = theta; flo = f; } else { hi = theta; }
        double tn = (fp != 0.0) ? theta - f / fp : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - theta) <= 1e-15 * (1.0 + fabs(theta))) { theta = tn; break; }
        theta = tn;
      }
    }
    pol_coefs(k, g, theta, coef);
    *bar = or_cheb_series(k, coef, a);
    if (*bar <= tau) { status = 0; break; }
  }
  if (k > max_deg) {
    /* max degree reached: return the max-degree filter with the last centre */
    k = max_deg;
    or_damping(damping, k, g);
    pol_coefs(k, g, theta, coef);
    *bar = or_cheb_series(k, coef, (bnd == -1) ? b : a);
  }
  *deg = k;
  *gamma = cos(theta);
  free(g);
  free(dT);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Filter application Y = sum_j coef_j T_j(A-hat) V, A-hat = (A - cc I)/dd
 * (eq:mapping, eq:Cheb0): W_0 = V, W_1 = A-hat V, W_{j+1} = 2 A-hat W_j - W_{j-1}. */
void or_filter_apply(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                     double cc, double dd, int k, const double *coef, int nvec,
                     const double *V, double *Y) {
  size_t sz = (size_t)n * nvec;
  double *w0 = (double *)malloc(sizeof(double) * sz);
  double *w1 = (double *)malloc(sizeof(double) * sz);
  double *w2 = (double *)malloc(sizeof(double) * sz);
  memcpy(w0, V, sizeof(double) * sz);
  for (size_t e = 0; e < sz; ++e) Y[e] = coef[0] * w0[e];
  if (k >= 1) {
    /* W_1 = (A W_0 - cc W_0)/dd */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int l = 0; l < nvec; ++l) {
        double s = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * w0[(size_t)ci[p] * nvec + l];
        w1[i * nvec + l] = (s - cc * w0[i * nvec + l]) / dd;
        Y[i * nvec + l] += coef[1] * w1[i * nvec + l];
      }
  }
  for (int j = 1; j < k; ++j) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int l = 0; l < nvec; ++l) {
        double s = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * w1[(size_t)ci[p] * nvec + l];
        w2[i * nvec + l] = 2.0 * (s - cc * w1[i * nvec + l]) / dd - w0[i * nvec + l];
        Y[i * nvec + l] += coef[j + 1] * w2[i * nvec + l];
      }
    double *t = w0;
    w0 = w1;
    w1 = w2;
    w2 = t;
  }
  free(w0);
  free(w1);
  free(w2);
}

/* ------------------------------------------------------------------------ */
/* KPM (Section 2.1; the paper defers the formulas to Lin, Saad and Yang 2016):
 * zeta_k = (1/nvec) sum_l v_l^T T_k(A-hat) v_l estimates trace(T_k(A-hat)). */
void or_kpm_moments(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                    double lmin, double lmax, int K, int nvec, const double *V, double *mom) {
  double c = 0.5 * (lmax + lmin), d = 0.5 * (lmax - lmin);
  size_t sz = (size_t)n * nvec;
  double *w0 = (double *)malloc(sizeof(double) * sz);
  double *w1 = (double *)malloc(sizeof(double) * sz);
  double *w2 = (double *)malloc(sizeof(double) * sz);
  memcpy(w0, V, sizeof(double) * sz);
  for (int k = 0; k <= K; ++k) {
    if (k == 1) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i)
        for (int l = 0; l < nvec; ++l) {
          double s = 0.0;
          for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * w0[(size_t)ci[p] * nvec + l];
          w1[i * nvec + l] = (s - c * w0[i * nvec + l]) / d;
        }
    } else if (k >= 2) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i)
        for (int l = 0; l < nvec; ++l) {
          double s = 0.0;
          for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * w1[(size_t)ci[p] * nvec + l];
          w2[i * nvec + l] = 2.0 * (s - c * w1[i * nvec + l]) / d - w0[i * nvec + l];
        }
      double *t = w0;
      w0 = w1;
      w1 = w2;
      w2 = t;
    }
    const double *wk = (k == 0) ? w0 : w1; /* T_k(A-hat) V */
    double acc = 0.0;
    for (size_t e = 0; e < sz; ++e) acc += V[e] * wk[e];
    mom[k] = acc / nvec;
  }
  free(w0);
  free(w1);
  free(w2);
}

/* Count in [x0, x1] from the damped KPM DOS (eq:DOS0 integrated):
 *   phi(t) ~ sum_k g_k (2 - delta_k0) (zeta_k / n) T_k(t) / (pi sqrt(1 - t^2)),
 *   n * int T_k / (pi sqrt(1-t^2)) over [x0, x1] = (sin k th0 - sin k th1)/(k pi),
 * th = acos(mapped x); (th0 - th1)/pi for k = 0. */
double or_kpm_count(int K, const double *mom, int damping, double lmin, double lmax,
                    double x0, double x1) {
  double c = 0.5 * (lmax + lmin), d = 0.5 * (lmax - lmin);
  double t0 = (x0 - c) / d, t1 = (x1 - c) / d;
  if (t0 < -1.0) t0 = -1.0;
  if (t0 > 1.0) t0 = 1.0;
  if (t1 < -1.0) t1 = -1.0;
  if (t1 > 1.0) t1 = 1.0;
  double th0 = acos(t0), th1 = acos(t1);
  double *g = (double *)malloc(sizeof(double) * (K + 1));
  or_damping(damping, K, g);
  double s = g[0] * mom[0] * (th0 - th1) / M_PI;
  for (int k = 1; k <= K; ++k)
    s += 2.0 * g[k] * mom[k] * (sin(k * th0) - sin(k * th1)) / (k * M_PI);
  free(g);
  return s;
}

/* Slicer (eq:slice-ti): an npts-point uniform grid x_0 = xi < ... < x_{N-1} =
 * eta; C_j = estimated count on [xi, x_j], made non-decreasing; t_i is the
 * first grid point after t_{i-1} with C_j >= i C_{N-1} / n_s. */
int or_slicer(int K, const double *mom, int damping, const double intv[4], int nslices,
              int npts, double *sli) {
  if (nslices < 1 || npts < nslices + 1 || !(intv[1] > intv[0])) return -1;
  double xi = intv[0], eta = intv[1];
  double *C = (double *)malloc(sizeof(double) * npts);
  double run = -INFINITY;
  for (int j = 0; j < npts; ++j) {
    double x = xi + (eta - xi) * (double)j / (double)(npts - 1);
    double v = or_kpm_count(K, mom, damping, intv[2], intv[3], xi, x);
    run = v > run ? v : run;
    C[j] = run;
  }
  double total = C[npts - 1];
  sli[0] = xi;
  sli[nslices] = eta;
  int prev = 0, rc = 0;
  for (int i = 1; i < nslices; ++i) {
    double target = total * (double)i / (double)nslices;
    int j = prev + 1;
    while (j < npts - 1 && C[j] < target) ++j;
    if (j >= npts - 1) { rc = -1; break; }
    sli[i] = xi + (eta - xi) * (double)j / (double)(npts - 1);
    prev = j;
  }
  free(C);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi (Golub and Van Loan, Matrix Computations, Section 8.5): sweep
 * over all (p, q), zero a_pq with a rotation from the 2 x 2 symmetric Schur
 * decomposition, until the off-diagonal mass is negligible. */
int or_jacobi_eig(int m, double *A, double *w, double *V) {
  for (int i = 0; i < m * m; ++i) V[i] = 0.0;
  for (int i = 0; i < m; ++i) V[i + (size_t)i * m] = 1.0;
  double fro = 0.0;
  for (int i = 0; i < m * m; ++i) fro += A[i] * A[i];
  /* an off-diagonal entry below skip is treated as zero */
  double skip = 1e-18 * sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double apq = A[p + (size_t)q * m];
        if (fabs(apq) <= skip) continue;
        rotated = 1;
        double app = A[p + (size_t)p * m], aqq = A[q + (size_t)q * m];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        /* A <- J^T A J: rows/columns p and q rotate; the 2 x 2 block becomes
         * diag(a_pp - t a_pq, a_qq + t a_pq) with a_pq annihilated */
        for (int k = 0; k < m; ++k) {
          if (k == p || k == q) continue;
          double akp = A[k + (size_t)p * m], akq = A[k + (size_t)q * m];
          double nkp = c * akp - s * akq, nkq = s * akp + c * akq;
          A[k + (size_t)p * m] = nkp;
          A[p + (size_t)k * m] = nkp;
          A[k + (size_t)q * m] = nkq;
          A[q + (size_t)k * m] = nkq;
        }
        A[p + (size_t)p * m] = app - t * apq;
        A[q + (size_t)q * m] = aqq + t * apq;
        A[p + (size_t)q * m] = 0.0;
        A[q + (size_t)p * m] = 0.0;
        for (int k = 0; k < m; ++k) { /* V <- V J */
          double vkp = V[k + (size_t)p * m], vkq = V[k + (size_t)q * m];
          V[k + (size_t)p * m] = c * vkp - s * vkq;
          V[k + (size_t)q * m] = s * vkp + c * vkq;
        }
      }
    if (!rotated) break;
  }
  for (int i = 0; i < m; ++i) w[i] = A[i + (size_t)i * m];
  /* selection sort, ascending, moving the vectors along */
  for (int i = 0; i < m - 1; ++i) {
    int mi = i;
    for (int j = i + 1; j < m; ++j)
      if (w[j] < w[mi]) mi = j;
    if (mi != i) {
      double t = w[i];
      w[i] = w[mi];
      w[mi] = t;
      for (int k = 0; k < m; ++k) {
        double v = V[k + (size_t)i * m];
        V[k + (size_t)i * m] = V[k + (size_t)mi * m];
        V[k + (size_t)mi * m] = v;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Classical Gram-Schmidt of z against the columns of [B1, B2] (column-major,
 * n rows each): all coefficients come from the same z, then are subtracted.
 * The pass is repeated once when the norm drops below 1/sqrt(2) of its value
 * before the pass (DGKS criterion, Section 2.3). */
static void cgs_dgks(int64_t n, double *z, const double *B1, int n1, const double *B2, int n2,
                     double *h) {
  for (int pass = 0; pass < 2; ++pass) {
    double before = nrm2(n, z);
    for (int j = 0; j < n1; ++j) h[j] = dot(n, B1 + (size_t)j * n, z);
    for (int j = 0; j < n2; ++j) h[n1 + j] = dot(n, B2 + (size_t)j * n, z);
    for (int j = 0; j < n1 + n2; ++j) {
      const double *bj = (j < n1) ? B1 + (size_t)j * n : B2 + (size_t)(j - n1) * n;
      for (int64_t i = 0; i < n; ++i) z[i] -= h[j] * bj[i];
    }
    double after = nrm2(n, z);
    if (after >= before / sqrt(2.0)) break;
  }
}

/* Spectrum bounds (Section 2.2.1: a few Lanczos steps estimate lambda_min and
 * lambda_max; LanBounds in Section 3.1). Widened by |beta_{m+1} y_{m,j}|, the
 * residual norm of the extreme Ritz pairs. */
int or_lanczos_bounds(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                      int nsteps, uint64_t seed, double *lmin, double *lmax) {
  int m = nsteps < n ? nsteps : (int)n;
  if (m < 1) return -1;
  double *Q = (double *)calloc((size_t)n * (m + 1), sizeof(double));
  double *T = (double *)calloc((size_t)m * m, sizeof(double));
  double *z = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (m + 1));
  or_lanczos_start(seed, n, 0, Q);
  double nq = nrm2(n, Q);
  for (int64_t i = 0; i < n; ++i) Q[i] /= nq;
  double beta = 0.0, scale = 0.0;
  int dim = m;
  for (int i = 0; i < m; ++i) {
    double *qi = Q + (size_t)i * n;
    or_spmv(n, rp, ci, va, qi, z);
    double alpha = dot(n, qi, z);
    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * qi[r] + (i > 0 ? beta * qi[r - n] : 0.0);
    cgs_dgks(n, z, Q, i + 1, NULL, 0, h);
    T[i + (size_t)i * m] = alpha;
    scale = fmax(scale, fabs(alpha) + beta);
    beta = nrm2(n, z);
    if (beta <= 1e-12 * scale) { dim = i + 1; beta = 0.0; break; }
    for (int64_t r = 0; r < n; ++r) Q[(size_t)(i + 1) * n + r] = z[r] / beta;
    if (i + 1 < m) {
      T[i + (size_t)(i + 1) * m] = beta;
      T[(i + 1) + (size_t)i * m] = beta;
    }
  }
  double *Tm = (double *)malloc(sizeof(double) * dim * dim);
  for (int j = 0; j < dim; ++j)
    for (int i = 0; i < dim; ++i) Tm[i + (size_t)j * dim] = T[i + (size_t)j * m];
  double *w = (double *)malloc(sizeof(double) * dim);
  double *Y = (double *)malloc(sizeof(double) * dim * dim);
  or_jacobi_eig(dim, Tm, w, Y);
  *lmin = w[0] - fabs(beta * Y[(dim - 1) + 0]);
  *lmax = w[dim - 1] + fabs(beta * Y[(dim - 1) + (size_t)(dim - 1) * dim]);
  free(Q); free(T); free(z); free(h); free(Tm); free(w); free(Y);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Filtered thick-restart Lanczos with locking: Algorithm alg:FiltLanTR
 * (Section 2.5), Lanczos step eq:3term with full reorthogonalisation by
 * classical Gram-Schmidt with the DGKS test (Section 2.3), Ritz pairs of T_m
 * (eq:Tm). Readings of the points the paper leaves open:
 *  - candidates are Ritz values >= bar, the filter's value at the slice ends;
 *  - the special TR step couples q_{l+1} to the l thick-restart Ritz vectors
 *    through s_j = beta_{m+1} y_{m,j} (arrowhead T, as in Wu and Simon 2000);
 *  - full reorthogonalisation runs against the locked vectors and the basis;
 *  - the early-restart sums carry over from one cycle to the next (the
 *    algorithm sets t_old = t_new at each test and initialises neither per
 *    cycle);
 *  - a restart that accepts no candidate (none with a Rayleigh quotient in the
 *    slice) starts the next cycle from a fresh random vector orthogonalised
 *    against the locked set (the extra restart), and two such restarts in a
 *    row end the run;
 *  - at most m - max(Ncycle, 10) Ritz vectors are kept for the thick restart. */
static void fresh_vector(int64_t n, uint64_t seed, int idx, double *z, const double *B1, int n1,
                         const double *B2, int n2, double *h, double *nrm) {
  or_lanczos_start(seed, n, idx, z);
  double n0 = nrm2(n, z);
  cgs_dgks(n, z, B1, n1, B2, n2, h);
  cgs_dgks(n, z, B1, n1, B2, n2, h);
  double nz = nrm2(n, z);
  *nrm = nz;
  if (nz > 1e-10 * n0)
    for (int64_t r = 0; r < n; ++r) z[r] /= nz;
  else
    *nrm = 0.0;
}

int or_filtered_lanczos(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                        const double intv[4], int deg, const double *coef, double bar,
                        const or_lan_opts *opt, double *lam, double *res, double *Y,
                        or_lan_stats *st) {
  memset(st, 0, sizeof(*st));
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  /* a slice that reaches a bound of the spectrum owns every eigenvalue
   * beyond it: the bound is an estimate, within rounding of the extreme
   * eigenvalue when the bounding Lanczos run has converged */
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  double normA = fabs(lmin) > fabs(lmax) ? fabs(lmin) : fabs(lmax);
  double cc = 0.5 * (lmax + lmin), dd = 0.5 * (lmax - lmin);
  int m = opt->m;
  if (m > n - 1) m = (int)(n - 1);
  if (m < 2 || deg < 1 || opt->ncycle < 1) return -1;
  double *Q = (double *)calloc((size_t)n * (m + 1), sizeof(double));
  double *TR = (double *)malloc(sizeof(double) * (size_t)n * m);
  double *T = (double *)calloc((size_t)(m + 1) * (m + 1), sizeof(double));
  double *Tw = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *w = (double *)malloc(sizeof(double) * m);
  double *Yv = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *z = (double *)malloc(sizeof(double) * n);
  double *u = (double *)malloc(sizeof(double) * n);
  double *au = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (opt->nev_cap + m + 2));
  double *thTR = (double *)malloc(sizeof(double) * m);
  double *sTR = (double *)malloc(sizeof(double) * m);
  const int M1 = m + 1;
#define TT(i, j) T[(i) + (size_t)(j) * M1]
  int nlock = 0, l = 0, its = 0, nmv = 0, nrand = 0, nocand = 0, nrestart = 0;
  int status = 0;
  double nz;

  /* q_1: seeded random unit vector */
  fresh_vector(n, opt->seed, nrand++, Q, NULL, 0, NULL, 0, h, &nz);

  /* the early-restart sums are initialised once, before the outer loop, and
   * carry over from one cycle to the next */
  double t_old = NAN, t_new = NAN;
  while (its <= opt->max_its) {
    /* Lanczos steps i = l+1..m (0-based column i = l..m-1 produces column i+1) */
    int dim = m, next_ok = 1;
    for (int i = l; i < m; ++i) {
      its++;
      double *qi = Q + (size_t)i * n;
      or_filter_apply(n, rp, ci, va, cc, dd, deg, coef, 1, qi, z);
      nmv += deg;
      /* deflation: z <- (I - U U^T) z */
      for (int j = 0; j < nlock; ++j) h[j] = dot(n, Y + (size_t)j * n, z);
      for (int j = 0; j < nlock; ++j)
        for (int64_t r = 0; r < n; ++r) z[r] -= h[j] * Y[(size_t)j * n + r];
      double alpha = dot(n, qi, z);
      if (i == l && l > 0) { /* special TR step: couplings to the TR vectors */
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * qi[r];
        for (int j = 0; j < l; ++j) {
          double sj = TT(j, l);
          for (int64_t r = 0; r < n; ++r) z[r] -= sj * Q[(size_t)j * n + r];
        }
      } else if (i > l) {
        double bi = TT(i - 1, i);
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * qi[r] + bi * qi[r - n];
      } else {
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * qi[r];
      }
      TT(i, i) = alpha;
      /* full reorthogonalisation against [U, q_1..q_i] */
      cgs_dgks(n, z, Y, nlock, Q, i + 1, h);
      double beta = nrm2(n, z);
      if (beta <= 1e-12) {
        /* invariant subspace of the filtered operator: new direction, coupling 0 */
        fresh_vector(n, opt->seed, nrand++, z, Y, nlock, Q, i + 1, h, &nz);
        TT(i, i + 1) = TT(i + 1, i) = 0.0;
        if (nz == 0.0) { dim = i + 1; next_ok = 0; break; }
        memcpy(Q + (size_t)(i + 1) * n, z, sizeof(double) * n);
      } else {
        for (int64_t r = 0; r < n; ++r) Q[(size_t)(i + 1) * n + r] = z[r] / beta;
        TT(i, i + 1) = beta;
        TT(i + 1, i) = beta;
      }
      if (((i + 1) - l) % opt->ncycle == 0) {
        int k = i + 1;
        for (int jj = 0; jj < k; ++jj)
          for (int ii = 0; ii < k; ++ii) Tw[ii + (size_t)jj * k] = TT(ii, jj);
        or_jacobi_eig(k, Tw, w, Yv);
        t_old = t_new;
        t_new = 0.0;
        for (int jj = 0; jj < k; ++jj)
          if (w[jj] >= bar) t_new += w[jj];
        if (fabs(t_new - t_old) < 1e-10 * (fabs(t_new) > 1.0 ? fabs(t_new) : 1.0)) {
          dim = i + 1;
          break;
        }
      }
      if (its > opt->max_its) { dim = i + 1; break; }
    }
    /* Rayleigh-Ritz on T_dim */
    nrestart++;
    for (int jj = 0; jj < dim; ++jj)
      for (int ii = 0; ii < dim; ++ii) Tw[ii + (size_t)jj * dim] = TT(ii, jj);
    or_jacobi_eig(dim, Tw, w, Yv);
    double beta_last = next_ok ? TT(dim - 1, dim) : 0.0;
    int lnew = 0, naccept = 0;
    int cap_tr = m - (opt->ncycle > 10 ? opt->ncycle : 10);
    if (cap_tr < 1) cap_tr = 1;
    for (int jj = dim - 1; jj >= 0; --jj) { /* largest Ritz values first */
      if (w[jj] < bar) break;
      const double *y = Yv + (size_t)jj * dim;
      for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int p = 0; p < dim; ++p) s += Q[(size_t)p * n + r] * y[p];
        u[r] = s;
      }
      or_spmv(n, rp, ci, va, u, au);
      nmv++;
      double uu = dot(n, u, u);
      double lam_j = dot(n, u, au) / uu;
      if (lam_j < tlo || lam_j > thi) continue; /* outside the slice: ignored */
      naccept++;
      double rr = 0.0;
      for (int64_t r = 0; r < n; ++r) {
        double e = au[r] - lam_j * u[r];
        rr += e * e;
      }
      rr = sqrt(rr / uu) / normA;
      if (rr <= opt->tol) {
        if (nlock >= opt->nev_cap) { status = 2; goto done; }
        double nu = sqrt(uu);
        for (int64_t r = 0; r < n; ++r) Y[(size_t)nlock * n + r] = u[r] / nu;
        lam[nlock] = lam_j;
        res[nlock] = rr;
        nlock++;
      } else if (lnew < cap_tr) {
        memcpy(TR + (size_t)lnew * n, u, sizeof(double) * n);
        thTR[lnew] = w[jj];
        sTR[lnew] = beta_last * y[dim - 1];
        lnew++;
      }
    }
    if (naccept == 0) {
      nocand++;
      if (nocand >= 2) break;
    } else {
      nocand = 0;
    }
    /* rebuild the basis for the next cycle */
    memset(T, 0, sizeof(double) * (size_t)M1 * M1);
    if (naccept == 0) {
      /* extra restart from a fresh random vector orthogonal to the locked set */
      fresh_vector(n, opt->seed, nrand++, z, Y, nlock, NULL, 0, h, &nz);
      if (nz == 0.0) break;
      memcpy(Q, z, sizeof(double) * n);
      l = 0;
    } else {
      if (next_ok) memcpy(z, Q + (size_t)dim * n, sizeof(double) * n); /* q_{dim+1} */
      memcpy(Q, TR, sizeof(double) * (size_t)n * lnew);
      if (!next_ok) {
        fresh_vector(n, opt->seed, nrand++, z, Y, nlock, Q, lnew, h, &nz);
        if (nz == 0.0) break;
        for (int j = 0; j < lnew; ++j) sTR[j] = 0.0;
      }
      memcpy(Q + (size_t)lnew * n, z, sizeof(double) * n);
      for (int j = 0; j < lnew; ++j) {
        TT(j, j) = thTR[j];
        TT(j, lnew) = sTR[j];
        TT(lnew, j) = sTR[j];
      }
      l = lnew;
    }
  }
  if (its > opt->max_its) status = 1;
done:
  /* sort ascending by eigenvalue (vectors move along) */
  for (int i = 0; i < nlock - 1; ++i) {
    int mi = i;
    for (int j = i + 1; j < nlock; ++j)
      if (lam[j] < lam[mi]) mi = j;
    if (mi != i) {
      double t = lam[i]; lam[i] = lam[mi]; lam[mi] = t;
      t = res[i]; res[i] = res[mi]; res[mi] = t;
      memcpy(u, Y + (size_t)i * n, sizeof(double) * n);
      memcpy(Y + (size_t)i * n, Y + (size_t)mi * n, sizeof(double) * n);
      memcpy(Y + (size_t)mi * n, u, sizeof(double) * n);
    }
  }
#undef TT
  st->nev = nlock;
  st->niter = its;
  st->nmv = nmv;
  st->nrestart = nrestart;
  st->status = status;
  free(Q); free(TR); free(T); free(Tw); free(w); free(Yv); free(z); free(u); free(au);
  free(h); free(thTR); free(sTR);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Filtered non-restart Lanczos. The paper names the method without giving its
 * steps; this reading keeps every choice of the thick-restart solver above that
 * applies without a restart: the same Lanczos step, full reorthogonalisation,
 * invariant-subspace rule (a fresh random direction with coupling 0), the
 * same settled-sum test, and the same candidates (Ritz values >= bar) and
 * acceptance (Rayleigh quotient in the slice, residual <= tol). */
int or_filtered_lanczos_nr(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                           const double intv[4], int deg, const double *coef, double bar,
                           const or_lan_opts *opt, double *lam, double *res, double *Y,
                           or_lan_stats *st) {
  memset(st, 0, sizeof(*st));
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  /* a slice that reaches a bound of the spectrum owns every eigenvalue
   * beyond it: the bound is an estimate, within rounding of the extreme
   * eigenvalue when the bounding Lanczos run has converged */
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  double normA = fabs(lmin) > fabs(lmax) ? fabs(lmin) : fabs(lmax);
  double cc = 0.5 * (lmax + lmin), dd = 0.5 * (lmax - lmin);
  int m = opt->m;
  if (m > n - 1) m = (int)(n - 1);
  if (m < 2 || deg < 1 || opt->ncycle < 1) return -1;
  const int M1 = m + 1;
  double *Q = (double *)calloc((size_t)n * M1, sizeof(double));
  double *T = (double *)calloc((size_t)M1 * M1, sizeof(double));
  double *Tw = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *w = (double *)malloc(sizeof(double) * m);
  double *Yv = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *z = (double *)malloc(sizeof(double) * n);
  double *u = (double *)malloc(sizeof(double) * n);
  double *au = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (M1 + 1));
#define TT(i, j) T[(i) + (size_t)(j) * M1]
  int its = 0, nmv = 0, nrand = 0, status = 1, nev = 0;
  double nz;
  fresh_vector(n, opt->seed, nrand++, Q, NULL, 0, NULL, 0, h, &nz);
  double t_old = NAN, t_new = NAN;
  int dim = m;
  for (int i = 0; i < m; ++i) {
    its++;
    double *qi = Q + (size_t)i * n;
    or_filter_apply(n, rp, ci, va, cc, dd, deg, coef, 1, qi, z);
    nmv += deg;
    double alpha = dot(n, qi, z);
    double bi = i > 0 ? TT(i - 1, i) : 0.0;
    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * qi[r] + (i > 0 ? bi * qi[r - n] : 0.0);
    TT(i, i) = alpha;
    cgs_dgks(n, z, Q, i + 1, NULL, 0, h);
    double beta = nrm2(n, z);
    if (beta <= 1e-12) {
      fresh_vector(n, opt->seed, nrand++, z, Q, i + 1, NULL, 0, h, &nz);
      if (nz == 0.0) { dim = i + 1; status = 0; break; }
      memcpy(Q + (size_t)(i + 1) * n, z, sizeof(double) * n);
    } else {
      for (int64_t r = 0; r < n; ++r) Q[(size_t)(i + 1) * n + r] = z[r] / beta;
      TT(i, i + 1) = beta;
      TT(i + 1, i) = beta;
    }
    if ((i + 1) % opt->ncycle == 0) {
      int k = i + 1;
      for (int jj = 0; jj < k; ++jj)
        for (int ii = 0; ii < k; ++ii) Tw[ii + (size_t)jj * k] = TT(ii, jj);
      or_jacobi_eig(k, Tw, w, Yv);
      t_old = t_new;
      t_new = 0.0;
      for (int jj = 0; jj < k; ++jj)
        if (w[jj] >= bar) t_new += w[jj];
      if (fabs(t_new - t_old) < 1e-10 * (fabs(t_new) > 1.0 ? fabs(t_new) : 1.0)) {
        dim = k;
        status = 0;
        break;
      }
    }
  }
  /* Ritz pairs of T_dim with values >= bar, checked against A */
  for (int jj = 0; jj < dim; ++jj)
    for (int ii = 0; ii < dim; ++ii) Tw[ii + (size_t)jj * dim] = TT(ii, jj);
  or_jacobi_eig(dim, Tw, w, Yv);
  for (int jj = dim - 1; jj >= 0 && w[jj] >= bar; --jj) {
    const double *y = Yv + (size_t)jj * dim;
    for (int64_t r = 0; r < n; ++r) {
      double s = 0.0;
      for (int p = 0; p < dim; ++p) s += Q[(size_t)p * n + r] * y[p];
      u[r] = s;
    }
    or_spmv(n, rp, ci, va, u, au);
    nmv++;
    double uu = dot(n, u, u);
    double lam_j = dot(n, u, au) / uu;
    if (lam_j < tlo || lam_j > thi) continue;
    double rr = 0.0;
    for (int64_t r = 0; r < n; ++r) {
      double e = au[r] - lam_j * u[r];
      rr += e * e;
    }
    rr = sqrt(rr / uu) / normA;
    if (rr > opt->tol) continue;
    if (nev >= opt->nev_cap) { status = 2; break; }
    double nu = sqrt(uu);
    for (int64_t r = 0; r < n; ++r) Y[(size_t)nev * n + r] = u[r] / nu;
    lam[nev] = lam_j;
    res[nev] = rr;
    nev++;
  }
  for (int i = 0; i < nev - 1; ++i) {
    int mi = i;
    for (int j = i + 1; j < nev; ++j)
      if (lam[j] < lam[mi]) mi = j;
    if (mi != i) {
      double t = lam[i]; lam[i] = lam[mi]; lam[mi] = t;
      t = res[i]; res[i] = res[mi]; res[mi] = t;
      memcpy(u, Y + (size_t)i * n, sizeof(double) * n);
      memcpy(Y + (size_t)i * n, Y + (size_t)mi * n, sizeof(double) * n);
      memcpy(Y + (size_t)mi * n, u, sizeof(double) * n);
    }
  }
#undef TT
  st->nev = nev;
  st->niter = its;
  st->nmv = nmv;
  st->nrestart = 0;
  st->status = status;
  free(Q); free(T); free(Tw); free(w); free(Yv); free(z); free(u); free(au); free(h);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Filtered subspace iteration. The paper names the method and notes that its
 * block size comes from the DOS count; the stopping rule, the start block and
 * the orthonormalisation are this reading's. */
static int orthonormalise_block(int64_t n, int b, double *W, double *h, uint64_t seed,
                                int *next) {
  /* column j <- column j minus its projections on columns < j (two passes),
   * normalised; a column that vanishes (relative norm < 1e-10) is replaced by
   * the next random vector of the stream and orthogonalised again; returns
   * the number of replacements */
  int refills = 0;
  for (int j = 0; j < b; ++j) {
    double *w = W + (size_t)j * n;
    for (int attempt = 0; attempt < 3; ++attempt) {
      double n0 = nrm2(n, w);
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < j; ++i) h[i] = dot(n, W + (size_t)i * n, w);
        for (int i = 0; i < j; ++i)
          for (int64_t r = 0; r < n; ++r) w[r] -= h[i] * W[(size_t)i * n + r];
      }
      double nw = nrm2(n, w);
      if (nw > 1e-10 * n0) {
        for (int64_t r = 0; r < n; ++r) w[r] /= nw;
        break;
      }
      or_lanczos_start(seed, n, (*next)++, w);
      refills++;
    }
  }
  return refills;
}

int or_filtered_subspace(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                         const double intv[4], int deg, const double *coef, double bar,
                         const or_si_opts *opt, double *lam, double *res, double *Y,
                         or_lan_stats *st) {
  memset(st, 0, sizeof(*st));
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  /* a slice that reaches a bound of the spectrum owns every eigenvalue
   * beyond it: the bound is an estimate, within rounding of the extreme
   * eigenvalue when the bounding Lanczos run has converged */
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  const double normA = fabs(lmin) > fabs(lmax) ? fabs(lmin) : fabs(lmax);
  const double cc = 0.5 * (lmax + lmin), dd = 0.5 * (lmax - lmin);
  const int b = opt->block;
  if (b < 1 || b > n || deg < 1 || opt->max_its < 1) return -1;
  double *V = (double *)malloc(sizeof(double) * (size_t)n * b);
  double *W = (double *)malloc(sizeof(double) * (size_t)n * b);
  double *AQ = (double *)malloc(sizeof(double) * (size_t)n * b);
  double *H = (double *)malloc(sizeof(double) * (size_t)b * b);
  double *S = (double *)malloc(sizeof(double) * (size_t)b * b);
  double *th = (double *)malloc(sizeof(double) * b);
  double *rs = (double *)malloc(sizeof(double) * b);
  double *mu = (double *)malloc(sizeof(double) * b);
  double *h = (double *)malloc(sizeof(double) * (b + 1));
  double *z = (double *)malloc(sizeof(double) * n);
  int its = 0, nmv = 0, status = 1, prev = -1, have_ritz = 0;
  int next = b;  /* next random block of the stream (refills) */
  for (int j = 0; j < b; ++j) or_lanczos_start(opt->seed, n, j, V + (size_t)j * n);
  orthonormalise_block(n, b, V, h, opt->seed, &next);
  while (its < opt->max_its) {
    /* W = p(A-hat) V */
    for (int j = 0; j < b; ++j)
      or_filter_apply(n, rp, ci, va, cc, dd, deg, coef, 1, V + (size_t)j * n, W + (size_t)j * n);
    its++;
    nmv += deg * b;
    if (have_ritz) {
      int nconv = 0, bad = 0, nin = 0;
      for (int j = 0; j < b; ++j) {
        mu[j] = dot(n, V + (size_t)j * n, W + (size_t)j * n);
        if (th[j] < tlo || th[j] > thi) continue;
        nin++;
        if (rs[j] <= opt->tol) nconv++;
        else if (mu[j] >= bar) bad++;
      }
      if (nin == b) { status = 3; break; }
      if (nconv == prev && bad == 0) { status = 0; break; }
      prev = nconv;
    }
    /* orthonormal basis Q of span(W) (in W), A Q, Rayleigh-Ritz */
    orthonormalise_block(n, b, W, h, opt->seed, &next);
    for (int j = 0; j < b; ++j) or_spmv(n, rp, ci, va, W + (size_t)j * n, AQ + (size_t)j * n);
    nmv += b;
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) H[i + (size_t)j * b] = dot(n, W + (size_t)i * n, AQ + (size_t)j * n);
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < j; ++i) {
        double avg = 0.5 * (H[i + (size_t)j * b] + H[j + (size_t)i * b]);
        H[i + (size_t)j * b] = H[j + (size_t)i * b] = avg;
      }
    or_jacobi_eig(b, H, th, S);
    /* V = Q S, residuals ||A v - theta v|| = ||AQ s - theta Q s|| */
    for (int j = 0; j < b; ++j) {
      double *v = V + (size_t)j * n;
      for (int64_t r = 0; r < n; ++r) {
        double sv = 0.0, sa = 0.0;
        for (int p = 0; p < b; ++p) {
          sv += W[(size_t)p * n + r] * S[p + (size_t)j * b];
          sa += AQ[(size_t)p * n + r] * S[p + (size_t)j * b];
        }
        v[r] = sv;
        z[r] = sa;
      }
      double rr = 0.0;
      for (int64_t r = 0; r < n; ++r) {
        double e = z[r] - th[j] * v[r];
        rr += e * e;
      }
      rs[j] = sqrt(rr) / normA;
    }
    have_ritz = 1;
  }
  /* converged pairs inside the slice, ascending (the Ritz values are sorted) */
  int nev = 0;
  for (int j = 0; j < b; ++j) {
    if (th[j] < tlo || th[j] > thi || rs[j] > opt->tol) continue;
    if (nev >= opt->nev_cap) { status = 2; break; }
    memcpy(Y + (size_t)nev * n, V + (size_t)j * n, sizeof(double) * n);
    lam[nev] = th[j];
    res[nev] = rs[j];
    nev++;
  }
  st->nev = nev;
  st->niter = its;
  st->nmv = nmv;
  st->nrestart = 0;
  st->status = status;
  free(V); free(W); free(AQ); free(H); free(S); free(th); free(rs); free(mu); free(h); free(z);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lanczos DOS with Gaussian quadrature (Section 2.1). The paper cites the
 * method without formulas; the quadrature is the classical one (Golub and
 * Meurant): nodes = eigenvalues of T_m, weights = squared first eigenvector
 * components. */
int or_lanczos_dos(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, int m,
                   int nvec, uint64_t seed, double *nodes, double *weights, int *dims) {
  if (m < 1 || nvec < 1) return -1;
  if (m > n) m = (int)n;
  double *Q = (double *)calloc((size_t)n * (m + 1), sizeof(double));
  double *z = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (m + 1));
  double *al = (double *)malloc(sizeof(double) * m);
  double *be = (double *)malloc(sizeof(double) * m);
  double *T = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *Y = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *w = (double *)malloc(sizeof(double) * m);
  for (int l = 0; l < nvec; ++l) {
    or_lanczos_start(seed, n, l, Q);
    double nq = nrm2(n, Q);
    for (int64_t i = 0; i < n; ++i) Q[i] /= nq;
    int dim = m;
    double scale = 0.0;
    for (int i = 0; i < m; ++i) {
      double *qi = Q + (size_t)i * n;
      or_spmv(n, rp, ci, va, qi, z);
      al[i] = dot(n, qi, z);
      for (int64_t r = 0; r < n; ++r) z[r] -= al[i] * qi[r] + (i > 0 ? be[i - 1] * qi[r - n] : 0.0);
      cgs_dgks(n, z, Q, i + 1, NULL, 0, h);
      be[i] = nrm2(n, z);
      scale = fmax(scale, fabs(al[i]) + (i > 0 ? be[i - 1] : 0.0));
      if (i + 1 < m && be[i] <= 1e-12 * scale) { dim = i + 1; break; }
      if (i + 1 < m)
        for (int64_t r = 0; r < n; ++r) Q[(size_t)(i + 1) * n + r] = z[r] / be[i];
    }
    for (int j = 0; j < dim * dim; ++j) T[j] = 0.0;
    for (int i = 0; i < dim; ++i) {
      T[i + (size_t)i * dim] = al[i];
      if (i + 1 < dim) T[i + (size_t)(i + 1) * dim] = T[(i + 1) + (size_t)i * dim] = be[i];
    }
    or_jacobi_eig(dim, T, w, Y);
    for (int k = 0; k < m; ++k) {
      nodes[(size_t)l * m + k] = k < dim ? w[k] : 0.0;
      weights[(size_t)l * m + k] = k < dim ? Y[(size_t)k * dim] * Y[(size_t)k * dim] : 0.0;
    }
    dims[l] = dim;
  }
  free(Q); free(z); free(h); free(al); free(be); free(T); free(Y); free(w);
  return 0;
}

double or_lanczos_count(const double *nodes, const double *weights, const int *dims, int nvec,
                        int m, int64_t n, double sigma, double x0, double x1) {
  double s = 0.0;
  for (int l = 0; l < nvec; ++l)
    for (int k = 0; k < dims[l]; ++k) {
      const double t = nodes[(size_t)l * m + k], wk = weights[(size_t)l * m + k];
      if (sigma > 0.0) {
        const double r = 1.0 / (sigma * sqrt(2.0));
        s += wk * 0.5 * (erf((x1 - t) * r) - erf((x0 - t) * r));
      } else if (t >= x0 && t <= x1) {
        s += wk;
      }
    }
  return (double)n * s / nvec;
}

int or_lanczos_slicer(const double *nodes, const double *weights, const int *dims, int nvec,
                      int m, int64_t n, double sigma, double xi, double eta, int nslices,
                      int npts, double *sli) {
  if (nslices < 1 || npts < nslices + 1 || !(eta > xi)) return -1;
  double *C = (double *)malloc(sizeof(double) * npts);
  for (int j = 0; j < npts; ++j) {
    double x = xi + (eta - xi) * (double)j / (double)(npts - 1);
    C[j] = or_lanczos_count(nodes, weights, dims, nvec, m, n, sigma, xi, x);
  }
  double total = C[npts - 1];
  sli[0] = xi;
  sli[nslices] = eta;
  int prev = 0, rc = 0;
  for (int i = 1; i < nslices; ++i) {
    double target = total * (double)i / (double)nslices;
    int j = prev + 1;
    while (j < npts - 1 && C[j] < target) ++j;
    if (j >= npts - 1) { rc = -1; break; }
    sli[i] = xi + (eta - xi) * (double)j / (double)(npts - 1);
    prev = j;
  }
  free(C);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Generalized problems (Section 2.4). */
int or_lspol(int kind, double lo, double hi, int deg, double *coef) {
  if (!(hi > lo) || !(lo > 0.0) || deg < 0 || (kind != 0 && kind != 1)) return -1;
  const int N = 1024;
  const double c = 0.5 * (hi + lo), d = 0.5 * (hi - lo);
  for (int j = 0; j <= deg; ++j) coef[j] = 0.0;
  for (int k = 0; k < N; ++k) {
    const double th = M_PI * (k + 0.5) / N;
    const double t = c + d * cos(th);
    const double f = kind == 0 ? 1.0 / t : 1.0 / sqrt(t);
    for (int j = 0; j <= deg; ++j) coef[j] += f * cos(j * th);
  }
  for (int j = 0; j <= deg; ++j) coef[j] *= (j == 0 ? 1.0 : 2.0) / N;
  return 0;
}

int or_cg_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *vb,
                const double *r, double *x) {
  double *res = (double *)malloc(sizeof(double) * n);
  double *p = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; res[i] = r[i]; p[i] = r[i]; }
  const double r0 = nrm2(n, r);
  double rr = dot(n, res, res);
  int it = 0;
  for (; it < 10000 && sqrt(rr) > 1e-15 * r0; ++it) {
    or_spmv(n, rp, ci, vb, p, q);
    const double a = rr / dot(n, p, q);
    for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; res[i] -= a * q[i]; }
    const double rn = dot(n, res, res);
    const double bb = rn / rr;
    rr = rn;
    for (int64_t i = 0; i < n; ++i) p[i] = res[i] + bb * p[i];
  }
  free(res); free(p); free(q);
  return it;
}

/* B-orthonormal random start: w = v / ||v||_B, z = B w. */
static void gen_start(int64_t n, const int32_t *rpb, const int32_t *cib, const double *vb,
                      uint64_t seed, int64_t block, double *w, double *z) {
  or_lanczos_start(seed, n, block, w);
  or_spmv(n, rpb, cib, vb, w, z);
  const double nb = sqrt(dot(n, w, z));
  for (int64_t i = 0; i < n; ++i) { w[i] /= nb; z[i] /= nb; }
}

int or_lanczos_bounds_gen(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                          const int32_t *rpb, const int32_t *cib, const double *vb, int nsteps,
                          uint64_t seed, double *lmin, double *lmax) {
  int m = nsteps < n ? nsteps : (int)n;
  if (m < 1) return -1;
  double *W = (double *)calloc((size_t)n * (m + 1), sizeof(double));
  double *Z = (double *)calloc((size_t)n * (m + 1), sizeof(double));
  double *z = (double *)malloc(sizeof(double) * n);
  double *T = (double *)calloc((size_t)m * m, sizeof(double));
  double *h = (double *)malloc(sizeof(double) * (m + 1));
  gen_start(n, rpb, cib, vb, seed, 0, W, Z);
  double beta = 0.0, scale = 0.0;
  int dim = m;
  for (int i = 0; i < m; ++i) {
    double *wi = W + (size_t)i * n, *zi = Z + (size_t)i * n;
    /* one step of Algorithm alg:LanAB */
    or_spmv(n, rp, ci, va, wi, z);
    if (i > 0)
      for (int64_t r = 0; r < n; ++r) z[r] -= beta * Z[(size_t)(i - 1) * n + r];
    const double alpha = dot(n, z, wi);
    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r];
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j <= i; ++j) h[j] = dot(n, z, W + (size_t)j * n);
      for (int j = 0; j <= i; ++j)
        for (int64_t r = 0; r < n; ++r) z[r] -= h[j] * Z[(size_t)j * n + r];
    }
    T[i + (size_t)i * m] = alpha;
    double *wn = W + (size_t)(i + 1) * n;
    or_cg_solve(n, rpb, cib, vb, z, wn);
    scale = fmax(scale, fabs(alpha) + beta);
    beta = sqrt(fmax(dot(n, wn, z), 0.0));
    if (beta <= 1e-12 * scale) { dim = i + 1; beta = 0.0; break; }
    for (int64_t r = 0; r < n; ++r) { wn[r] /= beta; Z[(size_t)(i + 1) * n + r] = z[r] / beta; }
    if (i + 1 < m) T[i + (size_t)(i + 1) * m] = T[(i + 1) + (size_t)i * m] = beta;
  }
  double *Tm = (double *)malloc(sizeof(double) * dim * dim);
  for (int j = 0; j < dim; ++j)
    for (int i = 0; i < dim; ++i) Tm[i + (size_t)j * dim] = T[i + (size_t)j * m];
  double *w = (double *)malloc(sizeof(double) * dim), *Y = (double *)malloc(sizeof(double) * dim * dim);
  or_jacobi_eig(dim, Tm, w, Y);
  *lmin = w[0] - fabs(beta * Y[(dim - 1) + 0]);
  *lmax = w[dim - 1] + fabs(beta * Y[(dim - 1) + (size_t)(dim - 1) * dim]);
  free(W); free(Z); free(z); free(T); free(h); free(Tm); free(w); free(Y);
  return 0;
}

/* y = rho(A-hat B^(-1)) x by the Chebyshev recurrence in M = A-hat B^(-1):
 * M v = (A u - c v)/d with u = B^(-1) v (exact solve). */
static void gen_filter(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                       const int32_t *rpb, const int32_t *cib, const double *vb, double c,
                       double d, int deg, const double *coef, const double *x, double *y) {
  double *w0 = (double *)malloc(sizeof(double) * n), *w1 = (double *)malloc(sizeof(double) * n);
  double *w2 = (double *)malloc(sizeof(double) * n), *u = (double *)malloc(sizeof(double) * n);
  double *au = (double *)malloc(sizeof(double) * n);
  memcpy(w0, x, sizeof(double) * n);
  or_cg_solve(n, rpb, cib, vb, w0, u);
  or_spmv(n, rp, ci, va, u, au);
  for (int64_t i = 0; i < n; ++i) {
    w1[i] = (au[i] - c * w0[i]) / d;
    y[i] = coef[0] * w0[i] + coef[1] * w1[i];
  }
  for (int j = 1; j < deg; ++j) {
    or_cg_solve(n, rpb, cib, vb, w1, u);
    or_spmv(n, rp, ci, va, u, au);
    for (int64_t i = 0; i < n; ++i) {
      w2[i] = 2.0 * (au[i] - c * w1[i]) / d - w0[i];
      y[i] += coef[j + 1] * w2[i];
    }
    double *t = w0; w0 = w1; w1 = w2; w2 = t;
  }
  free(w0); free(w1); free(w2); free(u); free(au);
}

int or_filtered_lanczos_gen(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                            const int32_t *rpb, const int32_t *cib, const double *vb,
                            const double intv[4], int deg, const double *coef, double bar,
                            const or_lan_opts *opt, double *lam, double *res, double *Y,
                            or_lan_stats *st) {
  memset(st, 0, sizeof(*st));
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  /* a slice that reaches a bound of the spectrum owns every eigenvalue
   * beyond it: the bound is an estimate, within rounding of the extreme
   * eigenvalue when the bounding Lanczos run has converged */
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  const double normA = fabs(lmin) > fabs(lmax) ? fabs(lmin) : fabs(lmax);
  const double cc = 0.5 * (lmax + lmin), dd = 0.5 * (lmax - lmin);
  int m = opt->m;
  if (m > n - 1) m = (int)(n - 1);
  if (m < 2 || deg < 1 || opt->ncycle < 1) return -1;
  const int M1 = m + 1;
  double *W = (double *)calloc((size_t)n * M1, sizeof(double));
  double *Z = (double *)calloc((size_t)n * M1, sizeof(double));
  double *T = (double *)calloc((size_t)M1 * M1, sizeof(double));
  double *Tw = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *w = (double *)malloc(sizeof(double) * m), *Yv = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *z = (double *)malloc(sizeof(double) * n), *x = (double *)malloc(sizeof(double) * n);
  double *ax = (double *)malloc(sizeof(double) * n), *bx = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (M1 + 1));
#define TT(i, j) T[(i) + (size_t)(j) * M1]
  int its = 0, nmv = 0, status = 1, nev = 0, dim = m;
  double t_old = NAN, t_new = NAN, beta = 0.0;
  gen_start(n, rpb, cib, vb, opt->seed, 0, W, Z);
  for (int i = 0; i < m; ++i) {
    its++;
    double *wi = W + (size_t)i * n, *zi = Z + (size_t)i * n;
    /* eq:polyapp1: z = rho(A-hat B^(-1)) z_i - beta_i z_{i-1} */
    gen_filter(n, rp, ci, va, rpb, cib, vb, cc, dd, deg, coef, zi, z);
    nmv += deg;
    if (i > 0)
      for (int64_t r = 0; r < n; ++r) z[r] -= beta * Z[(size_t)(i - 1) * n + r];
    const double alpha = dot(n, z, wi);
    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r];
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j <= i; ++j) h[j] = dot(n, z, W + (size_t)j * n);
      for (int j = 0; j <= i; ++j)
        for (int64_t r = 0; r < n; ++r) z[r] -= h[j] * Z[(size_t)j * n + r];
    }
    TT(i, i) = alpha;
    double *wn = W + (size_t)(i + 1) * n;
    or_cg_solve(n, rpb, cib, vb, z, wn);
    beta = sqrt(fmax(dot(n, wn, z), 0.0));
    if (beta <= 1e-12) { dim = i + 1; status = 0; break; }
    for (int64_t r = 0; r < n; ++r) { wn[r] /= beta; Z[(size_t)(i + 1) * n + r] = z[r] / beta; }
    TT(i, i + 1) = TT(i + 1, i) = beta;
    if ((i + 1) % opt->ncycle == 0) {
      const int k = i + 1;
      for (int jj = 0; jj < k; ++jj)
        for (int ii = 0; ii < k; ++ii) Tw[ii + (size_t)jj * k] = TT(ii, jj);
      or_jacobi_eig(k, Tw, w, Yv);
      t_old = t_new;
      t_new = 0.0;
      for (int jj = 0; jj < k; ++jj)
        if (w[jj] >= bar) t_new += w[jj];
      if (fabs(t_new - t_old) < 1e-10 * (fabs(t_new) > 1.0 ? fabs(t_new) : 1.0)) {
        dim = k;
        status = 0;
        break;
      }
    }
  }
  for (int jj = 0; jj < dim; ++jj)
    for (int ii = 0; ii < dim; ++ii) Tw[ii + (size_t)jj * dim] = TT(ii, jj);
  or_jacobi_eig(dim, Tw, w, Yv);
  for (int jj = dim - 1; jj >= 0 && w[jj] >= bar; --jj) {
    const double *y = Yv + (size_t)jj * dim;
    for (int64_t r = 0; r < n; ++r) {
      double s = 0.0;
      for (int p = 0; p < dim; ++p) s += W[(size_t)p * n + r] * y[p];
      x[r] = s;
    }
    or_spmv(n, rp, ci, va, x, ax);
    or_spmv(n, rpb, cib, vb, x, bx);
    nmv++;
    const double xbx = dot(n, x, bx), lam_j = dot(n, x, ax) / xbx;
    if (lam_j < tlo || lam_j > thi) continue;
    double rr = 0.0;
    for (int64_t r = 0; r < n; ++r) {
      const double e = ax[r] - lam_j * bx[r];
      rr += e * e;
    }
    const double rj = sqrt(rr) / (nrm2(n, bx) * normA);
    if (rj > opt->tol) continue;
    if (nev >= opt->nev_cap) { status = 2; break; }
    const double nb = sqrt(xbx);
    for (int64_t r = 0; r < n; ++r) Y[(size_t)nev * n + r] = x[r] / nb;
    lam[nev] = lam_j;
    res[nev] = rj;
    nev++;
  }
  for (int i = 0; i < nev - 1; ++i) {
    int mi = i;
    for (int j = i + 1; j < nev; ++j)
      if (lam[j] < lam[mi]) mi = j;
    if (mi != i) {
      double t = lam[i]; lam[i] = lam[mi]; lam[mi] = t;
      t = res[i]; res[i] = res[mi]; res[mi] = t;
      memcpy(x, Y + (size_t)i * n, sizeof(double) * n);
      memcpy(Y + (size_t)i * n, Y + (size_t)mi * n, sizeof(double) * n);
      memcpy(Y + (size_t)mi * n, x, sizeof(double) * n);
    }
  }
#undef TT
  st->nev = nev;
  st->niter = its;
  st->nmv = nmv;
  st->status = status;
  free(W); free(Z); free(T); free(Tw); free(w); free(Yv); free(z); free(x); free(ax); free(bx);
  free(h);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Generalized problems, thick-restart form: Algorithm alg:FiltLanTR carried
 * out in the B-inner product with the two bases of Algorithm alg:LanAB (W
 * B-orthonormal, Z = B W) and the filtered step of eq:polyapp1. The locked
 * vectors U are B-orthonormal and kept with B U; in the z-representation the
 * deflation subtracts B U (U^T z) and the full reorthogonalisation (two
 * classical Gram-Schmidt passes, as in the non-restart form) subtracts
 * B U (U^T z) and Z (W^T z). Ritz vectors of T are u = W y with B u = Z y; a
 * candidate is accepted when lambda = u^T A u / u^T B u lies in the slice and
 * ||A u - lambda B u|| / (||B u|| max(|lambda_min|, |lambda_max|)) <= tol.
 * Every other reading (candidates, arrowhead T, early-restart sums, extra
 * restart, kept Ritz vectors) is that of or_filtered_lanczos. Y holds the
 * B-normalised locked vectors. */
static void gen_fresh(int64_t n, const int32_t *rpb, const int32_t *cib, const double *vb,
                      uint64_t seed, int idx, const double *U, const double *BU, int nlock,
                      const double *W, const double *Z, int k, double *w, double *z, double *nrm) {
  or_lanczos_start(seed, n, idx, w);
  or_spmv(n, rpb, cib, vb, w, z);
  const double n0 = sqrt(fmax(dot(n, w, z), 0.0));
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < nlock; ++j) {
      const double hj = dot(n, BU + (size_t)j * n, w);
      for (int64_t r = 0; r < n; ++r) w[r] -= hj * U[(size_t)j * n + r];
    }
    for (int j = 0; j < k; ++j) {
      const double hj = dot(n, Z + (size_t)j * n, w);
      for (int64_t r = 0; r < n; ++r) w[r] -= hj * W[(size_t)j * n + r];
    }
  }
  or_spmv(n, rpb, cib, vb, w, z);
  const double nb = sqrt(fmax(dot(n, w, z), 0.0));
  *nrm = nb > 1e-10 * n0 ? nb : 0.0;
  if (*nrm > 0.0)
    for (int64_t r = 0; r < n; ++r) { w[r] /= nb; z[r] /= nb; }
}

int or_filtered_lanczos_gen_tr(int64_t n, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *rpb, const int32_t *cib, const double *vb,
                               const double intv[4], int deg, const double *coef, double bar,
                               const or_lan_opts *opt, double *lam, double *res, double *Y,
                               or_lan_stats *st) {
  memset(st, 0, sizeof(*st));
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  /* a slice that reaches a bound of the spectrum owns every eigenvalue
   * beyond it */
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  const double normA = fabs(lmin) > fabs(lmax) ? fabs(lmin) : fabs(lmax);
  const double cc = 0.5 * (lmax + lmin), dd = 0.5 * (lmax - lmin);
  int m = opt->m;
  if (m > n - 1) m = (int)(n - 1);
  if (m < 2 || deg < 1 || opt->ncycle < 1) return -1;
  const int M1 = m + 1;
  double *W = (double *)calloc((size_t)n * M1, sizeof(double));
  double *Z = (double *)calloc((size_t)n * M1, sizeof(double));
  double *BU = (double *)calloc((size_t)n * (opt->nev_cap > 0 ? opt->nev_cap : 1), sizeof(double));
  double *TRw = (double *)malloc(sizeof(double) * (size_t)n * m);
  double *TRz = (double *)malloc(sizeof(double) * (size_t)n * m);
  double *T = (double *)calloc((size_t)M1 * M1, sizeof(double));
  double *Tw = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *w = (double *)malloc(sizeof(double) * m);
  double *Yv = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *z = (double *)malloc(sizeof(double) * n), *zw = (double *)malloc(sizeof(double) * n);
  double *u = (double *)malloc(sizeof(double) * n), *bu = (double *)malloc(sizeof(double) * n);
  double *au = (double *)malloc(sizeof(double) * n);
  double *h = (double *)malloc(sizeof(double) * (opt->nev_cap + m + 2));
  double *thTR = (double *)malloc(sizeof(double) * m), *sTR = (double *)malloc(sizeof(double) * m);
#define TT(i, j) T[(i) + (size_t)(j) * M1]
  int nlock = 0, l = 0, its = 0, nmv = 0, nrand = 0, nocand = 0, nrestart = 0, status = 0;
  double nz;
  gen_fresh(n, rpb, cib, vb, opt->seed, nrand++, Y, BU, 0, W, Z, 0, W, Z, &nz);
  double t_old = NAN, t_new = NAN;
  while (its <= opt->max_its) {
    int dim = m, next_ok = 1;
    for (int i = l; i < m; ++i) {
      its++;
      double *wi = W + (size_t)i * n, *zi = Z + (size_t)i * n;
      /* eq:polyapp1: z = rho(A-hat B^(-1)) z_i */
      gen_filter(n, rp, ci, va, rpb, cib, vb, cc, dd, deg, coef, zi, z);
      nmv += deg;
      /* deflation: z <- z - B U (U^T z) */
      for (int j = 0; j < nlock; ++j) h[j] = dot(n, Y + (size_t)j * n, z);
      for (int j = 0; j < nlock; ++j)
        for (int64_t r = 0; r < n; ++r) z[r] -= h[j] * BU[(size_t)j * n + r];
      const double alpha = dot(n, z, wi);
      if (i == l && l > 0) { /* special TR step: couplings to the TR vectors */
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r];
        for (int j = 0; j < l; ++j) {
          const double sj = TT(j, l);
          for (int64_t r = 0; r < n; ++r) z[r] -= sj * Z[(size_t)j * n + r];
        }
      } else if (i > l) {
        const double bi = TT(i - 1, i);
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r] + bi * zi[r - n];
      } else {
        for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r];
      }
      TT(i, i) = alpha;
      /* full reorthogonalisation against [U, w_1..w_i] (two passes) */
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < nlock; ++j) h[j] = dot(n, Y + (size_t)j * n, z);
        for (int j = 0; j <= i; ++j) h[nlock + j] = dot(n, W + (size_t)j * n, z);
        for (int j = 0; j < nlock; ++j)
          for (int64_t r = 0; r < n; ++r) z[r] -= h[j] * BU[(size_t)j * n + r];
        for (int j = 0; j <= i; ++j)
          for (int64_t r = 0; r < n; ++r) z[r] -= h[nlock + j] * Z[(size_t)j * n + r];
      }
      double *wn = W + (size_t)(i + 1) * n, *zn = Z + (size_t)(i + 1) * n;
      or_cg_solve(n, rpb, cib, vb, z, wn);
      const double beta = sqrt(fmax(dot(n, wn, z), 0.0));
      if (beta <= 1e-12) {
        /* invariant subspace of the filtered operator: new direction, coupling 0 */
        gen_fresh(n, rpb, cib, vb, opt->seed, nrand++, Y, BU, nlock, W, Z, i + 1, wn, zn, &nz);
        TT(i, i + 1) = TT(i + 1, i) = 0.0;
        if (nz == 0.0) { dim = i + 1; next_ok = 0; break; }
      } else {
        for (int64_t r = 0; r < n; ++r) { wn[r] /= beta; zn[r] = z[r] / beta; }
        TT(i, i + 1) = TT(i + 1, i) = beta;
      }
      if (((i + 1) - l) % opt->ncycle == 0) {
        const int k = i + 1;
        for (int jj = 0; jj < k; ++jj)
          for (int ii = 0; ii < k; ++ii) Tw[ii + (size_t)jj * k] = TT(ii, jj);
        or_jacobi_eig(k, Tw, w, Yv);
        t_old = t_new;
        t_new = 0.0;
        for (int jj = 0; jj < k; ++jj)
          if (w[jj] >= bar) t_new += w[jj];
        if (fabs(t_new - t_old) < 1e-10 * (fabs(t_new) > 1.0 ? fabs(t_new) : 1.0)) {
          dim = k;
          break;
        }
      }
      if (its > opt->max_its) { dim = i + 1; break; }
    }
    /* Rayleigh-Ritz on T_dim */
    nrestart++;
    for (int jj = 0; jj < dim; ++jj)
      for (int ii = 0; ii < dim; ++ii) Tw[ii + (size_t)jj * dim] = TT(ii, jj);
    or_jacobi_eig(dim, Tw, w, Yv);
    const double beta_last = next_ok ? TT(dim - 1, dim) : 0.0;
    const int cap_tr = m - (opt->ncycle > 10 ? opt->ncycle : 10) > 0
                           ? m - (opt->ncycle > 10 ? opt->ncycle : 10) : 1;
    int lnew = 0, naccept = 0;
    for (int jj = dim - 1; jj >= 0 && w[jj] >= bar; --jj) {
      const double *y = Yv + (size_t)jj * dim;
      for (int64_t r = 0; r < n; ++r) {
        double s = 0.0, sb = 0.0;
        for (int p = 0; p < dim; ++p) {
          s += W[(size_t)p * n + r] * y[p];
          sb += Z[(size_t)p * n + r] * y[p];
        }
        u[r] = s;
        bu[r] = sb;
      }
      or_spmv(n, rp, ci, va, u, au);
      nmv++;
      const double ubu = dot(n, u, bu);
      const double lam_j = dot(n, u, au) / ubu;
      if (lam_j < tlo || lam_j > thi) continue; /* outside the slice: ignored */
      naccept++;
      double rr = 0.0;
      for (int64_t r = 0; r < n; ++r) {
        const double e = au[r] - lam_j * bu[r];
        rr += e * e;
      }
      rr = sqrt(rr) / (nrm2(n, bu) * normA);
      if (rr <= opt->tol) {
        if (nlock >= opt->nev_cap) { status = 2; goto done; }
        const double nb = sqrt(ubu);
        for (int64_t r = 0; r < n; ++r) {
          Y[(size_t)nlock * n + r] = u[r] / nb;
          BU[(size_t)nlock * n + r] = bu[r] / nb;
        }
        lam[nlock] = lam_j;
        res[nlock] = rr;
        nlock++;
      } else if (lnew < cap_tr) {
        memcpy(TRw + (size_t)lnew * n, u, sizeof(double) * n);
        memcpy(TRz + (size_t)lnew * n, bu, sizeof(double) * n);
        thTR[lnew] = w[jj];
        sTR[lnew] = beta_last * y[dim - 1];
        lnew++;
      }
    }
    if (naccept == 0) {
      nocand++;
      if (nocand >= 2) break;
    } else {
      nocand = 0;
    }
    memset(T, 0, sizeof(double) * (size_t)M1 * M1);
    if (naccept == 0) {
      /* extra restart from a fresh random vector B-orthogonal to the locked set */
      gen_fresh(n, rpb, cib, vb, opt->seed, nrand++, Y, BU, nlock, W, Z, 0, zw, z, &nz);
      if (nz == 0.0) break;
      memcpy(W, zw, sizeof(double) * n);
      memcpy(Z, z, sizeof(double) * n);
      l = 0;
    } else {
      if (next_ok) {
        memcpy(zw, W + (size_t)dim * n, sizeof(double) * n);
        memcpy(z, Z + (size_t)dim * n, sizeof(double) * n);
      }
      memcpy(W, TRw, sizeof(double) * (size_t)n * lnew);
      memcpy(Z, TRz, sizeof(double) * (size_t)n * lnew);
      if (!next_ok) {
        gen_fresh(n, rpb, cib, vb, opt->seed, nrand++, Y, BU, nlock, W, Z, lnew, zw, z, &nz);
        if (nz == 0.0) break;
        for (int j = 0; j < lnew; ++j) sTR[j] = 0.0;
      }
      memcpy(W + (size_t)lnew * n, zw, sizeof(double) * n);
      memcpy(Z + (size_t)lnew * n, z, sizeof(double) * n);
      for (int j = 0; j < lnew; ++j) {
        TT(j, j) = thTR[j];
        TT(j, lnew) = sTR[j];
        TT(lnew, j) = sTR[j];
      }
      l = lnew;
    }
  }
  if (its > opt->max_its) status = 1;
done:
  for (int i = 0; i < nlock - 1; ++i) {
    int mi = i;
    for (int j = i + 1; j < nlock; ++j)
      if (lam[j] < lam[mi]) mi = j;
    if (mi != i) {
      double t = lam[i]; lam[i] = lam[mi]; lam[mi] = t;
      t = res[i]; res[i] = res[mi]; res[mi] = t;
      memcpy(u, Y + (size_t)i * n, sizeof(double) * n);
      memcpy(Y + (size_t)i * n, Y + (size_t)mi * n, sizeof(double) * n);
      memcpy(Y + (size_t)mi * n, u, sizeof(double) * n);
    }
  }
#undef TT
  st->nev = nlock;
  st->niter = its;
  st->nmv = nmv;
  st->nrestart = nrestart;
  st->status = status;
  free(W); free(Z); free(BU); free(TRw); free(TRz); free(T); free(Tw); free(w); free(Yv);
  free(z); free(zw); free(u); free(bu); free(au); free(h); free(thTR); free(sTR);
  return 0;
}
