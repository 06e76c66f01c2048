// Generalized problems A x = lambda B x with B symmetric positive definite
// (Section 2.4). Algorithm alg:LanAB keeps two bases, W (B-orthonormal) and
// Z = B W, so that inner products need no product with B; the filtered form
// applies it to the pencil (B rho(B^(-1) A-hat), B) of eq:gen1, whose product
// step becomes eq:polyapp1: z = rho(A-hat B^(-1)) z_i - beta_i z_{i-1} with
// A-hat = (A - cB)/d. The Chebyshev recurrence in M = A-hat B^(-1) needs, per
// degree step, one solve with B and one product with A (Table tab:itercomp):
// M v = (A u - c v)/d with u = B^(-1) v. Solves with B use the least-squares
// Chebyshev approximation of 1/t on B's spectrum (lsPol, Section 3.1), itself
// a Chebyshev recurrence in B. Non-restart form only: the run ends when the
// sum of the Ritz values >= bar has settled, as for standard problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "context.hpp"
#include "host_poly.hpp"
#include "kernels.hpp"

using namespace evc;

namespace {

__global__ void k_gen_scalars(const double *h1, const double *h2, int idx, const double *nrm2,
                              double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = h1[idx] + h2[idx];
    out[1] = sqrt(nrm2[0]);
  }
}

// One outer degree step of rho(A-hat B^(-1)) v given t = A B^(-1) W:
//   first: Wn = s1 t + s0 W,        Y = c0 W + c1 Wn
//   next : Wn = s1 t + s0 W - Wp,   Y += c1 Wn
template <bool FIRST>
__global__ __launch_bounds__(256) void k_gen_combine(int n, const double *__restrict__ t,
                                                     const double *__restrict__ W,
                                                     const double *Wp, double *Wn, double *Y,
                                                     double s1, double s0, double c0, double c1) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const double w = W[r];
  double wn = s1 * t[r] + s0 * w;
  if (!FIRST) wn -= Wp[r];
  Wn[r] = wn;
  Y[r] = (FIRST ? c0 * w : Y[r]) + c1 * wn;
}

// Chebyshev coefficients of f on [lo, hi] (kind 0: 1/t, kind 1: 1/sqrt(t)),
// from the Chebyshev-Gauss rule with N nodes: c_j = (2 - [j = 0]) / N *
// sum_k f(t_k) cos(j theta_k); cos(j theta) by its three-term recurrence.
void lspol_coef(int kind, double lo, double hi, int deg, double *coef) {
  const int N = 1024;
  const double c = 0.5 * (hi + lo), d = 0.5 * (hi - lo);
  const double pi = 3.14159265358979323846;
  std::fill(coef, coef + deg + 1, 0.0);
  for (int k = 0; k < N; ++k) {
    const double th = pi * (k + 0.5) / N;
    const double x = std::cos(th);
    const double t = c + d * x;
    const double f = kind == 0 ? 1.0 / t : 1.0 / std::sqrt(t);
    double tm1 = 1.0, tj = x;
    coef[0] += f;
    for (int j = 1; j <= deg; ++j) {
      coef[j] += f * tj;
      const double tn = 2.0 * x * tj - tm1;
      tm1 = tj;
      tj = tn;
    }
  }
  coef[0] /= N;
  for (int j = 1; j <= deg; ++j) coef[j] *= 2.0 / N;
}

struct GenSolver {
  evsl_ctx_t ctx = nullptr;
  const evsl_csr_t *A = nullptr, *B = nullptr;
  int n = 0;
  int64_t ld = 0;
  // solves with B: lsPol of 1/t on [blo, bhi]
  double cb = 0, db = 0;
  int kb = 0;
  std::vector<double> bcoef;
  // filter rho (absent for the plain pencil Lanczos of the bounds)
  bool filtered = false;
  double cc = 0, dd = 0, bar = 0, pbound = 0;
  int deg = 0;
  std::vector<double> coef;
  // device
  std::vector<void *> owned;
  double *bcoef_dev = nullptr, *W = nullptr, *Z = nullptr, *zb = nullptr, *wb = nullptr;
  double *u = nullptr, *t = nullptr, *f1 = nullptr, *f2 = nullptr, *s1 = nullptr, *s2 = nullptr;
  double *partial = nullptr, *h1 = nullptr, *h2 = nullptr, *nrm2 = nullptr, *scal = nullptr;
  double *hs = nullptr;
  int m = 0;
  std::vector<double> alpha, beta;
  int its = 0, nmv = 0, nsolve = 0;

  ~GenSolver() {
    for (void *p : owned) dfree(ctx, p);
    if (hs) (void)hipHostFree(hs);
  }
  double *alloc(size_t count) {
    double *p = (double *)dalloc(ctx, sizeof(double) * std::max<size_t>(count, 1));
    owned.push_back(p);
    return p;
  }
  hipStream_t st() const { return ctx->stream; }

  // ncols_max: the most columns a Gram-Schmidt product spans (the basis, or
  // the locked block of the thick-restart form when that is larger)
  void setup(evsl_ctx_t c, const evsl_csr_t *Am, const evsl_csr_t *Bm, const double bb[2],
             int bdeg, int msteps, int ncols_max = 0) {
    ctx = c;
    A = Am;
    B = Bm;
    n = (int)A->n;
    if (B->n != A->n || !(bb[1] > bb[0]) || !(bb[0] > 0.0) || bdeg < 1) fail(EVSL_EINVAL);
    ld = ((int64_t)n + 63) / 64 * 64;
    cb = 0.5 * (bb[1] + bb[0]);
    db = 0.5 * (bb[1] - bb[0]);
    kb = bdeg;
    bcoef.resize(kb + 1);
    lspol_coef(0, bb[0], bb[1], kb, bcoef.data());
    m = msteps;
    bcoef_dev = alloc(kb + 1);
    HC(ctx, hipMemcpyAsync(bcoef_dev, bcoef.data(), sizeof(double) * (kb + 1),
                           hipMemcpyHostToDevice, st()));
    W = alloc((size_t)ld * (m + 1));
    Z = alloc((size_t)ld * (m + 1));
    for (double **p : {&zb, &wb, &u, &t, &f1, &f2, &s1, &s2}) *p = alloc(ld);
    partial = alloc(std::max(evk::gemv_partials(n, std::max(m + 2, ncols_max)),
                             evk::dot_partials(n, 2)));
    h1 = alloc(m + 2);
    h2 = alloc(m + 2);
    nrm2 = alloc(8);
    scal = alloc(8);
    void *p = nullptr;
    HC(ctx, hipHostMalloc(&p, sizeof(double) * (2 * m + 8), hipHostMallocDefault));
    hs = (double *)p;
    HC(ctx, hipStreamSynchronize(st()));
  }

  // y = p_B(B) x ~ B^(-1) x (x is not written; s1, s2 are work).
  void bsolve(const double *x, double *y) {
    const evk::Csr Bc = to_csr(B);
    evk::cheb_vec<double>(st(), Bc, 3, evk::STEP_FIRST, 1.0 / db, -cb / db, x, nullptr, s1, y, ld,
                          1, bcoef_dev, kb + 1, 1);
    const double *wprev = x;
    double *wcur = s1;
    for (int j = 1; j < kb; ++j) {
      double *dst = (wprev == x) ? s2 : const_cast<double *>(wprev);
      evk::cheb_vec<double>(st(), Bc, 3, evk::STEP_NEXT, 2.0 / db, -2.0 * cb / db, wcur, wprev,
                            dst, y, ld, 1, bcoef_dev, kb + 1, j + 1);
      wprev = wcur;
      wcur = dst;
    }
    nsolve++;
  }

  // t = A B^(-1) v
  void a_binv(const double *v) {
    bsolve(v, u);
    const evk::Csr Ac = to_csr(A);
    evk::cheb_vec<double>(st(), Ac, 3, evk::STEP_PLAIN, 1.0, 0.0, u, nullptr, t, nullptr, ld, 1,
                          nullptr, 0, 0);
  }

  // y = rho(A-hat B^(-1)) x, the operator of eq:polyapp1 (x is not written).
  void apply_filter(const double *x, double *y) {
    const int g = (n + 255) / 256;
    a_binv(x);
    hipLaunchKernelGGL(k_gen_combine<true>, dim3(g), dim3(256), 0, st(), n, t, x, nullptr, f1, y,
                       1.0 / dd, -cc / dd, coef[0], coef[1]);
    const double *wprev = x;
    double *wcur = f1;
    for (int j = 1; j < deg; ++j) {
      double *dst = (wprev == x) ? f2 : const_cast<double *>(wprev);
      a_binv(wcur);
      hipLaunchKernelGGL(k_gen_combine<false>, dim3(g), dim3(256), 0, st(), n, t, wcur, wprev,
                         dst, y, 2.0 / dd, -2.0 * cc / dd, 0.0, coef[j + 1]);
      wprev = wcur;
      wcur = dst;
    }
    nmv += deg;
  }

  double *col(double *Bs, int j) const { return Bs + (int64_t)j * ld; }

  // Algorithm alg:LanAB. The subtraction of beta_i z_{i-1} and alpha_i z_i and
  // the full reorthogonalisation are one classical Gram-Schmidt step against
  // all (w_j, z_j), j <= i, made twice: h = W^T z, z -= Z h. Stops after m
  // steps, at an invariant subspace, or when `settled` returns true (tested
  // every ncycle steps on the eigenvalues of T). Returns the dimension.
  template <typename Settled>
  int run(uint64_t seed, int ncycle, Settled settled, bool *converged) {
    hipStream_t s = st();
    const evk::Csr Ac = to_csr(A), Bc = to_csr(B);
    evk::lanczos_start(s, n, seed, 0, wb);
    evk::cheb_vec<double>(s, Bc, 3, evk::STEP_PLAIN, 1.0, 0.0, wb, nullptr, zb, nullptr, ld, 1,
                          nullptr, 0, 0);
    evk::col_dots(s, n, 1, wb, ld, zb, ld, partial, nrm2);
    evk::normalize(s, n, wb, col(W, 0), nrm2, nullptr);
    evk::normalize(s, n, zb, col(Z, 0), nrm2, nullptr);
    alpha.assign(m, 0.0);
    beta.assign(m, 0.0);
    *converged = false;
    int dim = m;
    for (int i = 0; i < m; ++i) {
      its++;
      if (filtered) {
        apply_filter(col(Z, i), zb);
      } else {
        evk::cheb_vec<double>(s, Ac, 3, evk::STEP_PLAIN, 1.0, 0.0, col(W, i), nullptr, zb,
                              nullptr, ld, 1, nullptr, 0, 0);
        nmv++;
      }
      evk::gemv_t(s, n, i + 1, W, ld, zb, partial, h1);
      evk::gemv_n_sub(s, n, i + 1, Z, ld, h1, zb);
      evk::gemv_t(s, n, i + 1, W, ld, zb, partial, h2);
      evk::gemv_n_sub(s, n, i + 1, Z, ld, h2, zb);
      bsolve(zb, wb);
      evk::col_dots(s, n, 1, wb, ld, zb, ld, partial, nrm2);
      hipLaunchKernelGGL(k_gen_scalars, dim3(1), dim3(64), 0, s, h1, h2, i, nrm2, scal);
      evk::normalize(s, n, wb, col(W, i + 1), nrm2, nullptr);
      evk::normalize(s, n, zb, col(Z, i + 1), nrm2, nullptr);
      HC(ctx, hipMemcpyAsync(hs, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      HC(ctx, hipStreamSynchronize(s));
      alpha[i] = hs[0];
      beta[i] = hs[1];
      if (!std::isfinite(alpha[i]) || !std::isfinite(beta[i])) fail(EVSL_ESPECTRUM);
      if (!(beta[i] > 1e-12)) {  // invariant subspace (or an indefinite approximate solve)
        dim = i + 1;
        *converged = true;
        break;
      }
      if ((i + 1) % ncycle == 0 && settled(i + 1)) {
        dim = i + 1;
        *converged = true;
        break;
      }
    }
    return dim;
  }

  // eigenvalues of T_k (tridiagonal), ascending
  std::vector<double> ritz_values(int k) const {
    std::vector<double> d(alpha.begin(), alpha.begin() + k), e(std::max(k - 1, 1), 0.0), w(k);
    std::copy(beta.begin(), beta.begin() + (k - 1), e.begin());
    evh::tridiag_eig(k, d.data(), e.data(), w.data(), nullptr);
    return w;
  }
};

// Thick-restart form for the pencil: Algorithm alg:FiltLanTR in the
// B-inner product, on the bases of the solver above (W B-orthonormal, Z = B W)
// and the filtered step of eq:polyapp1. Locked vectors UL (B-orthonormal)
// are kept with BUL = B UL. Each step makes two classical Gram-Schmidt passes
// against [UL, W_0..W_i] (coefficients from W^T z, updates with Z; for the
// locked block from UL^T z, updates with BUL), which also removes the
// three-term and arrowhead components. T = the kept Ritz values with their
// couplings s_j to index l, then the step coefficients; its tridiagonal form
// comes from evh::ArrowForm. Every reading (candidates >= bar, carried
// early-restart sums, extra restart, two no-candidate restarts end the run,
// at most m - max(Ncycle, 10) kept Ritz vectors) is that of the standard
// thick-restart solver.
struct GenTR {
  GenSolver &g;
  int n;
  int64_t ld;
  double tlo, thi, normA, tol;
  int m, ncycle, nev_cap, max_its;
  uint64_t seed;
  double *UL = nullptr, *BUL = nullptr, *hL1 = nullptr, *hL2 = nullptr;
  std::vector<double> alpha, beta, th_tr, s_tr, lam, res;
  evh::ArrowForm arrow;
  std::vector<double> arrow_d, arrow_e;
  bool arrow_ok = false;
  int nlock = 0, l = 0, i = 0, its = 0, nrand = 0, nocand = 0, nrestart = 0;
  int status = EVSL_OK;
  bool done = false, next_ok = true;
  double t_old = NAN, t_new = NAN;

  explicit GenTR(GenSolver &gs) : g(gs), n(gs.n), ld(gs.ld) {}
  hipStream_t st() const { return g.st(); }
  double *W(int j) const { return g.W + (int64_t)j * ld; }
  double *Z(int j) const { return g.Z + (int64_t)j * ld; }

  void setup() {
    UL = g.alloc((size_t)ld * nev_cap);
    BUL = g.alloc((size_t)ld * nev_cap);
    hL1 = g.alloc(nev_cap + 2);
    hL2 = g.alloc(nev_cap + 2);
    alpha.assign(m + 1, 0.0);
    beta.assign(m + 1, 0.0);
    if (fresh(0, W(0), Z(0)) == 0.0) fail(EVSL_EINVAL);
  }

  // z -= BUL (UL^T z), then z -= Z (W_0..k-1^T z); coefficients into hL, h
  void project_z(double *z, int k, double *hL, double *h) {
    evk::gemv_t(st(), n, nlock, UL, ld, z, g.partial, hL);
    evk::gemv_n_sub(st(), n, nlock, BUL, ld, hL, z);
    evk::gemv_t(st(), n, k, g.W, ld, z, g.partial, h);
    evk::gemv_n_sub(st(), n, k, g.Z, ld, h, z);
  }

  // Random vector from restart block `nrand`, B-orthogonalised twice against
  // the locked vectors and W_0..k-1, B-normalised into (w, z). Returns its
  // B-norm relative to before (0 when it vanished). Synchronous.
  double fresh(int k, double *w, double *z) {
    const evk::Csr Bc = to_csr(g.B);
    hipStream_t s = st();
    evk::lanczos_start(s, n, seed, nrand++, g.wb);
    evk::cheb_vec<double>(s, Bc, 1, evk::STEP_PLAIN, 1.0, 0.0, g.wb, nullptr, g.zb, nullptr, ld, 1,
                          nullptr, 0, 0);
    evk::col_dots(s, n, 1, g.wb, ld, g.zb, ld, g.partial, g.nrm2 + 1);
    for (int pass = 0; pass < 2; ++pass) {
      // w -= UL (BUL^T w), w -= W (Z^T w)
      evk::gemv_t(s, n, nlock, BUL, ld, g.wb, g.partial, hL1);
      evk::gemv_n_sub(s, n, nlock, UL, ld, hL1, g.wb);
      evk::gemv_t(s, n, k, g.Z, ld, g.wb, g.partial, g.h1);
      evk::gemv_n_sub(s, n, k, g.W, ld, g.h1, g.wb);
    }
    evk::cheb_vec<double>(s, Bc, 1, evk::STEP_PLAIN, 1.0, 0.0, g.wb, nullptr, g.zb, nullptr, ld, 1,
                          nullptr, 0, 0);
    evk::col_dots(s, n, 1, g.wb, ld, g.zb, ld, g.partial, g.nrm2);
    HC(g.ctx, hipMemcpyAsync(g.hs, g.nrm2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HC(g.ctx, hipStreamSynchronize(s));
    const double after = std::sqrt(std::max(g.hs[0], 0.0));
    const double before = std::sqrt(std::max(g.hs[1], 0.0));
    if (!(after > 1e-10 * before)) return 0.0;
    evk::normalize(s, n, g.wb, w, g.nrm2, nullptr);
    evk::normalize(s, n, g.zb, z, g.nrm2, nullptr);
    return after / before;
  }

  void tri_form(int k, std::vector<double> &d, std::vector<double> &e) {
    d.assign(k, 0.0);
    e.assign(std::max(k - 1, 1), 0.0);
    if (l > 0) {
      if (!arrow_ok) {
        arrow_d.assign(l + 1, 0.0);
        arrow_e.assign(std::max(l, 1), 0.0);
        arrow.reduce(l, th_tr.data(), s_tr.data(), alpha[l], arrow_d.data(), arrow_e.data());
        arrow_ok = true;
      }
      std::copy(arrow_d.begin(), arrow_d.begin() + (l + 1), d.begin());
      std::copy(arrow_e.begin(), arrow_e.begin() + l, e.begin());
    }
    for (int r = l > 0 ? l + 1 : 0; r < k; ++r) d[r] = alpha[r];
    for (int r = l; r + 1 < k; ++r) e[r] = beta[r];
  }

  void check(const std::vector<double> &w) const {
    for (double x : w)
      if (!(std::fabs(x) <= 1.01 * g.pbound + 1e-12)) fail(EVSL_ESPECTRUM);
  }

  // one Lanczos step of the current cycle (column i -> i + 1)
  void step() {
    hipStream_t s = st();
    its++;
    g.apply_filter(Z(i), g.zb);
    project_z(g.zb, i + 1, hL1, g.h1);
    project_z(g.zb, i + 1, hL2, g.h2);
    g.bsolve(g.zb, g.wb);
    evk::col_dots(s, n, 1, g.wb, ld, g.zb, ld, g.partial, g.nrm2);
    hipLaunchKernelGGL(k_gen_scalars, dim3(1), dim3(64), 0, s, g.h1, g.h2, i, g.nrm2, g.scal);
    evk::normalize(s, n, g.wb, W(i + 1), g.nrm2, nullptr);
    evk::normalize(s, n, g.zb, Z(i + 1), g.nrm2, nullptr);
    HC(g.ctx, hipMemcpyAsync(g.hs, g.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HC(g.ctx, hipStreamSynchronize(s));
    const double a_i = g.hs[0], b_i = g.hs[1];
    if (!std::isfinite(a_i) || !std::isfinite(b_i)) fail(EVSL_ESPECTRUM);
    alpha[i] = a_i;
    bool end_cycle = false;
    next_ok = true;
    if (!(b_i > 1e-12)) {
      // invariant subspace of the filtered operator: new direction, coupling 0
      beta[i] = 0.0;
      if (fresh(i + 1, W(i + 1), Z(i + 1)) == 0.0) {
        next_ok = false;
        end_cycle = true;
      }
    } else {
      beta[i] = b_i;
    }
    if (!end_cycle && ((i + 1) - l) % ncycle == 0) {
      const int k = i + 1;
      std::vector<double> w(k), d, e;
      tri_form(k, d, e);
      evh::tridiag_eig(k, d.data(), e.data(), w.data(), nullptr);
      check(w);
      t_old = t_new;
      t_new = 0.0;
      for (double x : w)
        if (x >= g.bar) t_new += x;
      if (std::fabs(t_new - t_old) < 1e-10 * std::max(1.0, std::fabs(t_new))) end_cycle = true;
    }
    if (its > max_its) end_cycle = true;
    if (!end_cycle && i + 1 >= m) end_cycle = true;
    if (end_cycle) {
      restart(i + 1);
      if (!done && its > max_its) {
        status = EVSL_ENOCONV;
        done = true;
      }
    } else {
      i++;
    }
  }

  void restart(int dim) {
    hipStream_t s = st();
    nrestart++;
    std::vector<double> d, e, w(dim), Ysel((size_t)dim * dim);
    tri_form(dim, d, e);
    const int nsel = evh::tridiag_eig_sel(dim, d.data(), e.data(), w.data(), g.bar, Ysel.data());
    if (l > 0 && nsel > 0) arrow.back(nsel, Ysel.data(), dim);
    arrow_ok = false;
    check(w);
    const int first = dim - nsel;
    const double beta_last = next_ok ? beta[dim - 1] : 0.0;
    const int lc = nsel;
    int naccept = 0;
    std::vector<int> lock_sel, tr_sel;
    std::vector<double> lock_lam, lock_res;
    int cap_tr = m - std::max(ncycle, 10);
    if (cap_tr < 1) cap_tr = 1;
    double *U = nullptr, *BU = nullptr;
    if (lc > 0) {
      // candidates largest first: column t of Yc is Ritz value w[dim - 1 - t]
      std::vector<double> Yh((size_t)dim * lc);
      for (int t = 0; t < lc; ++t) {
        const double *y = Ysel.data() + (size_t)(dim - 1 - t - first) * dim;
        std::copy(y, y + dim, Yh.begin() + (size_t)t * dim);
      }
      U = (double *)ws(g.ctx, 80, sizeof(double) * ld * lc);
      BU = (double *)ws(g.ctx, 81, sizeof(double) * ld * lc);
      double *AU = (double *)ws(g.ctx, 82, sizeof(double) * ld * lc);
      double *Yd = (double *)ws(g.ctx, 83, sizeof(double) * (size_t)dim * lc);
      double *dv = (double *)ws(g.ctx, 84, sizeof(double) * 4 * lc);
      double *pp = (double *)ws(g.ctx, 85, sizeof(double) * evk::dot_partials(n, lc));
      HC(g.ctx, hipMemcpyAsync(Yd, Yh.data(), sizeof(double) * Yh.size(), hipMemcpyHostToDevice, s));
      evk::gemm_nn(s, n, dim, lc, g.W, ld, Yd, dim, U, ld);
      evk::gemm_nn(s, n, dim, lc, g.Z, ld, Yd, dim, BU, ld);
      const evk::Csr Ac = to_csr(g.A);
      evk::cheb_vec<double>(s, Ac, 1, evk::STEP_PLAIN, 1.0, 0.0, U, nullptr, AU, nullptr, ld, lc,
                            nullptr, 0, 0);
      g.nmv += lc;
      double *uau = dv, *ubu = dv + lc, *r2 = dv + 2 * lc, *bb = dv + 3 * lc;
      evk::col_dots(s, n, lc, U, ld, AU, ld, pp, uau);
      evk::col_dots(s, n, lc, U, ld, BU, ld, pp, ubu);
      evk::col_resid2(s, n, lc, BU, AU, ld, uau, ubu, pp, r2);  // ||AU - lambda BU||^2
      evk::col_dots(s, n, lc, BU, ld, BU, ld, pp, bb);
      evk::normalize_cols(s, n, lc, U, ld, ubu);  // B-normalised
      evk::normalize_cols(s, n, lc, BU, ld, ubu);
      std::vector<double> h(4 * lc);
      HC(g.ctx, hipMemcpyAsync(h.data(), dv, sizeof(double) * 4 * lc, hipMemcpyDeviceToHost, s));
      HC(g.ctx, hipStreamSynchronize(s));
      for (int t = 0; t < lc; ++t) {
        const double lamt = h[t] / h[lc + t];
        if (!std::isfinite(lamt)) fail(EVSL_ESPECTRUM);
        if (lamt < tlo || lamt > thi) continue;  // outside the slice: ignored
        naccept++;
        const double r = std::sqrt(std::max(h[2 * lc + t], 0.0)) /
                         (std::sqrt(std::max(h[3 * lc + t], 0.0)) * normA);
        if (r <= tol) {
          lock_sel.push_back(t);
          lock_lam.push_back(lamt);
          lock_res.push_back(r);
        } else if ((int)tr_sel.size() < cap_tr) {
          tr_sel.push_back(t);
        }
      }
      if (nlock + (int)lock_sel.size() > nev_cap) {
        status = EVSL_ENOMEM;
        done = true;
        return;
      }
      for (size_t q = 0; q < lock_sel.size(); ++q) {
        HC(g.ctx, hipMemcpyAsync(UL + (int64_t)nlock * ld, U + (int64_t)lock_sel[q] * ld,
                                 sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        HC(g.ctx, hipMemcpyAsync(BUL + (int64_t)nlock * ld, BU + (int64_t)lock_sel[q] * ld,
                                 sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        lam.push_back(lock_lam[q]);
        res.push_back(lock_res[q]);
        nlock++;
      }
    }
    if (naccept == 0) {
      nocand++;
      th_tr.clear();
      s_tr.clear();
      if (nocand >= 2) {
        done = true;
        return;
      }
      // extra restart: fresh random vector B-orthogonal to the locked set
      l = 0;
      i = 0;
      if (fresh(0, W(0), Z(0)) == 0.0) done = true;
      return;
    }
    nocand = 0;
    // [kept Ritz vectors | w_dim] as the new basis
    if (next_ok) {
      HC(g.ctx, hipMemcpyAsync(g.f1, W(dim), sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      HC(g.ctx, hipMemcpyAsync(g.f2, Z(dim), sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    th_tr.clear();
    s_tr.clear();
    for (size_t q = 0; q < tr_sel.size(); ++q) {
      const int t = tr_sel[q];
      HC(g.ctx, hipMemcpyAsync(W((int)q), U + (int64_t)t * ld, sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s));
      HC(g.ctx, hipMemcpyAsync(Z((int)q), BU + (int64_t)t * ld, sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s));
      th_tr.push_back(w[dim - 1 - t]);
      s_tr.push_back(beta_last * Ysel[(size_t)(dim - 1 - t - first) * dim + (dim - 1)]);
    }
    l = (int)tr_sel.size();
    if (next_ok) {
      HC(g.ctx, hipMemcpyAsync(W(l), g.f1, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      HC(g.ctx, hipMemcpyAsync(Z(l), g.f2, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {
      if (fresh(l, W(l), Z(l)) == 0.0) {
        done = true;
        return;
      }
      std::fill(s_tr.begin(), s_tr.end(), 0.0);
    }
    i = l;
  }
};

}  // namespace

extern "C" {

int evsl_lspol(int kind, double lo, double hi, int deg, double *coef) {
  if ((kind != 0 && kind != 1) || !(hi > lo) || !(lo > 0.0) || deg < 0 || !coef)
    return EVSL_EINVAL;
  lspol_coef(kind, lo, hi, deg, coef);
  return EVSL_OK;
}

int evsl_spectrum_bounds_gen(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_csr_t *B,
                             const double bbounds[2], int bdeg, int nsteps, uint64_t seed,
                             double *lmin, double *lmax) {
  if (!ctx || !bbounds || !lmin || !lmax || nsteps < 1) return EVSL_EINVAL;
  EVSL_GUARD_BEGIN
  check_csr(A);
  check_csr(B);
  if (A->dtype != EVSL_F64 || B->dtype != EVSL_F64) return EVSL_ENOTIMPL;
  GenSolver g;
  const int m = (int)std::min<int64_t>(nsteps, A->n - 1);
  if (m < 1) return EVSL_EINVAL;
  g.setup(ctx, A, B, bbounds, bdeg, m);
  bool conv = false;
  const int dim = g.run(seed, m + 1, [](int) { return false; }, &conv);
  std::vector<double> T((size_t)dim * dim, 0.0), w(dim), Y((size_t)dim * dim);
  for (int i = 0; i < dim; ++i) {
    T[i + (size_t)i * dim] = g.alpha[i];
    if (i + 1 < dim) T[i + (size_t)(i + 1) * dim] = T[(i + 1) + (size_t)i * dim] = g.beta[i];
  }
  evh::sym_eig(dim, T.data(), w.data(), Y.data());
  const double blast = conv ? 0.0 : g.beta[dim - 1];
  *lmin = w[0] - std::fabs(blast * Y[(dim - 1) + 0]);
  *lmax = w[dim - 1] + std::fabs(blast * Y[(dim - 1) + (size_t)(dim - 1) * dim]);
  return EVSL_OK;
  EVSL_GUARD_END
}

int evsl_filtered_lanczos_gen(evsl_ctx_t ctx, const evsl_csr_t *A, const evsl_csr_t *B,
                              const double bbounds[2], int bdeg, const double intv[4],
                              const evsl_pol_t *pol, const evsl_lan_opts_t *opt,
                              evsl_eigs_t *out) {
  if (!ctx || !bbounds || !intv || !pol || !out) return EVSL_EINVAL;
  std::memset(out, 0, sizeof(*out));
  EVSL_GUARD_BEGIN
  check_csr(A);
  check_csr(B);
  if (A->dtype != EVSL_F64 || B->dtype != EVSL_F64) return EVSL_ENOTIMPL;
  if (opt && opt->prec != EVSL_F64) return EVSL_ENOTIMPL;
  if (opt && opt->method != EVSL_LAN_TR && opt->method != EVSL_LAN_NR) return EVSL_EINVAL;
  const bool tr = opt && opt->method == EVSL_LAN_TR;
  const double t0 = now_s();
  double tlo = intv[0], thi = intv[1];
  const double lmin = intv[2], lmax = intv[3];
  if (!(thi > tlo) || !(lmax > lmin) || !pol->coef || pol->deg < 1) return EVSL_EINVAL;
  // a slice that reaches a bound of the spectrum owns every eigenvalue beyond it
  if (tlo <= lmin) tlo = -INFINITY;
  if (thi >= lmax) thi = INFINITY;
  const double normA = std::max(std::fabs(lmin), std::fabs(lmax));
  GenSolver g;
  g.filtered = true;
  g.cc = 0.5 * (lmax + lmin);
  g.dd = 0.5 * (lmax - lmin);
  if (std::fabs(pol->cc - g.cc) > 1e-12 * (1 + std::fabs(g.cc)) ||
      std::fabs(pol->dd - g.dd) > 1e-12 * (1 + std::fabs(g.dd)))
    return EVSL_EINVAL;
  g.deg = pol->deg;
  g.bar = pol->bar;
  g.coef.assign(pol->coef, pol->coef + g.deg + 1);
  for (double c : g.coef) g.pbound += std::fabs(c);
  const int nev_est = (opt && opt->nev_est > 0) ? opt->nev_est : 50;
  int m = (opt && opt->m > 0) ? opt->m
                              : (tr ? std::max(3 * nev_est + 30, 60) : std::max(5 * nev_est + 200, 400));
  m = (int)std::min<int64_t>(m, A->n - 1);
  if (m < 2) return EVSL_EINVAL;
  const int ncycle = (opt && opt->ncycle > 0) ? opt->ncycle : 30;
  const double tol = (opt && opt->tol > 0) ? opt->tol : 1e-8;
  const uint64_t seed = opt ? opt->seed : 0;
  const int nev_cap = (opt && opt->nev_cap > 0) ? opt->nev_cap : std::max(2 * nev_est + 40, 100);
  g.setup(ctx, A, B, bbounds, bdeg, m, tr ? nev_cap : 0);
  if (tr) {
    GenTR t(g);
    t.tlo = tlo;
    t.thi = thi;
    t.normA = normA;
    t.tol = tol;
    t.m = m;
    t.ncycle = ncycle;
    t.nev_cap = nev_cap;
    t.max_its = (opt && opt->max_its > 0) ? opt->max_its : std::max(20 * m, 2000);
    t.seed = seed;
    t.setup();
    while (!t.done) t.step();
    HC(ctx, hipStreamSynchronize(ctx->stream));
    const int k = t.nlock;
    std::vector<int> idx(k);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return t.lam[a] < t.lam[b]; });
    out->nev = k;
    out->lam = (double *)std::malloc(sizeof(double) * std::max(k, 1));
    out->res = (double *)std::malloc(sizeof(double) * std::max(k, 1));
    if (!out->lam || !out->res) fail(EVSL_ENOMEM);
    out->Y = nullptr;
    if (k > 0) out->Y = (double *)dalloc(ctx, sizeof(double) * (size_t)g.n * k);
    for (int j = 0; j < k; ++j) {
      out->lam[j] = t.lam[idx[j]];
      out->res[j] = t.res[idx[j]];
      HC(ctx, hipMemcpyAsync(out->Y + (int64_t)j * g.n, t.UL + (int64_t)idx[j] * g.ld,
                             sizeof(double) * g.n, hipMemcpyDeviceToDevice, ctx->stream));
    }
    HC(ctx, hipStreamSynchronize(ctx->stream));
    out->niter = t.its;
    out->nmv = g.nmv;
    out->nrestart = g.nsolve;  // solves with B
    out->status = t.status == EVSL_ENOMEM ? EVSL_ENOCONV : t.status;
    out->t_tot = now_s() - t0;
    return out->status;
  }
  auto check = [&](const std::vector<double> &w) {
    for (double x : w)
      if (!(std::fabs(x) <= 1.01 * g.pbound + 1e-12)) fail(EVSL_ESPECTRUM);
  };
  double t_old = NAN, t_new = NAN;
  auto settled = [&](int k) {
    const std::vector<double> w = g.ritz_values(k);
    check(w);
    t_old = t_new;
    t_new = 0.0;
    for (double x : w)
      if (x >= g.bar) t_new += x;
    return std::fabs(t_new - t_old) < 1e-10 * std::max(1.0, std::fabs(t_new));
  };
  bool conv = false;
  const int dim = g.run(seed, ncycle, settled, &conv);
  // candidates: Ritz values >= bar; Ritz vectors x = W y (eq:gen1), checked
  // with A and B: lambda = x^T A x / x^T B x, res = ||A x - lambda B x|| /
  // (||B x|| ||A||)
  const std::vector<double> w = g.ritz_values(dim);
  check(w);
  int first = dim;
  while (first > 0 && w[first - 1] >= g.bar) --first;
  const int nc = dim - first;
  std::vector<double> lam, res;
  double *Yout = nullptr;
  if (nc > 0) {
    std::vector<double> d(g.alpha.begin(), g.alpha.begin() + dim), e(std::max(dim - 1, 1), 0.0);
    std::copy(g.beta.begin(), g.beta.begin() + (dim - 1), e.begin());
    std::vector<double> Zc((size_t)dim * nc);
    evh::tridiag_eigvecs(dim, d.data(), e.data(), nc, w.data() + first, Zc.data());
    hipStream_t s = ctx->stream;
    double *U = (double *)dalloc(ctx, sizeof(double) * g.ld * nc);
    double *AU = (double *)dalloc(ctx, sizeof(double) * g.ld * nc);
    double *BU = (double *)dalloc(ctx, sizeof(double) * g.ld * nc);
    double *Yd = (double *)dalloc(ctx, sizeof(double) * (size_t)dim * nc);
    double *dv = (double *)dalloc(ctx, sizeof(double) * 4 * nc);
    double *pp = (double *)dalloc(ctx, sizeof(double) * evk::dot_partials((int)A->n, nc));
    struct Free {
      evsl_ctx_t c;
      std::vector<void *> p;
      ~Free() {
        for (void *q : p) dfree(c, q);
      }
    } fr{ctx, {U, AU, BU, Yd, dv, pp}};
    HC(ctx, hipMemcpyAsync(Yd, Zc.data(), sizeof(double) * Zc.size(), hipMemcpyHostToDevice, s));
    evk::gemm_nn(s, g.n, dim, nc, g.W, g.ld, Yd, dim, U, g.ld);
    const evk::Csr Ac = to_csr(A), Bc = to_csr(B);
    evk::cheb_vec<double>(s, Ac, 1, evk::STEP_PLAIN, 1.0, 0.0, U, nullptr, AU, nullptr, g.ld, nc,
                          nullptr, 0, 0);
    evk::cheb_vec<double>(s, Bc, 1, evk::STEP_PLAIN, 1.0, 0.0, U, nullptr, BU, nullptr, g.ld, nc,
                          nullptr, 0, 0);
    g.nmv += nc;
    double *xax = dv, *xbx = dv + nc, *r2 = dv + 2 * nc, *bb = dv + 3 * nc;
    evk::col_dots(s, g.n, nc, U, g.ld, AU, g.ld, pp, xax);
    evk::col_dots(s, g.n, nc, U, g.ld, BU, g.ld, pp, xbx);
    // ||AU - (xax / xbx) BU||^2 and ||BU||^2
    evk::col_resid2(s, g.n, nc, BU, AU, g.ld, xax, xbx, pp, r2);
    evk::col_dots(s, g.n, nc, BU, g.ld, BU, g.ld, pp, bb);
    evk::normalize_cols(s, g.n, nc, U, g.ld, xbx);  // B-normalised
    std::vector<double> h(4 * nc);
    HC(ctx, hipMemcpyAsync(h.data(), dv, sizeof(double) * 4 * nc, hipMemcpyDeviceToHost, s));
    HC(ctx, hipStreamSynchronize(s));
    std::vector<int> acc;
    for (int c = nc - 1; c >= 0; --c) {  // largest filter values first
      const double l = h[c] / h[nc + c];
      if (!std::isfinite(l)) fail(EVSL_ESPECTRUM);
      if (l < tlo || l > thi) continue;
      const double r = std::sqrt(std::max(h[2 * nc + c], 0.0)) / (std::sqrt(h[3 * nc + c]) * normA);
      if (r > tol) continue;
      if ((int)acc.size() >= nev_cap) break;
      acc.push_back(c);
    }
    std::sort(acc.begin(), acc.end(),
              [&](int a, int b) { return h[a] / h[nc + a] < h[b] / h[nc + b]; });
    if (!acc.empty()) {
      Yout = (double *)dalloc(ctx, sizeof(double) * (size_t)g.n * acc.size());
      for (size_t q = 0; q < acc.size(); ++q) {
        lam.push_back(h[acc[q]] / h[nc + acc[q]]);
        res.push_back(std::sqrt(std::max(h[2 * nc + acc[q]], 0.0)) /
                      (std::sqrt(h[3 * nc + acc[q]]) * normA));
        HC(ctx, hipMemcpyAsync(Yout + (int64_t)q * g.n, U + (int64_t)acc[q] * g.ld,
                               sizeof(double) * g.n, hipMemcpyDeviceToDevice, s));
      }
      HC(ctx, hipStreamSynchronize(s));
    }
  }
  const int k = (int)lam.size();
  out->nev = k;
  out->lam = (double *)std::malloc(sizeof(double) * std::max(k, 1));
  out->res = (double *)std::malloc(sizeof(double) * std::max(k, 1));
  if (!out->lam || !out->res) fail(EVSL_ENOMEM);
  std::copy(lam.begin(), lam.end(), out->lam);
  std::copy(res.begin(), res.end(), out->res);
  out->Y = Yout;
  out->niter = g.its;
  out->nmv = g.nmv;
  out->nrestart = g.nsolve;  // solves with B
  out->status = conv ? EVSL_OK : EVSL_ENOCONV;
  out->t_tot = now_s() - t0;
  return out->status;
  EVSL_GUARD_END
}

}  // extern "C"
