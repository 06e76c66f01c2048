// Filtered subspace iteration (ChebSI; the paper lists it beside the Lanczos
// solvers at the end of Section 2.5 and in Section 3.1, with the block size
// taken from the DOS count). One iteration on a slice's block V (n x b):
//   W = p(A-hat) V                       (block filter, all active slices of a
//                                         batch in one launch per degree step)
//   mu_j = v_j^T w_j                     (filter Rayleigh quotients of V)
//   stop test on (theta, res, mu)        (below)
//   Q = orthonormal basis of span(W)     (SVQB twice: Gram matrix on FP64 MFMA,
//                                         its eigen-decomposition on the host)
//   H = Q^T A Q, H = S diag(theta) S^T   (Rayleigh-Ritz with A)
//   V = Q S, residuals ||A v - theta v|| / ||A||.
// The run stops when the count of converged Ritz pairs inside the slice is
// the same as at the previous test and no unconverged Ritz value inside the
// slice has mu_j >= bar (the filter's value at the slice ends): a wanted
// eigenvector still converging has mu -> p(lambda) >= bar, while a mixture of
// eigenvectors outside the slice has mu < bar.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <vector>

#include "context.hpp"
#include "host_poly.hpp"
#include "kernels.hpp"
#include "polish.hpp"

using namespace evc;

namespace {

struct SiSlice {
  evsl_ctx_t ctx = nullptr;
  const evsl_csr_t *A = nullptr;
  int n = 0;
  int64_t ld = 0;
  double tlo = 0, thi = 0, normA = 0, cc = 0, dd = 0, bar = 0;
  int deg = 0;
  std::vector<double> coef;
  double pbound = 0.0;  // |p(t)| <= sum |coef_j| on [-1, 1]
  int b = 0, max_its = 0;
  double tol = 0;
  uint64_t seed = 0;
  int next_rand = 0;
  // device: V (Ritz vectors), W (filter output / basis), X (work), all n x b
  double *V = nullptr, *W = nullptr, *X = nullptr;
  double *Gd = nullptr, *tnp = nullptr, *dots = nullptr, *partial = nullptr;
  double *hbuf = nullptr;  // pinned host: 3 b
  std::vector<double> th, rs, mu;
  int its = 0, nmv = 0, prev = -1, status = EVSL_OK, nrefill = 0;
  bool have_ritz = false, done = false;
  double t_mv = 0, t_orth = 0, t_ritz = 0, t_done = 0;

  SiSlice() = default;
  SiSlice(const SiSlice &) = delete;
  SiSlice &operator=(const SiSlice &) = delete;
  bool own_v = true;  // false in the polish: V is the caller's block
  ~SiSlice() {
    if (own_v) dfree(ctx, V);
    for (double *p : {W, X, Gd, tnp, dots, partial}) dfree(ctx, p);
    if (hbuf) (void)hipHostFree(hbuf);
  }

  hipStream_t st() const { return ctx->stream; }
  double *col(double *B, int j) const { return B + (int64_t)j * ld; }

  void setup(evsl_ctx_t c, const evsl_csr_t *Am, const double intv[4], const evsl_pol_t *pol,
             const evsl_si_opts_t *opt) {
    ctx = c;
    A = Am;
    n = (int)Am->n;
    tlo = intv[0];
    thi = intv[1];
    const double lmin = intv[2], lmax = intv[3];
    if (!(thi > tlo) || !(lmax > lmin) || !pol || !pol->coef || pol->deg < 1) fail(EVSL_EINVAL);
    // a slice that reaches a bound of the spectrum owns every eigenvalue beyond it
    if (tlo <= lmin) tlo = -INFINITY;
    if (thi >= lmax) thi = INFINITY;
    normA = std::max(std::fabs(lmin), std::fabs(lmax));
    cc = 0.5 * (lmax + lmin);
    dd = 0.5 * (lmax - lmin);
    if (std::fabs(pol->cc - cc) > 1e-12 * (1 + std::fabs(cc)) ||
        std::fabs(pol->dd - dd) > 1e-12 * (1 + std::fabs(dd)))
      fail(EVSL_EINVAL);
    bar = pol->bar;
    deg = pol->deg;
    coef.assign(pol->coef, pol->coef + deg + 1);
    pbound = 0.0;
    for (double c : coef) pbound += std::fabs(c);
    const int nev_est = (opt && opt->nev_est > 0) ? opt->nev_est : 50;
    b = (opt && opt->block > 0) ? opt->block : 3 * nev_est + 8;
    b = std::min(b, n);
    max_its = (opt && opt->max_its > 0) ? opt->max_its : 100;
    tol = (opt && opt->tol > 0) ? opt->tol : 1e-8;
    seed = opt ? opt->seed : 0;
    alloc_buffers();
    // start block: column j is the start vector of restart block j
    next_rand = b;
    for (int j = 0; j < b; ++j) evk::lanczos_start(st(), n, seed, j, col(V, j));
    orthonormalise(V);
  }

  // The precision form's FP64 phase on one slice: the block is the job's k
  // vectors, refined in place (take_back compacts the in-slice pairs).
  void setup_polish(evsl_ctx_t c, const evsl_csr_t *Am, const evsi::PolishJob &job, double cc_,
                    double dd_) {
    ctx = c;
    A = Am;
    n = (int)Am->n;
    tlo = job.tlo;
    thi = job.thi;
    normA = job.normA;
    cc = cc_;
    dd = dd_;
    bar = job.bar;
    deg = job.deg;
    coef.assign(job.coef, job.coef + deg + 1);
    pbound = 0.0;
    for (double x : coef) pbound += std::fabs(x);
    b = job.k;
    if (b < 1 || b > n || job.ldv != ((int64_t)n + 63) / 64 * 64) fail(EVSL_EINVAL);
    tol = job.tol;
    seed = job.seed;
    own_v = false;
    V = job.V;
    alloc_buffers();
    // refill vectors (rank deficiency only) from a part of the stream that the
    // Lanczos start vectors do not reach
    next_rand = 1 << 20;
  }

  // Ritz pairs inside the slice after a Rayleigh-Ritz step: count and
  // converged count
  void count_in(int &nin, int &nconv) const {
    nin = nconv = 0;
    for (int j = 0; j < b; ++j) {
      if (th[j] < tlo || th[j] > thi) continue;
      nin++;
      if (rs[j] <= tol) nconv++;
    }
  }

  // The in-slice Ritz pairs (ascending) into the job: vectors to its first
  // columns, values and residuals to lam and res.
  void take_back(evsi::PolishJob &job) {
    job.lam.clear();
    job.res.clear();
    int t = 0;
    for (int j = 0; j < b; ++j) {
      if (th[j] < tlo || th[j] > thi) continue;
      job.lam.push_back(th[j]);
      job.res.push_back(rs[j]);
      // in place: column t <= j, and columns below j were read before
      if (job.V + (int64_t)t * job.ldv != col(V, j))
        HC(ctx, hipMemcpyAsync(job.V + (int64_t)t * job.ldv, col(V, j), sizeof(double) * n,
                               hipMemcpyDeviceToDevice, st()));
      t++;
    }
    count_in(job.nin, job.nconv);
    job.ok = job.nconv == job.nin;
    job.nfilter = its;
    job.nmv = nmv;
    job.t_mv = t_mv;
    job.t_ritz = t_ritz;
    HC(ctx, hipStreamSynchronize(st()));
  }

  void alloc_buffers() {
    ld = ((int64_t)n + 63) / 64 * 64;
    if (own_v) V = (double *)dalloc(ctx, sizeof(double) * ld * b);
    W = (double *)dalloc(ctx, sizeof(double) * ld * b);
    X = (double *)dalloc(ctx, sizeof(double) * ld * b);
    Gd = (double *)dalloc(ctx, sizeof(double) * (size_t)b * b);
    tnp = (double *)dalloc(ctx, sizeof(double) * evk::gemm_tn_partials_bound(n, b, b));
    dots = (double *)dalloc(ctx, sizeof(double) * (3 * b + 8));
    partial = (double *)dalloc(ctx, sizeof(double) * evk::dot_partials(n, b));
    void *hp = nullptr;
    HC(ctx, hipHostMalloc(&hp, sizeof(double) * (3 * b + 8), hipHostMallocDefault));
    hbuf = (double *)hp;
    th.assign(b, 0.0);
    rs.assign(b, 0.0);
    mu.assign(b, 0.0);
  }

  // One SVQB pass on the b columns of B: B <- B D U_k diag(w_k)^(-1/2) from
  // the eigen-decomposition of the unit-diagonal Gram matrix D B^T B D; keeps
  // the directions with w > 1e-14 and returns their number (in the first
  // columns of B; B and X swap roles).
  int svqb(double *&B) {
    hipStream_t s = st();
    evk::gemm_tn(s, n, b, b, B, ld, B, ld, Gd, b, tnp);
    std::vector<double> G((size_t)b * b), U((size_t)b * b), w(b), d(b);
    HC(ctx, hipMemcpyAsync(G.data(), Gd, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
    HC(ctx, hipStreamSynchronize(s));
    for (int j = 0; j < b; ++j) d[j] = G[j + (size_t)j * b] > 0 ? 1.0 / std::sqrt(G[j + (size_t)j * b]) : 0.0;
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) G[i + (size_t)j * b] *= d[i] * d[j];
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < j; ++i) {
        const double a = 0.5 * (G[i + (size_t)j * b] + G[j + (size_t)i * b]);
        G[i + (size_t)j * b] = G[j + (size_t)i * b] = a;
      }
    evh::sym_eig(b, G.data(), w.data(), U.data());
    std::vector<double> M((size_t)b * b, 0.0);
    int k = 0;
    for (int c = b - 1; c >= 0; --c) {
      if (!(w[c] > 1e-14)) break;
      const double sw = 1.0 / std::sqrt(w[c]);
      for (int r = 0; r < b; ++r) M[r + (size_t)k * b] = d[r] * U[r + (size_t)c * b] * sw;
      k++;
    }
    if (k == 0) return 0;
    HC(ctx, hipMemcpyAsync(Gd, M.data(), sizeof(double) * (size_t)b * k, hipMemcpyHostToDevice, s));
    evk::gemm_nn(s, n, b, k, B, ld, Gd, b, X, ld);
    HC(ctx, hipStreamSynchronize(s));
    std::swap(B, X);
    return k;
  }

  // Orthonormal basis of span(B) in B (two SVQB passes); directions lost to
  // rank deficiency are replaced by the next random vectors of the stream.
  void orthonormalise(double *&B) {
    for (int attempt = 0; attempt < 3; ++attempt) {
      const int k = svqb(B);
      if (k == b) break;
      for (int j = k; j < b; ++j) evk::lanczos_start(st(), n, seed, next_rand++, col(B, j));
      nrefill += b - k;
    }
    if (svqb(B) != b) fail(EVSL_ESPECTRUM);
  }

  // Host part after W = p(A-hat) V has been computed on the stream.
  void after_filter() {
    its++;
    nmv += deg * b;
    hipStream_t s = st();
    if (have_ritz) {
      evk::col_dots(s, n, b, V, ld, W, ld, partial, dots);
      HC(ctx, hipMemcpyAsync(hbuf, dots, sizeof(double) * b, hipMemcpyDeviceToHost, s));
      HC(ctx, hipStreamSynchronize(s));
      int nin = 0, nconv = 0, bad = 0;
      for (int j = 0; j < b; ++j) {
        mu[j] = hbuf[j];
        // a filter Rayleigh quotient beyond the bound of p on [-1, 1]: the
        // spectrum leaves [lambda_min, lambda_max]
        if (!(std::fabs(mu[j]) <= 1.01 * pbound + 1e-12)) fail(EVSL_ESPECTRUM);
        if (th[j] < tlo || th[j] > thi) continue;
        nin++;
        if (rs[j] <= tol)
          nconv++;
        else if (mu[j] >= bar)
          bad++;
      }
      if (nin == b) {  // the slice fills the subspace: the block is too small
        status = EVSL_ENOCONV;
        done = true;
        return;
      }
      if (nconv == prev && bad == 0) {
        done = true;
        return;
      }
      prev = nconv;
    }
    const double t0 = now_s();
    rayleigh_ritz();
    t_ritz += now_s() - t0;
    have_ritz = true;
    if (its >= max_its) {
      status = EVSL_ENOCONV;
      done = true;
    }
  }

  void rayleigh_ritz() {
    hipStream_t s = st();
    orthonormalise(W);  // W = Q
    // X = A Q
    const evk::Csr Ac = to_csr(A);
    evk::cheb_vec<double>(s, Ac, 1, evk::STEP_PLAIN, 1.0, 0.0, W, nullptr, X, nullptr, ld, b,
                          nullptr, 0, 0);
    nmv += b;
    evk::gemm_tn(s, n, b, b, W, ld, X, ld, Gd, b, tnp);
    std::vector<double> H((size_t)b * b), S((size_t)b * b);
    HC(ctx, hipMemcpyAsync(H.data(), Gd, sizeof(double) * H.size(), hipMemcpyDeviceToHost, s));
    HC(ctx, hipStreamSynchronize(s));
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < j; ++i) {
        const double a = 0.5 * (H[i + (size_t)j * b] + H[j + (size_t)i * b]);
        H[i + (size_t)j * b] = H[j + (size_t)i * b] = a;
      }
    evh::sym_eig(b, H.data(), th.data(), S.data());
    HC(ctx, hipMemcpyAsync(Gd, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s));
    // V = Q S, then A V = (A Q) S written over Q
    evk::gemm_nn(s, n, b, b, W, ld, Gd, b, V, ld);
    evk::gemm_nn(s, n, b, b, X, ld, Gd, b, W, ld);
    double *xx = dots, *xax = dots + b, *rr = dots + 2 * b;
    evk::col_dots(s, n, b, V, ld, V, ld, partial, xx);
    evk::col_dots(s, n, b, V, ld, W, ld, partial, xax);
    evk::col_resid2(s, n, b, V, W, ld, xax, xx, partial, rr);
    HC(ctx, hipMemcpyAsync(hbuf, dots, sizeof(double) * 3 * b, hipMemcpyDeviceToHost, s));
    HC(ctx, hipStreamSynchronize(s));
    for (int j = 0; j < b; ++j) {
      if (!std::isfinite(hbuf[b + j])) fail(EVSL_ESPECTRUM);
      rs[j] = std::sqrt(std::max(hbuf[2 * b + j], 0.0) / hbuf[j]) / normA;
    }
  }

  void emit(evsl_eigs_t *out) {
    HC(ctx, hipStreamSynchronize(st()));
    std::vector<int> keep;
    if (have_ritz)
      for (int j = 0; j < b; ++j)
        if (th[j] >= tlo && th[j] <= thi && rs[j] <= tol) keep.push_back(j);
    const int k = (int)keep.size();  // theta ascending from the eigensolver
    out->nev = k;
    out->lam = (double *)std::malloc(sizeof(double) * std::max(k, 1));
    out->res = (double *)std::malloc(sizeof(double) * std::max(k, 1));
    if (!out->lam || !out->res) fail(EVSL_ENOMEM);
    out->Y = nullptr;
    if (k > 0) out->Y = (double *)dalloc(ctx, sizeof(double) * (size_t)n * k);
    for (int j = 0; j < k; ++j) {
      out->lam[j] = th[keep[j]];
      out->res[j] = rs[keep[j]];
      HC(ctx, hipMemcpyAsync(out->Y + (int64_t)j * n, col(V, keep[j]), sizeof(double) * n,
                             hipMemcpyDeviceToDevice, st()));
    }
    HC(ctx, hipStreamSynchronize(st()));
    out->niter = its;
    out->nmv = nmv;
    out->nrestart = nrefill;
    out->npolish = 0;
    out->status = status;
    out->t_mv = t_mv;
    out->t_orth = t_orth;
    out->t_ritz = t_ritz;
  }
};

// W = p_q(A-hat) V for every column of a batch of slices (in non-increasing
// degree), as block Clenshaw recurrences over chunks of at most `chunk`
// consecutive columns: a chunk's columns are gathered into a row-major block,
// B_k is written over B_{k+2} (four passes per degree step), columns join as k
// reaches their slice's degree, and the result is scattered back to each
// slice's W. Buffers: workspace slots 70-74, sized for one chunk and degree
// kmax.
struct BlockFilter {
  evsl_ctx_t ctx;
  const evsl_csr_t *A;
  evk::Csr Ac;
  int n;
  double cc, dd;
  int chunk;
  double *X0 = nullptr, *X1 = nullptr, *Yb = nullptr, *ctab = nullptr;
  double **ptrs = nullptr;
  void *hpin = nullptr;
  std::vector<double> tab;
  std::vector<int> ncs;

  BlockFilter(evsl_ctx_t c, const evsl_csr_t *Am, double cc_, double dd_, int cols, int kmax,
              int max_chunk)
      : ctx(c), A(Am), n((int)Am->n), cc(cc_), dd(dd_),
        chunk(std::max(1, std::min(cols, max_chunk))) {
    const int64_t ldb_max = (chunk + 1) / 2 * 2;  // even: two FP64 columns per lane
    X0 = (double *)ws(ctx, 70, sizeof(double) * (size_t)n * ldb_max);
    X1 = (double *)ws(ctx, 71, sizeof(double) * (size_t)n * ldb_max);
    Yb = (double *)ws(ctx, 72, sizeof(double) * (size_t)n * ldb_max);
    ctab = (double *)ws(ctx, 73, sizeof(double) * (size_t)chunk * (kmax + 1));
    ptrs = (double **)ws(ctx, 74, sizeof(double *) * 2 * (size_t)chunk);
    HC(ctx, hipHostMalloc(&hpin, sizeof(double *) * 2 * (size_t)chunk, hipHostMallocDefault));
    Ac = to_csr(A);
    attach_col_offsets(ctx, A, Ac);
    ncs.resize(kmax + 2);
  }
  BlockFilter(const BlockFilter &) = delete;
  BlockFilter &operator=(const BlockFilter &) = delete;
  ~BlockFilter() {
    if (hpin) (void)hipHostFree(hpin);
  }

  // Filters the V columns of `act` into their W; returns the wall time and
  // adds it to each slice's t_mv.
  double run(const std::vector<SiSlice *> &act) {
    hipStream_t s = ctx->stream;
    const double **hp = (const double **)hpin;
    struct ColRef {
      SiSlice *q;
      int j;
    };
    std::vector<ColRef> all;
    for (SiSlice *q : act)
      for (int j = 0; j < q->b; ++j) all.push_back({q, j});
    const int ntot = (int)all.size();
    const double tf0 = now_s();
    for (int c0 = 0; c0 < ntot; c0 += chunk) {
      const int nc = std::min(chunk, ntot - c0);
      int km = 0;
      for (int c = 0; c < nc; ++c) km = std::max(km, all[c0 + c].q->deg);
      const int64_t ldb = (nc + 1) / 2 * 2;
      tab.assign((size_t)nc * (km + 1), 0.0);
      for (int c = 0; c < nc; ++c) {
        SiSlice *q = all[c0 + c].q;
        std::copy(q->coef.begin(), q->coef.end(), tab.begin() + (size_t)c * (km + 1));
        hp[c] = q->col(q->V, all[c0 + c].j);
        hp[nc + c] = q->col(q->W, all[c0 + c].j);
      }
      // columns in non-increasing degree: those active at step k are a prefix
      for (int k = 0; k <= km; ++k) {
        int a = 0;
        while (a < nc && all[c0 + a].q->deg >= k) ++a;
        ncs[k] = std::max(a, 1);
      }
      HC(ctx, hipMemcpyAsync(ctab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice,
                             s));
      HC(ctx, hipMemcpyAsync(ptrs, hp, sizeof(double *) * 2 * nc, hipMemcpyHostToDevice, s));
      FilterTimer tm(ctx);
      evk::gather_cols<double>(s, n, nc, (const double *const *)ptrs, X0, ldb);
      evk::fill_zero<double>(s, (int64_t)n * ldb, X1);
      evk::fill_zero<double>(s, (int64_t)n * ldb, Yb);
      double bytes = 2.0 * (double)n * (double)ldb * 8.0;
      double *bk1 = X1, *bk2 = Yb;
      for (int k = km; k >= 0; --k) {
        const double sc = k > 0 ? 2.0 : 1.0;
        evk::cheb_blk<double>(s, Ac, evk::STEP_CLEN, sc / dd, -sc * cc / dd, bk1, bk2, bk2,
                              nullptr, ldb, ncs[k], ctab, km + 1, k, X0, nullptr,
                              &ctx->blk_sched);
        bytes += step_bytes(A, ncs[k], 8, 4);
        std::swap(bk1, bk2);
      }
      evk::scatter_cols<double>(s, n, nc, bk1, ldb, (double *const *)(ptrs + nc));
      tm.stop(km + 1, bytes);
      // the staging buffers are reused by the next chunk: wait for them
      HC(ctx, hipStreamSynchronize(s));
    }
    const double tf = now_s() - tf0;
    for (SiSlice *q : act) q->t_mv += tf;
    return tf;
  }
};

// Columns per block recurrence in the polish: bounds its row-major buffers
// (3 n x 32 FP64) whatever the block size, at a few percent more reads of A.
constexpr int kPolishChunk = 32;

// The precision form's FP64 phase on a group of jobs (see polish.hpp).
void polish_group(evsl_ctx_t ctx, const evsl_csr_t *A, double cc, double dd, int max_filter,
                  const std::vector<evsi::PolishJob *> &jobs, size_t j0, size_t j1, int cols) {
  const size_t nj = j1 - j0;
  const char *trace_env = std::getenv("EVSL_TRACE");
  const bool progress = trace_env && std::atoi(trace_env) > 0;
  std::vector<SiSlice> sl(nj);
  int kmax = 0;
  for (size_t t = 0; t < nj; ++t) {
    sl[t].setup_polish(ctx, A, *jobs[j0 + t], cc, dd);
    kmax = std::max(kmax, sl[t].deg);
  }
  // Rayleigh-Ritz with A on the span of the FP32-phase vectors
  std::vector<char> ok(nj, 0);
  for (size_t t = 0; t < nj; ++t) {
    SiSlice &q = sl[t];
    HC(ctx, hipMemcpyAsync(q.W, q.V, sizeof(double) * q.ld * q.b, hipMemcpyDeviceToDevice,
                           q.st()));
    const double t0 = now_s();
    q.rayleigh_ritz();
    q.t_ritz += now_s() - t0;
    int nin, nconv;
    q.count_in(nin, nconv);
    ok[t] = nconv == nin;
    if (progress)
      std::fprintf(stderr, "[evsl] polish: %d vectors, Rayleigh-Ritz: %d in the slice, %d at tol\n",
                   q.b, nin, nconv);
  }
  // then FP64 filter applications (subspace iteration), all unfinished
  // slices of the group in one block recurrence, in non-increasing degree
  std::vector<size_t> order(nj);
  std::iota(order.begin(), order.end(), (size_t)0);
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return sl[a].deg > sl[b].deg; });
  std::vector<SiSlice *> act;
  std::unique_ptr<BlockFilter> bf;
  for (int it = 0; it < max_filter; ++it) {
    act.clear();
    for (size_t t : order)
      if (!ok[t]) act.push_back(&sl[t]);
    if (act.empty()) break;
    if (!bf) bf.reset(new BlockFilter(ctx, A, cc, dd, cols, kmax, kPolishChunk));
    bf->run(act);
    for (size_t t : order) {
      if (ok[t]) continue;
      SiSlice &q = sl[t];
      q.its++;
      q.nmv += q.deg * q.b;
      const double t0 = now_s();
      q.rayleigh_ritz();
      q.t_ritz += now_s() - t0;
      int nin, nconv;
      q.count_in(nin, nconv);
      ok[t] = nconv == nin;
      if (progress)
        std::fprintf(stderr, "[evsl] polish: filter %d (degree %d): %d in the slice, %d at tol\n",
                     q.its, q.deg, nin, nconv);
    }
  }
  for (size_t t = 0; t < nj; ++t) sl[t].take_back(*jobs[j0 + t]);
}

}  // namespace

namespace evsi {

void polish(evsl_ctx_t ctx, const evsl_csr_t *A, double cc, double dd, int max_filter,
            const std::vector<PolishJob *> &jobs) {
  // one slice at a time: a slice's block (about its eigenvalue count, tens to
  // hundreds of columns) already shares each read of A over its columns, and
  // the device memory stays that of one slice
  for (size_t j = 0; j < jobs.size(); ++j)
    polish_group(ctx, A, cc, dd, max_filter, jobs, j, j + 1, jobs[j]->k);
  // the block buffers are the polish's alone: they do not outlive it
  for (int slot = 70; slot <= 74; ++slot) ws_release(ctx, slot);
}

}  // namespace evsi

extern "C" {

int evsl_filtered_subspace_batch(evsl_ctx_t ctx, const evsl_csr_t *A, int nslices,
                                 const double *intv, const evsl_pol_t *pols,
                                 const evsl_si_opts_t *opts, evsl_eigs_t *outs) {
  if (!ctx || nslices < 1 || !intv || !pols || !outs) return EVSL_EINVAL;
  for (int q = 0; q < nslices; ++q) std::memset(&outs[q], 0, sizeof(outs[q]));
  EVSL_GUARD_BEGIN
  check_csr(A);
  if (A->dtype != EVSL_F64) return EVSL_ENOTIMPL;
  const double t0 = now_s();
  std::vector<SiSlice> sl(nslices);
  for (int q = 0; q < nslices; ++q)
    sl[q].setup(ctx, A, intv + 4 * q, &pols[q], opts ? &opts[q] : nullptr);
  const double cc = sl[0].cc, dd = sl[0].dd;
  for (int q = 1; q < nslices; ++q)
    if (std::fabs(sl[q].cc - cc) > 1e-13 * (1 + std::fabs(cc)) ||
        std::fabs(sl[q].dd - dd) > 1e-13 * (1 + std::fabs(dd)))
      return EVSL_EINVAL;
  // slices in non-increasing degree: the active columns form a shrinking prefix
  std::vector<int> order(nslices);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sl[a].deg > sl[b].deg; });
  int btot = 0, kmax = 0;
  for (auto &x : sl) {
    btot += x.b;
    kmax = std::max(kmax, x.deg);
  }
  BlockFilter bf(ctx, A, cc, dd, btot, kmax, btot);
  const char *prog_env = std::getenv("EVSL_PROGRESS");
  const bool progress = prog_env && std::atoi(prog_env) > 0;
  int iteration = 0;
  std::vector<SiSlice *> act;
  while (true) {
    act.clear();
    for (int q : order)
      if (!sl[q].done) act.push_back(&sl[q]);
    if (act.empty()) break;
    bf.run(act);
    int nc = 0;
    for (SiSlice *q : act) {
      nc += q->b;
      q->after_filter();
      if (q->done) q->t_done = now_s() - t0;
    }
    ++iteration;
    if (progress) {
      int ndone = 0;
      for (auto &x : sl) ndone += x.done ? 1 : 0;
      std::fprintf(stderr, "[evsl] subspace iteration %d: %d columns filtered, %d of %d slices done, %.1f s\n",
                   iteration, nc, ndone, nslices, now_s() - t0);
    }
  }
  int rc = EVSL_OK;
  for (int q = 0; q < nslices; ++q) {
    sl[q].emit(&outs[q]);
    outs[q].t_tot = sl[q].t_done;
    if (outs[q].status != EVSL_OK) rc = outs[q].status;
  }
  return rc;
  EVSL_GUARD_END
}

int evsl_filtered_subspace(evsl_ctx_t ctx, const evsl_csr_t *A, const double intv[4],
                           const evsl_pol_t *pol, const evsl_si_opts_t *opt, evsl_eigs_t *out) {
  if (!intv || !pol || !out) return EVSL_EINVAL;
  return evsl_filtered_subspace_batch(ctx, A, 1, intv, pol, opt, out);
}

}  // extern "C"
