// Library-internal: the FP64 phase of the precision form (not part of the
// C-ABI). The FP32-filter Lanczos phase ends with Ritz vectors whose error
// has two parts: mixing among the slice's own eigenvectors (the FP32 filter
// perturbs a filtered spectrum whose values inside the slice lie close
// together), which a Rayleigh-Ritz projection with A removes exactly, and
// components along eigenvectors outside the slice, which the slice's filter
// damps. So the block of FP32-phase vectors is refined in FP64 by
// Rayleigh-Ritz with A, then, for slices where pairs still miss the
// tolerance, by iterations of the filtered subspace iteration (Section 2.5,
// ChebSI, Section 3.1) started from that block.
#pragma once
#include <cstdint>
#include <vector>

#include "context.hpp"

namespace evsi {

struct PolishJob {
  // in: k FP64 vectors (device, column-major, leading dimension ldv), refined
  // in place
  double *V = nullptr;
  int64_t ldv = 0;
  int k = 0;
  double tlo = 0, thi = 0;  // the slice (a bound of the spectrum widened to +-inf)
  double normA = 0, bar = 0, tol = 0;
  int deg = 0;
  const double *coef = nullptr;  // deg + 1 Chebyshev coefficients (host)
  uint64_t seed = 0;
  // out: the Ritz pairs inside the slice, ascending, vectors in V[:, 0, nin)
  int nin = 0, nconv = 0;
  int nfilter = 0;  // FP64 filter applications
  int nmv = 0;
  bool ok = false;  // every Ritz pair inside the slice meets tol
  std::vector<double> lam, res;
  double t_mv = 0, t_ritz = 0;
};

// Refines every job (all with the same cc, dd), one after another:
// Rayleigh-Ritz with A on the span of its vectors, then up to max_filter FP64
// filter applications (one block Clenshaw recurrence over its k columns),
// each followed by Rayleigh-Ritz, until every Ritz pair inside the slice
// meets tol. The job's vectors are refined in place. Device memory, for the
// job in progress: two FP64 n-vectors per column (its filtered block and a
// work block), three row-major n x 32 blocks (the recurrence runs over chunks
// of at most 32 columns), its Gram matrix and partial sums; freed on return.
void polish(evsl_ctx_t ctx, const evsl_csr_t *A, double cc, double dd, int max_filter,
            const std::vector<PolishJob *> &jobs);

}  // namespace evsi
