// HIP kernels for gfx950 (MI355X): the Chebyshev filter recurrence over CSR
// (Section 2.2.1, eq:Cheb0, eq:mapping), the reductions of the Lanczos step
// (eq:3term with full reorthogonalisation, Section 2.3), and helpers.
//
// All reductions use a fixed order (per-lane sums in index order, a fixed
// butterfly inside the 64-wide wavefront, wave partials summed in wave order,
// then workgroup partials summed in workgroup order), so every result is
// reproducible bit for bit for a given problem size and launch shape.
#include "kernels.hpp"

#include <algorithm>

namespace evk {

static constexpr int TPB = 256;  // 4 wavefronts of 64

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a workgroup; valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds4[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  return s;
}

// ---------------------------------------------------------------- SplitMix64
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Remapping gives XCD x a contiguous range of logical blocks, so rows
// that are neighbours in the matrix (and read each other's vector entries)
// are processed by the same XCD, one after another.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int x = bid & 7, local = bid >> 3;
  const int q = nblk >> 3, rem = nblk & 7;
  return x * q + min(x, rem) + local;
}

// ---------------------------------------------------------------- filter step, single vectors
// One row per thread; grid.y selects the column of a column-major multivector.
template <typename T, int KIND>
__global__ __launch_bounds__(TPB) void k_cheb_vec_direct(int n, const int *__restrict__ rp,
                                                         const int *__restrict__ ci,
                                                         const T *__restrict__ va, T s1, T s0,
                                                         const T *__restrict__ W, const T *Wp,
                                                         T *Wn, T *Y, int64_t ld,
                                                         const double *__restrict__ coef,
                                                         int cld, int jnext, const T *__restrict__ Vd) {
  constexpr bool IS_CLEN = (KIND == STEP_CLEN);
  constexpr bool HAS_PREV = (KIND == STEP_NEXT || IS_CLEN);
  constexpr bool HAS_Y = (KIND == STEP_FIRST || KIND == STEP_NEXT);
  constexpr bool Y_INIT = (KIND == STEP_FIRST);
  const int r = blockIdx.x * TPB + threadIdx.x;
  if (r >= n) return;
  const int64_t off = (int64_t)blockIdx.y * ld;
  const T *w = W + off;
  T acc = 0;
  const int kb = rp[r], ke = rp[r + 1];
  for (int k = kb; k < ke; ++k) acc += va[k] * w[ci[k]];
  const T wr = w[r];
  T wn = s1 * acc + s0 * wr;
  if (HAS_PREV) wn -= Wp[off + r];
  if (IS_CLEN) wn += (T)coef[(int64_t)blockIdx.y * cld + jnext] * Vd[off + r];
  Wn[off + r] = wn;
  if (HAS_Y) {
    const double *cc = coef + (int64_t)blockIdx.y * cld;
    const T y = Y_INIT ? (T)cc[0] * wr : Y[off + r];
    Y[off + r] = y + (T)cc[jnext] * wn;
  }
}

// LDS-staged CSR stream: the workgroup's 256 rows of row_ptr, col and val are
// loaded into LDS with coalesced loads, then each thread sums its row from LDS.
// Falls back to direct reads when the rows hold more than CAP entries.
template <typename T, int KIND>
__global__ __launch_bounds__(TPB) void k_cheb_vec_lds(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const T *__restrict__ va, T s1, T s0,
                                                      const T *__restrict__ W, const T *Wp, T *Wn,
                                                      T *Y, int64_t ld,
                                                      const double *__restrict__ coef, int cld,
                                                      int jnext, const T *__restrict__ Vd) {
  constexpr int CAP = 2048;
  constexpr bool IS_CLEN = (KIND == STEP_CLEN);
  constexpr bool HAS_PREV = (KIND == STEP_NEXT || IS_CLEN);
  constexpr bool HAS_Y = (KIND == STEP_FIRST || KIND == STEP_NEXT);
  constexpr bool Y_INIT = (KIND == STEP_FIRST);
  __shared__ int s_rp[TPB + 1];
  __shared__ int s_ci[CAP];
  __shared__ T s_va[CAP];
  const int r0 = blockIdx.x * TPB;
  const int nr = min(TPB, n - r0);
  for (int i = threadIdx.x; i <= nr; i += TPB) s_rp[i] = rp[r0 + i];
  __syncthreads();
  const int nz0 = s_rp[0];
  const int cnt = s_rp[nr] - nz0;
  const bool staged = cnt <= CAP;
  if (staged) {
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      s_ci[i] = ci[nz0 + i];
      s_va[i] = va[nz0 + i];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= nr) return;
  const int r = r0 + t;
  const int64_t off = (int64_t)blockIdx.y * ld;
  const T *w = W + off;
  T acc = 0;
  const int kb = s_rp[t], ke = s_rp[t + 1];
  if (staged) {
    for (int k = kb - nz0; k < ke - nz0; ++k) acc += s_va[k] * w[s_ci[k]];
  } else {
    for (int k = kb; k < ke; ++k) acc += va[k] * w[ci[k]];
  }
  const T wr = w[r];
  T wn = s1 * acc + s0 * wr;
  if (HAS_PREV) wn -= Wp[off + r];
  if (IS_CLEN) wn += (T)coef[(int64_t)blockIdx.y * cld + jnext] * Vd[off + r];
  Wn[off + r] = wn;
  if (HAS_Y) {
    const double *cc = coef + (int64_t)blockIdx.y * cld;
    const T y = Y_INIT ? (T)cc[0] * wr : Y[off + r];
    Y[off + r] = y + (T)cc[jnext] * wn;
  }
}

// LDS-staged CSR stream with the nonzero loop unrolled by 8: the column
// indices and values of 8 entries come from LDS, their 8 gathers are issued
// together (padding entries read the row's own element and are multiplied by
// 0), then accumulated in index order. XCD=true remaps workgroups per XCD.
// With DELTA the columns come as 16-bit offsets from the row (cd).
template <typename T, int KIND, bool XCD, bool DELTA>
__global__ __launch_bounds__(TPB) void k_cheb_vec_lds8(int n, const int *__restrict__ rp,
                                                       const int *__restrict__ ci,
                                                       const int16_t *__restrict__ cd,
                                                       const T *__restrict__ va, T s1, T s0,
                                                       const T *__restrict__ W, const T *Wp, T *Wn,
                                                       T *Y, int64_t ld,
                                                       const double *__restrict__ coef, int cld,
                                                       int jnext, const T *__restrict__ Vd) {
  constexpr int CAP = 2048;
  constexpr bool IS_CLEN = (KIND == STEP_CLEN);
  constexpr bool HAS_PREV = (KIND == STEP_NEXT || IS_CLEN);
  constexpr bool HAS_Y = (KIND == STEP_FIRST || KIND == STEP_NEXT);
  constexpr bool Y_INIT = (KIND == STEP_FIRST);
  __shared__ int s_rp[TPB + 1];
  __shared__ int s_ci[CAP];
  __shared__ T s_va[CAP];
  const int bx = XCD ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int r0 = bx * TPB;
  const int nr = min(TPB, n - r0);
  for (int i = threadIdx.x; i <= nr; i += TPB) s_rp[i] = rp[r0 + i];
  __syncthreads();
  const int nz0 = s_rp[0];
  const int cnt = s_rp[nr] - nz0;
  const bool staged = cnt <= CAP;
  if (staged) {
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      s_ci[i] = DELTA ? (int)cd[nz0 + i] : ci[nz0 + i];
      s_va[i] = va[nz0 + i];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= nr) return;
  const int r = r0 + t;
  const int64_t off = (int64_t)blockIdx.y * ld;
  const T *w = W + off;
  T acc = 0;
  const int kb = s_rp[t] - nz0, ke = s_rp[t + 1] - nz0;
  if (staged) {
    for (int k = kb; k < ke; k += 8) {
      T a[8], g[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = k + u < ke;
        const int c = ok ? (DELTA ? r + s_ci[k + u] : s_ci[k + u]) : r;
        a[u] = ok ? s_va[k + u] : (T)0;
        g[u] = w[c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += a[u] * g[u];
    }
  } else {
    for (int k = kb + nz0; k < ke + nz0; ++k) acc += va[k] * w[DELTA ? r + (int)cd[k] : ci[k]];
  }
  const T wr = w[r];
  T wn = s1 * acc + s0 * wr;
  if (HAS_PREV) wn -= Wp[off + r];
  if (IS_CLEN) wn += (T)coef[(int64_t)blockIdx.y * cld + jnext] * Vd[off + r];
  Wn[off + r] = wn;
  if (HAS_Y) {
    const double *cc = coef + (int64_t)blockIdx.y * cld;
    const T y = Y_INIT ? (T)cc[0] * wr : Y[off + r];
    Y[off + r] = y + (T)cc[jnext] * wn;
  }
}

template <typename T>
void cheb_vec(hipStream_t s, const Csr &A, int variant, int kind, double s1, double s0,
              const T *W, const T *Wp, T *Wn, T *Y, int64_t ld, int ncol, const double *coef,
              int cld, int jnext, const T *Vd) {
  if (A.n <= 0 || ncol <= 0) return;
  dim3 grid((A.n + TPB - 1) / TPB, ncol);
  const T *va = (const T *)A.va;
#define EVK_LAUNCH_VEC(KERN, K)                                                               \
  hipLaunchKernelGGL((KERN<T, K>), grid, dim3(TPB), 0, s, A.n, A.rp, A.ci, va, (T)s1, (T)s0, W, \
                     Wp, Wn, Y, ld, coef, cld, jnext, Vd)
  if (variant == 3 || variant == 4) {
#define EVK_LAUNCH_LDS8(K, X, D)                                                                \
  hipLaunchKernelGGL((k_cheb_vec_lds8<T, K, X, D>), grid, dim3(TPB), 0, s, A.n, A.rp, A.ci, A.cd, \
                     va, (T)s1, (T)s0, W, Wp, Wn, Y, ld, coef, cld, jnext, Vd)
#define EVK_LAUNCH_LDS8_K(X, D)                                      \
  switch (kind) {                                                    \
    case STEP_PLAIN: EVK_LAUNCH_LDS8(STEP_PLAIN, X, D); break;       \
    case STEP_FIRST: EVK_LAUNCH_LDS8(STEP_FIRST, X, D); break;       \
    case STEP_CLEN: EVK_LAUNCH_LDS8(STEP_CLEN, X, D); break;         \
    default: EVK_LAUNCH_LDS8(STEP_NEXT, X, D); break;                \
  }
    const bool xcd = variant == 3;
    if (A.cd) {
      if (xcd) {
        EVK_LAUNCH_LDS8_K(true, true)
      } else {
        EVK_LAUNCH_LDS8_K(false, true)
      }
    } else {
      if (xcd) {
        EVK_LAUNCH_LDS8_K(true, false)
      } else {
        EVK_LAUNCH_LDS8_K(false, false)
      }
    }
#undef EVK_LAUNCH_LDS8_K
#undef EVK_LAUNCH_LDS8
  } else if (variant == 2) {
    switch (kind) {
      case STEP_PLAIN: EVK_LAUNCH_VEC(k_cheb_vec_lds, STEP_PLAIN); break;
      case STEP_FIRST: EVK_LAUNCH_VEC(k_cheb_vec_lds, STEP_FIRST); break;
      case STEP_CLEN: EVK_LAUNCH_VEC(k_cheb_vec_lds, STEP_CLEN); break;
      default: EVK_LAUNCH_VEC(k_cheb_vec_lds, STEP_NEXT); break;
    }
  } else {
    switch (kind) {
      case STEP_PLAIN: EVK_LAUNCH_VEC(k_cheb_vec_direct, STEP_PLAIN); break;
      case STEP_FIRST: EVK_LAUNCH_VEC(k_cheb_vec_direct, STEP_FIRST); break;
      case STEP_CLEN: EVK_LAUNCH_VEC(k_cheb_vec_direct, STEP_CLEN); break;
      default: EVK_LAUNCH_VEC(k_cheb_vec_direct, STEP_NEXT); break;
    }
  }
#undef EVK_LAUNCH_VEC
}

template void cheb_vec<double>(hipStream_t, const Csr &, int, int, double, double, const double *,
                               const double *, double *, double *, int64_t, int, const double *,
                               int, int, const double *);
template void cheb_vec<float>(hipStream_t, const Csr &, int, int, double, double, const float *,
                              const float *, float *, float *, int64_t, int, const double *, int,
                              int, const float *);

// ---------------------------------------------------------------- filter step, row-major block
// Row-major n x ld block, the first nc columns active. With nc <= 256 a
// workgroup covers 256/nc rows per pass (lanes of a row read nc contiguous
// values of each gathered row); wider blocks split the columns over grid.y.
template <typename T, int KIND>
__global__ __launch_bounds__(TPB) void k_cheb_blk(int n, int nc, int rows_per_wg,
                                                  const int *__restrict__ rp,
                                                  const int *__restrict__ ci,
                                                  const T *__restrict__ va, T s1, T s0,
                                                  const T *__restrict__ W, const T *Wp, T *Wn,
                                                  T *Y, int64_t ld,
                                                  const double *__restrict__ coef, int cld,
                                                  int jnext, const T *__restrict__ Vd,
                                                  double *partial) {
  constexpr bool IS_CLEN = (KIND == STEP_CLEN);
  constexpr bool HAS_PREV = (KIND == STEP_NEXT || KIND == STEP_KPM_NEXT || IS_CLEN);
  constexpr bool HAS_Y = (KIND == STEP_FIRST || KIND == STEP_NEXT);
  constexpr bool Y_INIT = (KIND == STEP_FIRST);
  constexpr bool HAS_DOT = (KIND == STEP_KPM_FIRST || KIND == STEP_KPM_NEXT);
  __shared__ double red[4];
  const int tid = threadIdx.x;
  int R0, rsub, col;
  bool active;
  if (nc <= TPB) {
    R0 = TPB / nc;
    rsub = tid / nc;
    col = tid - rsub * nc;
    active = rsub < R0;
  } else {
    R0 = 1;
    rsub = 0;
    col = blockIdx.y * TPB + tid;
    active = col < nc;
  }
  double dacc = 0.0;
  if (active) {
    T c0 = 0, c1 = 0;
    if (HAS_Y || IS_CLEN) c1 = (T)coef[(int64_t)col * cld + jnext];
    if (Y_INIT) c0 = (T)coef[(int64_t)col * cld];
    const int rbeg = blockIdx.x * rows_per_wg;
    const int rend = min(rbeg + rows_per_wg, n);
    for (int r = rbeg + rsub; r < rend; r += R0) {
      T acc = 0;
      const int kb = rp[r], ke = rp[r + 1];
      for (int k = kb; k < ke; ++k) acc = fma_t(va[k], W[(int64_t)ci[k] * ld + col], acc);
      const int64_t e = (int64_t)r * ld + col;
      const T w = W[e];
      // the same fused multiply-adds, in the same order, as the LDS-staged kernel
      T wn = fma_t(s1, acc, s0 * w);
      if (HAS_PREV) wn = wn - Wp[e];
      if (IS_CLEN) wn = fma_t(c1, Vd[e], wn);
      Wn[e] = wn;
      if (HAS_Y) Y[e] = fma_t(c1, wn, Y_INIT ? c0 * w : Y[e]);
      if (HAS_DOT) dacc += (double)Vd[e] * (double)wn;
    }
  }
  if (HAS_DOT) {
    const double b = block_sum(dacc, red);
    if (tid == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = b;
  }
}

// Row-major block, LDS-staged: the workgroup's rows of the CSR matrix are
// loaded into LDS with coalesced loads; each thread owns VEC adjacent columns
// of a group of rows (columns fastest, so the epilogue is contiguous), reads
// the row's entries from LDS and issues 8 gathers of VEC values at a time.
// Element offsets are 32-bit when n * ld < 2^31, else (WIDE) 32 x 32 -> 64-bit
// products; VEC > 1 needs nc and ld divisible by VEC and VEC-aligned base
// pointers. With DELTA the column indices come as 16-bit offsets from the row
// (cd), half the index bytes of a matrix whose bandwidth is below 2^15.
//
// Schedule (runtime `map`; a workgroup covers rows_per_wg rows of one chunk of
// cw columns; nrb row blocks per chunk):
//   0  one chunk (cw = nc), row blocks in launch order;
//   1  one chunk, row blocks renumbered so each of the 8 XCDs sweeps a
//      contiguous row range (neighbouring rows share an L2);
//   2  column chunks of cw columns, chunk 0 over all rows, then chunk 1, ...;
//      within a chunk the row blocks go to the XCDs in runs of grp blocks
//      (run j to XCD j mod 8; npad >= nrb blocks per chunk, a multiple of
//      8 grp, the padding blocks exit at once). All XCDs then sweep the same
//      rows of the same narrow chunk together: a row of W gathered again far
//      away (a neighbouring plane of a 3-D stencil) is re-read while it is
//      still in the Infinity Cache, and rows gathered from close by (the
//      neighbouring lines) are mostly in the XCD's own L2.
template <typename T, int KIND, int VEC, bool WIDE, bool DELTA>
__global__ __launch_bounds__(TPB) void k_cheb_blk_lds(int n, int nc, int rows_per_wg,
                                                      const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const int16_t *__restrict__ cd,
                                                      const T *__restrict__ va, T s1, T s0,
                                                      const T *__restrict__ W, const T *Wp, T *Wn,
                                                      T *Y, int64_t ld64,
                                                      const double *__restrict__ coef, int cld,
                                                      int jnext, const T *__restrict__ Vd,
                                                      double *partial, int map, int cw, int nrb,
                                                      int npad, int grp) {
  typedef T vt __attribute__((ext_vector_type(VEC)));
  constexpr int CAP = 1792;
  constexpr bool IS_CLEN = (KIND == STEP_CLEN);
  constexpr bool HAS_PREV = (KIND == STEP_NEXT || KIND == STEP_KPM_NEXT || IS_CLEN);
  constexpr bool HAS_Y = (KIND == STEP_FIRST || KIND == STEP_NEXT);
  constexpr bool Y_INIT = (KIND == STEP_FIRST);
  constexpr bool HAS_DOT = (KIND == STEP_KPM_FIRST || KIND == STEP_KPM_NEXT);
  __shared__ int s_rp[TPB + 1];
  __shared__ int s_ci[CAP];
  __shared__ T s_va[CAP];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int bid = blockIdx.x;
  int bx, chunk = 0;
  if (map == 2) {
    const int x = bid & 7, local = bid >> 3, per = npad >> 3;
    chunk = local / per;
    const int lc = local - chunk * per;
    bx = ((lc / grp) * 8 + x) * grp + lc % grp;
    if (bx >= nrb) return;  // padding block (uniform over the workgroup)
  } else {
    bx = map == 1 ? xcd_remap(bid, gridDim.x) : bid;
  }
  const int cbase = chunk * cw;  // first column of the chunk
  const int r0 = bx * rows_per_wg;
  const int nr = min(rows_per_wg, n - r0);
  for (int i = tid; i <= nr; i += TPB) s_rp[i] = rp[r0 + i];
  __syncthreads();
  const int nz0 = s_rp[0];
  const int cnt = s_rp[nr] - nz0;
  const bool staged = cnt <= CAP;
  if (staged) {
    for (int i = tid; i < cnt; i += TPB) {
      s_ci[i] = DELTA ? (int)cd[nz0 + i] : ci[nz0 + i];
      s_va[i] = va[nz0 + i];
    }
  }
  __syncthreads();
  const int ncv = cw / VEC;  // vector slots per row of the chunk
  int R0, rsub, slot;
  bool active;
  if (ncv <= TPB) {
    R0 = TPB / ncv;
    rsub = tid / ncv;
    slot = tid - rsub * ncv;
    active = rsub < R0;
  } else {
    R0 = 1;
    rsub = 0;
    slot = blockIdx.y * TPB + tid;
    active = slot < ncv;
  }
  const int col = cbase + slot * VEC;
  active = active && col < nc;
  const int ld = (int)ld64;
  // offset of element (row, 0) of the block
  auto roff = [&](int row) -> size_t {
    return WIDE ? (size_t)(uint32_t)row * (uint32_t)ld : (size_t)(row * ld);
  };
  double dacc = 0.0;
  if (active) {
    vt c0 = (T)0, c1 = (T)0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      if (HAS_Y || IS_CLEN) c1[v] = (T)coef[(col + v) * cld + jnext];
      if (Y_INIT) c0[v] = (T)coef[(col + v) * cld];
    }
    const T *wc = W + col;
    for (int rl = rsub; rl < nr; rl += R0) {
      const int kb = s_rp[rl] - nz0, ke = s_rp[rl + 1] - nz0;
      const int row = r0 + rl;
      const size_t e = roff(row) + col;
      // the row's own operands are loaded first, so that their loads are in
      // flight together with the gathers below (Wn may alias Wp, but only
      // element e, which this thread reads before it writes)
      const vt w = *(const vt *)(W + e);
      const vt wp = HAS_PREV ? *(const vt *)(Wp + e) : (vt)(T)0;
      const vt vd = (IS_CLEN || HAS_DOT) ? *(const vt *)(Vd + e) : (vt)(T)0;
      const vt yo = (HAS_Y && !Y_INIT) ? *(const vt *)(Y + e) : (vt)(T)0;
      vt acc = (T)0;
      if (staged) {
        for (int k = kb; k < ke; k += 8) {
          T a[8];
          vt g[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const bool ok = k + u < ke;
            const int c = ok ? (DELTA ? row + s_ci[k + u] : s_ci[k + u]) : row;
            a[u] = ok ? s_va[k + u] : (T)0;
            g[u] = *(const vt *)(wc + roff(c));
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fma_t(a[u], g[u][v], acc[v]);
        }
      } else {
        for (int k = kb + nz0; k < ke + nz0; ++k) {
          const vt g = *(const vt *)(wc + roff(DELTA ? row + (int)cd[k] : ci[k]));
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] = fma_t(va[k], g[v], acc[v]);
        }
      }
      // element by element with explicit fused multiply-adds, so that every
      // lane width (and so every schedule) rounds the same way
      vt wn;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        T x = fma_t(s1, acc[v], s0 * w[v]);
        if (HAS_PREV) x = x - wp[v];
        if (IS_CLEN) x = fma_t(c1[v], vd[v], x);
        wn[v] = x;
      }
      *(vt *)(Wn + e) = wn;
      if (HAS_Y) {
        vt y;
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          y[v] = fma_t(c1[v], wn[v], Y_INIT ? c0[v] * w[v] : yo[v]);
        *(vt *)(Y + e) = y;
      }
      if (HAS_DOT) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) dacc += (double)vd[v] * (double)wn[v];
      }
    }
  }
  if (HAS_DOT) {
    const double b = block_sum(dacc, red);
    if (tid == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = b;
  }
}

// 1: global loads; 2: LDS-staged, 16-byte lanes, scheduled; 3: LDS-staged,
// one column per lane, launch order; 4: 2 with one column per lane
static int g_blk_variant = 2;

void set_blk_variant(int v) { g_blk_variant = (v >= 1 && v <= 4) ? v : 2; }

// Columns per lane for a launch: 2 (16-byte loads) when the block allows it.
static int blk_vec(int nc, int64_t ld, size_t es, const void *const *ptrs, int np, int want) {
  if (g_blk_variant != 2) return 1;
  int v = es == 8 ? 2 : 4;  // 16-byte loads
  if (want == 4 || want == 2 || want == 1) v = want;  // the schedule's lane width
  while (v > 1) {
    bool ok = (nc % v == 0) && (ld % v == 0);
    for (int i = 0; ok && i < np; ++i)
      if (ptrs[i] && ((uintptr_t)ptrs[i] % (v * es))) ok = false;
    if (ok) break;
    v >>= 1;
  }
  return v;
}

// Rows per workgroup and grid for nc columns (one chunk of cw = nc columns).
// lds: the LDS-staged kernel, whose row-pointer stage holds at most TPB rows;
// rows > 0 asks for that many rows per workgroup (rounded to whole passes).
static void blk_shape(int n, int nc, int vec, int *rows_per_wg, dim3 *grid, bool lds = true,
                      int rows = 0) {
  const int ncv = nc / vec;
  const int R0 = ncv <= TPB ? TPB / ncv : 1;
  int passes = (ncv <= TPB && R0 > 2) ? 4 : 8;
  if (rows > 0) passes = std::max(1, rows / R0);
  if (lds) passes = std::max(1, std::min(passes, TPB / R0));
  *rows_per_wg = R0 * passes;
  const int gx = (n + *rows_per_wg - 1) / *rows_per_wg;
  const int gy = ncv <= TPB ? 1 : (ncv + TPB - 1) / TPB;
  *grid = dim3(gx, gy);
}

int blk_partials(int n, int nc) {
  // an upper bound over the launch shapes (VEC 1 has the most workgroups)
  int rpw;
  dim3 g;
  blk_shape(n, nc, 1, &rpw, &g, g_blk_variant != 1);
  return (int)(g.x * g.y);
}

// The schedule actually used for a launch: map 2 needs a chunk width that is
// a multiple of VEC with at most 256 slots and below nc, and grp >= 1;
// otherwise (and for the KPM kinds, whose partial sums are indexed by
// workgroup) the launch is one chunk with contiguous row ranges per XCD.
static BlkSched blk_resolve(const BlkSched *sc, int nc, int vec, int kind) {
  BlkSched r;
  r.map = g_blk_variant == 3 ? 0 : 1;
  r.cw = nc;
  r.grp = 1;
  if (!sc || g_blk_variant == 3 || kind == STEP_KPM_FIRST || kind == STEP_KPM_NEXT) return r;
  r.rows = sc->rows;
  if (sc->map == 0 || sc->map == 1) {
    r.map = sc->map;
    return r;
  }
  const int cw = sc->cw;
  if (cw < vec || cw % vec || cw / vec > TPB || cw >= nc || sc->grp < 1) return r;
  r.map = 2;
  r.cw = cw;
  r.grp = sc->grp;
  return r;
}

template <typename T>
void cheb_blk(hipStream_t s, const Csr &A, int kind, double s1, double s0, const T *W,
              const T *Wp, T *Wn, T *Y, int64_t ld, int nc, const double *coef, int cld, int jnext,
              const T *Vd, double *partial, const BlkSched *sched) {
  if (A.n <= 0 || nc <= 0) return;
  const bool wide = (int64_t)A.n * ld >= ((int64_t)1 << 31);
  const bool ok32 = ld < ((int64_t)1 << 31) && (int64_t)A.n < ((int64_t)1 << 31) &&
                    (int64_t)nc * cld < ((int64_t)1 << 31);
  const bool kpm = kind == STEP_KPM_FIRST || kind == STEP_KPM_NEXT;
  int var = ok32 ? g_blk_variant : 1;
  if (var != 1 && sched && sched->lds == 0 && !kpm) var = 1;  // the schedule's kernel choice
  const void *ptrs[5] = {W, Wp, Wn, Y, Vd};
  const int vec = var == 1 ? 1 : blk_vec(nc, ld, sizeof(T), ptrs, 5, sched ? sched->vec : 0);
  // the global-load kernel (variant 1) takes no schedule: one chunk
  const BlkSched sc = var == 1 ? BlkSched{0, nc, 1, 0, 0, 0} : blk_resolve(sched, nc, vec, kind);
  int rpw;
  dim3 grid;
  blk_shape(A.n, sc.cw, vec, &rpw, &grid, var != 1, sc.rows);
  const int nrb = (int)grid.x;
  int npad = nrb;
  if (sc.map == 2) {
    const int run = 8 * sc.grp;
    npad = (nrb + run - 1) / run * run;
    grid.x = (unsigned)((int64_t)npad * ((nc + sc.cw - 1) / sc.cw));
  }
  const T *va = (const T *)A.va;
#define EVK_BLK_ARGS                                                                          \
  grid, dim3(TPB), 0, s, A.n, nc, rpw, A.rp, A.ci, va, (T)s1, (T)s0, W, Wp, Wn, Y, ld, coef, cld, \
      jnext, Vd, partial
#define EVK_LDS_ARGS                                                                          \
  grid, dim3(TPB), 0, s, A.n, nc, rpw, A.rp, A.ci, A.cd, va, (T)s1, (T)s0, W, Wp, Wn, Y, ld,    \
      coef, cld, jnext, Vd, partial, sc.map, sc.cw, nrb, npad, sc.grp
#define EVK_LAUNCH_LDS(K, W, D)                                                              \
  do {                                                                                       \
    if (vec == 4)                                                                            \
      hipLaunchKernelGGL((k_cheb_blk_lds<T, K, 4, W, D>), EVK_LDS_ARGS);                     \
    else if (vec == 2)                                                                       \
      hipLaunchKernelGGL((k_cheb_blk_lds<T, K, 2, W, D>), EVK_LDS_ARGS);                     \
    else                                                                                     \
      hipLaunchKernelGGL((k_cheb_blk_lds<T, K, 1, W, D>), EVK_LDS_ARGS);                     \
  } while (0)
#define EVK_LAUNCH_BLK(K)                                                                    \
  do {                                                                                       \
    if (var == 1)                                                                            \
      hipLaunchKernelGGL((k_cheb_blk<T, K>), EVK_BLK_ARGS);                                  \
    else if (wide && A.cd)                                                                   \
      EVK_LAUNCH_LDS(K, true, true);                                                         \
    else if (wide)                                                                           \
      EVK_LAUNCH_LDS(K, true, false);                                                        \
    else if (A.cd)                                                                           \
      EVK_LAUNCH_LDS(K, false, true);                                                        \
    else                                                                                     \
      EVK_LAUNCH_LDS(K, false, false);                                                       \
  } while (0)
  switch (kind) {
    case STEP_PLAIN: EVK_LAUNCH_BLK(STEP_PLAIN); break;
    case STEP_FIRST: EVK_LAUNCH_BLK(STEP_FIRST); break;
    case STEP_NEXT: EVK_LAUNCH_BLK(STEP_NEXT); break;
    case STEP_KPM_FIRST: EVK_LAUNCH_BLK(STEP_KPM_FIRST); break;
    case STEP_CLEN: EVK_LAUNCH_BLK(STEP_CLEN); break;
    default: EVK_LAUNCH_BLK(STEP_KPM_NEXT); break;
  }
#undef EVK_LAUNCH_BLK
#undef EVK_LAUNCH_LDS
#undef EVK_LDS_ARGS
#undef EVK_BLK_ARGS
}

template void cheb_blk<double>(hipStream_t, const Csr &, int, double, double, const double *,
                               const double *, double *, double *, int64_t, int, const double *,
                               int, int, const double *, double *, const BlkSched *);
template void cheb_blk<float>(hipStream_t, const Csr &, int, double, double, const float *,
                              const float *, float *, float *, int64_t, int, const double *, int,
                              int, const float *, double *, const BlkSched *);

template <typename T>
__global__ __launch_bounds__(TPB) void k_fill_zero(int64_t count, T *p) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < count) p[i] = (T)0;
}

template <typename T>
void fill_zero(hipStream_t s, int64_t count, T *p) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)((count + TPB - 1) / TPB)), dim3(TPB), 0, s,
                     count, p);
}

template void fill_zero<double>(hipStream_t, int64_t, double *);
template void fill_zero<float>(hipStream_t, int64_t, float *);

// cd[k] = col[k] - row(k); flag[0] = 1 when an offset does not fit 16 bits
// (every writer stores the same value).
__global__ __launch_bounds__(TPB) void k_col_offsets(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, int16_t *cd,
                                                     int *flag) {
  const int r = blockIdx.x * TPB + threadIdx.x;
  if (r >= n) return;
  bool bad = false;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int d = ci[k] - r;
    if (d < -32768 || d > 32767) {
      bad = true;
      cd[k] = 0;
    } else {
      cd[k] = (int16_t)d;
    }
  }
  if (bad) flag[0] = 1;
}

bool make_col_offsets(hipStream_t s, const Csr &A, int16_t *cd, int *flag) {
  if (A.n <= 0) return false;
  int h = 0;
  if (hipMemcpyAsync(flag, &h, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) return false;
  hipLaunchKernelGGL(k_col_offsets, dim3((A.n + TPB - 1) / TPB), dim3(TPB), 0, s, A.n, A.rp, A.ci,
                     cd, flag);
  if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  return h == 0;
}

// ---------------------------------------------------------------- gather / scatter
// blk (row-major, value type TB) <-> FP64 columns given by a device pointer array.
template <typename TB>
__global__ __launch_bounds__(TPB) void k_gather_cols(int n, int nc, const double *const *src,
                                                     TB *blk, int64_t ldb) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= (int64_t)n * nc) return;
  const int r = (int)(e / nc), c = (int)(e - (int64_t)r * nc);
  blk[(int64_t)r * ldb + c] = (TB)src[c][r];
}

template <typename TB>
__global__ __launch_bounds__(TPB) void k_scatter_cols(int n, int nc, const TB *blk, int64_t ldb,
                                                      double *const *dst) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= (int64_t)n * nc) return;
  const int r = (int)(e / nc), c = (int)(e - (int64_t)r * nc);
  dst[c][r] = (double)blk[(int64_t)r * ldb + c];
}

template <typename TB>
void gather_cols(hipStream_t s, int n, int nc, const double *const *src, TB *blk, int64_t ldb) {
  int64_t tot = (int64_t)n * nc;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_gather_cols<TB>, dim3((unsigned)((tot + TPB - 1) / TPB)), dim3(TPB), 0, s,
                     n, nc, src, blk, ldb);
}

template <typename TB>
void scatter_cols(hipStream_t s, int n, int nc, const TB *blk, int64_t ldb, double *const *dst) {
  int64_t tot = (int64_t)n * nc;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_scatter_cols<TB>, dim3((unsigned)((tot + TPB - 1) / TPB)), dim3(TPB), 0, s,
                     n, nc, blk, ldb, dst);
}

template void gather_cols<double>(hipStream_t, int, int, const double *const *, double *, int64_t);
template void gather_cols<float>(hipStream_t, int, int, const double *const *, float *, int64_t);
template void scatter_cols<double>(hipStream_t, int, int, const double *, int64_t, double *const *);
template void scatter_cols<float>(hipStream_t, int, int, const float *, int64_t, double *const *);

// ---------------------------------------------------------------- reductions over columns
// out[c] = scale * sum_w partial[c * nw + w]; one workgroup per column.
__global__ __launch_bounds__(TPB) void k_reduce_partials(int nw, const double *partial,
                                                         double scale, double *out,
                                                         const int *gate) {
  __shared__ double red[4];
  if (gate && gate[0] == 0) {
    if (threadIdx.x == 0) out[blockIdx.x] = 0.0;
    return;
  }
  const double *p = partial + (int64_t)blockIdx.x * nw;
  double acc = 0.0;
  for (int w = threadIdx.x; w < nw; w += TPB) acc += p[w];
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = scale * b;
}

void reduce_partials(hipStream_t s, int nw, int ncol, const double *partial, double scale,
                     double *out, const int *gate) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_reduce_partials, dim3(ncol), dim3(TPB), 0, s, nw, partial, scale, out,
                     gate);
}

// h = B^T z, partial sums per 64*RPL-row chunk; wave w of the workgroup takes
// columns j = w, w+4, ...; z of the chunk stays in registers.
static constexpr int GEMV_RPL = 16;
static constexpr int GEMV_ROWS = 64 * GEMV_RPL;

// grid.x: 1024-row chunks; grid.y: groups of cpg columns, so that small n
// still fills the device: cpg = 64 unless fewer 1024-row chunks than that
// leave the grid short of about 512 workgroups, down to 4 (one per wave).
// Per column a lane sums its rows in increasing order and the wave reduces by
// a fixed butterfly.
static int gemv_cols_per_group(int nwg, int nb) {
  const int want = (int)(((int64_t)nb * nwg + 511) / 512);
  return std::max(4, std::min(64, (want + 3) / 4 * 4));
}

__global__ __launch_bounds__(TPB) void k_gemv_t_partial(int n, int nb, const double *__restrict__ B,
                                                        int64_t ld, const double *__restrict__ z,
                                                        double *partial, const int *gate,
                                                        int cpg) {
  if (gate && gate[0] == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.x * GEMV_ROWS;
  double zr[GEMV_RPL];
#pragma unroll
  for (int t = 0; t < GEMV_RPL; ++t) {
    const int r = r0 + lane + 64 * t;
    zr[t] = r < n ? z[r] : 0.0;
  }
  const int nwg = gridDim.x;
  const int jend = min(nb, (int)(blockIdx.y + 1) * cpg);
  for (int j = blockIdx.y * cpg + wave; j < jend; j += 4) {
    const double *b = B + (int64_t)j * ld;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < GEMV_RPL; ++t) {
      const int r = r0 + lane + 64 * t;
      if (r < n) acc += b[r] * zr[t];
    }
    acc = wave_sum(acc);
    if (lane == 0) partial[(int64_t)j * nwg + blockIdx.x] = acc;
  }
}

int gemv_partials(int n, int nb) { return ((n + GEMV_ROWS - 1) / GEMV_ROWS) * std::max(nb, 1); }

void gemv_t(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *z,
            double *partial, double *h, const int *gate) {
  if (nb <= 0 || n <= 0) return;
  const int nwg = (n + GEMV_ROWS - 1) / GEMV_ROWS;
  const int cpg = gemv_cols_per_group(nwg, nb);
  hipLaunchKernelGGL(k_gemv_t_partial, dim3(nwg, (nb + cpg - 1) / cpg), dim3(TPB), 0, s, n, nb, B,
                     ld, z, partial, gate, cpg);
  reduce_partials(s, nwg, nb, partial, 1.0, h, gate);
}

// z -= B h, one row per thread, h staged through LDS in chunks. With NRM the
// workgroup also writes the sum of squares of its rows of the updated z.
template <bool NRM>
__global__ __launch_bounds__(TPB) void k_gemv_n_sub(int n, int nb, const double *__restrict__ B,
                                                    int64_t ld, const double *__restrict__ h,
                                                    double *z, const int *gate,
                                                    double *nrm_partial) {
  __shared__ double sh[1024];
  __shared__ double red[4];
  if (gate && gate[0] == 0) return;
  const int r = blockIdx.x * TPB + threadIdx.x;
  double acc = 0.0;
  for (int j0 = 0; j0 < nb; j0 += 1024) {
    const int cnt = min(1024, nb - j0);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += TPB) sh[i] = h[j0 + i];
    __syncthreads();
    if (r < n) {
      const double *b = B + (int64_t)j0 * ld + r;
#pragma unroll 8
      for (int j = 0; j < cnt; ++j) acc += b[(int64_t)j * ld] * sh[j];
    }
  }
  double zn = 0.0;
  if (r < n) {
    zn = z[r] - acc;
    z[r] = zn;
  }
  if (NRM) {
    const double b = block_sum(zn * zn, red);
    if (threadIdx.x == 0) nrm_partial[blockIdx.x] = b;
  }
}

void gemv_n_sub(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *h,
                double *z, const int *gate) {
  if (nb <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_gemv_n_sub<false>, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, nb, B,
                     ld, h, z, gate, nullptr);
}

int nrm_partials(int n) { return std::max((n + TPB - 1) / TPB, 1); }

void gemv_n_sub_nrm(hipStream_t s, int n, int nb, const double *B, int64_t ld, const double *h,
                    double *z, double *nrm_partial) {
  if (nb <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_gemv_n_sub<true>, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, nb, B, ld,
                     h, z, nullptr, nrm_partial);
}

// DGKS test of a classical Gram-Schmidt pass (Section 2.3): with the
// orthonormal basis, the norm of z before the pass, taken without the
// components the three-term recurrence accounts for, is sqrt(after^2 + S),
// S = sum of h[j]^2 over the other columns [lo, hi). A second pass is made
// when after < before / sqrt(2), i.e. when after^2 < S.
__global__ __launch_bounds__(TPB) void k_dgks_gate(int nw, const double *nrm_partial,
                                                   const double *h, int lo, int hi, int force,
                                                   int *gate) {
  __shared__ double red[4];
  double a = 0.0, sq = 0.0;
  for (int w = threadIdx.x; w < nw; w += TPB) a += nrm_partial[w];
  for (int j = lo + threadIdx.x; j < hi; j += TPB) sq += h[j] * h[j];
  const double after2 = block_sum(a, red);
  __syncthreads();
  const double other = block_sum(sq, red);
  if (threadIdx.x == 0) gate[0] = (force || after2 < other) ? 1 : 0;
}

void dgks_gate(hipStream_t s, int n, const double *nrm_partial, const double *h, int lo, int hi,
               int *gate, int force) {
  hipLaunchKernelGGL(k_dgks_gate, dim3(1), dim3(TPB), 0, s, nrm_partials(n), nrm_partial, h, lo,
                     std::max(hi, lo), force, gate);
}

// z -= alpha[0] q + beta qp (qp may be null)
__global__ __launch_bounds__(TPB) void k_three_term(int n, double *__restrict__ z,
                                                    const double *__restrict__ q,
                                                    const double *__restrict__ qp,
                                                    const double *__restrict__ alpha,
                                                    double beta) {
  const int r = blockIdx.x * TPB + threadIdx.x;
  if (r >= n) return;
  double v = z[r] - alpha[0] * q[r];
  if (qp) v -= beta * qp[r];
  z[r] = v;
}

void three_term(hipStream_t s, int n, double *z, const double *q, const double *qp,
                const double *alpha, double beta) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_three_term, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, z, q, qp, alpha,
                     beta);
}

// Column dots and residual norms: 2048-row chunks, grid.y over columns.
static constexpr int DOT_ROWS = 2048;

__global__ __launch_bounds__(TPB) void k_col_dots(int n, const double *__restrict__ X, int64_t ldx,
                                                  const double *__restrict__ Y, int64_t ldy,
                                                  double *partial) {
  __shared__ double red[4];
  const double *x = X + (int64_t)blockIdx.y * ldx;
  const double *y = Y + (int64_t)blockIdx.y * ldy;
  const int r0 = blockIdx.x * DOT_ROWS;
  const int r1 = min(r0 + DOT_ROWS, n);
  double acc = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += TPB) acc += x[r] * y[r];
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = b;
}

int dot_partials(int n, int ncol) { return ((n + DOT_ROWS - 1) / DOT_ROWS) * std::max(ncol, 1); }

void col_dots(hipStream_t s, int n, int ncol, const double *X, int64_t ldx, const double *Y,
              int64_t ldy, double *partial, double *out) {
  if (ncol <= 0 || n <= 0) return;
  const int nwg = (n + DOT_ROWS - 1) / DOT_ROWS;
  hipLaunchKernelGGL(k_col_dots, dim3(nwg, ncol), dim3(TPB), 0, s, n, X, ldx, Y, ldy, partial);
  reduce_partials(s, nwg, ncol, partial, 1.0, out);
}

__global__ __launch_bounds__(TPB) void k_col_resid2(int n, const double *__restrict__ X,
                                                    const double *__restrict__ AX, int64_t ld,
                                                    const double *__restrict__ xax,
                                                    const double *__restrict__ xx,
                                                    double *partial) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  const double lam = xax[c] / xx[c];
  const double *x = X + (int64_t)c * ld;
  const double *ax = AX + (int64_t)c * ld;
  const int r0 = blockIdx.x * DOT_ROWS;
  const int r1 = min(r0 + DOT_ROWS, n);
  double acc = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += TPB) {
    const double e = ax[r] - lam * x[r];
    acc += e * e;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = b;
}

void col_resid2(hipStream_t s, int n, int ncol, const double *X, const double *AX, int64_t ld,
                const double *xax, const double *xx, double *partial, double *out) {
  if (ncol <= 0 || n <= 0) return;
  const int nwg = (n + DOT_ROWS - 1) / DOT_ROWS;
  hipLaunchKernelGGL(k_col_resid2, dim3(nwg, ncol), dim3(TPB), 0, s, n, X, AX, ld, xax, xx,
                     partial);
  reduce_partials(s, nwg, ncol, partial, 1.0, out);
}

// ---------------------------------------------------------------- scaling
__global__ __launch_bounds__(TPB) void k_normalize(int n, const double *src, double *dst,
                                                   const double *__restrict__ nrm2,
                                                   double *beta_out) {
  const double beta = sqrt(nrm2[0]);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int r = blockIdx.x * TPB + threadIdx.x;
  if (beta_out != nullptr && r == 0) beta_out[0] = beta;
  if (r < n) dst[r] = src[r] * inv;
}

void normalize(hipStream_t s, int n, const double *src, double *dst, const double *nrm2,
               double *beta_out) {
  hipLaunchKernelGGL(k_normalize, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, src, dst, nrm2,
                     beta_out);
}

__global__ __launch_bounds__(TPB) void k_normalize_cols(int n, double *X, int64_t ld,
                                                        const double *__restrict__ nrm2) {
  const int c = blockIdx.y;
  const double beta = sqrt(nrm2[c]);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int r = blockIdx.x * TPB + threadIdx.x;
  if (r < n) X[(int64_t)c * ld + r] *= inv;
}

void normalize_cols(hipStream_t s, int n, int ncol, double *X, int64_t ld, const double *nrm2) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_normalize_cols, dim3((n + TPB - 1) / TPB, ncol), dim3(TPB), 0, s, n, X, ld,
                     nrm2);
}

// ---------------------------------------------------------------- C = A B (tall A, small B)
// FP64 MFMA (v_mfma_f64_16x16x4f64, operand layout as in k_gemm_tn_mfma below):
// a workgroup owns 64 rows x 64 columns of C, each wavefront 16 rows x the 64
// columns (four 16 x 16 accumulators). A (column-major) is read straight from
// memory, 16 consecutive rows per k, once per 64-column block; B is staged in
// LDS 64 rows of K at a time (zero outside B).
typedef double v4d __attribute__((ext_vector_type(4)));
static constexpr int NN_ROWS = 64, NN_COLS = 64, NN_KC = 64;

__global__ __launch_bounds__(TPB) void k_gemm_nn_mfma(int n, int K, int N,
                                                      const double *__restrict__ A, int64_t lda,
                                                      const double *__restrict__ B, int64_t ldb,
                                                      double *C, int64_t ldc) {
  __shared__ double Bs[NN_KC][NN_COLS + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int rb = blockIdx.x * NN_ROWS + 16 * wave;
  const int j0 = blockIdx.y * NN_COLS;
  const int row = rb + i;
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += NN_KC) {
    __syncthreads();
    for (int e = tid; e < NN_KC * NN_COLS; e += TPB) {
      const int jj = e / NN_KC, kk = e - jj * NN_KC;
      Bs[kk][jj] = (k0 + kk < K && j0 + jj < N) ? B[(int64_t)(j0 + jj) * ldb + k0 + kk] : 0.0;
    }
    __syncthreads();
    const int kend = min(NN_KC, K - k0);
    for (int kk = 0; kk < kend; kk += 4) {
      const int k = k0 + kk + kq;
      const double a = (row < n && k < K) ? A[(int64_t)k * lda + row] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[kk + kq][16 * t + i], acc[t], 0, 0, 0);
    }
  }
  // lane l, register v: row 4 v + l / 16 of the wave's strip, column l % 16 of tile t
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = j0 + 16 * t + i;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rb + 4 * v + kq;
      if (r < n && col < N) C[(int64_t)col * ldc + r] = acc[t][v];
    }
  }
}

void gemm_nn(hipStream_t s, int n, int K, int N, const double *A, int64_t lda, const double *B,
             int64_t ldb, double *C, int64_t ldc) {
  if (n <= 0 || N <= 0 || K <= 0) return;
  hipLaunchKernelGGL(k_gemm_nn_mfma, dim3((n + NN_ROWS - 1) / NN_ROWS, (N + NN_COLS - 1) / NN_COLS),
                     dim3(TPB), 0, s, n, K, N, A, lda, B, ldb, C, ldc);
}

// ---------------------------------------------------------------- random inputs
__global__ __launch_bounds__(TPB) void k_rademacher(int n, int nvec, uint64_t seed, double *V) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= (int64_t)n * nvec) return;
  const int64_t i = e / nvec;
  const int64_t l = e - i * nvec;
  const uint64_t bits = sm64(seed, (uint64_t)l * (uint64_t)n + (uint64_t)i) >> 63;
  V[e] = bits ? -1.0 : 1.0;
}

void rademacher(hipStream_t s, int n, int nvec, uint64_t seed, double *V) {
  const int64_t tot = (int64_t)n * nvec;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_rademacher, dim3((unsigned)((tot + TPB - 1) / TPB)), dim3(TPB), 0, s, n,
                     nvec, seed, V);
}

__global__ __launch_bounds__(TPB) void k_lanczos_start(int n, uint64_t seed, int64_t restart,
                                                       double *x) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const uint64_t u = sm64(seed, (uint64_t)restart * (uint64_t)n + (uint64_t)i) >> 11;
  x[i] = 2.0 * ((double)u * (1.0 / 9007199254740992.0)) - 1.0;
}

void lanczos_start(hipStream_t s, int n, uint64_t seed, int64_t restart, double *x) {
  hipLaunchKernelGGL(k_lanczos_start, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, n, seed, restart,
                     x);
}

// ---------------------------------------------------------------- C = X^T Y (FP64 MFMA)
// X (n x p) and Y (n x q) column-major. Each workgroup owns a 32 x 32 tile of C
// and a chunk of rows; the chunk is staged through LDS 64 rows at a time and
// each wavefront accumulates one 16 x 16 quadrant with v_mfma_f64_16x16x4f64
// (A operand: lane l holds X^T[i][k], i = l % 16, k = l / 16; B operand: lane l
// holds Y[k][j], j = l % 16; result: lane l, register v holds row 4 v + l / 16 of
// column l % 16). Per-chunk tiles go to `partial`, summed in chunk order.
static constexpr int TN_RC = 64;

__global__ __launch_bounds__(TPB) void k_gemm_tn_mfma(int n, int p, int q, int rows_per_chunk,
                                                      const double *__restrict__ X, int64_t ldx,
                                                      const double *__restrict__ Y, int64_t ldy,
                                                      double *partial) {
  __shared__ double Xs[TN_RC][33];
  __shared__ double Ys[TN_RC][33];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = blockIdx.x, i0 = blockIdx.y * 32, j0 = blockIdx.z * 32;
  const int rbeg = chunk * rows_per_chunk;
  const int rend = min(rbeg + rows_per_chunk, n);
  const int qi = wave >> 1, qj = wave & 1;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = rbeg; r0 < rend; r0 += TN_RC) {
    __syncthreads();
    // stage 64 rows x 32 columns of X and of Y (zero outside the matrices)
    for (int e = tid; e < TN_RC * 32; e += TPB) {
      const int c = e / TN_RC, rr = e - c * TN_RC;
      const int r = r0 + rr;
      Xs[rr][c] = (r < rend && i0 + c < p) ? X[(int64_t)(i0 + c) * ldx + r] : 0.0;
      Ys[rr][c] = (r < rend && j0 + c < q) ? Y[(int64_t)(j0 + c) * ldy + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k4 = 0; k4 < TN_RC; k4 += 4) {
      const double a = Xs[k4 + (lane >> 4)][16 * qi + (lane & 15)];
      const double b = Ys[k4 + (lane >> 4)][16 * qj + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  // write this chunk's tile: partial[chunk][i][j], i < p, j < q
  const int j = j0 + 16 * qj + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 16 * qi + 4 * v + (lane >> 4);
    if (i < p && j < q) partial[((int64_t)chunk * p + i) * q + j] = acc[v];
  }
}

__global__ __launch_bounds__(TPB) void k_sum_chunks(int nchunk, int64_t pq,
                                                    const double *__restrict__ partial,
                                                    double *C, int p, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= pq) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)c * pq + e];
  const int64_t qcols = pq / p;
  const int64_t i = e / qcols, jj = e - i * qcols;
  C[jj * ldc + i] = s;  // C column-major p x q
}

static int tn_rows_per_chunk(int n, int p, int q) {
  // keep the partial tiles at most ~64 MB and at least 4096 rows per chunk
  int64_t tiles = (int64_t)((p + 31) / 32) * ((q + 31) / 32);
  int rpc = 4096;
  while ((int64_t)((n + rpc - 1) / rpc) * p * q * 8 > (64ll << 20) && rpc < n) rpc *= 2;
  (void)tiles;
  return rpc;
}

int64_t gemm_tn_partials(int n, int p, int q) {
  const int rpc = tn_rows_per_chunk(n, p, q);
  return (int64_t)((n + rpc - 1) / rpc) * p * q;
}

// Enough partials for every shape p' <= p, q' <= q (chunks are never smaller
// than 4096 rows).
int64_t gemm_tn_partials_bound(int n, int p, int q) {
  return (int64_t)((n + 4095) / 4096) * p * q;
}

void gemm_tn(hipStream_t s, int n, int p, int q, const double *X, int64_t ldx, const double *Y,
             int64_t ldy, double *C, int64_t ldc, double *partial) {
  if (n <= 0 || p <= 0 || q <= 0) return;
  const int rpc = tn_rows_per_chunk(n, p, q);
  const int nchunk = (n + rpc - 1) / rpc;
  dim3 grid(nchunk, (p + 31) / 32, (q + 31) / 32);
  hipLaunchKernelGGL(k_gemm_tn_mfma, grid, dim3(TPB), 0, s, n, p, q, rpc, X, ldx, Y, ldy, partial);
  const int64_t pq = (int64_t)p * q;
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((pq + TPB - 1) / TPB)), dim3(TPB), 0, s, nchunk,
                     pq, partial, C, p, ldc);
}

// ---------------------------------------------------------------- y += a x
__global__ __launch_bounds__(TPB) void k_axpy(int64_t len, double a, const double *__restrict__ x,
                                              double *y) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < len) y[i] += a * x[i];
}

void axpy(hipStream_t s, int64_t len, double a, const double *x, double *y) {
  if (len > 0)
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((len + TPB - 1) / TPB)), dim3(TPB), 0, s, len, a, x,
                       y);
}

// ---------------------------------------------------------------- copy (bandwidth calibration)
__global__ __launch_bounds__(TPB) void k_copy_probe(int64_t n2, const double2 *__restrict__ x,
                                                    double2 *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n2; i += (int64_t)gridDim.x * TPB)
    y[i] = x[i];
}

void copy_probe(hipStream_t s, int64_t bytes, const void *x, void *y) {
  const int64_t n2 = bytes / 16;
  if (n2 <= 0) return;
  const int64_t want = (n2 + TPB - 1) / TPB;
  const unsigned grid = (unsigned)std::min<int64_t>(want, 256 * 64);
  hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(TPB), 0, s, n2, (const double2 *)x,
                     (double2 *)y);
}

// ---------------------------------------------------------------- conversions
__global__ __launch_bounds__(TPB) void k_to_f32(int64_t n, const double *x, float *y) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ __launch_bounds__(TPB) void k_to_f64(int64_t n, const float *x, double *y) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
void to_f32(hipStream_t s, int64_t n, const double *x, float *y) {
  if (n > 0)
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, n, x, y);
}
void to_f64(hipStream_t s, int64_t n, const float *x, double *y) {
  if (n > 0)
    hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, n, x, y);
}

}  // namespace evk
