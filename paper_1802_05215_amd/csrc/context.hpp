// Library-internal context and helpers shared by the solver sources (not part
// of the C-ABI): the evsl_ctx_s state, error handling, device allocation with
// the context's memory ledger, workspace slots, filter timing by HIP events.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/evsl_mi355.h"
#include "kernels.hpp"

namespace evc {

struct Error {
  int code;
};

[[noreturn]] inline void fail(int code) { throw Error{code}; }

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace evc

struct evsl_ctx_s {
  hipStream_t stream = nullptr;
  int device = 0;
  int last_hip = 0;
  int spmv_variant = 0;  // 0 auto, 1 direct, 2 LDS-staged, 3/4 unrolled
  int group_width = 0;   // columns per block filter launch in batches (0: all)
  evk::BlkSched blk_sched;  // block filter schedule (evsl_set_block_schedule, autotuner)
  bool timing = true;
  bool use_graphs = true;  // batch group filters replayed from HIP graphs
  hipStream_t cap_stream = nullptr;  // private stream for graph capture (created on first use)
  // filter measurement
  int64_t filt_launches = 0;
  double filt_seconds = 0.0;
  double filt_bytes = 0.0;
  struct Pending {
    hipEvent_t a, b;
    int64_t launches;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  // grow-only workspace slots
  std::vector<void *> ws_ptr;
  std::vector<size_t> ws_size;
  double *pinned = nullptr;
  size_t pinned_cap = 0;
  // device memory held by this context (workspace, slice buffers, results)
  std::unordered_map<void *, size_t> live;
  int64_t mem_cur = 0, mem_peak = 0;
  // caller's device allocator (alloc == nullptr: hipMalloc / hipFree)
  evsl_alloc_t alloc{};
};

namespace evc {

inline void hipchk(evsl_ctx_t ctx, hipError_t e) {
  if (e != hipSuccess) {
    if (ctx) ctx->last_hip = (int)e;
    if (e == hipErrorOutOfMemory) fail(EVSL_ENOMEM);
    fail(EVSL_EHIP);
  }
}
#define HC(ctx, x) hipchk((ctx), (x))

inline void *dalloc(evsl_ctx_t ctx, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (ctx->alloc.alloc) {
    p = ctx->alloc.alloc(ctx->alloc.user, bytes, (void *)ctx->stream);
    if (!p) fail(EVSL_ENOMEM);
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ctx->last_hip = (int)e;
      fail(EVSL_ENOMEM);
    }
  }
  ctx->live[p] = bytes;
  ctx->mem_cur += (int64_t)bytes;
  ctx->mem_peak = std::max(ctx->mem_peak, ctx->mem_cur);
  return p;
}

// Frees a buffer from dalloc and takes it off the context's ledger.
inline void dfree(evsl_ctx_t ctx, void *p) {
  if (!p || !ctx) return;
  if (ctx->alloc.alloc)
    ctx->alloc.free(ctx->alloc.user, p, (void *)ctx->stream);
  else
    (void)hipFree(p);
  auto it = ctx->live.find(p);
  if (it != ctx->live.end()) {
    ctx->mem_cur -= (int64_t)it->second;
    ctx->live.erase(it);
  }
}

// Workspace slot `slot` of at least `bytes` bytes (contents not preserved on growth).
inline void *ws(evsl_ctx_t ctx, int slot, size_t bytes) {
  if ((int)ctx->ws_ptr.size() <= slot) {
    ctx->ws_ptr.resize(slot + 1, nullptr);
    ctx->ws_size.resize(slot + 1, 0);
  }
  if (ctx->ws_size[slot] < bytes) {
    if (ctx->ws_ptr[slot]) {
      HC(ctx, hipStreamSynchronize(ctx->stream));
      dfree(ctx, ctx->ws_ptr[slot]);
    }
    ctx->ws_ptr[slot] = nullptr;
    ctx->ws_size[slot] = 0;
    ctx->ws_ptr[slot] = dalloc(ctx, bytes);
    ctx->ws_size[slot] = bytes;
  }
  return ctx->ws_ptr[slot];
}

// Frees workspace slot `slot` (after the stream's pending work).
inline void ws_release(evsl_ctx_t ctx, int slot) {
  if ((int)ctx->ws_ptr.size() <= slot || !ctx->ws_ptr[slot]) return;
  HC(ctx, hipStreamSynchronize(ctx->stream));
  dfree(ctx, ctx->ws_ptr[slot]);
  ctx->ws_ptr[slot] = nullptr;
  ctx->ws_size[slot] = 0;
}

inline double *pinned(evsl_ctx_t ctx, size_t count) {
  if (ctx->pinned_cap < count) {
    if (ctx->pinned) {
      HC(ctx, hipStreamSynchronize(ctx->stream));
      (void)hipHostFree(ctx->pinned);
      ctx->pinned = nullptr;
      ctx->pinned_cap = 0;
    }
    void *p = nullptr;
    HC(ctx, hipHostMalloc(&p, count * sizeof(double), hipHostMallocDefault));
    ctx->pinned = (double *)p;
    ctx->pinned_cap = count;
  }
  return ctx->pinned;
}

inline hipEvent_t get_event(evsl_ctx_t ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HC(ctx, hipEventCreate(&e));
  return e;
}

// Resolve pending filter timings (waits for their completion).
inline void resolve_pending(evsl_ctx_t ctx) {
  for (auto &p : ctx->pending) {
    HC(ctx, hipEventSynchronize(p.b));
    float ms = 0.f;
    HC(ctx, hipEventElapsedTime(&ms, p.a, p.b));
    ctx->filt_seconds += ms * 1e-3;
    ctx->filt_launches += p.launches;
    ctx->filt_bytes += p.bytes;
    ctx->event_pool.push_back(p.a);
    ctx->event_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// Bracket a batch of filter launches with events (when timing is on).
struct FilterTimer {
  evsl_ctx_t ctx;
  hipEvent_t a = nullptr, b = nullptr;
  explicit FilterTimer(evsl_ctx_t c) : ctx(c) {
    if (ctx->timing) {
      a = get_event(ctx);
      HC(ctx, hipEventRecord(a, ctx->stream));
    }
  }
  void stop(int64_t launches, double bytes) {
    if (ctx->timing) {
      b = get_event(ctx);
      HC(ctx, hipEventRecord(b, ctx->stream));
      ctx->pending.push_back({a, b, launches, bytes});
      if (ctx->pending.size() > 4096) resolve_pending(ctx);
    } else {
      ctx->filt_launches += launches;
      ctx->filt_bytes += bytes;
    }
  }
};

// The context's capture stream (non-blocking, default priority).
inline hipStream_t capture_stream(evsl_ctx_t ctx) {
  if (!ctx->cap_stream) HC(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  return ctx->cap_stream;
}

// Ends a capture left open by an error, so the stream stays usable.
struct CaptureGuard {
  hipStream_t s;
  bool open = false;
  ~CaptureGuard() {
    if (open) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
    }
  }
};

inline evk::Csr to_csr(const evsl_csr_t *A) {
  evk::Csr c;
  c.n = (int)A->n;
  c.nnz = A->nnz;
  c.rp = A->row_ptr;
  c.ci = A->col;
  c.va = A->val;
  c.dtype = A->dtype;
  return c;
}

inline void check_csr(const evsl_csr_t *A) {
  if (!A || A->n <= 0 || A->n >= (int64_t)1 << 31 || A->nnz < 0 || !A->row_ptr || !A->col ||
      !A->val || (A->dtype != EVSL_F64 && A->dtype != EVSL_F32))
    fail(EVSL_EINVAL);
}

// Algorithmic bytes of one filter step over nc columns (value size s):
// the matrix once, plus P passes over the n x nc vectors.
inline double step_bytes(const evsl_csr_t *A, int nc, int s, int passes) {
  const double ma = (double)A->nnz * (s + 4) + 4.0 * (double)(A->n + 1);
  return ma + (double)passes * (double)A->n * nc * s;
}

// The block filter reads 16-bit column offsets from the row (half the index
// bytes) when every |col - row| < 2^15; they are built into workspace slots
// 26 and 27 (one pass over the matrix, synchronous). Ac.cd stays null for a
// matrix of larger bandwidth.
inline void attach_col_offsets(evsl_ctx_t ctx, const evsl_csr_t *A, evk::Csr &Ac) {
  if (A->nnz <= 0) return;
  int16_t *cd = (int16_t *)ws(ctx, 26, sizeof(int16_t) * (size_t)A->nnz);
  int *flag = (int *)ws(ctx, 27, sizeof(int) * 4);
  if (evk::make_col_offsets(ctx->stream, Ac, cd, flag)) Ac.cd = cd;
}

inline int pick_variant(evsl_ctx_t ctx) { return ctx->spmv_variant == 0 ? 3 : ctx->spmv_variant; }

}  // namespace evc

// Entry points run their body inside these: library errors become return codes.
#define EVSL_GUARD_BEGIN try {
#define EVSL_GUARD_END                  \
  }                                     \
  catch (const evc::Error &e) {         \
    return e.code;                      \
  }                                     \
  catch (const std::bad_alloc &) {      \
    return EVSL_ENOMEM;                 \
  }                                     \
  catch (...) {                         \
    return EVSL_EINVAL;                 \
  }
