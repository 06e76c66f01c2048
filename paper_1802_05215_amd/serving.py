"""Request serving for the spectrum-slicing library.

A stream of requests, each on its own matrix (a Laplacian with its own
potential), is served on one device:

* ``dos`` requests compute KPM moments of the whole spectrum (Section 2.1);
* ``eigs`` requests compute every eigenpair in an interval [xi, eta] placed
  by the KPM density (xi at a quantile of the cumulative count, eta where the
  estimated count reaches the request's target), sliced by the DOS into
  slices of about 100 eigenvalues, each solved by the filtered thick-restart
  Lanczos method with locking (Section 2.2, Algorithm 2), all slices of the
  request in one batch call.

Scheduling lives here; every numerical step is a call into the C-ABI. The
policy:

* requests wait in arrival order; the head of the queue is admitted when its
  device-memory footprint (an upper bound computed from the library's own
  sizing rules) fits in the budget next to the running requests and a worker
  slot is free. When the head does not fit, the earliest later request that
  does may start instead (a bypass), at most ``max_bypass`` times per head
  request; after that nothing overtakes it, so every request is admitted in
  bounded time (``max_bypass = 0``: strict FIFO);
* a request whose footprint exceeds the whole budget is rejected (status
  ``rejected``), a queued request can be cancelled until it is admitted;
* an admitted request runs on a worker thread with its own library context
  bound to its own HIP stream, so the device overlaps the work of all running
  requests; the ledger entry and the slot are returned when it finishes;
* every kernel choice is fixed by the request alone (group width, seeds,
  slice count), and the library's reductions have a fixed order, so a
  request computes the same bits alone or in any mix;
* an eigenpair request whose slices did not all converge (a slice status
  other than EVSL_OK) is reported as ``partial``: its pairs are returned but
  not counted as served eigenpairs.

The executor is pluggable: ``DeviceExecutor`` runs requests on the device;
tests run the admission logic on the CPU with a simulated one.
"""
from __future__ import annotations

import dataclasses
import math
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np

# ---------------------------------------------------------------- requests


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    kind: str               # "dos" or "eigs"
    dim: int                # 2 or 3
    N: int                  # grid points per side
    pot_seed: int
    kpm_degree: int = 100
    kpm_vectors: int = 20
    quantile: float = 0.3   # eigs: xi at this fraction of the spectrum's count
    target: int = 100       # eigs: wanted count in [xi, eta]

    @property
    def n(self) -> int:
        return self.N ** self.dim

    @property
    def nnz(self) -> int:
        N = self.N
        return 5 * N * N - 4 * N if self.dim == 2 else 7 * N ** 3 - 6 * N * N

    @property
    def nslices(self) -> int:
        return max(1, math.ceil(self.target / 100)) if self.kind == "eigs" else 0

    @property
    def nev_plan(self) -> int:
        """Per-slice eigenvalue estimate the solve is sized for (an upper
        clamp on what the executor passes as nev_est)."""
        return math.ceil(1.5 * self.target / max(self.nslices, 1)) + 10


def poisson_stream(seed: int, count: int, rate: float, n_min: float = 1e4, n_max: float = 4e6,
                   eig_range=(50, 400), first_at_zero: bool = False) -> List[Request]:
    """Seeded request stream: exponential inter-arrival times with mean
    1/rate; 2-D or 3-D with probability 1/2; n log-uniform in [n_min, n_max]
    and N the rounded dim-th root; DOS or eigenpair request with probability
    1/2; an eigenpair request targets a count uniform in eig_range from a
    count quantile uniform in [0.05, 0.6] of the spectrum."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        gap = rng.exponential(1.0 / rate) if rate > 0 else 0.0
        t += 0.0 if (first_at_zero and i == 0) else gap
        dim = 2 if rng.random() < 0.5 else 3
        n = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        N = max(8, int(round(n ** (1.0 / dim))))
        kind = "dos" if rng.random() < 0.5 else "eigs"
        out.append(Request(rid=i, arrival=t, kind=kind, dim=dim, N=N,
                           pot_seed=int(rng.integers(1, 2 ** 31)),
                           quantile=float(rng.uniform(0.05, 0.6)),
                           target=int(rng.integers(eig_range[0], eig_range[1] + 1))))
    return out


# ---------------------------------------------------------------- footprint
# The sizes below follow the library's allocation rules: Krylov dimension
# m = max(3 nev_est + 30, 60), lock capacity max(2 nev_est + 40, 100), a
# basis of (capacity + m + 1) columns with leading dimension n rounded up to
# 64, workspace slots that grow to the largest use and live until the
# context is destroyed, result vectors (at most the lock capacity per slice)
# held until they are copied out, and, in the precision form, the FP64
# polish (one slice at a time: two n-vectors per column of at most the lock
# capacity and three row-major blocks of 32 columns, freed when it ends).

_TPB = 256


def _ld(n: int) -> int:
    return (n + 63) // 64 * 64


def _blk_partials(n: int, nc: int) -> int:
    r0 = _TPB // nc if nc <= _TPB else 1
    passes = max(1, min(4 if (nc <= _TPB and r0 > 2) else 8, _TPB // r0))
    rpw = r0 * passes
    gy = 1 if nc <= _TPB else (nc + _TPB - 1) // _TPB
    return (n + rpw - 1) // rpw * gy


def _lan_sizes(nev_est: int, n: int):
    m = min(max(3 * nev_est + 30, 60), n - 1)
    cap = min(max(2 * nev_est + 40, 100), n)
    return m, cap


def footprint_parts(req: Request) -> Dict[str, int]:
    """Upper bounds (bytes) of the device memory a request holds: `matrix`
    (CSR with 32-bit indices and FP64 values), `library` (everything the
    library context allocates, comparable with its memory ledger) and
    `results` (the caller's copies of the eigenvectors)."""
    n, nnz = req.n, req.nnz
    ld = _ld(n)
    nv, K = req.kpm_vectors, req.kpm_degree
    parts = {"matrix": 12 * nnz + 4 * (n + 1)}
    # spectrum bounds (80 Lanczos steps) and KPM share workspace slots 0-4
    ws = 8 * (max(81 * ld, n * nv) + max(ld, n * nv)
              + max(((n + 1023) // 1024) * 82, n * nv)
              + max(82, _blk_partials(n, nv) * (K + 1) + (n * nv + 2047) // 2048 + 8)
              + max(K + 2, 82) + 256)
    if req.kind == "dos":
        parts["library"] = ws + 2 * nnz + 16   # with the 16-bit column offsets
        parts["results"] = 0
        return parts
    ns = req.nslices
    m, cap = _lan_sizes(req.nev_plan, n)
    cols = cap + m + 1
    # basis, filter output, two recurrence vectors and the staged input; Ritz
    # block; partial sums; Gram-Schmidt coefficients, norms and the DGKS gate;
    # coefficients
    per_slice = 8 * (ld * (cols + 4) + m * m
                     + max(((n + 1023) // 1024) * (cols + 8),
                           ((n + 2047) // 2048) * (max(m, cap) + 2))
                     + 2 * (cols + 8) + 3 * m + 16 + (n + 255) // 256 + 2 + 10001)
    # group blocks, coefficient table, pointer arrays, Ritz scratch, and the
    # 16-bit column offsets of the block filter
    batch = 8 * (3 * n * ns + ns * 10001 + 2 * (ns + 1)) + 8 * 2 * ld * m + 2 * nnz + 16
    vectors = 8 * n * cap * ns
    # precision form: the FP64 polish, one slice at a time and in place, of a
    # block of at most `cap` columns: its filtered block and work block, the
    # Gram matrix, the Gram partial sums (4096-row chunks), the dot partials,
    # and for the recurrence (chunks of at most 32 columns) three row-major
    # blocks, the coefficient table (degree <= 10000) and the column pointers
    ch = min(cap, 32)
    polish = 8 * (2 * ld * cap + cap * cap + ((n + 4095) // 4096) * cap * cap + 3 * cap + 8
                  + ((n + 2047) // 2048) * cap + 3 * n * ((ch + 1) // 2 * 2) + ch * 10001
                  + 2 * ch)
    parts["library"] = ws + batch + ns * per_slice + vectors + polish
    parts["results"] = vectors
    return parts


def footprint_bytes(req: Request) -> int:
    return sum(footprint_parts(req).values())


# ---------------------------------------------------------------- scheduler


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    start: float = 0.0
    end: float = 0.0
    status: str = "ok"            # ok | partial | failed | rejected | cancelled
    nev: int = 0
    lam: Optional[np.ndarray] = None
    res: Optional[np.ndarray] = None
    ycheck: Optional[np.ndarray] = None   # 1-norms of the eigenvectors
    moments: Optional[np.ndarray] = None
    interval: Optional[tuple] = None
    lib_peak: int = 0             # the context's measured device high-water mark
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.end - self.arrival


class Ledger:
    """Device-memory ledger and worker-slot count for admission."""

    def __init__(self, budget_bytes: int, max_running: int):
        self.budget = int(budget_bytes)
        self.max_running = int(max_running)
        self.used = 0
        self.high_water = 0
        self.running = 0

    def never_fits(self, req: Request) -> bool:
        return footprint_bytes(req) > self.budget

    def fits(self, req: Request) -> bool:
        return (self.running < self.max_running
                and self.used + footprint_bytes(req) <= self.budget)

    def admit(self, req: Request):
        fb = footprint_bytes(req)
        if self.running >= self.max_running or self.used + fb > self.budget:
            raise RuntimeError(f"request {req.rid} admitted over the budget")
        self.used += fb
        self.running += 1
        self.high_water = max(self.high_water, self.used)

    def release(self, req: Request):
        self.used -= footprint_bytes(req)
        self.running -= 1


class Server:
    """Admission in arrival order with bounded bypass against a Ledger; one
    worker thread per running request."""

    def __init__(self, ledger: Ledger, execute: Callable[[Request, float], Result],
                 clock: Callable[[], float] = time.perf_counter,
                 on_tick: Optional[Callable[[], None]] = None,
                 on_result: Optional[Callable[[Result], None]] = None,
                 max_bypass: int = 0):
        self.ledger = ledger
        self.max_bypass = int(max_bypass)
        self.bypassed: Dict[int, int] = {}   # head request id -> times it was passed over
        self.execute = execute
        self.clock = clock
        self.on_tick = on_tick
        self.on_result = on_result
        self._cv = threading.Condition()
        self._cancel = set()
        self.admission_order: List[int] = []

    def cancel(self, rid: int):
        """Cancels a request that has not been admitted yet (no effect after)."""
        with self._cv:
            self._cancel.add(rid)
            self._cv.notify_all()

    def run(self, requests: List[Request]) -> List[Result]:
        """Serves the stream; requests become visible at their arrival times.
        Returns one Result per request, in the order given."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queue: List[Request] = []
        results: Dict[int, Result] = {}
        threads = []
        t0 = self.clock()
        led = self.ledger

        def worker(req: Request):
            try:
                res = self.execute(req, t0)
            except Exception as exc:  # a failed request is reported, not fatal
                now = self.clock() - t0
                res = Result(req.rid, req.kind, req.arrival, now, now, status="failed",
                             error=repr(exc))
            with self._cv:
                results[req.rid] = res
                led.release(req)
                if self.on_result:
                    self.on_result(res)
                self._cv.notify_all()

        i = 0
        with self._cv:
            while len(results) < len(requests):
                now = self.clock() - t0
                while i < len(pending) and pending[i].arrival <= now:
                    queue.append(pending[i])
                    i += 1
                # cancelled and impossible requests leave the queue at once
                keep = []
                for r in queue:
                    if r.rid in self._cancel:
                        results[r.rid] = Result(r.rid, r.kind, r.arrival, now, now,
                                                status="cancelled")
                    elif led.never_fits(r):
                        results[r.rid] = Result(
                            r.rid, r.kind, r.arrival, now, now, status="rejected",
                            error=f"footprint {footprint_bytes(r)} B exceeds the budget "
                                  f"{led.budget} B")
                    else:
                        keep.append(r)
                queue = keep
                while queue:
                    head = queue[0]
                    if led.fits(head):
                        req = queue.pop(0)
                    elif self.bypassed.get(head.rid, 0) < self.max_bypass:
                        k = next((k for k in range(1, len(queue)) if led.fits(queue[k])), 0)
                        if k == 0:
                            break
                        req = queue.pop(k)
                        self.bypassed[head.rid] = self.bypassed.get(head.rid, 0) + 1
                    else:
                        break
                    led.admit(req)
                    self.admission_order.append(req.rid)
                    th = threading.Thread(target=worker, args=(req,), daemon=True)
                    threads.append(th)
                    th.start()
                if self.on_tick:
                    self.on_tick()
                if len(results) < len(requests):
                    wait = 0.25
                    if i < len(pending):
                        wait = min(wait, max(pending[i].arrival - (self.clock() - t0), 0.0))
                    self._cv.wait(timeout=wait)
        for th in threads:
            th.join()
        return [results[r.rid] for r in requests]


# ---------------------------------------------------------------- device executor


class DeviceExecutor:
    """Runs one request on the device: its own stream and library context;
    the matrix is generated on the host from the seeded input recipe and
    copied to the device; bounds, KPM, slicing, filters and the filtered
    Lanczos of all slices run in the library. prec "f32": the precision form
    (FP32 filter phase locking at tol_lo, then the FP64 phase; Ritz,
    reorthogonalisation and residuals FP64 throughout); "f64": FP64."""

    def __init__(self, tol: float = 1e-8, group_width: int = 0, device: str = "cuda:0",
                 prec: str = "f32", tol_lo: float = 0.0):
        if prec not in ("f32", "f64"):
            raise ValueError("prec must be f32 or f64")
        self.tol = tol
        self.group_width = group_width
        self.device = device
        self.prec = prec
        self.tol_lo = tol_lo

    def __call__(self, req: Request, t0: float) -> Result:
        import torch

        import evsl_inputs as I
        import paper_1802_05215_amd as ev

        start = time.perf_counter() - t0
        A = I.laplacian(req.N, req.dim, pot_seed=req.pot_seed)
        stream = torch.cuda.Stream(device=self.device)
        try:
            with torch.cuda.stream(stream):
                ctx = ev.Ctx(stream)
                try:
                    Ad = ev.DeviceCsr.from_host(A, device=self.device)
                    stream.synchronize()
                    out = self._solve(ev, torch, ctx, Ad, req)
                    stream.synchronize()
                    out.lib_peak = ctx.mem_stats()[1]
                finally:
                    ctx.close()
                del Ad
        finally:
            torch.cuda.empty_cache()
        out.start = start
        out.end = time.perf_counter() - t0
        return out

    def _solve(self, ev, torch, ctx, Ad, req):
        lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
        mom, _ = ev.evsl_kpm_dos(ctx, Ad, [lo, hi, lo, hi], req.kpm_degree, req.kpm_vectors,
                                 seed=1, damping=ev.DAMP_JACKSON)
        if req.kind == "dos":
            return Result(req.rid, "dos", req.arrival, moments=mom)
        xi, eta = eig_interval(ev, mom, lo, hi, req.quantile, req.target)
        ns = req.nslices
        intv = [xi, eta, lo, hi]
        sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, ns, 2000) if ns > 1 else \
            np.array([xi, eta])
        ivs, pols, opts = [], [], []
        for q in range(ns):
            iv = [float(sli[q]), float(sli[q + 1]), lo, hi]
            cnt = ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, iv[0], iv[1])
            ivs.append(iv)
            pols.append(ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON))
            nev_est = min(max(int(cnt * 1.3) + 5, 10), req.nev_plan)
            opts.append(ev.lan_opts(tol=self.tol, seed=2 + q, nev_est=nev_est,
                                    prec=ev.EVSL_F32 if self.prec == "f32" else ev.EVSL_F64,
                                    tol_lo=self.tol_lo))
        ctx.set_group_width(self.group_width)
        outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
        lams, ress, ychk = [], [], []
        status = "ok"
        for q, (lam, Y, res, st) in enumerate(outs):
            if st["status"] != ev.EVSL_OK:
                status = "partial"
            # a slice that starts at the lower spectrum bound owns everything below it
            keep = ((lam >= ivs[q][0]) | (ivs[q][0] <= lo)) & ((lam < ivs[q][1]) | (q == ns - 1)) \
                & (res <= self.tol)
            lams.append(lam[keep])
            ress.append(res[keep])
            if keep.any():
                ychk.append(torch.linalg.vector_norm(Y, 1, dim=0).cpu().numpy()[keep])
        del outs
        return Result(req.rid, "eigs", req.arrival, status=status,
                      nev=int(sum(len(x) for x in lams)),
                      lam=np.concatenate(lams), res=np.concatenate(ress),
                      ycheck=np.concatenate(ychk) if ychk else np.empty(0),
                      moments=mom, interval=(xi, eta))


def eig_interval(ev, mom, lo, hi, quantile, target):
    """[xi, eta] of an eigenpair request from the KPM count: xi where the
    cumulative count reaches `quantile` of the total, eta where the count
    from xi reaches `target` (bisection, 60 halvings each)."""
    total = ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, lo, hi)

    def at_count(c0, base):
        a, b = base, hi
        for _ in range(60):
            mid = 0.5 * (a + b)
            if ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, base, mid) < c0:
                a = mid
            else:
                b = mid
        return 0.5 * (a + b)

    xi = at_count(quantile * total, lo)
    eta = at_count(float(target), xi)
    return xi, eta


def summarize(results: List[Result], wall: float, ledger: Ledger) -> dict:
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok])
    nev = sum(r.nev for r in ok)
    return {
        "requests": len(results),
        "completed": len(ok),
        "partial": sum(r.status == "partial" for r in results),
        "failed": sum(r.status == "failed" for r in results),
        "rejected": sum(r.status == "rejected" for r in results),
        "cancelled": sum(r.status == "cancelled" for r in results),
        "eigenpairs": int(nev),
        "wall_s": wall,
        "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "eigenpairs_per_s": nev / wall if wall > 0 else None,
        "requests_per_s": len(ok) / wall if wall > 0 else None,
        "ledger_high_water_bytes": int(ledger.high_water),
    }
