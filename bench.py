"""Benchmark of the polynomial-filtered spectrum-slicing hot path on one MI355X.

One step is one pass of the whole path over one synthetic matrix resident in
HBM: Lanczos spectrum bounds -> KPM moments -> DOS slicing -> one Chebyshev
filter per slice -> filtered thick-restart Lanczos with locking on every
slice (all slices advance together, their filters applied as one block SpMM
per degree step) -> eigenpairs with residual <= tol.

Default workload: 3-D 7-point Laplacian on a 100^3 grid (n = 1e6, nnz =
6.94e6, CSR FP64) plus a diagonal potential uniform in [0, 1) (SplitMix64,
seed 0); all eigenvalues in [0.60, 0.70], cut into 10 slices by a KPM density
estimate (degree 80, 20 Rademacher vectors, Jackson damping); Jackson
filters with tau = 0.8; tolerance 1e-8 on ||A u - lambda u|| / ||A||.

The default run does one warm-up solve, then whole timed solves while the
next one still ends before --time-budget seconds from the start (at most
--steps), then the batched 200^3 filter leg (one FP64 Clenshaw degree step
over a 512-column block per launch, reported under "c3_filter"), then the
oracle's bounded sample ("cpu_baseline"). Only slices whose solver status is
EVSL_OK count towards eigenpairs/s.

Prints one JSON line (see the keys below); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.perf_counter()
METRIC = "eigenpairs/s + filter SpMM HBM GB/s at resid<=1e-8; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="at most this many timed solves (fewer when --time-budget ends them)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up solves (at most 1 is run)")
    ap.add_argument("--time-budget", type=float, default=330.0,
                    help="seconds from the start after which no further timed solve begins "
                         "(0: run all --steps)")
    ap.add_argument("--no-c3", dest="c3", action="store_false",
                    help="skip the 200^3 x 512-column filter leg of the default run")
    ap.add_argument("--c3-only", action="store_true",
                    help="only the 200^3 x 512-column filter leg (its own JSON line)")
    ap.add_argument("--c3-kpm-degree", type=int, default=2000,
                    help="200^3 leg: KPM degree of the cut (degree 80 cannot resolve the "
                         "spectrum's lower edge)")
    ap.add_argument("--c3-degree", type=int, default=24,
                    help="200^3 leg: degree of the truncated filters (launches per application "
                         "= degree + 1)")
    ap.add_argument("--c3-launches", type=int, default=25,
                    help="200^3 leg: at least this many timed launches")
    ap.add_argument("--grid", type=int, default=100, help="N of the N^3 grid")
    ap.add_argument("--interval", type=float, nargs=2, default=[0.60, 0.70])
    ap.add_argument("--nslices", type=int, default=10)
    ap.add_argument("--interval-count", type=int, default=0,
                    help="interval [lambda_min, eta] with eta where the KPM count reaches this "
                         "number (replaces --interval)")
    ap.add_argument("--slices", type=int, nargs="+", default=None,
                    help="solve only these slices of the KPM cut (default: all)")
    ap.add_argument("--dos", choices=["kpm", "lanczos"], default="kpm",
                    help="density estimate for slicing: KPM moments or Lanczos quadrature "
                         "(--kpm-degree steps, --kpm-vectors probes)")
    ap.add_argument("--dos-sigma", type=float, default=0.0,
                    help="Lanczos DOS: Gaussian spread of each quadrature node "
                         "(0: (lambda_max - lambda_min) / (2 steps))")
    ap.add_argument("--kpm-degree", type=int, default=80)
    ap.add_argument("--kpm-vectors", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--m-factor", type=float, default=0.0,
                    help="Lanczos dimension m = factor * nev_est + 30 (0: the library default)")
    ap.add_argument("--tune-schedule", choices=["auto", "on", "off"], default="auto",
                    help="autotune the block filter's launch schedule for the batch's group "
                         "width (auto: matrices of 4e6 rows or more)")
    ap.add_argument("--ncycle", type=int, default=0,
                    help="Lanczos steps between early-restart tests (0: the library default)")
    ap.add_argument("--max-its", type=int, default=0,
                    help="cap on Lanczos steps per slice (profiling runs only; 0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--group-width", type=int, default=-1,
                    help="slices per block filter launch (-1: autotuned, 0: all)")
    ap.add_argument("--no-precision-leg", action="store_true",
                    help="skip the precision form's solve of the same cut after the timed "
                         "FP64 steps")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64",
                    help="filter arithmetic (f32: precision form, FP32 phase then FP64 phase)")
    ap.add_argument("--tol-lo", type=float, default=0.0, help="FP32-phase lock tolerance")
    ap.add_argument("--precision-out", default="",
                    help="--precision-study: write the per-eigenvalue table (CSV) here")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain copy kernel (1 GiB) used to calibrate counters")
    ap.add_argument("--method", choices=["tr", "nr", "si"], default="tr",
                    help="slice solver: thick-restart Lanczos (default), non-restart Lanczos, "
                         "subspace iteration")
    ap.add_argument("--si-block", type=int, default=0,
                    help="subspace iteration: vectors per slice (0: 3 nev_est + 8)")
    ap.add_argument("--mode", choices=["batch", "serial"], default="batch",
                    help="batch: all slices in lock-step; serial: one slice after another")
    ap.add_argument("--filter-only", action="store_true",
                    help="filter SpMM only: FP64 and FP32 on an n x columns block")
    ap.add_argument("--columns", type=int, default=512)
    ap.add_argument("--degrees", type=int, nargs="+", default=[50, 100, 200, 300])
    ap.add_argument("--paper-table", action="store_true",
                    help="the twelve Laplacian problems of the paper's Section 4.1 tables, "
                         "solved by the non-restart filtered Lanczos")
    ap.add_argument("--rows", type=int, nargs="+", default=None,
                    help="--paper-table: rows to run (0-11, default all)")
    ap.add_argument("--methods", nargs="+", default=["nr"], choices=["nr", "tr"])
    ap.add_argument("--precision-study", action="store_true",
                    help="FP64 and FP32-filter solves of the same slices, eigenvalue by eigenvalue "
                         "(default slices [0.50,0.60], [0.60,0.65], [0.60,0.625] of the grid)")
    ap.add_argument("--small", action="store_true",
                    help="the 40x40 plain case: whole-path latency over repeated solves, "
                         "with and without HIP graphs")
    ap.add_argument("--repeats", type=int, default=50)
    ap.add_argument("--pencil", action="store_true",
                    help="generalized problem: a finite-element pencil (A, B) with a closed-form "
                         "spectrum, both Lanczos forms")
    ap.add_argument("--pencil-n", type=int, default=100, help="N of the N x N pencil grid")
    ap.add_argument("--pencil-count", type=int, default=100,
                    help="eigenvalues in the pencil's interval")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: a Poisson stream of DOS and eigenpair requests")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--serve-seed", type=int, default=7)
    ap.add_argument("--serve-nmax", type=float, default=4e6)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="arrivals per second (0: 0.7 x the capacity of a calibration run)")
    ap.add_argument("--calib", type=int, default=4, help="requests served alone to calibrate")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-running", type=int, default=4)
    ap.add_argument("--max-bypass", type=int, default=8,
                    help="serving: times a waiting head request may be passed over")
    ap.add_argument("--serve-prec", choices=["f32", "f64"], default="f32",
                    help="serving: FP32-filter precision form (default) or FP64")
    ap.add_argument("--serve-log", default="",
                    help="serving: append one JSON record per finished request to this file")
    return ap.parse_args()


def one_step(ctx, ev, Ad, args):
    """Runs the whole path once; returns the per-step record."""
    import torch
    t0 = time.perf_counter()
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    xi, eta = args.interval
    if args.interval_count > 0:
        xi, eta = lo, hi
    intv = [xi, eta, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, args.kpm_degree, args.kpm_vectors, seed=1,
                               damping=ev.DAMP_JACKSON)
    if args.dos == "lanczos":
        quad = ev.evsl_lanczos_dos(ctx, Ad, args.kpm_degree, args.kpm_vectors, seed=1)
        # the quadrature has m nodes per probe: spread each over the spacing of
        # m points on the spectrum, so the count is smooth enough to cut
        sigma = args.dos_sigma or (hi - lo) / (2 * args.kpm_degree)
        count = lambda x0, x1: ev.evsl_lanczos_count(quad, Ad.n, sigma, x0, x1)
    else:
        count = lambda x0, x1: ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, x0, x1)
    if args.interval_count > 0:
        # eta where the estimated count from lambda_min reaches interval_count
        a, b = lo, hi
        for _ in range(60):
            mid = 0.5 * (a + b)
            if count(lo, mid) < args.interval_count:
                a = mid
            else:
                b = mid
        eta = 0.5 * (a + b)
        intv = [lo, eta, lo, hi]
        est = count(lo, eta)
    if args.dos == "lanczos":
        est = count(intv[0], intv[1])
        sli = ev.evsl_slice_spectrum_lanczos(quad, Ad.n, sigma, intv[0], intv[1], args.nslices,
                                             2000)
    else:
        sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, args.nslices, 2000)
    sel = args.slices if args.slices else list(range(args.nslices))
    ivs, pols, opts = [], [], []
    for q in sel:
        iv = [sli[q], sli[q + 1], lo, hi]
        cnt = count(sli[q], sli[q + 1])
        ivs.append(iv)
        pols.append(ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON, tau=0.8, tau_ext=0.4))
        nev_est = max(int(cnt * 1.1) + 5, 10)
        if args.method == "si":
            opts.append(ev.si_opts(tol=args.tol, seed=2 + q, nev_est=nev_est,
                                   max_its=args.max_its, block=args.si_block))
        else:
            opts.append(ev.lan_opts(tol=args.tol, seed=2 + q, nev_est=nev_est, ncycle=args.ncycle,
                                    m=int(args.m_factor * nev_est) + 30 if args.m_factor else 0,
                                    max_its=args.max_its,
                                    prec=ev.EVSL_F32 if args.prec == "f32" else ev.EVSL_F64,
                                    tol_lo=args.tol_lo,
                                    method=ev.EVSL_LAN_NR if args.method == "nr" else ev.EVSL_LAN_TR))
    if args.group_width < 0:
        gw, us = ev.evsl_autotune(ctx, Ad, len(sel),
                                  ev.EVSL_F32 if args.prec == "f32" else ev.EVSL_F64)
    else:
        ctx.set_group_width(args.group_width)
        gw, us = args.group_width, None
    sched = None
    tune = args.tune_schedule == "on" or (args.tune_schedule == "auto" and Ad.n >= 4_000_000)
    if tune and min(gw or len(sel), len(sel)) >= 4:
        # large matrices: the block filter's launch schedule for the group width
        sched = ev.evsl_autotune_schedule(ctx, Ad, min(gw or len(sel), len(sel)),
                                          ev.EVSL_F32 if args.prec == "f32" else ev.EVSL_F64)
    t_setup = time.perf_counter() - t0
    if args.method == "si":
        if args.mode == "batch":
            outs = ev.evsl_filtered_subspace_batch(ctx, Ad, ivs, pols, opts)
        else:
            outs = [ev.evsl_filtered_subspace(ctx, Ad, ivs[q], pols[q], opts[q])
                    for q in range(len(sel))]
    elif args.mode == "batch":
        outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
    else:
        outs = [ev.evsl_filtered_lanczos(ctx, Ad, ivs[q], pols[q], opts[q])
                for q in range(len(sel))]
    torch.cuda.synchronize()
    t_tot = time.perf_counter() - t0
    lams, ress, per_slice = [], [], []
    for q, (lam, Y, res, st) in enumerate(outs):
        last = sel[q] == args.nslices - 1
        # a slice that starts at the lower spectrum bound owns everything below it
        keep = ((lam >= ivs[q][0]) | (ivs[q][0] <= ivs[q][2])) & ((lam < ivs[q][1]) | last) \
            & (res <= args.tol)
        if st["status"] != ev.EVSL_OK:
            # an unconverged slice may miss eigenpairs: none of its pairs count
            keep &= False
        lams.append(lam[keep])
        ress.append(res[keep])
        per_slice.append(dict(slice=sel[q], deg=pols[q].deg, nev=int(keep.sum()), niter=st["niter"],
                              nev_est=opts[q].nev_est,
                              nmv=st["nmv"], t_done=st["t_tot"], t_mv=st["t_mv"],
                              t_orth=st["t_orth"], t_ritz=st["t_ritz"], status=st["status"],
                              npolish=st["npolish"], north2=st["north2"]))
    lam_all = np.concatenate(lams)
    return dict(t=t_tot, t_setup=t_setup, group_width=gw, tune_us=us, schedule=sched,
                nev=len(lam_all), lam=lam_all,
                res=np.concatenate(ress), bounds=(lo, hi), kpm_est=est, slices=sli, interval=intv[:2],
                per_slice=per_slice, pols=pols, ivs=ivs)


def host_info():
    """CPU model and logical core count of this host (for the oracle timings)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def cpu_baseline(A, rec, args, c3=None, budget_s=25.0):
    """The oracle, timed on this host's cores, on a bounded sample of the
    default workload: its thick-restart filtered Lanczos (Algorithm
    alg:FiltLanTR) on the highest-degree slice of the GPU run's cut, stopped
    after a fixed number of Lanczos steps (filter, deflation, full
    reorthogonalisation, as in a full solve). Its time per Lanczos step per
    filter degree is then scaled to the Lanczos steps and degrees of every
    slice of the GPU run. The early steps reorthogonalise against a short
    basis, so the scaled time is a lower bound on the oracle's full solve
    and the rate an upper bound. With the 200^3 filter leg, the oracle also
    filters one column of that block (one of its degree-k filters), checked
    against the GPU's column."""
    import oracle
    model, nproc = host_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or nproc
    oracle.lib()
    q = int(np.argmax([p.deg for p in rec["pols"]]))
    p = rec["pols"][q]
    iv = rec["ivs"][q]
    opol = oracle.find_pol(iv, damping=2, tau=0.8, tau_ext=0.4)
    ps = rec["per_slice"][q]
    # one filter application (deg products with A) to size the sample
    t0 = time.perf_counter()
    oracle.filter_apply(A, p.cc, p.dd, p.coef, np.ones(A.n))
    t_filter = time.perf_counter() - t0
    steps = int(max(2, min(40, budget_s / max(t_filter, 1e-3))))
    t0 = time.perf_counter()
    _, _, _, ost = oracle.filtered_lanczos(A, iv, opol, tol=args.tol, seed=2 + ps["slice"],
                                           max_its=steps, nev_est=ps["nev_est"])
    dt = time.perf_counter() - t0
    per_step_deg = dt / max(ost["niter"], 1) / opol["deg"]
    est_time = sum(s["niter"] * s["deg"] for s in rec["per_slice"]) * per_step_deg
    out = {"value": rec["nev"] / est_time, "unit": "eigenpairs/s", "cores": threads,
           "kind": "oracle", "host_cpu": model, "host_nproc": nproc,
           "sample": (f"oracle thick-restart filtered Lanczos on slice {ps['slice']} "
                      f"(degree {opol['deg']}) of the same cut, on the full 100^3 matrix, stopped "
                      f"after {ost['niter']} Lanczos steps ({dt:.1f} s, "
                      f"{per_step_deg * 1e3:.3f} ms per step per degree); scaled to the "
                      f"{sum(s['niter'] for s in rec['per_slice'])} Lanczos steps x degree of "
                      f"all slices of the GPU run ({est_time:.0f} s). Early steps reorthogonalise "
                      f"against a short basis, so this rate is an upper bound on the oracle's")}
    if c3 is not None and c3.get("check_column") is not None:
        col = c3.pop("check_column")
        t0 = time.perf_counter()
        yo = oracle.filter_apply(c3.pop("A_host"), col["cc"], col["dd"], col["coef"], col["v"])
        out["c3_column_check"] = {
            "rel_err_vs_oracle": float(np.linalg.norm(col["y"] - yo) / np.linalg.norm(col["v"])),
            "degree": len(col["coef"]) - 1, "column": col["index"],
            "oracle_s": time.perf_counter() - t0}
    return out


def precision_leg(ctx, ev, Ad, args, rec64, value64, log):
    """The precision form on the same cut, one solve after the timed FP64
    steps: the FP32-filter Lanczos phase, then the FP64 polish (Rayleigh-Ritz
    and FP64 filter applications to each slice's block) and, where pairs
    remain, the FP64 thick-restart continuation, at the same tolerance.
    Reports its eigenpairs/s beside the FP64 value, whether the counts agree,
    the FP64 phase each slice took (npolish) and the largest residual. A
    failure is reported in the leg rather than raised, so that the rest of the
    line stands."""
    import copy
    import torch
    try:
        a = copy.copy(args)
        a.prec = "f32"
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = one_step(ctx, ev, Ad, a)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        v = r["nev"] / dt
        log(f"[precision] {r['nev']} eigenpairs in {dt:.1f} s ({v:.2f}/s; FP64 {value64:.2f}/s)")
        return {
            "workload": "the same cut in the precision form (FP32-filter Lanczos phase, then the "
                        "FP64 polish and, where pairs remain, the FP64 thick-restart "
                        f"continuation), tol {args.tol:g}",
            "value": v, "unit": "eigenpairs/s", "seconds": dt, "nev": r["nev"],
            "fp64_value": value64, "fp64_nev": rec64["nev"],
            "ratio_to_fp64": v / value64 if value64 > 0 else None,
            "counts_equal": r["nev"] == rec64["nev"],
            "group_width": r["group_width"],
            "npolish": [p["npolish"] for p in r["per_slice"]],
            "status": [p["status"] for p in r["per_slice"]],
            "max_residual": float(r["res"].max()) if r["nev"] else None,
        }
    except Exception as e:  # the leg must not cost the measured line
        log(f"[precision] failed: {e!r}")
        return {"error": repr(e)}


def c3_filter_leg(ctx, ev, args, log):
    """The batched 200^3 workload's filter step: 3-D 7-point Laplacian 200^3 +
    U[0,1) potential (seed 0), interval [lambda_min, eta] with eta where the
    KPM count (degree 2000, 20 probes) reaches 512, cut into 32 KPM slices; the
    512-column block (16 columns per slice, Gaussian, torch generator seed 0)
    filtered by one Clenshaw degree step per launch over all 512 columns
    (FP64). Every slice's filter is truncated to the same degree so that each
    timed launch is a full-width step; the slices' own degrees are reported
    beside. Times come from HIP events on the context stream around the filter
    application (k + 1 launches, the two zero fills of the Clenshaw buffers
    included in time and bytes)."""
    import concurrent.futures as cf
    import torch

    import evsl_inputs as I
    t0 = time.perf_counter()
    N, ncols, nsl, kstep = 200, 512, 32, args.c3_degree
    A = I.laplacian(N, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A, device="cuda:0")
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    mom, _ = ev.evsl_kpm_dos(ctx, Ad, [lo, hi, lo, hi], args.c3_kpm_degree, 20, seed=1,
                             damping=ev.DAMP_JACKSON)
    cnt = lambda x0, x1: ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, x0, x1)
    a, b = lo, hi
    for _ in range(60):
        mid = 0.5 * (a + b)
        a, b = (mid, b) if cnt(lo, mid) < 512 else (a, mid)
    eta = 0.5 * (a + b)
    sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, [lo, eta, lo, hi], nsl, 2000)
    ivs = [[sli[q], sli[q + 1], lo, hi] for q in range(nsl)]
    with cf.ThreadPoolExecutor(8) as ex:
        real = list(ex.map(lambda iv: ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON), ivs))
    pols = [ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON, max_deg=kstep) for iv in ivs]
    assert all(p.deg == kstep for p in pols)
    cg = np.arange(ncols) // (ncols // nsl)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(0)
    V = torch.randn((A.n, ncols), dtype=torch.float64, device="cuda:0", generator=g)
    Y = torch.empty_like(V)
    # the block filter's launch schedule for this matrix and width (kept in ctx)
    sched = ev.evsl_autotune_schedule(ctx, Ad, ncols, ev.EVSL_F64)
    t_setup = time.perf_counter() - t0
    ev.evsl_filter_apply(ctx, Ad, pols, cg, V, Y)  # warm-up
    torch.cuda.synchronize()
    ctx.reset_stats()
    reps = max(1, -(-args.c3_launches // (kstep + 1)))
    for _ in range(reps):
        ev.evsl_filter_apply(ctx, Ad, pols, cg, V, Y)
    torch.cuda.synchronize()
    fs = ctx.filter_stats()
    ctx.reset_stats()
    gbps = fs["bytes"] / fs["seconds"] / 1e9
    m_a = 12.0 * A.nnz + 4.0 * (A.n + 1)
    step_bytes = m_a + 4.0 * A.n * ncols * 8
    out = {
        "workload": (f"batched filter: 3-D 7-point Laplacian {N}^3 + U[0,1) potential (seed 0), "
                     f"[lambda_min, eta_512] = [{lo:.6g}, {eta:.6g}] cut into {nsl} KPM slices "
                     f"(degree {args.c3_kpm_degree}), "
                     f"{ncols} columns ({ncols // nsl} per slice), FP64 Clenshaw degree step "
                     f"over all {ncols} columns per launch"),
        "n": A.n, "nnz": A.nnz, "columns": ncols,
        "slice_degrees": [p.deg for p in real],
        "timed_degree": kstep, "launches": fs["launches"],
        "schedule": {"map": sched[0], "chunk_cols": sched[1], "group": sched[2],
                     "lane_cols": sched[3], "rows_per_wg": sched[4], "lds_staging": sched[5],
                     "tuner_ms_per_step": sched[6]},
        "ms_per_launch": fs["seconds"] / fs["launches"] * 1e3,
        "bytes_per_step": step_bytes,
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBS, "traffic": None,
                     "traffic_bytes_per_launch": None,
                     "kernel": "k_cheb_blk_lds<double, STEP_CLEN> at 512 columns"},
        "setup_s": t_setup,
    }
    tb = measured_traffic(COUNTERS_C3, sched[:6])
    if tb is not None:
        out["roofline"]["traffic"] = tb / (fs["seconds"] / fs["launches"]) / 1e9
        out["roofline"]["traffic_bytes_per_launch"] = tb
    log(f"[c3] {fs['launches']} launches, {out['ms_per_launch']:.2f} ms each, {gbps:.0f} GB/s "
        f"({gbps / HBM_PEAK_GBS:.2f} of peak); degrees {min(out['slice_degrees'])}-"
        f"{max(out['slice_degrees'])}")
    if not args.no_cpu_baseline:
        j = int(ncols // 2)
        p = pols[cg[j]]
        out["check_column"] = {"index": j, "v": V[:, j].cpu().numpy(), "y": Y[:, j].cpu().numpy(),
                               "cc": p.cc, "dd": p.dd, "coef": p.coef}
        out["A_host"] = A
    del V, Y
    ctx.set_block_schedule(1, 0, 1, 0, 0, 1)
    torch.cuda.empty_cache()
    return out


KERNEL_SRC = os.path.join(ROOT, "paper_1802_05215_amd", "csrc", "kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "filter_step_100cube_counters.txt")
COUNTERS_C3 = os.path.join(ROOT, "profiles", "filter_block_200cube_512col_counters.txt")


def filter_kernel_source():
    """Source text of the measured filter kernel and its launch configuration
    (from the LDS-staged block kernel to the explicit instantiations of its
    launcher) in csrc/kernels.hip."""
    src = open(KERNEL_SRC).read()
    i = src.index("// Row-major block, LDS-staged")
    j = src.index("template void cheb_blk<float>")
    return src[i:j]


def measured_traffic(path=None, schedule=None):
    """HBM bytes per filter launch from a committed counter summary (default:
    the 100^3 step's), or None when the kernel source has changed since the
    counters were taken. With `schedule` (map, chunk_cols, group, lane_cols,
    rows_per_wg, lds_staging), the bytes of that schedule from the summary's
    per-schedule fetch table (None when it holds no such row)."""
    import hashlib
    path = path or COUNTERS
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(filter_kernel_source().encode()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or "hbm_bytes_per_launch" not in kv:
        return None
    if schedule is None:
        return float(kv["hbm_bytes_per_launch"])
    key = "fetch_kib[" + ",".join(str(int(x)) for x in schedule) + "]"
    if key not in kv:
        return None
    return (float(kv[key]) * 1024 * float(kv["fetch_scale"])
            + float(kv["write_kib_per_launch"]) * 1024 * float(kv["write_scale"]))


def copy_probe_main():
    import torch
    import paper_1802_05215_amd as ev
    ev.load()
    ctx = ev.Ctx()
    nbytes = 1 << 30
    t = ev.evsl_copy_probe(ctx, nbytes, 20)
    print(json.dumps({"copy_probe_bytes": nbytes, "seconds_per_copy": t,
                      "gbps_read_plus_write": 2 * nbytes / t / 1e9}), flush=True)


def filter_only_main(args):
    """Filter-only workload: Y = p_g(A-hat) V for an n x `columns` block, one
    filter per 16-column group (32 groups of degree exactly k, centred at
    evenly spaced points of [0.30, 0.50]), in FP64 and in FP32, for each k of
    `degrees`. Reports the filter SpMM rate in algorithmic HBM GB/s (events
    on the context stream), the FP32 relative error per column against FP64,
    and a full-size oracle check of one FP64 column at the smallest degree."""
    import torch

    import evsl_inputs as I
    import paper_1802_05215_amd as ev

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    N, nc = args.grid, args.columns
    A = I.laplacian(N, 3, pot_seed=0)
    n = A.n
    Ad = ev.DeviceCsr.from_host(A, device="cuda:0")
    A32 = Ad.with_values(Ad.val.float())
    ctx = ev.Ctx()
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    ngroups = max(1, nc // 16)
    cg = np.minimum(np.arange(nc) // 16, ngroups - 1)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(0)
    V64 = torch.randn((n, nc), dtype=torch.float64, device="cuda:0", generator=g)
    V32 = V64.float()
    Y64 = torch.empty_like(V64)
    Y32 = torch.empty_like(V32)
    recs = []
    oracle_check = None
    for k in sorted(args.degrees):
        centres = np.linspace(0.30, 0.50, ngroups)
        pols = [ev.evsl_cheb_coeffs([c - 1e-4, c + 1e-4, lo, hi], max_deg=k) for c in centres]
        assert all(p.deg == k for p in pols)
        row = {"degree": k}
        for name, V, Y, Am in (("f64", V64, Y64, Ad), ("f32", V32, Y32, A32)):
            ev.evsl_filter_apply(ctx, Am, pols, cg, V, Y)  # warm-up
            torch.cuda.synchronize()
            ctx.reset_stats()
            t0 = time.perf_counter()
            ev.evsl_filter_apply(ctx, Am, pols, cg, V, Y)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            fs = ctx.filter_stats()
            row[name] = {"gbps": fs["bytes"] / fs["seconds"] / 1e9,
                         "ms_per_step": fs["seconds"] / fs["launches"] * 1e3,
                         "bytes_per_step": fs["bytes"] / fs["launches"], "wall_s": wall}
            log(f"[filter] k {k} {name}: {row[name]['gbps']:.0f} GB/s, "
                f"{row[name]['ms_per_step']:.2f} ms per step")
        errs, errv = [], []
        for c0 in range(0, nc, 64):
            y = Y64[:, c0:c0 + 64]
            dn = (Y32[:, c0:c0 + 64].double() - y).norm(dim=0)
            errs.append((dn / y.norm(dim=0)).cpu().numpy())
            errv.append((dn / V64[:, c0:c0 + 64].norm(dim=0)).cpu().numpy())
        errs, errv = np.concatenate(errs), np.concatenate(errv)
        # relative to ||Y64|| (the filtered output is small: the filter keeps only
        # the components near its centre) and relative to ||V||
        row["f32_rel_err"] = {"max": float(errs.max()), "median": float(np.median(errs))}
        row["f32_err_rel_v"] = {"max": float(errv.max()), "median": float(np.median(errv))}
        if oracle_check is None and not args.no_cpu_baseline:
            import oracle
            v0 = V64[:, 0].cpu().numpy()
            p0 = pols[cg[0]]
            t0 = time.perf_counter()
            yo = oracle.filter_apply(A, p0.cc, p0.dd, p0.coef, v0)
            dt = time.perf_counter() - t0
            y0 = Y64[:, 0].cpu().numpy()
            oracle_check = {"degree": k, "column": 0,
                            "rel_err_vs_oracle": float(np.linalg.norm(y0 - yo) /
                                                       np.linalg.norm(v0)),
                            "oracle_s": dt}
            log(f"[filter] oracle check: {oracle_check}")
        recs.append(row)
    print(json.dumps({
        "metric": "filter SpMM HBM GB/s (algorithmic bytes), FP64 and FP32",
        "value": max(r["f64"]["gbps"] for r in recs),
        "unit": "GB/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": (f"filter only: 3-D 7-point Laplacian {N}^3 + U[0,1) potential "
                                f"(seed 0), {nc} Gaussian columns (seed 0), {ngroups} filters "
                                f"of degree k, one per 16 columns"),
                   "n": n, "nnz": A.nnz, "columns": nc},
        "per_degree": recs,
        "oracle_check": oracle_check,
        "peak_gbps": HBM_PEAK_GBS,
    }), flush=True)


# The Laplacian problems of Table tab:lap (grid, printed bounds [a, b],
# interval, count nu) with the ChebLanNr results the paper prints in Table
# tab:lap_pol_results (deg, niter, nmv, t-mv, t-orth, t-tot in seconds on the
# paper's CPU), quoted as context.
PAPER_ROWS = [
    # dim, N, [a, b], [xi, eta], nu, deg, niter, nmv, t_mv, t_orth, t_tot
    (2, 343, (0, 7.9998), (0.40, 0.436), 356, 157, 1290, 203200, 10.66, 24.11, 51.95),
    (2, 343, (0, 7.9998), (1.00, 1.033), 347, 256, 1310, 336219, 17.39, 25.48, 66.71),
    (2, 729, (0, 7.9998), (0.40, 0.410), 446, 557, 1610, 898330, 182.51, 168.20, 497.78),
    (2, 729, (0, 7.9998), (1.00, 1.009), 435, 936, 1590, 1490547, 294.33, 179.45, 679.08),
    (2, 1000, (0, 7.9998), (0.40, 0.405), 429, 1111, 1530, 1702481, 1451.40, 308.98, 2410.99),
    (2, 1000, (0, 7.9998), (1.00, 1.005), 460, 1684, 1670, 2816108, 2402.99, 367.49, 3804.91),
    (3, 49, (0, 11.9882), (0.40, 0.570), 343, 43, 1290, 55899, 3.81, 26.53, 41.03),
    (3, 49, (0, 11.9882), (1.00, 1.100), 345, 107, 1270, 136449, 9.80, 24.25, 47.00),
    (3, 81, (0, 11.9882), (0.40, 0.450), 433, 141, 1590, 224905, 77.24, 189.91, 359.61),
    (3, 81, (0, 11.9882), (1.00, 1.028), 420, 378, 1570, 594636, 191.42, 168.33, 494.66),
    (3, 100, (0, 11.9882), (0.40, 0.428), 454, 248, 1710, 425030, 563.36, 398.70, 1250.26),
    (3, 100, (0, 11.9882), (1.00, 1.018), 475, 588, 1830, 1077689, 1357.12, 426.17, 2314.43),
]


def paper_table_main(args):
    """The paper's Laplacian experiments on one GPU: for each problem, the
    filter (sigma damping, tau = 0.8, from the printed bounds) and the filtered
    Lanczos solve at tol 1e-8; the eigenvalues are checked against the closed
    form 4 - 2 cos(i pi/(N+1)) - 2 cos(j pi/(N+1)) (and the 3-D analogue)."""
    import torch

    import evsl_inputs as I
    import paper_1802_05215_amd as ev

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx = ev.Ctx()
    rows = args.rows if args.rows is not None else range(len(PAPER_ROWS))
    out = []
    for ri in rows:
        dim, N, ab, iv, nu, pdeg, pniter, pnmv, ptmv, ptorth, pttot = PAPER_ROWS[ri]
        A = I.laplacian(N, dim)
        Ad = ev.DeviceCsr.from_host(A, device="cuda:0")
        c = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
        ex = (c[:, None] + c[None, :]) if dim == 2 else \
            (c[:, None, None] + c[None, :, None] + c[None, None, :])
        ex = np.sort(ex.ravel())
        want = ex[(ex >= iv[0]) & (ex <= iv[1])]
        # degree with the printed bounds (the paper's filter); the solve uses
        # bounds that contain the spectrum: for 81^3 and 100^3 the printed b
        # (that of 49^3) lies below lambda_max, and the filter grows without
        # bound above it
        pdeg_printed = ev.evsl_cheb_coeffs([iv[0], iv[1], ab[0], ab[1]],
                                           damping=ev.DAMP_SIGMA, tau=0.8, tau_ext=0.4).deg
        lo_c, hi_c = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
        intv = [iv[0], iv[1], min(ab[0], lo_c), max(ab[1], hi_c)]
        pol = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_SIGMA, tau=0.8, tau_ext=0.4)
        for meth in args.methods:
            mcode = ev.EVSL_LAN_NR if meth == "nr" else ev.EVSL_LAN_TR
            opts = ev.lan_opts(tol=args.tol, seed=2, nev_est=len(want), method=mcode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, intv, pol, opts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            del Y
            err = float(np.abs(lam - want).max()) if len(lam) == len(want) else None
            rec = {"grid": f"{N}^{dim}", "interval": list(iv), "method": meth,
                   "nu_closed_form": int(len(want)), "nu_paper": nu, "found": int(len(lam)),
                   "max_abs_err": err, "max_res": float(res.max()) if len(res) else None,
                   "bounds_used": intv[2:], "deg": pol.deg,
                   "deg_printed_bounds": pdeg_printed, "deg_paper": pdeg, "niter": st["niter"], "niter_paper": pniter,
                   "nmv": st["nmv"], "nmv_paper": pnmv, "t_mv": st["t_mv"],
                   "t_orth": st["t_orth"], "t_ritz": st["t_ritz"], "t_tot": dt,
                   "t_tot_paper_cpu": pttot, "eig_per_s": len(lam) / dt, "status": st["status"]}
            out.append(rec)
            log(f"[paper] {rec['grid']} {iv} {meth}: found {rec['found']}/{len(want)} "
                f"deg {pol.deg} (printed bounds {pdeg_printed}, paper {pdeg}) niter {st['niter']} (paper {pniter}) "
                f"t {dt:.2f} s (paper {pttot} s CPU) err {err}")
        del Ad
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "eigenpairs/s on the paper's Laplacian problems (non-restart filtered Lanczos)",
        "unit": "eigenpairs/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Table tab:lap problems: 2-D 5-point / 3-D 7-point Laplacians, "
                               "bounds = printed [a, b] widened to the computed Lanczos bounds, "
                               "sigma damping, tau 0.8, "
                               f"tol {args.tol:g}"},
        "rows": out}), flush=True)


def small_main(args):
    """The small plain case: 2-D 40x40 Laplacian without potential, [1.0, 1.6]
    (91 eigenvalues, 44 of them exact double pairs). Each repeat runs the whole
    path (Lanczos bounds, KPM degree 40 with 10 vectors, slicing, Jackson
    filters, thick-restart solve at tol 1e-10) from a device-resident matrix;
    p50/p99 latency over the repeats, time per filter degree step and per
    Lanczos step, for one and two slices, with the filter replayed from HIP
    graphs and launched kernel by kernel. Every repeat is checked against the
    closed form 4 - 2 cos(i pi/41) - 2 cos(j pi/41)."""
    import torch

    import evsl_inputs as I
    import paper_1802_05215_amd as ev

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    N, intv0, tol = 40, (1.0, 1.6), 1e-10
    A = I.laplacian(N, 2)
    Ad = ev.DeviceCsr.from_host(A, device="cuda:0")
    c = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    ex = np.sort((c[:, None] + c[None, :]).ravel())
    want = ex[(ex >= intv0[0]) & (ex <= intv0[1])]
    ctx = ev.Ctx()

    def solve(ns):
        t0 = time.perf_counter()
        lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
        intv = [intv0[0], intv0[1], lo, hi]
        mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, 40, 10, seed=1, damping=ev.DAMP_JACKSON)
        sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, ns, 2000) if ns > 1 \
            else np.array(intv0)
        ivs, pols, opts = [], [], []
        for q in range(ns):
            iv = [sli[q], sli[q + 1], lo, hi]
            cnt = ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, sli[q], sli[q + 1])
            ivs.append(iv)
            pols.append(ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON, tau=0.8, tau_ext=0.4))
            opts.append(ev.lan_opts(tol=tol, seed=2 + q, nev_est=max(int(cnt * 1.1) + 5, 10)))
        t1 = time.perf_counter()
        if ns == 1:
            outs = [ev.evsl_filtered_lanczos(ctx, Ad, ivs[0], pols[0], opts[0])]
        else:
            outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        lams = []
        for q, (lam, Y, res, st) in enumerate(outs):
            keep = (lam >= ivs[q][0]) & ((lam < ivs[q][1]) | (q == ns - 1)) & (res <= tol)
            lams.append(lam[keep])
        lam = np.sort(np.concatenate(lams))
        err = float(np.abs(lam - want).max() / np.abs(want).max()) if len(lam) == len(want) \
            else float("inf")
        return dict(t=t2 - t0, t_solve=t2 - t1, nev=len(lam), err=err,
                    niter=sum(o[3]["niter"] for o in outs), degs=[p.deg for p in pols])

    rows = []
    for graphs in (True, False):
        ctx.set_graphs(graphs)
        for ns in (1, 2):
            for _ in range(3):
                solve(ns)
            torch.cuda.synchronize()
            ctx.reset_stats()
            recs = [solve(ns) for _ in range(args.repeats)]
            fs = ctx.filter_stats()
            t = np.array([r["t"] for r in recs])
            ts = np.array([r["t_solve"] for r in recs])
            steps = sum(r["niter"] for r in recs)
            row = {"graphs": graphs, "slices": ns, "degrees": recs[0]["degs"],
                   "nev": [r["nev"] for r in recs][0], "all_correct":
                   all(r["nev"] == len(want) and r["err"] <= 1e-10 for r in recs),
                   "max_rel_err": max(r["err"] for r in recs),
                   "p50_ms": float(np.percentile(t, 50)) * 1e3,
                   "p99_ms": float(np.percentile(t, 99)) * 1e3,
                   "solve_p50_ms": float(np.percentile(ts, 50)) * 1e3,
                   "lanczos_steps": recs[0]["niter"],
                   "us_per_lanczos_step": float(ts.sum()) / steps * 1e6,
                   "us_per_filter_step": fs["seconds"] / max(fs["launches"], 1) * 1e6,
                   "filter_steps_per_lanczos_step": fs["launches"] / max(steps, 1)}
            rows.append(row)
            log(f"[small] graphs {graphs} slices {ns}: p50 {row['p50_ms']:.1f} ms "
                f"p99 {row['p99_ms']:.1f} ms, {row['us_per_lanczos_step']:.1f} us per Lanczos "
                f"step, {row['us_per_filter_step']:.2f} us per filter step, nev {row['nev']}, "
                f"correct {row['all_correct']}")
    ctx.set_graphs(True)
    best = min(r["p50_ms"] for r in rows)
    print(json.dumps({
        "metric": "whole-path latency, 40x40 plain case (p50 over repeats)",
        "value": best, "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D 5-point Laplacian 40x40 (n 1600), no potential, "
                               "[1.0, 1.6] (91 eigenvalues), KPM degree 40 with 10 vectors, "
                               f"Jackson filters, thick-restart Lanczos, tol {tol:g}",
                   "repeats": args.repeats},
        "rows": rows}), flush=True)


def pencil_main(args):
    """Generalized problem A x = lambda B x on the bilinear finite-element pencil
    of an N x N grid (K1 x M1 + M1 x K1, M1 x M1), whose eigenvalues are
    mu_i + mu_j in closed form: bounds of B, bounds of the pencil, then the
    interval holding about `count` eigenvalues after index N^2/5 (its ends in the
    widest nearby gaps of the spectrum) solved by the
    non-restart and the thick-restart forms (solves with B by a degree-60
    Chebyshev fit of 1/t), tol 1e-10, every eigenvalue checked against the closed
    form."""
    import torch

    import evsl_inputs as I
    import paper_1802_05215_amd as ev

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    N, cnt, bdeg, tol = args.pencil_n, args.pencil_count, 60, 1e-10
    A, B = I.fe_pencil(N)
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    mu = (2 - 2 * np.cos(th)) / ((4 + 2 * np.cos(th)) / 6)
    ex = np.sort((mu[:, None] + mu[None, :]).ravel())
    # interval ends in the widest gap between consecutive eigenvalues within 20
    # places of the targets (the pencil has double eigenvalues mu_i + mu_j =
    # mu_j + mu_i, and a narrow end gap leaves the filter little separation)
    def end_at(k):
        return max(range(k - 20, k + 21), key=lambda j: ex[j] - ex[j - 1])
    k0 = end_at(A.n // 5)
    k1 = end_at(k0 + cnt)
    xi, eta = 0.5 * (ex[k0 - 1] + ex[k0]), 0.5 * (ex[k1 - 1] + ex[k1])
    want = ex[(ex >= xi) & (ex <= eta)]
    ctx = ev.Ctx()
    Ad, Bd = ev.DeviceCsr.from_host(A, device="cuda:0"), ev.DeviceCsr.from_host(B, device="cuda:0")
    rows = []
    for name, meth in (("non-restart", ev.EVSL_LAN_NR), ("thick restart", ev.EVSL_LAN_TR)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blo, bhi = ev.evsl_spectrum_bounds(ctx, Bd, 80, 3)
        bb = [0.98 * blo, 1.02 * bhi]
        lo, hi = ev.evsl_spectrum_bounds_gen(ctx, Ad, Bd, bb, bdeg, 80, 3)
        intv = [xi, eta, lo, hi]
        pol = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_JACKSON)
        lam, Y, res, st = ev.evsl_filtered_lanczos_gen(
            ctx, Ad, Bd, bb, bdeg, intv, pol, ev.lan_opts(tol=tol, nev_est=len(want), method=meth))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(np.abs(lam - want).max()) if len(lam) == len(want) else None
        row = {"method": name, "found": int(len(lam)), "want": int(len(want)), "deg": pol.deg,
               "niter": st["niter"], "b_solves": st["nrestart"], "t_s": dt,
               "eig_per_s": len(lam) / dt, "max_abs_err": err,
               "max_res": float(res.max()) if len(res) else None, "status": st["status"]}
        rows.append(row)
        log(f"[pencil] {name}: found {len(lam)}/{len(want)} deg {pol.deg} niter {st['niter']} "
            f"solves {st['nrestart']} t {dt:.2f} s err {err}")
    best = max(r["eig_per_s"] for r in rows)
    print(json.dumps({
        "metric": "eigenpairs/s on a generalized problem A x = lambda B x",
        "value": best, "unit": "eigenpairs/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"bilinear finite-element pencil {N}x{N} (n {A.n}), "
                               f"[{xi:.6g}, {eta:.6g}] ({len(want)} eigenvalues, closed form), "
                               f"Jackson filter, lsPol solves of degree {bdeg}, tol {tol:g}"},
        "rows": rows}), flush=True)


def match_eigs(ref, got):
    """Pairs every reference eigenvalue with the nearest unused computed one
    (both sorted; equal counts pair in order). Returns (pairs (i_ref, i_got),
    reference indices left unmatched, computed indices left unmatched)."""
    ref, got = np.asarray(ref), np.asarray(got)
    if len(ref) == len(got):
        return [(k, k) for k in range(len(ref))], [], []
    used = np.zeros(len(got), bool)
    pairs, miss = [], []
    for k, x in enumerate(ref):
        cand = np.where(~used)[0]
        if len(cand) == 0:
            miss.append(k)
            continue
        j = cand[np.argmin(np.abs(got[cand] - x))]
        if abs(got[j] - x) <= 1e-6 * max(abs(x), 1.0):
            used[j] = True
            pairs.append((k, int(j)))
        else:
            miss.append(k)
    return pairs, miss, [int(j) for j in np.where(~used)[0]]


def precision_main(args, ctx, ev, Ad, A):
    """The precision form (FP32 filter phase, then the FP64 phase) against the
    plain FP64 path on the same bounds, KPM, slices and filters: the 100^3
    workload's ten slices of [0.60, 0.70] (one batch each) and three single
    slices whose Jackson degrees span about 40-300 ([0.50, 0.60], [0.60, 0.65],
    [0.60, 0.625]). For every eigenvalue: |lambda_32 - lambda_64| / |lambda_64|
    (matched in order, or to the nearest when the counts differ, the unmatched
    ones listed), and for the slices the oracle solved (tests/golden, slices 0
    and 9 of the 100^3 cut) the same against the oracle's eigenvalues. Writes
    the per-eigenvalue table to --precision-out when given."""
    import copy
    import torch

    gold_path = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else {"solved": {}}
    runs = [("100^3 [0.60, 0.70], 10 KPM slices", [0.60, 0.70], 10)]
    runs += [(f"single slice [{a:.3f}, {b:.3f}]", [a, b], 1)
             for a, b in ((0.50, 0.60), (0.60, 0.65), (0.60, 0.625))]
    out, table = [], []
    for name, iv, ns in runs:
        rec = {"workload": name, "interval": iv}
        res_ = {}
        for prec in ("f64", "f32"):
            a = copy.copy(args)
            a.interval, a.nslices, a.prec, a.slices, a.interval_count = list(iv), ns, prec, None, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = one_step(ctx, ev, Ad, a)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res_[prec] = r
            rec[prec] = {"nev": r["nev"], "s": dt, "eigenpairs_per_s": r["nev"] / dt,
                         "degrees": [p["deg"] for p in r["per_slice"]],
                         "niter": [p["niter"] for p in r["per_slice"]],
                         "fp64_phase": [p["npolish"] for p in r["per_slice"]],
                         "group_width": r["group_width"],
                         "status": [p["status"] for p in r["per_slice"]],
                         "max_residual": float(r["res"].max()) if r["nev"] else None}
            print(f"[precision] {name} {prec}: {r['nev']} pairs in {dt:.1f} s, status "
                  f"{rec[prec]['status']}", file=sys.stderr, flush=True)
        l64, l32 = np.sort(res_["f64"]["lam"]), np.sort(res_["f32"]["lam"])
        pairs, miss, extra = match_eigs(l64, l32)
        err = np.array([abs(l32[j] - l64[k]) / abs(l64[k]) for k, j in pairs])
        rec["f32_vs_f64"] = {"matched": len(pairs), "missing_in_f32": [float(l64[k]) for k in miss],
                             "extra_in_f32": [float(l32[j]) for j in extra],
                             "rel_err_max": float(err.max()) if len(err) else None,
                             "rel_err_median": float(np.median(err)) if len(err) else None}
        for k, j in pairs:
            table.append((name, "gpu-f64", l64[k], l32[j], abs(l32[j] - l64[k]) / abs(l64[k])))
        for k in miss:
            table.append((name, "gpu-f64", l64[k], float("nan"), float("nan")))
        if ns == 10:
            # slices the oracle solved: every eigenvalue of the slice against it
            sli = res_["f32"]["slices"]
            for q, g in sorted(gold["solved"].items()):
                q = int(q)
                lo_, hi_ = g["interval"]
                ref = np.array(g["eigenvalues"])
                if abs(sli[q] - lo_) > 1e-9 or abs(sli[q + 1] - hi_) > 1e-9:
                    rec[f"oracle_slice_{q}"] = "slice ends differ from the oracle's; skipped"
                    continue
                last = q == ns - 1
                got = l32[(l32 >= lo_) & ((l32 < hi_) | last)]
                pr, ms, ex = match_eigs(ref, got)
                e = np.array([abs(got[j] - ref[k]) / abs(ref[k]) for k, j in pr])
                rec[f"f32_vs_oracle_slice_{q}"] = {
                    "oracle_count": len(ref), "f32_count": len(got),
                    "missing_in_f32": [float(ref[k]) for k in ms],
                    "rel_err_max": float(e.max()) if len(e) else None}
                for k, j in pr:
                    table.append((f"{name}, slice {q}", "oracle", ref[k], got[j],
                                  abs(got[j] - ref[k]) / abs(ref[k])))
                for k in ms:
                    table.append((f"{name}, slice {q}", "oracle", ref[k], float("nan"),
                                  float("nan")))
        rec["speedup_f32"] = rec["f64"]["s"] / rec["f32"]["s"]
        out.append(rec)
    if args.precision_out:
        import csv
        with open(args.precision_out, "w", newline="") as f:
            wr = csv.writer(f)
            wr.writerow(["workload", "reference", "lambda_ref", "lambda_f32", "rel_err"])
            for w, kind, a, b, e in table:
                wr.writerow([w, kind, f"{a:.17g}", f"{b:.17g}", f"{e:.3e}"])
    print(json.dumps({
        "metric": "FP32-filter precision form vs FP64: eigenpairs/s and per-eigenvalue error",
        "n_gpus": 1, "dtype": "f32-filter/f64 vs f64", "data": "synthetic",
        "config": {"workload": (f"3-D 7-point Laplacian {args.grid}^3 + U[0,1) potential "
                                f"(seed 0), tol {args.tol:g}, tol_lo "
                                f"{args.tol_lo or 'default'}")},
        "runs": out}), flush=True)


def serve_main(args):
    """Serving workload: a seeded Poisson stream of requests, each on its own
    matrix, admitted by device-memory footprint and run concurrently (one HIP
    stream and library context per request). The arrival rate is 0.7 x the
    capacity measured by serving the first `calib` requests alone, one after
    another; those requests' results in the mix are compared bit for bit with
    their solo results."""
    import torch

    from paper_1802_05215_amd import serving as S

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    ex = S.DeviceExecutor(tol=args.tol, prec=args.serve_prec, tol_lo=args.tol_lo)
    budget = int(args.budget_gb * 2 ** 30)
    base = S.poisson_stream(args.serve_seed, args.requests, 1.0, n_max=args.serve_nmax)
    solo = {}
    t_solo = []
    for r in base[:args.calib]:
        one = S.Ledger(budget, 1)
        t0 = time.perf_counter()
        res = S.Server(one, ex).run([S.Request(**{**r.__dict__, "arrival": 0.0})])[0]
        t_solo.append(time.perf_counter() - t0)
        solo[r.rid] = res
        log(f"[serve] calibration request {r.rid}: {r.kind} dim {r.dim} n {r.n} "
            f"target {r.target}: {t_solo[-1]:.2f} s, status {res.status}")
    rate = args.serve_rate or 0.7 / float(np.mean(t_solo))
    reqs = S.poisson_stream(args.serve_seed, args.requests, rate, n_max=args.serve_nmax)
    free0, total = torch.cuda.mem_get_info()
    hw = {"used": 0}

    def tick():
        f, _ = torch.cuda.mem_get_info()
        hw["used"] = max(hw["used"], free0 - f)

    reqs_by_id = {}
    jsonl = open(args.serve_log, "a") if args.serve_log else None

    def done(res):
        log(f"[serve] request {res.rid} {res.kind}: {res.status}, nev {res.nev}, "
            f"latency {res.latency:.2f} s")
        if jsonl:
            r = reqs_by_id.get(res.rid)
            jsonl.write(json.dumps({
                "rid": res.rid, "kind": res.kind, "status": res.status, "error": res.error,
                "dim": r.dim if r else None, "n": r.n if r else None,
                "target": r.target if r and r.kind == "eigs" else None,
                "arrival_s": res.arrival, "start_s": res.start, "end_s": res.end,
                "latency_s": res.latency, "nev": res.nev,
                "max_residual": float(res.res.max()) if res.res is not None and len(res.res) else None,
                "interval": list(res.interval) if res.interval else None,
                "device_peak_bytes": res.lib_peak,
                "footprint_bytes": S.footprint_bytes(r) if r else None}) + "\n")
            jsonl.flush()

    reqs_by_id.update({r.rid: r for r in reqs})
    led = S.Ledger(budget, args.max_running)
    srv = S.Server(led, ex, on_tick=tick, on_result=done, max_bypass=args.max_bypass)
    t0 = time.perf_counter()
    out = srv.run(reqs)
    wall = time.perf_counter() - t0
    summ = S.summarize(out, wall, led)
    same = 0
    for rid, r0 in solo.items():
        r1 = out[rid]
        eq = r0.status == r1.status and r0.status in ("ok", "partial") \
            and np.array_equal(r0.moments, r1.moments)
        if eq and r0.kind == "eigs":
            eq = (np.array_equal(r0.lam, r1.lam) and np.array_equal(r0.res, r1.res)
                  and np.array_equal(r0.ycheck, r1.ycheck))
        same += int(eq)
    ok = [r for r in out if r.status == "ok" and r.kind == "eigs"]
    print(json.dumps({
        "metric": "served eigenpairs/s at resid<=1e-8, p50/p99 request latency",
        "value": summ["eigenpairs_per_s"],
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32-filter/f64" if args.serve_prec == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"Poisson stream (seed {args.serve_seed}) of {args.requests} requests: "
                         f"2-D/3-D Laplacian + U[0,1) potential, n log-uniform in "
                         f"[1e4, {args.serve_nmax:g}], half KPM DOS (degree 100, 20 vectors), "
                         f"half eigenpair requests (count U{{50..400}} from a DOS quantile "
                         f"U[0.05, 0.6]), "
                         + ("FP32-filter phase then FP64 phase, FP64 Ritz and residuals"
                            if args.serve_prec == "f32" else "FP64")
                         + f", tol {args.tol:g}"),
            "rate_per_s": rate, "calibration_s": t_solo, "budget_bytes": budget,
            "max_running": args.max_running, "max_bypass": args.max_bypass,
        },
        **summ,
        "device_mem_high_water_bytes": int(hw["used"]),
        "max_residual": float(max((r.res.max() for r in ok if r.nev), default=0.0)),
        "solo_bitwise_equal": f"{same}/{len(solo)}",
    }), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe_main()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.serve or args.filter_only or args.paper_table or args.small or args.pencil:
        import torch
        import paper_1802_05215_amd as ev
        if not torch.cuda.is_available():
            print(json.dumps({"error": "no HIP device"}))
            sys.exit(2)
        ev.load()
        torch.cuda.set_device(0)
        if args.serve:
            serve_main(args)
        elif args.paper_table:
            paper_table_main(args)
        elif args.small:
            small_main(args)
        elif args.pencil:
            pencil_main(args)
        else:
            filter_only_main(args)
        return
    import torch

    import evsl_inputs as I
    import paper_1802_05215_amd as ev

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(2)
    ev.load()
    torch.cuda.set_device(0)
    N = args.grid
    A = I.laplacian(N, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A, device="cuda:0")
    ctx = ev.Ctx()
    # load the code objects outside the timed region (a filter on a tiny matrix)
    tiny = ev.DeviceCsr.from_host(I.laplacian(8, 2), device="cuda:0")
    pt = ev.evsl_cheb_coeffs([1.0, 1.5, 0.0, 8.0])
    xv = torch.ones(64, dtype=torch.float64, device="cuda:0")
    ev.evsl_filter_apply(ctx, tiny, [pt], [0], xv, torch.empty_like(xv))
    torch.cuda.synchronize()

    if args.precision_study:
        precision_main(args, ctx, ev, Ad, A)
        return
    if args.c3_only:
        c3 = c3_filter_leg(ctx, ev, args, lambda m: print(m, file=sys.stderr, flush=True))
        c3.pop("check_column", None)
        c3.pop("A_host", None)
        print(json.dumps({"metric": "filter SpMM HBM GB/s (algorithmic bytes)",
                          "value": c3["roofline"]["achieved"], "unit": "GB/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": c3["workload"]}, "c3_filter": c3}), flush=True)
        return

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    # At most one warm-up solve; then whole solves while the next one (timed
    # like the last) still ends before the deadline, so that the run, the
    # 200^3 filter leg and the oracle sample fit the measurement window.
    nwarm = min(args.warmup, 1)
    last = None
    for _ in range(nwarm):
        tw = time.perf_counter()
        one_step(ctx, ev, Ad, args)
        torch.cuda.synchronize()
        last = time.perf_counter() - tw
        log(f"[bench] warm-up solve {last:.1f} s")
    torch.cuda.synchronize()
    ctx.reset_stats()
    recs = []
    t0 = time.perf_counter()
    for i in range(max(args.steps, 1)):
        now = time.perf_counter()
        if i > 0 and args.time_budget > 0 and now - T_START + last > args.time_budget:
            break
        recs.append(one_step(ctx, ev, Ad, args))
        torch.cuda.synchronize()
        last = time.perf_counter() - now
        log(f"[bench] step {i}: {recs[-1]['nev']} eigenpairs in {last:.1f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fs = ctx.filter_stats()
    rec = recs[-1]
    nev_total = sum(r["nev"] for r in recs)
    value = nev_total / elapsed
    lat = np.array([s["t_done"] for r in recs for s in r["per_slice"]])
    achieved = fs["bytes"] / fs["seconds"] / 1e9 if fs["seconds"] > 0 else 0.0
    per_launch_bytes = fs["bytes"] / max(fs["launches"], 1)
    solver = {"tr": "thick-restart Lanczos", "nr": "non-restart Lanczos",
              "si": "subspace iteration"}[args.method]
    arith = ("FP32-filter phase then FP64 phase, FP64 reorthogonalisation/Rayleigh-Ritz"
             if args.prec == "f32"
             else "FP64")
    workload = (f"3-D 7-point Laplacian {N}^3 + U[0,1) diagonal potential (seed 0), "
                f"all eigenpairs in [{rec['interval'][0]:.6g}, {rec['interval'][1]:.6g}]"
                + (f" (lambda_min to the KPM count {args.interval_count})"
                   if args.interval_count > 0 else "")
                + (f", {args.nslices} KPM slices (degree {args.kpm_degree}, "
                   f"{args.kpm_vectors} vectors)" if args.dos == "kpm" else
                   f", {args.nslices} Lanczos-DOS slices ({args.kpm_degree} steps, "
                   f"{args.kpm_vectors} probes)")
                + f", Jackson filters, {solver}, tol {args.tol:g}, {arith}, "
                f"slices {args.mode}"
                + (f"; only slices {args.slices} of the cut solved" if args.slices else ""))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": len(recs),
        "warmup": nwarm,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": elapsed / len(recs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-filter/f64" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n": A.n, "nnz": A.nnz, "nslices": args.nslices, "nev": rec["nev"],
            "slices_solved": args.slices or "all",
            "kpm_estimate": round(rec["kpm_est"], 1),
            "filter_degrees": [s["deg"] for s in rec["per_slice"]],
            "max_its": args.max_its,
            "group_width": rec["group_width"],
            "block_schedule": rec["schedule"],
        },
        "setup_s": rec["t_setup"],
        "filter_gbps": achieved,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "max_residual": float(rec["res"].max()) if rec["nev"] else None,
        "split_s": {k: float(sum(s[k] for s in rec["per_slice"]))
                    for k in ("t_mv", "t_orth", "t_ritz")},
        "niter": [s["niter"] for s in rec["per_slice"]],
        "north2": [s["north2"] for s in rec["per_slice"]],
        "npolish": [s["npolish"] for s in rec["per_slice"]],
        "status": [s["status"] for s in rec["per_slice"]],
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "traffic_bytes_per_launch": None,
            "kernel": "k_cheb_blk_lds<double, STEP_CLEN> (Clenshaw filter degree step)",
            "bytes_per_launch": per_launch_bytes,
            "avg_launch_us": fs["seconds"] / max(fs["launches"], 1) * 1e6,
            "launches": fs["launches"],
        },
    }
    tb = measured_traffic()
    if tb is not None and fs["launches"] and N == 100 and args.prec == "f64":
        # the committed counters are those of this workload's FP64 filter
        avg_s = fs["seconds"] / fs["launches"]
        out["roofline"]["traffic"] = tb / avg_s / 1e9
        out["roofline"]["traffic_bytes_per_launch"] = tb
    if (not args.no_precision_leg and N == 100 and args.prec == "f64" and args.method == "tr"
            and args.mode == "batch" and not args.slices):
        out["precision_form"] = precision_leg(ctx, ev, Ad, args, rec, value, log)
    c3 = None
    if args.c3 and N == 100:
        c3 = c3_filter_leg(ctx, ev, args, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, rec, args, c3)
    if c3 is not None:
        c3.pop("check_column", None)
        c3.pop("A_host", None)
        out["c3_filter"] = c3
        out["config"]["workload"] = ("value, roofline: " + out["config"]["workload"]
                                     + "; c3_filter: " + c3["workload"])
    out["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
