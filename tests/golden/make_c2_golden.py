"""Writes c2_oracle.json: the oracle's result on the 100^3 workload.

Workload: 3-D 7-point Laplacian on a 100^3 grid (h = 1, Dirichlet) plus the
diagonal potential U[0,1) of seed 0; interval [0.60, 0.70]; KPM density
estimate of degree 80 with 20 Rademacher probes (seed 1, Jackson damping) cut
into 10 slices on a 2000-point grid; Jackson filters with tau = 0.8 (boundary
tau_ext = 0.4); thick-restart filtered Lanczos (Algorithm alg:FiltLanTR) at
tolerance 1e-8 with the start vector of stream 2 + slice index and
nev_est = 1.1 x the slice's KPM count + 5.

Every number comes from `oracle/` (FP64 C, OpenMP on row loops): the
Lanczos spectrum bounds, the KPM moments, the slice ends, the filter degrees
and the eigenvalues of the solved slices. Nothing is read from the HIP
library. Slices default to 0 and 9 (the lowest and the highest filter
degree of the cut).

Usage: OMP_NUM_THREADS=8 python tests/golden/make_c2_golden.py [slice ...]
Takes about 20-40 minutes per slice on 8 host cores.
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import evsl_inputs as I  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "c2_oracle.json")
JACKSON = 2
INTERVAL = (0.60, 0.70)
NSLICES = 10
KPM_DEGREE, KPM_VECTORS = 80, 20
TOL = 1e-8


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(slices):
    A = I.laplacian(100, 3, pot_seed=0)
    oracle.lib()
    t0 = time.perf_counter()
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    log(f"bounds [{lo!r}, {hi!r}] in {time.perf_counter() - t0:.1f} s")
    intv = [INTERVAL[0], INTERVAL[1], lo, hi]
    V = oracle.rademacher(1, A.n, KPM_VECTORS)
    mom = oracle.kpm_moments(A, lo, hi, KPM_DEGREE, V)
    sli = oracle.slicer(mom, JACKSON, intv, NSLICES, 2000)
    est = oracle.kpm_count(mom, JACKSON, lo, hi, INTERVAL[0], INTERVAL[1])
    log(f"KPM estimate {est:.1f}; slices {np.round(sli, 6).tolist()}")
    prev = json.load(open(OUT)) if os.path.exists(OUT) else {}
    rec = {
        "workload": ("3-D 7-point Laplacian 100^3 + U[0,1) potential (seed 0), [0.60, 0.70], "
                     "KPM degree 80 x 20 Rademacher probes (seed 1, Jackson), 10 slices, "
                     "Jackson filters tau 0.8, thick-restart filtered Lanczos, tol 1e-8"),
        "script": "tests/golden/make_c2_golden.py",
        "bounds": [lo, hi],
        "kpm_moments": mom.tolist(),
        "kpm_estimate": est,
        "slices": sli.tolist(),
        "solved": prev.get("solved", {}),
    }
    for q in slices:
        iv = [float(sli[q]), float(sli[q + 1]), lo, hi]
        cnt = oracle.kpm_count(mom, JACKSON, lo, hi, iv[0], iv[1])
        pol = oracle.find_pol(iv, damping=JACKSON, tau=0.8, tau_ext=0.4)
        nev_est = max(int(cnt * 1.1) + 5, 10)
        log(f"slice {q}: [{iv[0]:.6f}, {iv[1]:.6f}], degree {pol['deg']}, KPM count {cnt:.1f}")
        t1 = time.perf_counter()
        lam, Y, res, st = oracle.filtered_lanczos(A, iv, pol, tol=TOL, seed=2 + q,
                                                  nev_est=nev_est)
        dt = time.perf_counter() - t1
        last = q == NSLICES - 1
        keep = (lam >= iv[0]) & ((lam < iv[1]) | last)
        order = np.argsort(lam[keep])
        lk, rk = lam[keep][order], res[keep][order]
        log(f"slice {q}: {len(lk)} eigenpairs in {dt:.0f} s, status {st['status']}, "
            f"{st['niter']} steps, max residual {rk.max() if len(rk) else 0:.2e}")
        rec["solved"][str(q)] = {
            "interval": iv[:2], "degree": pol["deg"], "kpm_count": cnt, "nev_est": nev_est,
            "eigenvalues": lk.tolist(), "residuals": rk.tolist(), "status": st["status"],
            "niter": st["niter"], "nmv": st["nmv"], "oracle_seconds": dt,
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "omp_threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0)},
        }
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1)
    if not slices:
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0, 9])
