"""Writes c3_oracle.json: the oracle's result on two slices of the batched
200^3 workload.

Workload: 3-D 7-point Laplacian on a 200^3 grid (h = 1, Dirichlet) plus the
diagonal potential U[0,1) of seed 0; interval [lambda_min, eta] with lambda_min
the Lanczos lower bound and eta where the KPM count (degree 2000, 20
Rademacher probes of seed 1, Jackson damping) from lambda_min reaches 512 (60
bisection halvings); that interval cut into 32 slices on a 2000-point grid (a
degree-80 estimate cannot resolve the spectrum's lower edge: it places 512
eigenvalues below 0.4953, where degrees 1000-4000 agree on about 201); Jackson
filters with tau = 0.8 (boundary slices tau_ext = 0.4); thick-restart filtered
Lanczos (Algorithm alg:FiltLanTR) at tolerance 1e-8 with the start vector of
stream 2 + slice index and nev_est = 1.1 x the slice's KPM count + 5.

Every number comes from `oracle/` (FP64 C, OpenMP on row loops). Slices
default to 0 (the boundary slice, Table tab:lapslicing's boundary filter) and
1 (the interior slice of lowest degree).

Usage: OMP_NUM_THREADS=8 python tests/golden/make_c3_golden.py [slice ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import evsl_inputs as I  # noqa: E402
import oracle  # noqa: E402
from tests.golden.make_c2_golden import cpu_model, log  # noqa: E402

OUT = os.path.join(HERE, "c3_oracle.json")
JACKSON = 2
NSLICES, TARGET = 32, 512
KPM_DEGREE, KPM_VECTORS = 2000, 20
TOL = 1e-8


def main(slices):
    A = I.laplacian(200, 3, pot_seed=0)
    oracle.lib()
    t0 = time.perf_counter()
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    log(f"bounds [{lo!r}, {hi!r}] in {time.perf_counter() - t0:.1f} s")
    V = oracle.rademacher(1, A.n, KPM_VECTORS)
    mom = oracle.kpm_moments(A, lo, hi, KPM_DEGREE, V)
    del V
    a, b = lo, hi
    for _ in range(60):
        mid = 0.5 * (a + b)
        if oracle.kpm_count(mom, JACKSON, lo, hi, lo, mid) < TARGET:
            a = mid
        else:
            b = mid
    eta = 0.5 * (a + b)
    sli = oracle.slicer(mom, JACKSON, [lo, eta, lo, hi], NSLICES, 2000)
    log(f"eta {eta!r}; slices {np.round(sli, 6).tolist()}")
    prev = json.load(open(OUT)) if os.path.exists(OUT) else {}
    rec = {
        "workload": ("3-D 7-point Laplacian 200^3 + U[0,1) potential (seed 0), [lambda_min, "
                     "eta_512] by the KPM count (degree 2000 x 20 Rademacher probes, seed 1, "
                     "Jackson), 32 slices, Jackson filters tau 0.8, thick-restart filtered "
                     "Lanczos, tol 1e-8"),
        "script": "tests/golden/make_c3_golden.py",
        "bounds": [lo, hi], "eta": eta,
        "kpm_moments": mom.tolist(),
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
        del Y
        dt = time.perf_counter() - t1
        # a slice that starts at the lower spectrum bound owns everything below it
        keep = ((lam >= iv[0]) | (q == 0)) & ((lam < iv[1]) | (q == NSLICES - 1))
        order = np.argsort(lam[keep])
        lk, rk = lam[keep][order], res[keep][order]
        log(f"slice {q}: {len(lk)} eigenpairs in {dt:.0f} s, status {st['status']}, "
            f"{st['niter']} steps, max residual {rk.max() if len(rk) else 0:.2e}")
        rec["solved"][str(q)] = {
            "interval": iv[:2], "degree": pol["deg"], "boundary": pol["boundary"],
            "kpm_count": cnt, "nev_est": nev_est,
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
    main([int(a) for a in sys.argv[1:]] or [0, 1])
