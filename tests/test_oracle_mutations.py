"""The oracle's pins catch planted mistakes. Each case copies the oracle's C
source, plants one plausible mistake (a wrong index, a flipped sign, a dropped
factor or term), builds the copy with gcc and runs a set of closed-form and
paper-table checks against it: at least one check must fail. The unmodified
source passes every check. CPU only; the mistakes live in temporary copies.
(A mistake that full reorthogonalisation repairs, such as a wrong coefficient
on the explicit three-term subtraction, changes no result and is not listed.)"""
import ctypes as C
import json
import os
import subprocess

import numpy as np
import pytest

import evsl_inputs as I
import oracle
from tests.closed_form import lap_eigs, lap_eigvec, lap_eig_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "evsl_oracle.c")
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))

# (name, exact text in the source, replacement)
MUTATIONS = [
    ("spmv gathers the row's own entry",
     "for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * x[ci[p]];",
     "for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * x[i];"),
    ("Jackson damping: sine term with the wrong sign",
     "g[j] = ((N - j + 1.0) * cos(j * al) + sin(j * al) * cos(al) / sin(al)) / (N + 1.0);",
     "g[j] = ((N - j + 1.0) * cos(j * al) - sin(j * al) * cos(al) / sin(al)) / (N + 1.0);"),
    ("sigma damping without theta in the denominator",
     "for (int j = 1; j <= k; ++j) g[j] = sin(j * th) / (j * th);",
     "for (int j = 1; j <= k; ++j) g[j] = sin(j * th) / j;"),
    ("filter coefficient mu_0 = 1 instead of 1/2",
     "coef[0] = 0.5 * g[0] / den;",
     "coef[0] = g[0] / den;"),
    ("filter recurrence adds W_{j-1}",
     "w2[i * nvec + l] = 2.0 * (s - cc * w1[i * nvec + l]) / dd - w0[i * nvec + l];",
     "w2[i * nvec + l] = 2.0 * (s - cc * w1[i * nvec + l]) / dd + w0[i * nvec + l];"),
    ("filter's first step shifts by +c",
     "w1[i * nvec + l] = (s - cc * w0[i * nvec + l]) / dd;",
     "w1[i * nvec + l] = (s + cc * w0[i * nvec + l]) / dd;"),
    ("KPM moments not averaged over the probes",
     "mom[k] = acc / nvec;",
     "mom[k] = acc;"),
    ("KPM count drops the factor 2 of the k >= 1 terms",
     "s += 2.0 * g[k] * mom[k] * (sin(k * th0) - sin(k * th1)) / (k * M_PI);",
     "s += g[k] * mom[k] * (sin(k * th0) - sin(k * th1)) / (k * M_PI);"),
    ("spectrum bounds narrowed instead of widened",
     "*lmin = w[0] - fabs(beta * Y[(dim - 1) + 0]);",
     "*lmin = w[0] + fabs(beta * Y[(dim - 1) + 0]);"),
    ("Gram-Schmidt adds the projections",
     "for (int64_t i = 0; i < n; ++i) z[i] -= h[j] * bj[i];",
     "for (int64_t i = 0; i < n; ++i) z[i] += h[j] * bj[i];"),
    ("lsPol fit without the factor 2 of the j >= 1 coefficients",
     "for (int j = 0; j <= deg; ++j) coef[j] *= (j == 0 ? 1.0 : 2.0) / N;",
     "for (int j = 0; j <= deg; ++j) coef[j] *= 1.0 / N;"),
    ("conjugate gradients with the residual update's sign flipped",
     "for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; res[i] -= a * q[i]; }",
     "for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; res[i] += a * q[i]; }"),
    ("pencil bounds: the Lanczos step subtracts alpha w_i instead of alpha z_i",
     "    or_spmv(n, rp, ci, va, wi, z);\n    if (i > 0)\n      for (int64_t r = 0; r < n; ++r) z[r] -= beta * Z[(size_t)(i - 1) * n + r];\n    const double alpha = dot(n, z, wi);\n    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * zi[r];",
     "    or_spmv(n, rp, ci, va, wi, z);\n    if (i > 0)\n      for (int64_t r = 0; r < n; ++r) z[r] -= beta * Z[(size_t)(i - 1) * n + r];\n    const double alpha = dot(n, z, wi);\n    for (int64_t r = 0; r < n; ++r) z[r] -= alpha * wi[r];"),
    ("thick restart couples through the first component",
     "        sTR[lnew] = beta_last * y[dim - 1];\n        lnew++;",
     "        sTR[lnew] = beta_last * y[0];\n        lnew++;"),
]


def _build(src_text, tmp_path, tag):
    c = tmp_path / f"o_{tag}.c"
    c.write_text(src_text)
    so = tmp_path / f"lib_{tag}.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-I",
                    os.path.join(ROOT, "oracle"), str(c), "-o", str(so), "-lm"], check=True)
    L = C.CDLL(str(so))
    oracle._setup(L)
    return L


def _checks():
    """Names of the checks that fail on the loaded oracle library."""
    failed = []

    def run(name, fn):
        try:
            if not fn():
                failed.append(name)
        except Exception:
            failed.append(name)

    A = I.laplacian(12, 2)
    v = lap_eigvec(12, 2, (2, 3))
    lam = lap_eig_of(12, (2, 3))
    run("spmv on a Laplacian mode", lambda: np.linalg.norm(oracle.spmv(A, v) - lam * v) < 1e-12)

    def degrees():
        rows = GOLD["lap_degrees"]["rows"]
        got = [oracle.find_pol([r["intv"][0], r["intv"][1], r["ab"][0], r["ab"][1]],
                               damping=oracle.DAMP_SIGMA)["deg"] for r in rows]
        return all(abs(a - r["deg"]) <= 1 for a, r in zip(got, rows))
    run("find_pol degrees of Table tab:lap_pol_results", degrees)

    def filter_on_mode():
        iv = [1.0, 1.4, 0.0, 8.0]
        p = oracle.find_pol(iv, damping=oracle.DAMP_JACKSON)
        y = oracle.filter_apply(A, p["cc"], p["dd"], p["coef"], v)
        rho = oracle.cheb_series(p["coef"], (lam - p["cc"]) / p["dd"])
        return np.linalg.norm(y - rho * v) < 1e-12 and p["bar"] > 0.0
    run("filter on a Laplacian mode", filter_on_mode)

    def kpm_count():
        B = I.laplacian(30, 2)
        ex = lap_eigs(30, 2)
        V = oracle.rademacher(5, B.n, 40)
        mom = oracle.kpm_moments(B, 0.0, 8.0, 60, V)
        est = oracle.kpm_count(mom, oracle.DAMP_JACKSON, 0.0, 8.0, 2.0, 4.0)
        true = np.count_nonzero((ex >= 2.0) & (ex <= 4.0))
        return abs(est - true) <= 0.1 * true
    run("KPM count on a 30 x 30 Laplacian", kpm_count)

    def bounds():
        lo, hi = oracle.lanczos_bounds(A, 40, 3)
        ex = lap_eigs(12, 2)
        return lo <= ex[0] and hi >= ex[-1]
    run("Lanczos bounds contain the spectrum", bounds)

    def lanczos():
        B = I.laplacian(20, 2)
        ex = lap_eigs(20, 2)
        lo, hi = oracle.lanczos_bounds(B, 80, 3)
        iv = [1.0, 1.4, lo, hi]
        want = ex[(ex >= 1.0) & (ex <= 1.4)]
        p = oracle.find_pol(iv, damping=oracle.DAMP_JACKSON)
        lam_, _, _, st = oracle.filtered_lanczos(B, iv, p, tol=1e-10, nev_est=len(want), m=40,
                                                 max_its=400)
        return len(lam_) == len(want) and np.abs(lam_ - want).max() < 1e-10 * 8
    run("thick-restart Lanczos on a 20 x 20 Laplacian", lanczos)

    def lspol_fit():
        c = oracle.lspol(0, 0.5, 2.0, 40)
        t = np.linspace(0.5, 2.0, 7)
        x = (t - 1.25) / 0.75
        return np.abs(np.polynomial.chebyshev.chebval(x, c) - 1.0 / t).max() < 1e-10
    run("lsPol fit of 1/t", lspol_fit)

    def pencil():
        Ap, Bp = I.fe_pencil(12)
        th = np.arange(1, 13) * np.pi / 13
        mu = (2 - 2 * np.cos(th)) / ((4 + 2 * np.cos(th)) / 6)
        ex = np.sort((mu[:, None] + mu[None, :]).ravel())
        r = np.linspace(1.0, 2.0, Bp.n)
        if np.linalg.norm(Bp.to_dense() @ oracle.cg_solve(Bp, r) - r) > 1e-10 * np.linalg.norm(r):
            return False
        lo, hi = oracle.lanczos_bounds_gen(Ap, Bp, 60, 3)
        # the bounds contain the spectrum up to rounding and sit close to its ends
        tol_b = 1e-6 * ex[-1]
        if not (ex[0] - tol_b <= lo <= ex[0] + 1e-12 * ex[-1]
                and ex[-1] - 1e-12 * ex[-1] <= hi <= ex[-1] + tol_b):
            return False
        iv = [3.0, 5.0, lo, hi]
        want = ex[(ex >= 3.0) & (ex <= 5.0)]
        p = oracle.find_pol(iv, damping=oracle.DAMP_JACKSON)
        lam_, _, _, st = oracle.filtered_lanczos_gen(Ap, Bp, iv, p, tol=1e-10, nev_est=len(want))
        return len(lam_) == len(want) and np.abs(lam_ - want).max() < 1e-10 * ex[-1]
    run("pencil solves and non-restart Lanczos on a 12 x 12 pencil", pencil)
    return failed


@pytest.fixture()
def restore():
    saved = oracle._lib
    yield
    oracle._lib = saved


def test_unmodified_oracle_passes_every_check(tmp_path, restore):
    oracle._lib = _build(open(SRC).read(), tmp_path, "orig")
    assert _checks() == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, restore, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    oracle._lib = _build(src.replace(old, new, 1), tmp_path, "mut")
    assert _checks() != [], name
