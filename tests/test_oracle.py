"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a closed
form, a number printed in the paper (tests/golden/paper_tables.json, each block
citing its table), an independent library routine (numpy), a brute-force
computation, or a statistical bound.
"""
import json
import os

import numpy as np
import pytest

import evsl_inputs as I
import oracle
from tests.closed_form import lap_count, lap_eig_of, lap_eigs, lap_eigvec

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


# ---------------------------------------------------------------- generator
def test_generator_nnz_matches_tab_lap():
    for r in GOLD["lap_problems"]["rows"]:
        N, dim = r["N"], r["dim"]
        assert N ** dim == r["n"]
        nnz = 5 * N * N - 4 * N if dim == 2 else 7 * N ** 3 - 6 * N * N
        assert nnz == r["nnz"]
    for N, dim in ((343, 2), (49, 3)):
        A = I.laplacian(N, dim)
        r = [x for x in GOLD["lap_problems"]["rows"] if x["N"] == N][0]
        assert A.n == r["n"] and A.nnz == r["nnz"]


def test_generator_structure_and_potential():
    A = I.laplacian(7, 3)
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    for i in range(A.n):
        cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    B = I.laplacian(7, 3, pot_seed=0)
    dv = B.diag() - A.diag()
    assert np.allclose(dv, I.potential(0, A.n), rtol=0, atol=1e-15)
    assert dv.min() >= 0.0 and dv.max() < 1.0


def test_splitmix64_known_answer_and_independent_copies():
    # Published SplitMix64 reference output for state 1234567 (first five outputs).
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    got = [oracle.splitmix64(1234567, i) for i in range(5)]
    assert got == ref
    assert [int(x) for x in I.splitmix64(1234567, np.arange(5))] == ref
    assert np.array_equal(oracle.rademacher(1, 333, 7), I.rademacher(1, 333, 7))
    assert np.array_equal(oracle.lanczos_start(5, 100, 3), I.lanczos_start(5, 100, 3))


# ---------------------------------------------------------------- SpMV
@pytest.mark.parametrize("N,dim,modes", [(12, 2, (1, 1)), (12, 2, (3, 7)), (6, 3, (2, 5, 1)),
                                          (6, 3, (6, 6, 6))])
def test_spmv_closed_form_eigenvectors(N, dim, modes):
    A = I.laplacian(N, dim)
    u = lap_eigvec(N, dim, modes)
    lam = lap_eig_of(N, modes)
    r = oracle.spmv(A, u) - lam * u
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(u) * 8


def test_spmv_matches_dense_product():
    A = I.laplacian(9, 3, pot_seed=4)
    x = np.random.default_rng(0).standard_normal(A.n)
    assert np.allclose(oracle.spmv(A, x), A.to_dense() @ x, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- damping
def test_damping_closed_forms():
    for k in (1, 5, 40):
        assert np.array_equal(oracle.damping(oracle.DAMP_NONE, k), np.ones(k + 1))
        s = oracle.damping(oracle.DAMP_SIGMA, k)
        th = np.pi / (k + 1)
        j = np.arange(1, k + 1)
        assert s[0] == 1.0
        assert np.allclose(s[1:], np.sin(j * th) / (j * th), rtol=1e-15, atol=0)
        g = oracle.damping(oracle.DAMP_JACKSON, k)
        assert abs(g[0] - 1.0) < 1e-15
        # g_1 = cos(pi/(N+1)) with N = k+1 moments
        assert abs(g[1] - np.cos(np.pi / (k + 2))) < 1e-15
    assert abs(oracle.damping(oracle.DAMP_SIGMA, 1)[1] - 2 / np.pi) < 1e-16


def test_jackson_kernel_is_nonnegative():
    # The Jackson-damped delta expansion g_0 + 2 sum g_k T_k(x) T_k(y) is >= 0.
    for k in (10, 41, 100):
        g = oracle.damping(oracle.DAMP_JACKSON, k)
        x = np.cos(np.linspace(0, np.pi, 401))
        for y in (-0.7, 0.0, 0.33, 0.95):
            T = np.cos(np.outer(np.arccos(x), np.arange(k + 1)))
            Ty = np.cos(np.arange(k + 1) * np.arccos(y))
            K = g[0] + 2 * (T[:, 1:] * (g[1:] * Ty[1:])).sum(axis=1)
            assert K.min() > -1e-10
        # while the undamped kernel oscillates below zero
    T = np.cos(np.outer(np.arccos(x), np.arange(101)))
    assert (1 + 2 * T[:, 1:].sum(axis=1)).min() < -1


def test_cheb_series_matches_numpy():
    rng = np.random.default_rng(1)
    c = rng.standard_normal(30)
    for t in (-1.3, -1.0, -0.4, 0.0, 0.77, 1.0, 1.05):
        ref = np.polynomial.chebyshev.chebval(t, c)
        assert abs(oracle.cheb_series(c, t) - ref) <= 1e-12 * max(1, abs(ref))


# ---------------------------------------------------------------- find_pol
def _fp(ab, intv, **kw):
    return oracle.find_pol([intv[0], intv[1], ab[0], ab[1]], damping=oracle.DAMP_SIGMA, **kw)


def test_find_pol_reproduces_laplacian_degrees():
    got = [(_fp(r["ab"], r["intv"])["deg"], r["deg"]) for r in GOLD["lap_degrees"]["rows"]]
    exact = sum(a == b for a, b in got)
    assert exact >= 10 and all(abs(a - b) <= 1 for a, b in got), got
    # the two +-1 cases become exact with b = 12.0 (printed b is rounded)
    assert _fp([0, 12.0], [0.40, 0.450])["deg"] == 141
    assert _fp([0, 12.0], [1.00, 1.018])["deg"] == 588


def test_find_pol_reproduces_maxwell_and_parsec_degrees():
    for r in GOLD["maxwell_degrees"]["rows"]:
        assert _fp(r["ab"], r["intv"])["deg"] == r["deg"], r["name"]
    got = {r["name"]: (_fp(r["ab"], r["intv"])["deg"], r["deg"]) for r in GOLD["parsec_degrees"]["rows"]}
    assert sum(a == b for a, b in got.values()) >= 3
    assert all(abs(a - b) <= 2 for a, b in got.values()), got


def test_find_pol_reproduces_slicing_degrees():
    s = GOLD["slicing_49cube"]
    for row in s["rows"]:
        for (xi, eta), deg in zip(row["slices"], row["deg"]):
            p = oracle.find_pol([xi, eta] + s["ab"], damping=oracle.DAMP_SIGMA, tau_ext=0.4)
            assert p["deg"] == deg, (xi, eta)
            assert p["boundary"] == (-1 if xi == 0.0 else 0)


@pytest.mark.parametrize("damp", [oracle.DAMP_SIGMA, oracle.DAMP_JACKSON])
@pytest.mark.parametrize("intv", [[1.0, 1.6, 0.0117, 7.9883], [0.6, 0.61, 0.4, 13.0],
                                  [-0.5, 0.2, -1.0, 3.0], [2.0, 2.9, 0.0, 3.0]])
def test_find_pol_invariants(damp, intv):
    p = oracle.find_pol(intv, damping=damp)
    a = (intv[0] - p["cc"]) / p["dd"]
    b = (intv[1] - p["cc"]) / p["dd"]
    cheb = np.polynomial.chebyshev.chebval
    if p["boundary"] == 0:
        assert abs(cheb(p["gamma"], p["coef"]) - 1.0) < 1e-12
        assert abs(cheb(a, p["coef"]) - cheb(b, p["coef"])) < 1e-12
        assert p["bar"] <= 0.8 and a < p["gamma"] < b
    # minimality: the degree below the returned one does not meet the threshold
    q = oracle.find_pol(intv, damping=damp, max_deg=p["deg"] - 1)
    assert q["status"] == 1


def test_find_pol_boundary_and_jackson_wider():
    p = oracle.find_pol([0.0, 0.5, 0.0, 12.0], damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    assert p["boundary"] == -1 and p["gamma"] == -1.0 and p["bar"] <= 0.4
    # mirrored slice at the upper end has the same degree
    q = oracle.find_pol([11.5, 12.0, 0.0, 12.0], damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    assert q["boundary"] == 1 and q["deg"] == p["deg"]
    # Jackson damping needs a higher degree than sigma for the same threshold
    s = oracle.find_pol([0.6, 0.61, 0.4, 13.0], damping=oracle.DAMP_SIGMA)
    j = oracle.find_pol([0.6, 0.61, 0.4, 13.0], damping=oracle.DAMP_JACKSON)
    assert 1.2 < j["deg"] / s["deg"] < 1.5


# ---------------------------------------------------------------- filter
def test_filter_on_closed_form_eigenvectors():
    N = 30
    A = I.laplacian(N, 2)
    p = oracle.find_pol([1.0, 1.2, 0.0, 8.0], damping=oracle.DAMP_JACKSON)
    for modes in ((1, 1), (7, 9), (30, 29), (5, 12)):
        u = lap_eigvec(N, 2, modes)
        lam = lap_eig_of(N, modes)
        rho = np.polynomial.chebyshev.chebval((lam - p["cc"]) / p["dd"], p["coef"])
        y = oracle.filter_apply(A, p["cc"], p["dd"], p["coef"], u)
        assert np.linalg.norm(y - rho * u) <= 1e-12 * np.linalg.norm(u)


def test_filter_matches_dense_spectral_formula():
    A = I.laplacian(20, 2, pot_seed=0)
    w, U = np.linalg.eigh(A.to_dense())
    p = oracle.find_pol([2.0, 2.3, 0.0, 9.0], damping=oracle.DAMP_SIGMA)
    rho = np.polynomial.chebyshev.chebval((w - p["cc"]) / p["dd"], p["coef"])
    V = np.random.default_rng(3).standard_normal((A.n, 3))
    Y = oracle.filter_apply(A, p["cc"], p["dd"], p["coef"], V)
    ref = U @ (rho[:, None] * (U.T @ V))
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(V).max()
    # columns are independent: the block equals column-by-column application
    for c in range(3):
        assert np.array_equal(Y[:, c], oracle.filter_apply(A, p["cc"], p["dd"], p["coef"], V[:, c]))


# ---------------------------------------------------------------- KPM
def test_kpm_exact_trace_with_unit_probes():
    N = 10
    A = I.laplacian(N, 2)
    lmin, lmax = 0.0, 8.0
    K = 30
    mom = oracle.kpm_moments(A, lmin, lmax, K, np.eye(A.n))
    lam = lap_eigs(N, 2)
    x = (lam - 4.0) / 4.0
    exact = np.array([np.cos(k * np.arccos(x)).sum() for k in range(K + 1)])
    assert np.allclose(mom * A.n, exact, rtol=0, atol=1e-10)


def _exact_moments(lam, lmin, lmax, K):
    x = np.clip((lam - (lmin + lmax) / 2) / ((lmax - lmin) / 2), -1, 1)
    th = np.arccos(x)
    return np.array([np.cos(k * th).sum() for k in range(K + 1)])


def test_kpm_count_converges_to_true_count():
    lam = lap_eigs(40, 2)
    errs = []
    for K in (40, 150, 600):
        mom = _exact_moments(lam, 0.0, 8.0, K)
        c = oracle.kpm_count(mom, oracle.DAMP_JACKSON, 0.0, 8.0, 1.0, 1.6)
        errs.append(abs(c - 91))
    assert errs[2] < errs[0] and errs[2] < 3.0
    # the whole spectrum counts n
    mom = _exact_moments(lam, 0.0, 8.0, 40)
    assert abs(oracle.kpm_count(mom, oracle.DAMP_JACKSON, 0.0, 8.0, 0.0, 8.0) - 1600) < 1e-9


def test_kpm_rademacher_estimator_unbiased():
    A = I.laplacian(6, 2, pot_seed=2)
    n = A.n
    K = 6
    nvec = 4000
    V = oracle.rademacher(11, n, nvec)
    mom = oracle.kpm_moments(A, 0.0, 9.0, K, V)
    w, U = np.linalg.eigh(A.to_dense())
    x = (w - 4.5) / 4.5
    for k in range(K + 1):
        M = (U * np.cos(k * np.arccos(x))) @ U.T
        tr = np.trace(M)
        var = 2 * (np.sum(M * M) - np.sum(np.diag(M) ** 2)) / nvec
        assert abs(mom[k] - tr) <= 5 * np.sqrt(max(var, 0.0)) + 1e-9, k
    assert mom[0] == n


def test_slicer_on_exact_moments_balances_the_49cube():
    s = GOLD["slicing_49cube"]
    lam = lap_eigs(49, 3)
    lmin, lmax = s["ab"]
    mom = _exact_moments(lam, lmin, lmax, 600)
    for row in s["rows"][1:]:
        ns = len(row["nu"])
        sli = oracle.slicer(mom, oracle.DAMP_JACKSON, [0.0, 1.0, lmin, lmax], ns, npts=2000)
        counts = [np.count_nonzero((lam >= sli[i]) & (lam <= sli[i + 1])) for i in range(ns)]
        assert sum(counts) == s["total"]
        assert max(abs(c - s["total"] / ns) for c in counts) <= 0.15 * s["total"] / ns
        paper = [sl[0] for sl in row["slices"]][1:]
        assert np.allclose(sli[1:-1], paper, atol=0.02)


def test_slicer_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.slicer(np.ones(5), 2, [1.0, 0.5, 0.0, 2.0], 2)
    with pytest.raises(ValueError):
        oracle.slicer(np.ones(5), 2, [0.0, 1.0, 0.0, 2.0], 10, npts=5)


# ---------------------------------------------------------------- Jacobi
def test_jacobi_against_numpy_and_closed_form():
    rng = np.random.default_rng(5)
    for m in (1, 2, 7, 60):
        B = rng.standard_normal((m, m))
        S = B + B.T
        w, V = oracle.jacobi_eig(S)
        assert np.allclose(w, np.linalg.eigvalsh(S), rtol=0, atol=1e-12 * max(1, np.abs(S).max()))
        assert np.abs(V.T @ V - np.eye(m)).max() < 1e-13
        assert np.abs(S @ V - V * w).max() < 1e-12 * max(1, np.abs(S).max())
    A = I.laplacian(9, 2).to_dense()          # repeated eigenvalues
    w, V = oracle.jacobi_eig(A)
    assert np.abs(w - lap_eigs(9, 2)).max() < 1e-13


# ---------------------------------------------------------------- bounds
@pytest.mark.parametrize("N,dim,pot", [(40, 2, None), (12, 3, 0), (30, 3, 0)])
def test_bounds_contain_spectrum_within_gershgorin(N, dim, pot):
    A = I.laplacian(N, dim, pot_seed=pot)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    ex = lap_eigs(N, dim)
    elo, ehi = ex[0], ex[-1]
    if pot is not None:
        if A.n <= 2000:
            w = np.linalg.eigvalsh(A.to_dense())
            elo, ehi = w[0], w[-1]
        else:
            # Rayleigh quotients of the extreme sine modes bound the extreme eigenvalues
            u = lap_eigvec(N, dim, (1,) * dim)
            v = lap_eigvec(N, dim, (N,) * dim)
            elo = u @ oracle.spmv(A, u) / (u @ u)
            ehi = v @ oracle.spmv(A, v) / (v @ v)
    assert lo <= elo + 1e-12 and hi >= ehi - 1e-12
    assert lo >= -1e-12 and hi <= 2 * 2 * dim + 1.0


# ---------------------------------------------------------------- TR Lanczos
@pytest.mark.parametrize("damp", [oracle.DAMP_SIGMA, oracle.DAMP_JACKSON])
def test_filtered_lanczos_40x40_all_91_with_multiplicity(damp):
    A = I.laplacian(40, 2)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [1.0, 1.6, lo, hi]
    p = oracle.find_pol(intv, damping=damp)
    lam, Y, res, st = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=91)
    ex = lap_eigs(40, 2)
    want = ex[(ex >= 1.0) & (ex <= 1.6)]
    assert len(want) == 91 and st["nev"] == 91 and st["status"] == 0
    assert np.abs(lam - want).max() <= 1e-12 * np.abs(want).max()
    assert res.max() <= 1e-10
    assert np.abs(Y.T @ Y - np.eye(91)).max() <= 1e-12


def test_filtered_lanczos_with_potential_matches_dense_eigh():
    A = I.laplacian(20, 2, pot_seed=0)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [2.0, 2.6, lo, hi]
    want = w[(w >= 2.0) & (w <= 2.6)]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-10 * np.abs(want).max()
    R = A.to_dense() @ Y - Y * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(lo), abs(hi))


def test_filtered_lanczos_boundary_slice_3d():
    N = 10
    A = I.laplacian(N, 3)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [lo, 1.4, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    assert p["boundary"] == -1
    ex = lap_eigs(N, 3)
    want = ex[ex <= 1.4]
    lam, Y, res, st = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)          # includes the triple eigenvalues of the cube
    assert np.abs(lam - want).max() <= 1e-12 * 12


@pytest.mark.parametrize("end", ["low", "high"])
def test_slice_reaching_a_spectrum_bound_owns_the_extreme_eigenvalue(end):
    """A slice whose end is the spectrum bound keeps every eigenvalue beyond
    that end: with the bound set exactly on the extreme eigenvalue (the
    closed form), the extreme eigenpair is returned, whichever way its
    computed Rayleigh quotient rounds."""
    N = 10
    A = I.laplacian(N, 3)
    ex = lap_eigs(N, 3)
    lo, hi = float(ex[0]), float(ex[-1])
    intv = [lo, 1.4, lo, hi] if end == "low" else [10.6, hi, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    want = ex[(ex >= intv[0]) & (ex <= intv[1])]
    lam, Y, res, st = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-12 * 12


def test_filtered_lanczos_empty_slice():
    A = I.laplacian(12, 2)
    ex = lap_eigs(12, 2)
    # a gap between two consecutive distinct eigenvalues
    u = np.unique(np.round(ex, 12))
    i = np.argmax(np.diff(u[10:50])) + 10
    a, b = u[i] + 0.2 * (u[i + 1] - u[i]), u[i + 1] - 0.2 * (u[i + 1] - u[i])
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [a, b, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_SIGMA)
    lam, Y, res, st = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=5)
    assert len(lam) == 0 and st["status"] == 0


# ---------------------------------------------------------------- non-restart Lanczos
def test_filtered_lanczos_nr_32x32_all_with_multiplicity():
    A = I.laplacian(32, 2)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [1.0, 1.5, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    ex = lap_eigs(32, 2)
    want = ex[(ex >= 1.0) & (ex <= 1.5)]
    # the square grid has double eigenvalues: one start vector still finds both copies
    assert len(np.unique(np.round(want, 10))) < len(want)
    lam, Y, res, st = oracle.filtered_lanczos_nr(A, intv, p, tol=1e-10, nev_est=len(want))
    assert st["nev"] == len(want) and st["status"] == 0 and st["nrestart"] == 0
    assert np.abs(lam - want).max() <= 1e-12 * np.abs(want).max()
    assert res.max() <= 1e-10
    assert np.abs(Y.T @ Y - np.eye(len(want))).max() <= 1e-10
    # the step count is a multiple of the test period, and nmv counts deg per step
    assert st["niter"] % 30 == 0
    assert st["nmv"] >= st["niter"] * p["deg"]


def test_filtered_lanczos_nr_with_potential_matches_dense_eigh_and_tr():
    A = I.laplacian(20, 2, pot_seed=0)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [2.0, 2.6, lo, hi]
    want = w[(w >= 2.0) & (w <= 2.6)]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_lanczos_nr(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-10 * np.abs(want).max()
    R = A.to_dense() @ Y - Y * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(lo), abs(hi))
    lam2, _, _, _ = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=len(want))
    assert np.abs(lam - lam2).max() <= 1e-12 * np.abs(want).max()


def test_filtered_lanczos_nr_boundary_and_empty_slices():
    A = I.laplacian(10, 3)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    ex = lap_eigs(10, 3)
    intv = [lo, 1.4, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    want = ex[ex <= 1.4]
    lam, Y, res, st = oracle.filtered_lanczos_nr(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)          # the cube's triple eigenvalues included
    assert np.abs(lam - want).max() <= 1e-12 * 12
    B = I.laplacian(12, 2)
    u = np.unique(np.round(lap_eigs(12, 2), 12))
    i = np.argmax(np.diff(u[10:50])) + 10
    a, b = u[i] + 0.2 * (u[i + 1] - u[i]), u[i + 1] - 0.2 * (u[i + 1] - u[i])
    lo, hi = oracle.lanczos_bounds(B, 80, 3)
    p = oracle.find_pol([a, b, lo, hi], damping=oracle.DAMP_SIGMA)
    lam, Y, res, st = oracle.filtered_lanczos_nr(B, [a, b, lo, hi], p, tol=1e-10, nev_est=5)
    assert len(lam) == 0 and st["status"] == 0


def test_filtered_lanczos_nr_step_cap_reports_unsettled():
    A = I.laplacian(24, 2, pot_seed=3)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [1.0, 1.5, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_lanczos_nr(A, intv, p, m=20, tol=1e-10, nev_est=30)
    assert st["status"] == 1 and st["niter"] == 20
    assert np.all(res <= 1e-10) and np.all((lam >= 1.0) & (lam <= 1.5))


# ---------------------------------------------------------------- subspace iteration
def test_filtered_subspace_32x32_all_with_multiplicity():
    A = I.laplacian(32, 2)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [1.0, 1.5, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    ex = lap_eigs(32, 2)
    want = ex[(ex >= 1.0) & (ex <= 1.5)]
    assert len(np.unique(np.round(want, 10))) < len(want)
    lam, Y, res, st = oracle.filtered_subspace(A, intv, p, tol=1e-10, nev_est=len(want))
    assert st["nev"] == len(want) and st["status"] == 0
    assert np.abs(lam - want).max() <= 1e-12 * np.abs(want).max()
    assert res.max() <= 1e-10
    assert np.abs(Y.T @ Y - np.eye(len(want))).max() <= 1e-10
    b = 3 * len(want) + 8
    assert st["nmv"] == st["niter"] * b * p["deg"] + (st["niter"] - 1) * b


def test_filtered_subspace_with_potential_matches_dense_and_lanczos():
    A = I.laplacian(20, 2, pot_seed=0)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [2.0, 2.6, lo, hi]
    want = w[(w >= 2.0) & (w <= 2.6)]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_subspace(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-10 * np.abs(want).max()
    R = A.to_dense() @ Y - Y * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(lo), abs(hi))
    lam2, _, _, _ = oracle.filtered_lanczos(A, intv, p, tol=1e-10, nev_est=len(want))
    assert np.abs(lam - lam2).max() <= 1e-12 * np.abs(want).max()


def test_filtered_subspace_boundary_empty_and_small_block():
    A = I.laplacian(10, 3)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    ex = lap_eigs(10, 3)
    intv = [lo, 1.4, lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_SIGMA, tau_ext=0.4)
    want = ex[ex <= 1.4]
    lam, Y, res, st = oracle.filtered_subspace(A, intv, p, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want) and st["status"] == 0
    assert np.abs(lam - want).max() <= 1e-12 * 12
    # a block smaller than the count: every Ritz value lands in the slice
    lam, Y, res, st = oracle.filtered_subspace(A, intv, p, block=len(want) - 5, tol=1e-10)
    assert st["status"] == 3
    B = I.laplacian(12, 2)
    u = np.unique(np.round(lap_eigs(12, 2), 12))
    i = np.argmax(np.diff(u[10:50])) + 10
    a, b = u[i] + 0.2 * (u[i + 1] - u[i]), u[i + 1] - 0.2 * (u[i + 1] - u[i])
    lo, hi = oracle.lanczos_bounds(B, 80, 3)
    p = oracle.find_pol([a, b, lo, hi], damping=oracle.DAMP_SIGMA)
    lam, Y, res, st = oracle.filtered_subspace(B, [a, b, lo, hi], p, tol=1e-10, nev_est=3)
    assert len(lam) == 0 and st["status"] == 0


# ---------------------------------------------------------------- Lanczos DOS
def test_lanczos_dos_gauss_quadrature_is_exact_to_degree_2m_minus_1():
    """For each probe v, sum_k w_k T_j(theta_k-hat) = v^T T_j(A-hat) v / v^T v for
    j < 2m (Gauss quadrature), with v the Lanczos start vector of its stream and
    the right side computed densely."""
    A = I.laplacian(12, 2, pot_seed=2)
    D = A.to_dense()
    m, nvec = 8, 3
    nodes, weights, dims = oracle.lanczos_dos(A, m, nvec, seed=5)
    w = np.linalg.eigvalsh(D)
    c, d = 0.5 * (w[-1] + w[0]) + 0.0, 0.5 * (w[-1] - w[0]) * 1.001
    Dh = (D - c * np.eye(A.n)) / d
    for l in range(nvec):
        assert dims[l] == m and abs(weights[l].sum() - 1.0) <= 1e-14
        v = I.lanczos_start(5, A.n, l)
        v = v / np.linalg.norm(v)
        th = (nodes[l] - c) / d
        t_prev, t_cur = v.copy(), Dh @ v
        q_prev, q_cur = np.ones(m), th.copy()
        for j in range(2 * m):
            if j == 0:
                lhs, rhs = weights[l].sum(), v @ v
            elif j == 1:
                lhs, rhs = weights[l] @ q_cur, v @ t_cur
            else:
                t_prev, t_cur = t_cur, 2 * Dh @ t_cur - t_prev
                q_prev, q_cur = q_cur, 2 * th * q_cur - q_prev
                lhs, rhs = weights[l] @ q_cur, v @ t_cur
            assert abs(lhs - rhs) <= 1e-12, (l, j, lhs, rhs)


def test_lanczos_dos_full_length_gives_the_spectrum():
    """With m = n the nodes are the eigenvalues and the weights the squared
    components of the start vector along the eigenvectors (numpy eigh)."""
    A = I.laplacian(7, 2, pot_seed=3)
    w, U = np.linalg.eigh(A.to_dense())
    nodes, weights, dims = oracle.lanczos_dos(A, A.n, 1, seed=9)
    assert dims[0] == A.n
    v = I.lanczos_start(9, A.n, 0)
    v = v / np.linalg.norm(v)
    assert np.abs(nodes[0] - w).max() <= 1e-12 * np.abs(w).max()
    assert np.abs(weights[0] - (U.T @ v) ** 2).max() <= 1e-10


def test_lanczos_dos_count_and_slicer_against_closed_form():
    A = I.laplacian(40, 2)
    q = oracle.lanczos_dos(A, 60, 40, seed=1)
    assert abs(oracle.lanczos_count(q, A.n, 0.0, -1.0, 9.0) - A.n) <= 1e-9
    exact = lap_count(40, 2, 1.0, 1.6)
    assert abs(oracle.lanczos_count(q, A.n, 0.0, 1.0, 1.6) - exact) <= 0.08 * exact
    assert abs(oracle.lanczos_count(q, A.n, 0.05, 1.0, 1.6) - exact) <= 0.08 * exact
    # slices of the 49^3 interval of Table tab:lapslicing hold similar closed-form counts
    B = I.laplacian(20, 3)
    qb = oracle.lanczos_dos(B, 80, 30, seed=2)
    sli = oracle.lanczos_slicer(qb, B.n, 0.02, 1.0, 3.0, 5)
    cnt = [lap_count(20, 3, sli[i], sli[i + 1]) for i in range(5)]
    assert max(cnt) <= 1.35 * min(cnt), (sli, cnt)


def test_lanczos_dos_smoothed_slices_balance_closed_form_counts():
    """Point masses give a step-function count that cannot be cut finely;
    spreading each node by sigma = (b - a) / (2m) balances ten slices of a
    300-eigenvalue-per-slice interval to within 35% (closed-form counts)."""
    A = I.laplacian(200, 2)
    q = oracle.lanczos_dos(A, 80, 20, seed=1)
    sli = oracle.lanczos_slicer(q, A.n, 8.0 / 160, 1.0, 1.3, 10)
    cnt = [lap_count(200, 2, sli[i], sli[i + 1]) for i in range(10)]
    assert max(cnt) <= 1.35 * min(cnt), cnt
    raw = oracle.lanczos_slicer(q, A.n, 0.0, 1.0, 1.3, 10)
    cnt0 = [lap_count(200, 2, raw[i], raw[i + 1]) for i in range(10)]
    assert max(cnt0) > 5 * max(min(cnt0), 1)


# ---------------------------------------------------------------- generalized problems
def _fe_eigs(N):
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    mu = (2 - 2 * np.cos(th)) / ((4 + 2 * np.cos(th)) / 6)
    return np.sort((mu[:, None] + mu[None, :]).ravel())


def test_fe_pencil_closed_form():
    import scipy.linalg as sl
    A, B = I.fe_pencil(9)
    w = sl.eigh(A.to_dense(), B.to_dense(), eigvals_only=True)
    assert np.abs(w - _fe_eigs(9)).max() <= 1e-12 * w.max()


@pytest.mark.parametrize("lo,hi,deg", [(0.1, 1.0, 20), (1.0, 3.0, 12), (0.11, 0.99, 40)])
def test_lspol_inverse_matches_closed_form_series(lo, hi, deg):
    """1/(c + d u) = (2/sqrt(c^2 - d^2)) sum' (-r)^j T_j(u), r = (c - sqrt(c^2 - d^2))/d."""
    c, d = 0.5 * (hi + lo), 0.5 * (hi - lo)
    q = np.sqrt(c * c - d * d)
    r = (c - q) / d
    ref = 2 * (-r) ** np.arange(deg + 1) / q
    ref[0] /= 2
    assert np.abs(oracle.lspol(0, lo, hi, deg) - ref).max() <= 1e-14 * ref[0]


def test_lspol_inverse_sqrt_converges():
    t = np.linspace(0.1, 1.0, 2001)
    u = (t - 0.55) / 0.45
    errs = []
    for deg in (10, 20, 40):
        cf = oracle.lspol(1, 0.1, 1.0, deg)
        errs.append(np.abs(np.polynomial.chebyshev.chebval(u, cf) - 1 / np.sqrt(t)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-9, errs


def test_cg_and_pencil_bounds():
    A, B = I.fe_pencil(16)
    r = I.lanczos_start(4, B.n)
    x = oracle.cg_solve(B, r)
    assert np.linalg.norm(B.to_dense() @ x - r) <= 1e-13 * np.linalg.norm(r)
    ex = _fe_eigs(16)
    lo, hi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    assert lo <= ex[0] + 1e-12 and hi >= ex[-1] - 1e-12
    assert ex[0] - lo <= 1e-3 * ex[-1] and hi - ex[-1] <= 1e-3 * ex[-1]


@pytest.mark.parametrize("ab", [(3.0, 5.0), (10.0, 11.0)])
def test_filtered_lanczos_gen_fe_pencil_closed_form(ab):
    A, B = I.fe_pencil(16)
    ex = _fe_eigs(16)
    want = ex[(ex >= ab[0]) & (ex <= ab[1])]
    lo, hi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    intv = [ab[0], ab[1], lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_lanczos_gen(A, B, intv, p, tol=1e-10, nev_est=len(want))
    assert st["status"] == 0 and len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-11 * ex[-1]
    assert res.max() <= 1e-10
    Db = B.to_dense()
    assert np.abs(Y.T @ Db @ Y - np.eye(len(lam))).max() <= 1e-10
    R = A.to_dense() @ Y - Db @ Y * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-9 * ex[-1]


@pytest.mark.parametrize("ab", [(0.5, 1.2), (2.0, 3.0)])
def test_filtered_lanczos_gen_thick_restart_fe_pencil_closed_form(ab):
    """The thick-restart form for the pencil finds every eigenvalue of the
    slice, the double ones (lambda = mu_i + mu_j = mu_j + mu_i) included, with
    B-orthonormal vectors."""
    A, B = I.fe_pencil(16)
    ex = _fe_eigs(16)
    want = ex[(ex >= ab[0]) & (ex <= ab[1])]
    assert np.any(np.diff(want) < 1e-12)            # the slice holds double eigenvalues
    lo, hi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    intv = [ab[0], ab[1], lo, hi]
    p = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = oracle.filtered_lanczos_gen_tr(A, B, intv, p, tol=1e-10,
                                                     nev_est=len(want))
    assert st["status"] == 0 and len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-11 * ex[-1]
    assert res.max() <= 1e-10
    Db = B.to_dense()
    assert np.abs(Y.T @ Db @ Y - np.eye(len(lam))).max() <= 1e-10
    R = A.to_dense() @ Y - Db @ Y * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-9 * ex[-1]


def test_paper_counts_from_closed_form():
    for r in GOLD["lap_problems"]["rows"]:
        if r["n"] > 600000:
            continue
        assert lap_count(r["N"], r["dim"], *r["intv"]) == r["nu"]
    s = GOLD["slicing_49cube"]
    for row in s["rows"]:
        for (xi, eta), nu in zip(row["slices"], row["nu"]):
            assert lap_count(49, 3, xi, eta) == nu


@pytest.mark.slow
def test_paper_counts_largest_grids():
    for r in GOLD["lap_problems"]["rows"]:
        if r["n"] > 600000:
            assert lap_count(r["N"], r["dim"], *r["intv"]) == r["nu"]
