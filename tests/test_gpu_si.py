"""GPU parity of the filtered subspace iteration (evsl_filtered_subspace)
against the oracle's subspace iteration, closed forms and dense solves.

Tolerances: eigenvalues 1e-10 relative (the device orthonormalises by SVQB and
the oracle by Gram-Schmidt: different bases of the same span, so the Ritz
pairs agree to rounding); residuals <= tol.
"""
import numpy as np
import pytest

import evsl_inputs as I
import oracle
import paper_1802_05215_amd as ev
from tests.closed_form import lap_eigs
from tests.eig_rules import assert_eigs_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ev.load()
    c = ev.Ctx()
    yield c
    c.close()


def _setup(A, ab, damp=ev.DAMP_JACKSON):
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [ab[0] if ab[0] is not None else lo, ab[1], lo, hi]
    pol = ev.evsl_cheb_coeffs(intv, damping=damp, tau=0.8, tau_ext=0.4)
    opol = oracle.find_pol(intv, damping=damp, tau=0.8, tau_ext=0.4)
    return Ad, intv, pol, opol


def test_si_32x32_matches_oracle_and_closed_form(ctx):
    A = I.laplacian(32, 2)
    Ad, intv, pol, opol = _setup(A, (1.0, 1.5))
    ex = lap_eigs(32, 2)
    want = ex[(ex >= 1.0) & (ex <= 1.5)]
    lam, Y, res, st = ev.evsl_filtered_subspace(
        ctx, Ad, intv, pol, ev.si_opts(tol=1e-10, nev_est=len(want)))
    olam, _, _, ost = oracle.filtered_subspace(A, intv, opol, tol=1e-10, nev_est=len(want))
    assert st["status"] == ev.EVSL_OK, st
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, np.abs(want).max())
    assert_eigs_match(lam, olam, np.abs(want).max())
    assert res.max() <= 1e-10
    Yh = Y.cpu().numpy()
    assert np.abs(Yh.T @ Yh - np.eye(len(want))).max() <= 1e-10
    assert abs(st["niter"] - ost["niter"]) <= 2


def test_si_potential_matches_dense_and_oracle(ctx):
    A = I.laplacian(20, 2, pot_seed=0)
    Ad, intv, pol, opol = _setup(A, (2.0, 2.6))
    w = np.linalg.eigvalsh(A.to_dense())
    want = w[(w >= 2.0) & (w <= 2.6)]
    lam, Y, res, st = ev.evsl_filtered_subspace(
        ctx, Ad, intv, pol, ev.si_opts(tol=1e-10, nev_est=len(want)))
    olam, _, _, _ = oracle.filtered_subspace(A, intv, opol, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, np.abs(want).max())
    assert_eigs_match(lam, olam, np.abs(want).max())
    Yh = Y.cpu().numpy()
    R = A.to_dense() @ Yh - Yh * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(intv[2]), abs(intv[3]))


def test_si_boundary_slice_finds_triples(ctx):
    A = I.laplacian(10, 3)
    Ad, intv, pol, opol = _setup(A, (None, 1.4), damp=ev.DAMP_SIGMA)
    ex = lap_eigs(10, 3)
    want = ex[ex <= 1.4]
    lam, Y, res, st = ev.evsl_filtered_subspace(
        ctx, Ad, intv, pol, ev.si_opts(tol=1e-10, nev_est=len(want)))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-12 * 12


def test_si_batch_matches_single_and_dense(ctx):
    A = I.laplacian(24, 2, pot_seed=1)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    w = np.linalg.eigvalsh(A.to_dense())
    cuts = [1.0, 1.3, 1.6, 1.9]
    ivs = [[cuts[q], cuts[q + 1], lo, hi] for q in range(3)]
    pols = [ev.evsl_cheb_coeffs(iv) for iv in ivs]
    cnts = [int(((w >= iv[0]) & (w <= iv[1])).sum()) for iv in ivs]
    opts = [ev.si_opts(tol=1e-10, seed=2 + q, nev_est=cnts[q]) for q in range(3)]
    outs = ev.evsl_filtered_subspace_batch(ctx, Ad, ivs, pols, opts)
    for q, (lam, Y, res, st) in enumerate(outs):
        want = w[(w >= ivs[q][0]) & (w <= ivs[q][1])]
        assert st["status"] == ev.EVSL_OK
        assert len(lam) == len(want), q
        assert_eigs_match(lam, want, np.abs(w).max())
        one = ev.evsl_filtered_subspace(ctx, Ad, ivs[q], pols[q], opts[q])
        assert len(one[0]) == len(lam)
        assert_eigs_match(one[0], lam, np.abs(w).max())


def test_si_small_block_and_empty_slice(ctx):
    A = I.laplacian(10, 3)
    Ad, intv, pol, opol = _setup(A, (None, 1.4), damp=ev.DAMP_SIGMA)
    want = lap_eigs(10, 3)
    want = want[want <= 1.4]
    lam, Y, res, st = ev.evsl_filtered_subspace(
        ctx, Ad, intv, pol, ev.si_opts(block=len(want) - 5, tol=1e-10))
    assert st["status"] == ev.EVSL_ENOCONV
    B = I.laplacian(12, 2)
    u = np.unique(np.round(lap_eigs(12, 2), 12))
    i = np.argmax(np.diff(u[10:50])) + 10
    a, b = u[i] + 0.2 * (u[i + 1] - u[i]), u[i + 1] - 0.2 * (u[i + 1] - u[i])
    Bd, intv, pol, opol = _setup(B, (a, b), damp=ev.DAMP_SIGMA)
    lam, Y, res, st = ev.evsl_filtered_subspace(ctx, Bd, intv, pol,
                                                ev.si_opts(tol=1e-10, nev_est=3))
    assert len(lam) == 0 and st["status"] == ev.EVSL_OK
