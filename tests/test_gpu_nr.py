"""GPU parity of the non-restart filtered Lanczos (EVSL_LAN_NR) against the
oracle's non-restart solver, closed forms and dense solves.

Tolerances: eigenvalues 1e-10 relative (FP64; the two sides differ only in
summation order, so step counts may differ by one test period while the
converged eigenvalues agree to rounding); residuals <= tol.
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


def _setup(A, ab, damp=ev.DAMP_JACKSON, tau_ext=0.4):
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [ab[0] if ab[0] is not None else lo, ab[1], lo, hi]
    pol = ev.evsl_cheb_coeffs(intv, damping=damp, tau=0.8, tau_ext=tau_ext)
    opol = oracle.find_pol(intv, damping=damp, tau=0.8, tau_ext=tau_ext)
    return Ad, intv, pol, opol


def test_nr_32x32_matches_oracle_and_closed_form(ctx):
    A = I.laplacian(32, 2)
    Ad, intv, pol, opol = _setup(A, (1.0, 1.5))
    ex = lap_eigs(32, 2)
    want = ex[(ex >= 1.0) & (ex <= 1.5)]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, pol, ev.lan_opts(tol=1e-10, nev_est=len(want), method=ev.EVSL_LAN_NR))
    olam, _, _, ost = oracle.filtered_lanczos_nr(A, intv, opol, tol=1e-10, nev_est=len(want))
    assert st["status"] == ev.EVSL_OK and st["nrestart"] == 0
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, np.abs(want).max())
    assert_eigs_match(lam, olam, np.abs(want).max())
    assert res.max() <= 1e-10
    Yh = Y.cpu().numpy()
    assert np.abs(Yh.T @ Yh - np.eye(len(want))).max() <= 1e-10
    assert abs(st["niter"] - ost["niter"]) <= 30


def test_nr_potential_matches_dense_and_oracle(ctx):
    A = I.laplacian(20, 2, pot_seed=0)
    Ad, intv, pol, opol = _setup(A, (2.0, 2.6))
    w = np.linalg.eigvalsh(A.to_dense())
    want = w[(w >= 2.0) & (w <= 2.6)]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, pol, ev.lan_opts(tol=1e-10, nev_est=len(want), method=ev.EVSL_LAN_NR))
    olam, _, _, _ = oracle.filtered_lanczos_nr(A, intv, opol, tol=1e-10, nev_est=len(want))
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, np.abs(want).max())
    assert_eigs_match(lam, olam, np.abs(want).max())
    Yh = Y.cpu().numpy()
    R = A.to_dense() @ Yh - Yh * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(intv[2]), abs(intv[3]))


def test_nr_boundary_slice_finds_triples(ctx):
    A = I.laplacian(10, 3)
    Ad, intv, pol, opol = _setup(A, (None, 1.4), damp=ev.DAMP_SIGMA)
    assert pol.boundary == -1
    ex = lap_eigs(10, 3)
    want = ex[ex <= 1.4]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, pol, ev.lan_opts(tol=1e-10, nev_est=len(want), method=ev.EVSL_LAN_NR))
    assert len(lam) == len(want)
    assert np.abs(lam - want).max() <= 1e-12 * 12


def test_nr_batch_matches_single(ctx):
    A = I.laplacian(24, 2, pot_seed=1)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    w = np.linalg.eigvalsh(A.to_dense())
    cuts = [1.0, 1.3, 1.6, 1.9]
    ivs = [[cuts[q], cuts[q + 1], lo, hi] for q in range(3)]
    pols = [ev.evsl_cheb_coeffs(iv) for iv in ivs]
    opts = [ev.lan_opts(tol=1e-10, seed=2 + q, nev_est=40, method=ev.EVSL_LAN_NR)
            for q in range(3)]
    for gw in (0, 1):
        ctx.set_group_width(gw)
        outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
        for q, (lam, Y, res, st) in enumerate(outs):
            want = w[(w >= ivs[q][0]) & (w <= ivs[q][1])]
            assert st["status"] == ev.EVSL_OK
            assert len(lam) == len(want), (q, gw)
            assert_eigs_match(lam, want, np.abs(w).max())
            one = ev.evsl_filtered_lanczos(ctx, Ad, ivs[q], pols[q], opts[q])
            assert_eigs_match(one[0], lam, np.abs(w).max())
    ctx.set_group_width(0)


def test_nr_step_cap_and_invalid_options(ctx):
    A = I.laplacian(24, 2, pot_seed=3)
    Ad, intv, pol, opol = _setup(A, (1.0, 1.5))
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, pol, ev.lan_opts(m=20, tol=1e-10, nev_est=30, method=ev.EVSL_LAN_NR))
    assert st["status"] == ev.EVSL_ENOCONV and st["niter"] == 20
    assert np.all(res <= 1e-10) and np.all((lam >= 1.0) & (lam <= 1.5))
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos(ctx, Ad, intv, pol, ev.lan_opts(method=ev.EVSL_LAN_NR,
                                                                 prec=ev.EVSL_F32))
    assert e.value.code == ev.EVSL_ENOTIMPL
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos(ctx, Ad, intv, pol, ev.lan_opts(method=7))
    assert e.value.code == ev.EVSL_EINVAL


def test_nr_paper_problem_100cube_all_475_eigenvalues(ctx):
    """The largest Laplacian of Table tab:lap_pol_results: 100^3, [1.0, 1.018],
    which holds 475 eigenvalues (closed form, many of them multiple). sigma
    damping, tau = 0.8, bounds from the device Lanczos run (they contain the
    spectrum; the printed b = 11.9882 lies below lambda_max of 100^3). The
    non-restart solver must return every one of them: an earlier version
    stopped at 183."""
    N = 100
    A = I.laplacian(N, 3)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.018, lo, hi]
    pol = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_SIGMA, tau=0.8, tau_ext=0.4)
    ex = lap_eigs(N, 3)
    want = ex[(ex >= 1.0) & (ex <= 1.018)]
    assert len(want) == 475
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, pol, ev.lan_opts(tol=1e-8, nev_est=len(want), method=ev.EVSL_LAN_NR))
    del Y
    assert st["status"] == ev.EVSL_OK, st
    assert len(lam) == 475 and res.max() <= 1e-8
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
