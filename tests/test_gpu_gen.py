"""GPU parity of the generalized-problem path (A x = lambda B x, B SPD) on a
bilinear finite-element pencil whose spectrum is known in closed form
(lambda_ij = mu_i + mu_j, mu = 1-D stiffness/mass eigenvalues), and against
the oracle's filtered Lanczos for (A, B), which uses exact (CG) solves.

Tolerances: eigenvalues 1e-10 relative to lambda_max; the device's solves
with B are a degree-60 Chebyshev fit of 1/t on B's spectrum (error ~1e-16 for
a condition number below 9), so its Ritz pairs agree with the exact-solve
oracle to rounding; residuals <= tol; Y^T B Y = I to 1e-10."""
import numpy as np
import pytest

import evsl_inputs as I
import oracle
import paper_1802_05215_amd as ev
from tests.eig_rules import assert_eigs_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
BDEG = 60


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ev.load()
    c = ev.Ctx()
    yield c
    c.close()


def _fe_eigs(N):
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    mu = (2 - 2 * np.cos(th)) / ((4 + 2 * np.cos(th)) / 6)
    return np.sort((mu[:, None] + mu[None, :]).ravel())


def _setup(ctx, N):
    A, B = I.fe_pencil(N)
    Ad, Bd = ev.DeviceCsr.from_host(A), ev.DeviceCsr.from_host(B)
    blo, bhi = ev.evsl_spectrum_bounds(ctx, Bd, 80, 3)
    bb = [0.98 * blo, 1.02 * bhi]
    return A, B, Ad, Bd, bb


def test_pencil_bounds_contain_the_spectrum(ctx):
    A, B, Ad, Bd, bb = _setup(ctx, 20)
    ex = _fe_eigs(20)
    lo, hi = ev.evsl_spectrum_bounds_gen(ctx, Ad, Bd, bb, BDEG, 80, 3)
    olo, ohi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    assert lo <= ex[0] + 1e-10 and hi >= ex[-1] - 1e-10
    # the widening terms |beta y_m| of the extreme Ritz pairs are tiny and
    # depend on rounding; the bounds agree with the oracle's to 1e-6 relative
    assert abs(lo - olo) <= 1e-6 * ex[-1] and abs(hi - ohi) <= 1e-6 * ex[-1]


@pytest.mark.parametrize("ab", [(3.0, 5.0), (10.0, 11.0)])
def test_filtered_lanczos_gen_matches_closed_form_and_oracle(ctx, ab):
    N = 16
    A, B, Ad, Bd, bb = _setup(ctx, N)
    ex = _fe_eigs(N)
    want = ex[(ex >= ab[0]) & (ex <= ab[1])]
    lo, hi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    intv = [ab[0], ab[1], lo, hi]
    pol = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_JACKSON)
    opol = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = ev.evsl_filtered_lanczos_gen(
        ctx, Ad, Bd, bb, BDEG, intv, pol,
        ev.lan_opts(tol=1e-10, nev_est=len(want), method=ev.EVSL_LAN_NR))
    olam, _, _, ost = oracle.filtered_lanczos_gen(A, B, intv, opol, tol=1e-10, nev_est=len(want))
    assert st["status"] == ev.EVSL_OK, st
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, ex[-1])
    assert_eigs_match(lam, olam, ex[-1])
    assert res.max() <= 1e-10
    Yh = Y.cpu().numpy()
    Db = B.to_dense()
    assert np.abs(Yh.T @ Db @ Yh - np.eye(len(lam))).max() <= 1e-10
    assert abs(st["niter"] - ost["niter"]) <= 30


@pytest.mark.parametrize("ab", [(0.5, 1.2), (2.0, 3.0), (10.0, 11.0)])
def test_filtered_lanczos_gen_thick_restart_matches_closed_form_and_oracle(ctx, ab):
    """The thick-restart form for the pencil: every eigenvalue of the slice,
    double ones included, equal to the closed form and to the oracle's
    thick-restart solver; B-orthonormal vectors."""
    N = 16
    A, B, Ad, Bd, bb = _setup(ctx, N)
    ex = _fe_eigs(N)
    want = ex[(ex >= ab[0]) & (ex <= ab[1])]
    lo, hi = oracle.lanczos_bounds_gen(A, B, 80, 3)
    intv = [ab[0], ab[1], lo, hi]
    pol = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_JACKSON)
    opol = oracle.find_pol(intv, damping=oracle.DAMP_JACKSON)
    lam, Y, res, st = ev.evsl_filtered_lanczos_gen(
        ctx, Ad, Bd, bb, BDEG, intv, pol,
        ev.lan_opts(tol=1e-10, nev_est=len(want), method=ev.EVSL_LAN_TR))
    olam, _, _, ost = oracle.filtered_lanczos_gen_tr(A, B, intv, opol, tol=1e-10,
                                                     nev_est=len(want))
    assert st["status"] == ev.EVSL_OK, st
    assert len(lam) == len(want) == len(olam)
    assert_eigs_match(lam, want, ex[-1])
    assert_eigs_match(lam, olam, ex[-1])
    assert res.max() <= 1e-10
    Yh = Y.cpu().numpy()
    Db = B.to_dense()
    assert np.abs(Yh.T @ Db @ Yh - np.eye(len(lam))).max() <= 1e-10
    R = A.to_dense() @ Yh - Db @ Yh * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-9 * ex[-1]


def test_generalized_rejects_unsupported_options(ctx):
    A, B, Ad, Bd, bb = _setup(ctx, 8)
    lo, hi = oracle.lanczos_bounds_gen(A, B, 40, 3)
    intv = [3.0, 5.0, lo, hi]
    pol = ev.evsl_cheb_coeffs(intv)
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos_gen(ctx, Ad, Bd, bb, BDEG, intv, pol,
                                     ev.lan_opts(method=ev.EVSL_LAN_TR, prec=ev.EVSL_F32))
    assert e.value.code == ev.EVSL_ENOTIMPL
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos_gen(ctx, Ad, Bd, [0.0, 1.0], BDEG, intv, pol)
    assert e.value.code == ev.EVSL_EINVAL
