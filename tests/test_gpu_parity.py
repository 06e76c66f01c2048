"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded inputs, and against closed forms at full size.

Tolerances (FP64):
* filter p(A-hat)V: ||Y_gpu - Y_oracle|| / ||V|| <= 1e-11 max(1, k/2000). Both
  sides run the forward three-term recurrence, whose rounding error grows
  O(k eps) on [-1, 1]; only the summation order differs.
* KPM moments: 1e-12 relative to n (the moments are O(n) sums).
* eigenvalues: |dlambda| <= 1e-10 max(|lambda|, 1e-6 ||A||); residuals <= tol;
  eigenvectors checked by residual and orthogonality, never elementwise.
"""
import numpy as np
import pytest

import evsl_inputs as I
import oracle
import paper_1802_05215_amd as ev
from tests.closed_form import lap_eig_of, lap_eigs, lap_eigvec
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


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _pol(intv, damp=ev.DAMP_JACKSON):
    return ev.evsl_cheb_coeffs(intv, damping=damp, tau=0.8, tau_ext=0.4)


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
@pytest.mark.parametrize("N,dim,pot,intv", [(40, 2, None, [1.0, 1.6, 0.0, 8.0]),
                                            (13, 3, 0, [2.0, 2.3, 0.0, 13.0]),
                                            (23, 2, 5, [0.0, 0.7, 0.0, 9.0])])
def test_filter_single_vector_matches_oracle(ctx, variant, N, dim, pot, intv):
    A = I.laplacian(N, dim, pot_seed=pot)
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol(intv)
    v = I.lanczos_start(9, A.n)
    ctx.set_spmv_variant(variant)
    V = _dev(v)
    Y = torch.empty_like(V)
    ev.evsl_filter_apply(ctx, Ad, [p], [0], V, Y)
    torch.cuda.synchronize()
    ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, v)
    err = np.linalg.norm(Y.cpu().numpy() - ref) / np.linalg.norm(v)
    assert err <= 1e-11 * max(1.0, p.deg / 2000), (err, p.deg)
    ctx.set_spmv_variant(0)


@pytest.mark.parametrize("blk_variant", [1, 2, 3])
@pytest.mark.parametrize("sorted_cols", [True, False])
def test_filter_block_matches_oracle(ctx, sorted_cols, blk_variant):
    ev.evsl_set_block_variant(blk_variant)
    A = I.laplacian(37, 2, pot_seed=1)             # n = 1369: ragged against every tile
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = 0.0, 9.0
    pols = [_pol([a, b, lo, hi]) for a, b in [(1.0, 1.3), (2.0, 2.1), (0.0, 0.9)]]
    groups = [1, 1, 0, 0, 2] if sorted_cols else [0, 2, 1, 0, 1]
    degs = [pols[g].deg for g in groups]
    if sorted_cols:
        assert all(degs[i] >= degs[i + 1] for i in range(len(degs) - 1))
    ncols, ld = 5, 8
    rng = np.random.default_rng(4)
    Vh = np.zeros((A.n, ld))
    Vh[:, :ncols] = rng.standard_normal((A.n, ncols))
    V = _dev(Vh)
    Y = torch.zeros_like(V)
    ev.evsl_filter_apply(ctx, Ad, pols, groups, V[:, :ncols], Y[:, :ncols])
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    for c in range(ncols):
        p = pols[groups[c]]
        ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, Vh[:, c])
        err = np.linalg.norm(Yh[:, c] - ref) / np.linalg.norm(Vh[:, c])
        assert err <= 1e-11, (c, err)
    assert np.all(Yh[:, ncols:] == 0.0)           # padding columns untouched
    ev.evsl_set_block_variant(2)


SCHEDULES = [(1, 0, 1, 0, 0, 1), (0, 0, 1, 0, 0, 1), (2, 8, 1, 0, 0, 1), (2, 16, 4, 0, 0, 1),
             (2, 64, 1, 0, 0, 1), (2, 16, 64, 0, 0, 1), (2, 8, 3, 0, 0, 1), (1, 0, 1, 4, 0, 1),
             (2, 16, 4, 4, 0, 1), (2, 8, 1, 1, 0, 1), (1, 0, 1, 0, 8, 1), (2, 16, 4, 0, 256, 1),
             (2, 32, 16, 0, 40, 1), (1, 0, 1, 0, 0, 0)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_filter_block_schedules_are_bitwise_equal_and_match_oracle(ctx, prec):
    """Every launch schedule of the block filter (launch order, XCD row
    ranges, column chunks one after another with row blocks dealt to the XCDs
    in runs) gives the same bits; FP64 matches the oracle. 21^3 + potential
    (n = 9261, ragged against every row tile), 120 of 128 columns (the last
    16-column chunk is half full), filters of three degrees so the Clenshaw
    step's active prefix changes with k."""
    A = I.laplacian(21, 3, pot_seed=3)
    Ad = ev.DeviceCsr.from_host(A)
    Am = Ad if prec == "f64" else Ad.with_values(Ad.val.float())
    lo, hi = 0.0, 13.0
    pols = [_pol([a, b, lo, hi]) for a, b in [(2.0, 2.2), (3.0, 3.6), (1.0, 1.05)]]
    order = np.argsort([-p.deg for p in pols])
    ncols, ld = 120, 128
    groups = [int(order[min(c // 40, 2)]) for c in range(ncols)]
    rng = np.random.default_rng(11)
    Vh = np.zeros((A.n, ld))
    Vh[:, :ncols] = rng.standard_normal((A.n, ncols))
    dt = torch.float64 if prec == "f64" else torch.float32
    V = _dev(Vh).to(dt)
    ref = None
    for sc in SCHEDULES:
        ctx.set_block_schedule(*sc)
        Y = torch.zeros_like(V)
        ev.evsl_filter_apply(ctx, Am, pols, groups, V[:, :ncols], Y[:, :ncols])
        torch.cuda.synchronize()
        assert torch.all(Y[:, ncols:] == 0)
        if ref is None:
            ref = Y
        else:
            assert torch.equal(Y, ref), sc
    ctx.set_block_schedule(1, 0, 1, 0, 0, 1)
    if prec == "f64":
        Yh = ref.cpu().numpy()
        for c in (0, 39, 40, 85, 119):
            p = pols[groups[c]]
            want = oracle.filter_apply(A, p.cc, p.dd, p.coef, Vh[:, c])
            assert np.linalg.norm(Yh[:, c] - want) / np.linalg.norm(Vh[:, c]) <= 1e-11


@pytest.mark.parametrize("blk_variant", [1, 2])
@pytest.mark.parametrize("ncols", [16, 300])
def test_filter_wide_block_matches_oracle(ctx, ncols, blk_variant):
    """Blocks wider than one workgroup row (300 > 256 columns) and rows with
    more nonzeros than the LDS stage holds fall back correctly."""
    ev.evsl_set_block_variant(blk_variant)
    A = I.laplacian(9, 3, pot_seed=2)
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol([2.0, 2.4, 0.0, 13.0])
    rng = np.random.default_rng(8)
    Vh = rng.standard_normal((A.n, ncols))
    V = _dev(Vh)
    Y = torch.empty_like(V)
    ev.evsl_filter_apply(ctx, Ad, [p], [0] * ncols, V, Y)
    torch.cuda.synchronize()
    ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, Vh)
    err = np.linalg.norm(Y.cpu().numpy() - ref, axis=0) / np.linalg.norm(Vh, axis=0)
    assert err.max() <= 1e-11
    ev.evsl_set_block_variant(2)


@pytest.mark.parametrize("prec,sched", [("f64", (1, 0, 1, 0, 0, 1)), ("f32", (1, 0, 1, 0, 0, 1)),
                                        ("f64", (2, 32, 16, 0, 0, 1)), ("f32", (2, 16, 1, 0, 0, 1)),
                                        ("f64", (2, 64, 64, 4, 64, 1)),
                                        ("f64", (1, 0, 1, 0, 0, 0))])
def test_filter_block_beyond_32bit_offsets(ctx, prec, sched):
    """n * ld >= 2^31 elements: the LDS kernel with 64-bit offsets, checked on
    sampled columns (first, middle, last) against the oracle at full size,
    under the default schedule and two chunked ones."""
    ctx.set_block_schedule(*sched)
    N, ncols = 2900, 256
    A = I.laplacian(N, 2, pot_seed=4)
    assert A.n * ncols >= 2 ** 31
    Ad = ev.DeviceCsr.from_host(A)
    p8 = ev.evsl_cheb_coeffs([2.0, 2.0001, 0.0, 9.0], max_deg=8)
    assert p8.deg == 8
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    dt = torch.float64 if prec == "f64" else torch.float32
    V = torch.randn((A.n, ncols), dtype=torch.float64, device="cuda", generator=g).to(dt)
    Y = torch.empty_like(V)
    Am = Ad if prec == "f64" else Ad.with_values(Ad.val.float())
    ev.evsl_filter_apply(ctx, Am, [p8], [0] * ncols, V, Y)
    torch.cuda.synchronize()
    for c in (0, ncols // 2 + 1, ncols - 1):
        v = V[:, c].double().cpu().numpy()
        ref = oracle.filter_apply(A, p8.cc, p8.dd, p8.coef, v)
        err = np.linalg.norm(Y[:, c].double().cpu().numpy() - ref) / np.linalg.norm(v)
        assert err <= (1e-13 if prec == "f64" else 8 * 6e-8 * 8), (c, err)
    ctx.set_block_schedule(1, 0, 1, 0, 0, 1)
    del V, Y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("permuted", [False, True])
def test_filter_block_column_offsets_and_wide_bandwidth(ctx, permuted):
    """The block filter reads 16-bit column offsets when the bandwidth allows
    (a 2-D Laplacian, bandwidth 200) and the 32-bit indices otherwise (the same
    matrix under a random symmetric permutation, bandwidth near n = 40,000);
    both agree with the oracle on every column."""
    A = I.laplacian(200, 2, pot_seed=3)
    if permuted:
        rng = np.random.default_rng(9)
        P = rng.permutation(A.n)
        inv = np.empty_like(P)
        inv[P] = np.arange(A.n)
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        r2, c2 = inv[rows], inv[A.col]
        order = np.lexsort((c2, r2))
        r2, c2, v2 = r2[order], c2[order], A.val[order]
        rp = np.zeros(A.n + 1, np.int64)
        np.add.at(rp, r2 + 1, 1)
        A = I.CSR(A.n, np.cumsum(rp).astype(np.int32), c2.astype(np.int32), v2.copy())
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        assert np.abs(A.col - rows).max() > 32767
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol([1.0, 1.2, 0.0, 9.0])
    rng = np.random.default_rng(10)
    Vh = rng.standard_normal((A.n, 6))
    V = _dev(Vh)
    Y = torch.empty_like(V)
    ev.evsl_filter_apply(ctx, Ad, [p], [0] * 6, V, Y)
    torch.cuda.synchronize()
    ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, Vh)
    err = np.linalg.norm(Y.cpu().numpy() - ref, axis=0) / np.linalg.norm(Vh, axis=0)
    assert err.max() <= 1e-11


def test_filter_dense_rows_fall_back(ctx):
    """A matrix whose rows exceed the LDS stage (a dense 300 x 300 block)."""
    rng = np.random.default_rng(2)
    n = 300
    M = rng.standard_normal((n, n))
    M = (M + M.T) / 2
    M /= np.abs(np.linalg.eigvalsh(M)).max()
    rows, cols = np.nonzero(np.ones((n, n)))
    A = I.CSR(n, np.arange(0, n * n + 1, n).astype(np.int32), cols.astype(np.int32),
              M[rows, cols].copy())
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol([0.1, 0.3, -1.0, 1.0])
    v = rng.standard_normal(n)
    ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, v)
    for var in (1, 2, 3, 4):
        ctx.set_spmv_variant(var)
        Y = torch.empty(n, dtype=torch.float64, device="cuda")
        ev.evsl_filter_apply(ctx, Ad, [p], [0], _dev(v), Y)
        torch.cuda.synchronize()
        assert np.linalg.norm(Y.cpu().numpy() - ref) <= 1e-11 * np.linalg.norm(v), var
    for bv in (1, 2, 3):
        ev.evsl_set_block_variant(bv)
        V2 = _dev(np.stack([v, 2 * v], axis=1))
        Y2 = torch.empty_like(V2)
        ev.evsl_filter_apply(ctx, Ad, [p], [0, 0], V2, Y2)
        torch.cuda.synchronize()
        assert np.linalg.norm(Y2.cpu().numpy()[:, 1] - 2 * ref) <= 2e-11 * np.linalg.norm(v), bv
    ctx.set_spmv_variant(0)
    ev.evsl_set_block_variant(2)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_filter_closed_form_eigenvector_full_size(ctx, variant):
    # 100^3 Laplacian (n = 1e6, the plain-method matrix without its potential)
    N = 100
    A = I.laplacian(N, 3)
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol([0.60, 0.61, 0.0, 12.0])
    ctx.set_spmv_variant(variant)
    for modes in ((1, 1, 1), (11, 17, 3), (60, 2, 41)):
        u = lap_eigvec(N, 3, modes)
        lam = lap_eig_of(N, modes)
        rho = np.polynomial.chebyshev.chebval((lam - p.cc) / p.dd, p.coef)
        U = _dev(u)
        Y = torch.empty_like(U)
        ev.evsl_filter_apply(ctx, Ad, [p], [0], U, Y)
        torch.cuda.synchronize()
        err = np.linalg.norm(Y.cpu().numpy() - rho * u) / np.linalg.norm(u)
        assert err <= 1e-11 * max(1.0, p.deg / 2000), (modes, err, p.deg)
    ctx.set_spmv_variant(0)


def test_filter_is_deterministic(ctx):
    A = I.laplacian(30, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    p = _pol([0.6, 0.7, 0.0, 13.0])
    V = _dev(I.lanczos_start(1, A.n))
    Y1, Y2 = torch.empty_like(V), torch.empty_like(V)
    ev.evsl_filter_apply(ctx, Ad, [p], [0], V, Y1)
    ev.evsl_filter_apply(ctx, Ad, [p], [0], V, Y2)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


@pytest.mark.parametrize("N,dim,pot,K,nv", [(40, 2, None, 40, 10), (17, 3, 0, 80, 20)])
def test_kpm_moments_match_oracle(ctx, N, dim, pot, K, nv):
    A = I.laplacian(N, dim, pot_seed=pot)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    intv = [1.0, 1.6, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, K, nv, seed=1, damping=ev.DAMP_JACKSON)
    V = oracle.rademacher(1, A.n, nv)
    ref = oracle.kpm_moments(A, lo, hi, K, V)
    assert np.abs(mom - ref).max() <= 1e-12 * A.n
    cnt = oracle.kpm_count(ref, oracle.DAMP_JACKSON, lo, hi, 1.0, 1.6)
    assert abs(est - cnt) <= 1e-9 * max(1.0, cnt)


@pytest.mark.parametrize("N,dim,pot", [(40, 2, None), (20, 3, 0), (60, 3, 0)])
def test_bounds_match_oracle_and_contain_spectrum(ctx, N, dim, pot):
    A = I.laplacian(N, dim, pot_seed=pot)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    rlo, rhi = oracle.lanczos_bounds(A, 80, 3)
    assert abs(lo - rlo) <= 1e-8 and abs(hi - rhi) <= 1e-8
    if pot is None:
        ex = lap_eigs(N, dim)
        elo, ehi = ex[0], ex[-1]
    elif A.n <= 8000:
        w = np.linalg.eigvalsh(A.to_dense())
        elo, ehi = w[0], w[-1]
    else:
        # Rayleigh quotients of the extreme sine modes bound the extreme eigenvalues
        u = lap_eigvec(N, dim, (1,) * dim)
        v = lap_eigvec(N, dim, (N,) * dim)
        elo = u @ oracle.spmv(A, u) / (u @ u)
        ehi = v @ oracle.spmv(A, v) / (v @ v)
    assert lo <= elo + 1e-12 and hi >= ehi - 1e-12


def _closed_form_interval(N, dim, a, b):
    ex = lap_eigs(N, dim)
    return ex[(ex >= a) & (ex <= b)]


def test_filtered_lanczos_40x40_all_91(ctx):
    """2-D 5-point Laplacian on 40 x 40, [1.0, 1.6]: 91 eigenvalues, 88 of them in
    exact double pairs, residual <= 1e-10."""
    A = I.laplacian(40, 2)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.6, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, 40, 10, seed=1, damping=ev.DAMP_JACKSON)
    p = _pol(intv)
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, intv, p,
                                               ev.lan_opts(tol=1e-10, seed=2, nev_est=int(est)))
    want = _closed_form_interval(40, 2, 1.0, 1.6)
    assert len(want) == 91 and st["nev"] == 91 and st["status"] == 0
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
    assert res.max() <= 1e-10
    Yh = Y.cpu().numpy()
    # pairs locked at different restarts are orthogonal to the level the basis
    # keeps against the locked vectors (about 1e-11 after a restart; the
    # second-pass gate holds the estimate below 1e-10)
    assert np.abs(Yh.T @ Yh - np.eye(91)).max() <= 1e-11
    # the oracle on the same inputs finds the same list
    olam, _, ores, _ = oracle.filtered_lanczos(A, intv, oracle.find_pol(intv, damping=2),
                                               tol=1e-10, nev_est=int(est))
    assert_eigs_match(lam, olam, max(abs(lo), abs(hi)))


def test_filtered_lanczos_potential_matches_dense(ctx):
    A = I.laplacian(20, 2, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [2.0, 2.6, lo, hi]
    w = np.linalg.eigvalsh(A.to_dense())
    want = w[(w >= 2.0) & (w <= 2.6)]
    p = _pol(intv)
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, intv, p,
                                               ev.lan_opts(tol=1e-10, nev_est=len(want)))
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
    R = A.to_dense() @ Y.cpu().numpy() - Y.cpu().numpy() * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * max(abs(lo), abs(hi))
    olam, _, _, _ = oracle.filtered_lanczos(A, intv, oracle.find_pol(intv, damping=2), tol=1e-10,
                                            nev_est=len(want))
    assert_eigs_match(lam, olam, max(abs(lo), abs(hi)))


def test_filtered_lanczos_boundary_slice_triples(ctx):
    N = 10
    A = I.laplacian(N, 3)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [lo, 1.4, lo, hi]
    p = _pol(intv)
    assert p.boundary == -1
    want = _closed_form_interval(N, 3, -1.0, 1.4)
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, intv, p,
                                               ev.lan_opts(tol=1e-10, nev_est=len(want)))
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))


@pytest.mark.parametrize("end", ["low", "high"])
def test_slice_reaching_a_spectrum_bound_owns_the_extreme_eigenvalue(ctx, end):
    """As in the oracle: bounds set exactly on the extreme eigenvalues; the
    boundary slice returns the extreme eigenpair and equals the oracle."""
    N = 10
    A = I.laplacian(N, 3)
    Ad = ev.DeviceCsr.from_host(A)
    ex = lap_eigs(N, 3)
    lo, hi = float(ex[0]), float(ex[-1])
    intv = [lo, 1.4, lo, hi] if end == "low" else [10.6, hi, lo, hi]
    p = ev.evsl_cheb_coeffs(intv, damping=ev.DAMP_SIGMA, tau=0.8, tau_ext=0.4)
    want = ex[(ex >= intv[0]) & (ex <= intv[1])]
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, intv, p,
                                               ev.lan_opts(tol=1e-10, nev_est=len(want)))
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
    olam, _, _, _ = oracle.filtered_lanczos(A, intv, oracle.find_pol(intv, damping=1),
                                            tol=1e-10, nev_est=len(want))
    assert_eigs_match(lam, olam, max(abs(lo), abs(hi)))


def test_filtered_lanczos_empty_slice(ctx):
    A = I.laplacian(12, 2)
    Ad = ev.DeviceCsr.from_host(A)
    u = np.unique(np.round(lap_eigs(12, 2), 12))
    i = np.argmax(np.diff(u[10:50])) + 10
    a, b = u[i] + 0.2 * (u[i + 1] - u[i]), u[i + 1] - 0.2 * (u[i + 1] - u[i])
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Ad, [a, b, lo, hi], _pol([a, b, lo, hi]),
                                               ev.lan_opts(tol=1e-10, nev_est=5))
    assert len(lam) == 0 and st["status"] == 0


@pytest.mark.parametrize("group", [0, 1, 2])
def test_batch_slices_match_single_and_closed_form(ctx, group):
    """Three KPM slices solved together; group 0 filters all slices in one
    block launch per degree step, 1 uses the single-vector kernel per slice,
    2 splits them into groups of two and one."""
    ctx.set_group_width(group)
    A = I.laplacian(40, 2)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.6, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, 40, 10, seed=1, damping=ev.DAMP_JACKSON)
    sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, 3, 2000)
    ivs = [[sli[q], sli[q + 1], lo, hi] for q in range(3)]
    pols = [_pol(iv) for iv in ivs]
    opts = [ev.lan_opts(tol=1e-10, seed=2 + q, nev_est=int(est / 3) + 5) for q in range(3)]
    outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
    got = []
    for q, (lam, Y, res, st) in enumerate(outs):
        keep = (lam >= ivs[q][0]) & ((lam < ivs[q][1]) | (q == 2))
        got.append(lam[keep])
        assert res.max() <= 1e-10
        one = ev.evsl_filtered_lanczos(ctx, Ad, ivs[q], pols[q], opts[q])[0]
        assert_eigs_match(lam, one, max(abs(lo), abs(hi)))
    got = np.sort(np.concatenate(got))
    want = _closed_form_interval(40, 2, 1.0, 1.6)
    assert len(got) == 91
    assert_eigs_match(got, want, max(abs(lo), abs(hi)))
    ctx.set_group_width(0)


@pytest.mark.parametrize("group,own_stream", [(0, False), (2, False), (2, True)])
def test_batch_graph_replays_equal_eager_launches(ctx, group, own_stream):
    """The batch driver replays each group's filter from a HIP graph every
    Lanczos step (with the step's eager orthogonalisation and host
    synchronisation between replays); the results must equal, bit for bit,
    those of the same launches issued eagerly. Checked on the null stream and
    on a stream of its own, with one group of three slices and with groups of
    two and one (a one-slice group replays the single-vector filter graph)."""
    A = I.laplacian(24, 2, pot_seed=1)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    cuts = [1.0, 1.3, 1.6, 1.9]
    ivs = [[cuts[q], cuts[q + 1], lo, hi] for q in range(3)]
    pols = [_pol(iv) for iv in ivs]
    opts = [ev.lan_opts(tol=1e-10, seed=2 + q, nev_est=40) for q in range(3)]
    stream = torch.cuda.Stream() if own_stream else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        c = ev.Ctx(stream) if own_stream else ctx
        Ad = ev.DeviceCsr.from_host(A)
        stream.synchronize()
        c.set_group_width(group)
        res = {}
        for on in (False, True, True):
            c.set_graphs(on)
            outs = ev.evsl_filtered_lanczos_batch(c, Ad, ivs, pols, opts)
            res.setdefault(on, []).append(
                [(lam, r, Y.cpu().numpy(), st["niter"]) for lam, Y, r, st in outs])
        c.set_graphs(True)
        c.set_group_width(0)
        if own_stream:
            c.close()
    eager = res[False][0]
    for run in res[True]:
        for (l0, r0, y0, n0), (l1, r1, y1, n1) in zip(eager, run):
            assert n0 == n1
            assert np.array_equal(l0, l1) and np.array_equal(r0, r1) and np.array_equal(y0, y1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_slice_graph_replays_equal_eager_launches(ctx, prec):
    """The single-slice solver stages each Lanczos vector in a fixed buffer
    and replays the captured degree-step launches; every replay (two solves,
    hundreds of replays each, with the orthogonalisation and host
    synchronisation in between) must give, bit for bit, what the same
    launches give issued one by one."""
    A = I.laplacian(30, 2, pot_seed=2)
    lo, hi = oracle.lanczos_bounds(A, 80, 3)
    iv = [1.0, 1.4, lo, hi]
    pol = _pol(iv)
    p = ev.EVSL_F32 if prec == "f32" else ev.EVSL_F64
    opts = ev.lan_opts(tol=1e-9 if prec == "f64" else 1e-8, seed=5, nev_est=60, prec=p)
    Ad = ev.DeviceCsr.from_host(A)
    res = {}
    for on in (False, True, True):
        ctx.set_graphs(on)
        lam, Y, r, st = ev.evsl_filtered_lanczos(ctx, Ad, iv, pol, opts)
        res.setdefault(on, []).append((lam, r, Y.cpu().numpy(), st["niter"]))
    ctx.set_graphs(True)
    l0, r0, y0, n0 = res[False][0]
    assert len(l0) > 20
    for l1, r1, y1, n1 in res[True]:
        assert n0 == n1
        assert np.array_equal(l0, l1) and np.array_equal(r0, r1) and np.array_equal(y0, y1)


def test_autotune_picks_a_width_and_batches_still_agree(ctx):
    A = I.laplacian(30, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    g, us = ev.evsl_autotune(ctx, Ad, 6)
    assert 1 <= g <= 6 and us > 0
    ctx.set_group_width(0)


def test_invalid_arguments_are_rejected(ctx):
    A = I.laplacian(10, 2)
    Ad = ev.DeviceCsr.from_host(A)
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_kpm_dos(ctx, Ad, [1.0, 2.0, 3.0, 3.0], 10, 2)
    assert e.value.code == ev.EVSL_EINVAL
    p = _pol([1.0, 1.5, 0.0, 8.0])
    with pytest.raises(ev.EvslError):
        ev.evsl_filtered_lanczos(ctx, Ad, [1.0, 1.5, 0.0, 9.0], p)   # filter built for other bounds


# ------------------------------------------------------------------ FP64 MFMA Gram product
@pytest.mark.parametrize("n,p,q", [(64, 16, 16), (10007, 5, 7), (5000, 33, 17), (131072, 100, 100),
                                   (3, 1, 1)])
def test_gram_mfma_matches_numpy(ctx, n, p, q):
    rng = np.random.default_rng(n + p)
    Xh = rng.standard_normal((p, n))          # row j = column j of the column-major X
    Yh = rng.standard_normal((q, n))
    X, Y = _dev(Xh).T, _dev(Yh).T             # n x p, n x q column-major views
    Ct = torch.empty((q, p), dtype=torch.float64, device="cuda")
    ev.evsl_gram(ctx, X, Y, Ct.T)
    torch.cuda.synchronize()
    ref = Xh @ Yh.T
    assert np.abs(Ct.T.cpu().numpy() - ref).max() <= 1e-12 * np.sqrt(n) * 4


# ------------------------------------------------------------------ precision form
def test_filter_fp32_error_against_fp64_oracle(ctx):
    A = I.laplacian(30, 3, pot_seed=0)
    p = _pol([0.6, 0.7, 0.0, 13.0])
    A32 = ev.DeviceCsr.from_host(A, dtype=torch.float32)
    v = I.lanczos_start(4, A.n)
    V = _dev(v).float()
    Y = torch.empty_like(V)
    ev.evsl_filter_apply(ctx, A32, [p], [0], V, Y)
    torch.cuda.synchronize()
    ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, v)
    err = np.linalg.norm(Y.double().cpu().numpy() - ref) / np.linalg.norm(v)
    # FP32 recurrence: rounding error of order k * eps32 relative to ||V||
    assert err <= p.deg * 6e-8, (err, p.deg)


@pytest.mark.parametrize("ncols,ld", [(2, 2), (3, 4), (4, 4), (6, 6), (8, 8), (12, 16)])
def test_filter_fp32_block_error_against_fp64_oracle(ctx, ncols, ld):
    """Row-major FP32 blocks at every lane width (1, 2 or 4 columns per lane)."""
    A = I.laplacian(30, 3, pot_seed=0)
    A32 = ev.DeviceCsr.from_host(A, dtype=torch.float32)
    pols = [_pol([0.6, 0.7, 0.0, 13.0]), _pol([1.0, 1.2, 0.0, 13.0])]
    groups = [0] * (ncols // 2) + [1] * (ncols - ncols // 2)
    rng = np.random.default_rng(ncols)
    Vh = np.zeros((A.n, ld))
    Vh[:, :ncols] = rng.standard_normal((A.n, ncols))
    V = _dev(Vh).float()
    Y = torch.zeros_like(V)
    ev.evsl_filter_apply(ctx, A32, pols, groups, V[:, :ncols], Y[:, :ncols])
    torch.cuda.synchronize()
    Yh = Y.double().cpu().numpy()
    for c in range(ncols):
        p = pols[groups[c]]
        ref = oracle.filter_apply(A, p.cc, p.dd, p.coef, Vh[:, c])
        err = np.linalg.norm(Yh[:, c] - ref) / np.linalg.norm(Vh[:, c])
        assert err <= p.deg * 6e-8, (c, err, p.deg)


@pytest.mark.parametrize("intv_ab", [(1.0, 1.15), (2.0, 2.05)])
def test_fp32_filter_lanczos_fp64_phase_reaches_fp64_tolerance(ctx, intv_ab):
    """16^3 Laplacian + potential: FP32 filter phase, then the FP64 phase;
    every eigenvalue in the slice (dense eigh) at residual <= 1e-8."""
    A = I.laplacian(16, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    a, b = intv_ab
    intv = [a, b, lo, hi]
    want = w[(w >= a) & (w <= b)]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, _pol(intv), ev.lan_opts(tol=1e-8, seed=2, nev_est=len(want) + 5,
                                               prec=ev.EVSL_F32))
    assert st["status"] == 0 and len(lam) == len(want), st
    assert res.max() <= 1e-8
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
    # the FP32 phase's block, refined by Rayleigh-Ritz and FP64 filter
    # applications, meets tol without the thick-restart continuation
    assert 1 <= st["npolish"] < 100, st


def test_fp32_phase_stopped_short_still_runs_the_stopping_rule(ctx):
    """16^3 Laplacian + potential, [1.0, 1.15]: max_its = 60 stops the FP32
    phase before its stopping rule (EVSL_ENOCONV with candidates left). The
    polish alone may not end such a slice: the FP64 continuation runs the
    stopping rule from the polished pairs, and every eigenvalue of the slice
    (dense eigh) is returned at tol with status EVSL_OK."""
    A = I.laplacian(16, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.15, lo, hi]
    want = w[(w >= 1.0) & (w <= 1.15)]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, _pol(intv), ev.lan_opts(tol=1e-8, seed=2, nev_est=len(want) + 5,
                                               max_its=60, prec=ev.EVSL_F32))
    assert st["status"] == 0 and len(lam) == len(want), st
    assert st["npolish"] >= 100, st
    assert res.max() <= 1e-8
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))


def test_fp32_filter_locked_at_tol_skips_the_fp64_phase(ctx):
    """When the FP32 phase locks at the requested tolerance (tol_lo = tol =
    1e-6, above the FP32 filter's floor) every pair already meets it in FP64:
    no FP64 phase runs, and the eigenvalues match the FP64 form's."""
    A = I.laplacian(16, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    w = np.linalg.eigvalsh(A.to_dense())
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.15, lo, hi]
    want = w[(w >= 1.0) & (w <= 1.15)]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, _pol(intv), ev.lan_opts(tol=1e-6, tol_lo=1e-6, seed=2,
                                               nev_est=len(want) + 5, prec=ev.EVSL_F32))
    assert st["status"] == 0 and len(lam) == len(want), st
    assert st["npolish"] == 0
    assert res.max() <= 1e-6
    # eigenvalue error of a residual-r pair is about r^2 / gap
    assert np.abs(lam - want).max() <= 1e-8 * max(abs(lo), abs(hi))


def test_fp32_filter_lanczos_40x40_eigenvalues(ctx):
    """40 x 40 Laplacian, [1.0, 1.6]: the FP32-filter form with its FP64
    phase finds all 91 eigenvalues (44 double pairs) at residual <= 1e-8."""
    A = I.laplacian(40, 2)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.6, lo, hi]
    lam, Y, res, st = ev.evsl_filtered_lanczos(
        ctx, Ad, intv, _pol(intv), ev.lan_opts(tol=1e-8, seed=2, nev_est=91, prec=ev.EVSL_F32))
    want = _closed_form_interval(40, 2, 1.0, 1.6)
    assert st["status"] == ev.EVSL_OK and st["nev"] == 91, st
    assert res.max() <= 1e-8
    assert_eigs_match(lam, want, max(abs(lo), abs(hi)))
    # the degree-20 filter leaves about a third of the pairs above tol after
    # the polish; the FP64 continuation then starts from a sum of nearly
    # converged vectors, where a single Gram-Schmidt pass loses orthogonality
    # geometrically unless the gate forces the second one
    assert st["npolish"] >= 100, st
    Yh = Y.cpu().numpy() if hasattr(Y, "cpu") else np.asarray(Y)
    G = Yh.T @ Yh
    assert np.abs(G - np.eye(91)).max() <= 1e-10


def test_fp32_batch_matches_fp64_batch(ctx):
    A = I.laplacian(20, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.3, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, 60, 10, seed=1)
    sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, 3, 2000)
    ivs = [[sli[q], sli[q + 1], lo, hi] for q in range(3)]
    pols = [_pol(iv) for iv in ivs]
    res64 = ev.evsl_filtered_lanczos_batch(
        ctx, Ad, ivs, pols, [ev.lan_opts(tol=1e-10, seed=2 + q, nev_est=int(est / 3) + 10)
                             for q in range(3)])
    res32 = ev.evsl_filtered_lanczos_batch(
        ctx, Ad, ivs, pols, [ev.lan_opts(tol=1e-8, seed=2 + q, nev_est=int(est / 3) + 10,
                                         prec=ev.EVSL_F32) for q in range(3)])
    w = np.linalg.eigvalsh(A.to_dense())
    for q in range(3):
        l64, _, r64, _ = res64[q]
        l32, _, r32, s32 = res32[q]
        want = w[(w >= ivs[q][0]) & (w <= ivs[q][1])]
        assert len(l64) == len(l32) == len(want)
        assert r32.max() <= 1e-8 and s32["status"] == 0, s32
        assert_eigs_match(l32, l64, max(abs(lo), abs(hi)))
        assert_eigs_match(l32, want, max(abs(lo), abs(hi)))


def test_bounds_below_the_spectrum_are_detected(ctx):
    """lambda_max = 11.65 for the 12^3 Laplacian; with b = 10.5 the filter grows
    without bound above b, and every solver reports EVSL_ESPECTRUM."""
    A = I.laplacian(12, 3)
    Ad = ev.DeviceCsr.from_host(A)
    intv = [1.0, 1.5, 0.0, 10.5]
    p = _pol(intv)
    for call in (lambda: ev.evsl_filtered_lanczos(ctx, Ad, intv, p, ev.lan_opts(nev_est=40)),
                 lambda: ev.evsl_filtered_lanczos(ctx, Ad, intv, p,
                                                  ev.lan_opts(nev_est=40, method=ev.EVSL_LAN_NR)),
                 lambda: ev.evsl_filtered_subspace(ctx, Ad, intv, p, ev.si_opts(nev_est=40))):
        with pytest.raises(ev.EvslError) as e:
            call()
        assert e.value.code == ev.EVSL_ESPECTRUM


@pytest.mark.parametrize("N,dim,pot", [(40, 2, None), (16, 3, 0)])
def test_lanczos_dos_matches_oracle(ctx, N, dim, pot):
    """Quadrature nodes, weights and counts of the device Lanczos DOS against
    the oracle's on the same probes; nodes to 1e-10 ||A||, counts to 1e-8 n."""
    A = I.laplacian(N, dim, pot_seed=pot)
    Ad = ev.DeviceCsr.from_host(A)
    m, nvec = 40, 6
    q = ev.evsl_lanczos_dos(ctx, Ad, m, nvec, seed=3)
    oq = oracle.lanczos_dos(A, m, nvec, seed=3)
    assert np.array_equal(q[2], oq[2])
    normA = np.abs(oq[0]).max()
    assert np.abs(q[0] - oq[0]).max() <= 1e-10 * normA
    assert np.abs(q[1].sum(axis=1) - 1.0).max() <= 1e-13
    for x0, x1 in ((1.0, 1.6), (0.5, 3.0), (4.0, 20.0)):
        for sigma in (0.0, 0.05):
            a = ev.evsl_lanczos_count(q, A.n, sigma, x0, x1)
            b = oracle.lanczos_count(oq, A.n, sigma, x0, x1)
            assert abs(a - b) <= 1e-8 * A.n, (x0, x1, sigma, a, b)


def test_precision_form_headline_slices_equal_the_oracle(ctx):
    """The precision form (FP32 filter, FP64 reorthogonalisation, Rayleigh-Ritz,
    polish and residuals) on slices 0 and 9 of the 100^3 workload's cut, solved
    together in one batch, against the oracle's FP64 run of them
    (tests/golden/c2_oracle.json): the same eigenvalue lists (same count, each
    within 1e-10 relative), residuals <= 1e-8, status EVSL_OK, and the FP64
    phase ended in the polish (no thick-restart continuation)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")))
    A = I.laplacian(100, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    normA = max(abs(lo), abs(hi))
    qs = sorted(int(q) for q in gold["solved"])
    ivs = [[gold["solved"][str(q)]["interval"][0], gold["solved"][str(q)]["interval"][1], lo, hi]
           for q in qs]
    pols = [_pol(iv) for iv in ivs]
    opts = [ev.lan_opts(tol=1e-8, seed=2 + q, nev_est=gold["solved"][str(q)]["nev_est"],
                        prec=ev.EVSL_F32) for q in qs]
    ev.evsl_autotune(ctx, Ad, len(qs), ev.EVSL_F32)
    outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
    ctx.set_group_width(0)
    for q, iv, (lam, Y, res, st) in zip(qs, ivs, outs):
        want = np.array(gold["solved"][str(q)]["eigenvalues"])
        keep = (lam >= iv[0]) & ((lam < iv[1]) | (q == 9))
        assert st["status"] == ev.EVSL_OK, st
        assert 1 <= st["npolish"] < 100, st
        assert keep.sum() == len(want), (q, int(keep.sum()), len(want))
        assert_eigs_match(lam[keep], want, normA)
        assert res.max() <= 1e-8


def test_headline_workload_slices_equal_the_oracle(ctx):
    """The 100^3 workload (3-D 7-point Laplacian + U[0,1) potential, KPM cut of
    [0.60, 0.70] into 10 slices, degree 80 x 20 probes) against the oracle's
    own run of it (tests/golden/c2_oracle.json, written by
    tests/golden/make_c2_golden.py from oracle/ alone): the device spectrum
    bounds, KPM moments and slice ends agree with the oracle's, and slices 0
    and 9 (the lowest and highest filter degree), solved together in one batch
    with the autotuned group width, return exactly the oracle's eigenvalue
    lists (same count, each within 1e-10 relative), residuals <= 1e-8 and
    orthonormal vectors; sampled pairs are re-checked with the oracle's FP64
    product on the host."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")))
    A = I.laplacian(100, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    normA = max(abs(lo), abs(hi))
    assert abs(lo - gold["bounds"][0]) <= 1e-8 * normA
    assert abs(hi - gold["bounds"][1]) <= 1e-8 * normA
    intv = [0.60, 0.70, lo, hi]
    mom, est = ev.evsl_kpm_dos(ctx, Ad, intv, 80, 20, seed=1, damping=ev.DAMP_JACKSON)
    omom = np.array(gold["kpm_moments"])
    assert np.abs(mom - omom).max() <= 1e-10 * A.n
    sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, intv, 10, 2000)
    grid_step = 0.1 / 1999
    assert np.abs(sli - np.array(gold["slices"])).max() <= grid_step * 1.0001
    qs = sorted(int(q) for q in gold["solved"])
    assert qs == [0, 9]
    ivs = [[gold["solved"][str(q)]["interval"][0], gold["solved"][str(q)]["interval"][1], lo, hi]
           for q in qs]
    pols = [_pol(iv) for iv in ivs]
    assert [p.deg for p in pols] == [gold["solved"][str(q)]["degree"] for q in qs]
    opts = [ev.lan_opts(tol=1e-8, seed=2 + q, nev_est=gold["solved"][str(q)]["nev_est"])
            for q in qs]
    ev.evsl_autotune(ctx, Ad, 10)
    outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
    ctx.set_group_width(0)
    for q, iv, (lam, Y, res, st) in zip(qs, ivs, outs):
        want = np.array(gold["solved"][str(q)]["eigenvalues"])
        keep = (lam >= iv[0]) & ((lam < iv[1]) | (q == 9))
        assert st["status"] == ev.EVSL_OK
        assert keep.sum() == len(want), (q, int(keep.sum()), len(want))
        assert_eigs_match(lam[keep], want, normA)
        assert res.max() <= 1e-8
        Yc = Y.contiguous()
        G = (Yc.T.contiguous() @ Yc).cpu().numpy()
        assert np.abs(G - np.eye(len(lam))).max() <= 1e-10
        for j in np.linspace(0, len(lam) - 1, 4).astype(int):
            y = Y[:, j].cpu().numpy()
            r = np.linalg.norm(oracle.spmv(A, y) - lam[j] * y) / np.linalg.norm(y) / normA
            assert r <= 1e-8, (q, j, r)


def test_failed_device_allocation_reports_enomem_and_context_survives(ctx):
    """A basis larger than the device (the lock capacity clamps to n, so about
    n x n doubles: 328 GB for n = 202,500) makes the allocation fail: the solve
    returns EVSL_ENOMEM, the context's memory ledger returns to where it was,
    and the next solve on it succeeds."""
    A = I.laplacian(450, 2, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    intv = [1.0, 1.01, lo, hi]
    p = _pol(intv)
    cur0, _ = ctx.mem_stats()
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos(ctx, Ad, intv, p, ev.lan_opts(nev_cap=10_000_000, nev_est=20))
    assert e.value.code == ev.EVSL_ENOMEM
    assert ctx.mem_stats()[0] == cur0
    S = I.laplacian(24, 2, pot_seed=0)
    Sd = ev.DeviceCsr.from_host(S)
    lo, hi = ev.evsl_spectrum_bounds(ctx, Sd, 80, 3)
    iv = [1.0, 1.5, lo, hi]
    w = np.linalg.eigvalsh(S.to_dense())
    lam, Y, res, st = ev.evsl_filtered_lanczos(ctx, Sd, iv, _pol(iv), ev.lan_opts(nev_est=40))
    assert st["status"] == ev.EVSL_OK and res.max() <= 1e-8
    assert len(lam) == int(((w >= 1.0) & (w <= 1.5)).sum())


def test_caller_allocator_serves_every_buffer_and_its_refusal_is_enomem():
    """evsl_create with a caller allocator (torch's caching allocator here):
    every device buffer of the context comes from it, the context's ledger
    equals what the allocator has handed out, results are bit for bit those of
    a default context, an allocator that refuses makes the solve return
    EVSL_ENOMEM and leaves the context usable, and destroying the context
    returns every buffer."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ev.load()
    live = {}
    state = {"limit": None, "refused": 0}
    dev = torch.cuda.current_device()

    def alloc(nbytes, stream):
        if state["limit"] is not None and sum(live.values()) + nbytes > state["limit"]:
            state["refused"] += 1
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, device=dev, stream=stream or 0)
        live[p] = nbytes
        return p

    def free(ptr, stream):
        live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    al = ev.make_allocator(alloc, free)
    c = ev.Ctx(alloc=al)
    ref = ev.Ctx()
    S = I.laplacian(24, 2, pot_seed=0)
    Sd = ev.DeviceCsr.from_host(S)
    outs = []
    for cx in (c, ref):
        lo, hi = ev.evsl_spectrum_bounds(cx, Sd, 80, 3)
        iv = [1.0, 1.5, lo, hi]
        outs.append(ev.evsl_filtered_lanczos(cx, Sd, iv, _pol(iv), ev.lan_opts(nev_est=40)))
    assert len(live) > 0 and c.mem_stats()[0] == sum(live.values())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][2], outs[1][2])
    # a larger solve under a budget the allocator enforces
    A = I.laplacian(160, 2)
    Ad = ev.DeviceCsr.from_host(A)
    lo, hi = ev.evsl_spectrum_bounds(c, Ad, 80, 3)
    iv = [1.0, 1.05, lo, hi]
    state["limit"] = sum(live.values()) + (1 << 20)
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filtered_lanczos(c, Ad, iv, _pol(iv), ev.lan_opts(nev_est=60))
    assert e.value.code == ev.EVSL_ENOMEM and state["refused"] >= 1
    assert c.mem_stats()[0] == sum(live.values())
    state["limit"] = None
    lam, Y, res, st = ev.evsl_filtered_lanczos(c, Ad, iv, _pol(iv), ev.lan_opts(nev_est=60))
    del Y
    assert st["status"] == ev.EVSL_OK and res.max() <= 1e-8
    assert_eigs_match(lam, _closed_form_interval(160, 2, 1.0, 1.05), max(abs(lo), abs(hi)))
    c.close()
    ref.close()
    assert live == {}
