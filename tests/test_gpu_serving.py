"""Serving on the device: a small request stream served concurrently (one
stream and library context per request) gives, for every request, the same
bits as the request served alone; eigenvalues agree with a dense solve; the
library's measured device high-water mark stays under the admission
footprint."""
import numpy as np
import pytest

from tests.eig_rules import assert_eigs_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def torch_cuda():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1802_05215_amd as ev
    ev.load()


def _stream():
    from paper_1802_05215_amd import serving as S
    reqs = S.poisson_stream(11, 6, 0.0, n_min=1500, n_max=4000, eig_range=(40, 130))
    return S, reqs


def test_mix_equals_solo_and_dense(torch_cuda):
    import evsl_inputs as I
    S, reqs = _stream()
    assert {r.kind for r in reqs} == {"dos", "eigs"}
    ex = S.DeviceExecutor(tol=1e-8)
    led = S.Ledger(40 * 2 ** 30, max_running=3)
    mix = S.Server(led, ex).run(reqs)
    assert led.high_water <= led.budget and led.used == 0
    for r, m in zip(reqs, mix):
        print(f"request {r.rid}: {r.kind} dim={r.dim} N={r.N} target={r.target}", flush=True)
        assert m.status == "ok", m.error
        one = S.Ledger(40 * 2 ** 30, 1)
        solo = S.Server(one, ex).run([S.Request(**{**r.__dict__, "arrival": 0.0})])[0]
        assert solo.status == "ok", solo.error
        assert np.array_equal(solo.moments, m.moments)
        fp = S.footprint_parts(r)
        assert 0 < m.lib_peak <= fp["library"], (m.lib_peak, fp)
        if r.kind == "dos":
            continue
        assert np.array_equal(solo.lam, m.lam)
        assert np.array_equal(solo.res, m.res)
        assert np.array_equal(solo.ycheck, m.ycheck)
        # every eigenvalue of the interval, checked against a dense solve
        A = I.laplacian(r.N, r.dim, pot_seed=r.pot_seed)
        w = np.linalg.eigvalsh(A.to_dense())
        xi, eta = m.interval
        want = w[(w >= xi) & (w <= eta)]
        assert m.nev == len(want), (m.nev, len(want))
        assert_eigs_match(m.lam, want, np.abs(w).max())
        assert m.res.max() <= 1e-8
        # the request got about its target count
        assert abs(m.nev - r.target) <= max(10, 0.25 * r.target)
