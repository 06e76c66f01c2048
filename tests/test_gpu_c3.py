"""The batched 200^3 workload against the oracle's run of two of its slices
(tests/golden/c3_oracle.json, written by tests/golden/make_c3_golden.py from
oracle/ alone): 3-D 7-point Laplacian 200^3 + U[0,1) potential (seed 0),
[lambda_min, eta_512] with eta_512 where the KPM count (degree 80, 20 probes)
reaches 512, cut into 32 slices; slice 0 is the boundary slice (its filter
has its centre at the spectrum's lower end), slice 1 the interior slice of
lowest degree."""
import json
import os

import numpy as np
import pytest

import evsl_inputs as I
import paper_1802_05215_amd as ev
from tests.eig_rules import assert_eigs_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c3_oracle.json")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ev.load()
    c = ev.Ctx()
    yield c
    c.close()


def test_c3_cut_and_two_slices_equal_the_oracle(ctx):
    gold = json.load(open(GOLD))
    A = I.laplacian(200, 3, pot_seed=0)
    Ad = ev.DeviceCsr.from_host(A)
    del A
    lo, hi = ev.evsl_spectrum_bounds(ctx, Ad, 80, 3)
    normA = max(abs(lo), abs(hi))
    assert abs(lo - gold["bounds"][0]) <= 1e-8 * normA
    assert abs(hi - gold["bounds"][1]) <= 1e-8 * normA
    mom, _ = ev.evsl_kpm_dos(ctx, Ad, [lo, hi, lo, hi], 2000, 20, seed=1,
                             damping=ev.DAMP_JACKSON)
    assert np.abs(mom - np.array(gold["kpm_moments"])).max() <= 1e-10 * Ad.n
    a, b = lo, hi
    for _ in range(60):
        mid = 0.5 * (a + b)
        if ev.evsl_kpm_count(mom, ev.DAMP_JACKSON, lo, hi, lo, mid) < 512:
            a = mid
        else:
            b = mid
    eta = 0.5 * (a + b)
    assert abs(eta - gold["eta"]) <= 1e-8
    sli = ev.evsl_slice_spectrum(mom, ev.DAMP_JACKSON, [lo, eta, lo, hi], 32, 2000)
    assert np.abs(sli - np.array(gold["slices"])).max() <= (eta - lo) / 1999 * 1.0001
    qs = sorted(int(q) for q in gold["solved"])
    assert qs == [0, 1]
    # the oracle's slice ends; the boundary slice starts at the device's own
    # lower bound (the two Lanczos bounds differ in the last digits), as a
    # slice starting at the spectrum's lower bound does in the cut
    ivs = [list(gold["solved"][str(q)]["interval"]) + [lo, hi] for q in qs]
    ivs[0][0] = lo
    pols = [ev.evsl_cheb_coeffs(iv, damping=ev.DAMP_JACKSON, tau=0.8, tau_ext=0.4) for iv in ivs]
    assert pols[0].boundary == -1
    assert [p.deg for p in pols] == [gold["solved"][str(q)]["degree"] for q in qs]
    opts = [ev.lan_opts(tol=1e-8, seed=2 + q, nev_est=gold["solved"][str(q)]["nev_est"])
            for q in qs]
    outs = ev.evsl_filtered_lanczos_batch(ctx, Ad, ivs, pols, opts)
    for q, iv, (lam, Y, res, st) in zip(qs, ivs, outs):
        want = np.array(gold["solved"][str(q)]["eigenvalues"])
        keep = ((lam >= iv[0]) | (q == 0)) & (lam < iv[1])
        assert st["status"] == ev.EVSL_OK
        assert keep.sum() == len(want), (q, int(keep.sum()), len(want))
        assert_eigs_match(lam[keep], want, normA)
        assert res.max() <= 1e-8
        Yc = Y.contiguous()
        G = (Yc.T.contiguous() @ Yc).cpu().numpy()
        assert np.abs(G - np.eye(len(lam))).max() <= 1e-10
