"""The allocation-free filter entry point against evsl_filter_apply, through
the C-ABI: the same bits on two calls in a row (the second smaller, so the
shared scratch holds the first call's values when it starts), a single
vector and an FP32 block, and EVSL_ESCRATCH for a problem larger than the
scratch, with no device memory taken by the calls."""
import numpy as np
import pytest

import evsl_inputs as I
import paper_1802_05215_amd as ev

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


def _case(N, ncols, seed, dtype=torch.float64):
    A = I.laplacian(N, 3, pot_seed=seed)
    Ad = ev.DeviceCsr.from_host(A)
    if dtype == torch.float32:
        Ad = Ad.with_values(Ad.val.float())
    lo, hi = 0.0, 13.0
    pols = [ev.evsl_cheb_coeffs([a, b, lo, hi]) for a, b in [(2.0, 2.3), (1.0, 1.2)]]
    order = sorted(range(2), key=lambda g: -pols[g].deg)
    groups = [order[0] if c < ncols // 2 else order[1] for c in range(ncols)]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    shape = (A.n, ncols) if ncols > 1 else (A.n,)
    V = torch.randn(shape, dtype=torch.float64, device="cuda", generator=g).to(dtype)
    return Ad, pols, groups, V


def _both(ctx, Ad, pols, groups, V):
    Y0 = torch.full_like(V, float("nan"))
    Y1 = torch.full_like(V, float("nan"))
    ev.evsl_filter_apply(ctx, Ad, pols, groups, V, Y0)
    torch.cuda.synchronize()
    cur0, _ = ctx.mem_stats()
    free0 = torch.cuda.mem_get_info()[0]
    ev.evsl_filter_apply_noalloc(ctx, Ad, pols, groups, V, Y1)
    torch.cuda.synchronize()
    assert ctx.mem_stats()[0] == cur0
    assert torch.cuda.mem_get_info()[0] == free0
    return Y0, Y1


def test_noalloc_equals_filter_apply_twice_second_smaller(ctx):
    for N, ncols, seed in ((24, 48, 1), (13, 10, 2)):
        Ad, pols, groups, V = _case(N, ncols, seed)
        Y0, Y1 = _both(ctx, Ad, pols, groups, V)
        assert torch.isfinite(Y0).all()
        assert torch.equal(Y0, Y1), (N, ncols)


def test_noalloc_single_vector_and_fp32_block(ctx):
    Ad, pols, groups, V = _case(20, 1, 3)
    Y0, Y1 = _both(ctx, Ad, pols[:1], [0], V)
    assert torch.equal(Y0, Y1)
    Ad, pols, groups, V = _case(16, 64, 4, dtype=torch.float32)
    Y0, Y1 = _both(ctx, Ad, pols, groups, V)
    assert torch.equal(Y0, Y1)


def test_noalloc_rejects_a_problem_beyond_its_scratch(ctx):
    # two 60^3 x 32 FP64 recurrence blocks are 110.6 MB > 64 MiB
    Ad, pols, groups, V = _case(60, 32, 5)
    assert 2 * V.numel() * 8 > ev.EVSL_NOALLOC_SCRATCH_BYTES
    Y = torch.zeros_like(V)
    with pytest.raises(ev.EvslError) as e:
        ev.evsl_filter_apply_noalloc(ctx, Ad, pols, groups, V, Y)
    assert e.value.code == ev.EVSL_ESCRATCH
    torch.cuda.synchronize()
    assert torch.count_nonzero(Y) == 0
    # the entry point still works after the refusal
    Ad, pols, groups, V = _case(12, 8, 6)
    Y0, Y1 = _both(ctx, Ad, pols, groups, V)
    assert torch.equal(Y0, Y1)
