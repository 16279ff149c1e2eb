"""The no-allocation variant of the c2r transform (pst_fft_c2r_noalloc),
called through the C ABI, against the plan-based pst_fft_c2r on the same
inputs: two calls in a row, the second with a smaller input (the static
scratch keeps the first call's contents), in both precisions; sizes beyond
the scratch limit are refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1808_01309_amd import pst
    return torch, pst


def _spec(torch, n, nf, seed, prec):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nf, n, n, n // 2 + 1)) + 1j * rng.standard_normal((nf, n, n, n // 2 + 1))
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(x).to(ct).cuda()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_plan_c2r(env, prec):
    torch, P = env
    rt = torch.float64 if prec == "fp64" else torch.float32
    for n, nf, seed in [(64, 3, 1), (32, 1, 2), (96, 2, 3)]:
        x = _spec(torch, n, nf, seed, prec)
        x0 = x.clone()
        plan = P.Plan(n, precision=prec)
        ref = torch.empty((nf, n, n, n), dtype=rt, device="cuda")
        plan.fft_c2r(x, ref, nf)
        got = torch.full((nf, n, n, n), float("nan"), dtype=rt, device="cuda")
        P.fft_c2r_noalloc(n, x, got, nf, precision=prec)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(g).all()
        e = rel(g, r)
        print(f"noalloc c2r n={n} nf={nf} {prec}: rel L2 vs plan {e:.2e}", flush=True)
        assert e < TOL[prec], (n, nf, e)
        assert torch.equal(x, x0)   # the input is not modified
        plan.close()


def test_noalloc_limits(env):
    torch, P = env
    lim = P.lib.pst_fft_c2r_noalloc_bytes
    assert P.fft_c2r_noalloc_bytes(128, 3, "fp64") <= 64 << 20
    assert P.fft_c2r_noalloc_bytes(128, 4, "fp64") > 64 << 20
    assert P.fft_c2r_noalloc_bytes(256, 1, "fp32") > 64 << 20
    assert lim(40, 0, 1) == 0
    x = torch.zeros((1, 256, 256, 129), dtype=torch.complex64, device="cuda")
    y = torch.zeros((1, 256, 256, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PstError, match="limit"):
        P.fft_c2r_noalloc(256, x, y, 1)
    assert P.lib.pst_fft_c2r_noalloc(64, 0, None, None, 1, None) == P.PST_ERR_INVALID_ARG
    assert P.lib.pst_fft_c2r_noalloc(40, 0, x.data_ptr(), y.data_ptr(), 1, None) == P.PST_ERR_UNSUPPORTED_N
