"""GPU FNO against the FP64 FNO oracle: forward output and every parameter
gradient, for the FP32 kernels (relative L2 <= 1e-5 forward, <= 1e-4 per
gradient group) and the BF16 matrix-core kernels (<= 2e-2 forward,
<= 5e-2 per gradient group: BF16 operands carry ~4e-3 relative rounding).
Inputs are the float32-rounded copies the GPU receives."""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

pytestmark = pytest.mark.gpu

CFG = dict(n=16, width=8, modes=3, layers=2, hidden=16)
B = 2


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def P():
    from paper_1808_01309_amd import pst
    return pst


@pytest.fixture(scope="module")
def case():
    import oracle.fno as F
    theta = I.fno_init_params(seed=3, out_scale=0.5, **CFG).astype(np.float32).astype(np.float64)
    n = CFG["n"]
    rng = np.random.default_rng(4)
    u = rng.standard_normal((B, 3, n, n, n)).astype(np.float32).astype(np.float64)
    tgt = (u + 0.2 * rng.standard_normal(u.shape)).astype(np.float32).astype(np.float64)
    out = F.forward(theta, u, CFG)
    L, g = F.loss_and_grad(theta, u, tgt, CFG)
    return theta, u, tgt, out, L, g


def groups():
    import oracle.fno as F
    off = 0
    for name, shape in F.param_shapes(CFG["width"], CFG["modes"], CFG["layers"], CFG["hidden"], CFG["n"]):
        size = int(np.prod(shape))
        yield name, off, size
        off += size


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("mfma,tf,tg", [(False, 1e-5, 1e-4), (True, 2e-2, 5e-2)])
def test_forward_and_gradients(P, torch, case, mfma, tf, tg):
    theta, u, tgt, out_ref, L_ref, g_ref = case
    fno = P.FNO(batch=B, mfma=mfma, **CFG)
    fno.set_params(theta)
    assert np.array_equal(fno.get_params(), theta.astype(np.float32))
    ud = torch.from_numpy(u).float().cuda()
    td = torch.from_numpy(tgt).float().cuda()
    od = torch.empty_like(ud)
    fno.forward(ud, od)
    torch.cuda.synchronize()
    y_ref = out_ref - u
    y = od.cpu().numpy() - u
    for b in range(B):
        assert rel(y[b], y_ref[b]) < tf, b
    L = fno.loss_grad(ud, td)
    assert abs(L - L_ref) < tf * L_ref
    g = fno.get_grad().astype(np.float64)
    for name, off, size in groups():
        assert rel(g[off:off + size], g_ref[off:off + size]) < tg, name


@pytest.mark.parametrize("mfma", [False, True])
def test_adam_reduces_loss(P, torch, case, mfma):
    theta, u, tgt, *_ = case
    fno = P.FNO(batch=B, mfma=mfma, **CFG)
    fno.set_params(theta)
    ud = torch.from_numpy(u).float().cuda()
    td = torch.from_numpy(tgt).float().cuda()
    losses = [fno.train_step(ud, td, 1e-3) for _ in range(8)]
    assert losses[-1] < 0.9 * losses[0] and all(np.diff(losses) < 0.02 * losses[0])


def test_adam_matches_formula(P, torch, case):
    """One Adam step from zero moments moves every parameter by lr * g / (|g| + eps')."""
    theta, u, tgt, *_ = case
    fno = P.FNO(batch=B, mfma=False, **CFG)
    fno.set_params(theta)
    ud = torch.from_numpy(u).float().cuda()
    td = torch.from_numpy(tgt).float().cuda()
    fno.loss_grad(ud, td)
    g = fno.get_grad().astype(np.float64)
    fno.adam(1e-3)
    th1 = fno.get_params().astype(np.float64)
    ref = theta - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.abs(th1 - ref).max() < 1e-6
