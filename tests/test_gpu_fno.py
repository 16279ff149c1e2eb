"""GPU FNO against the FP64 FNO oracle: forward output and every parameter
gradient, for the FP32 kernels (relative L2 <= 1e-5, forward and per gradient
group) and the BF16 matrix-core kernels (<= 2e-2: BF16 operands carry ~4e-3
relative rounding).  Inputs are the float32-rounded copies the GPU receives."""
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


# FP32 <= 1e-5 and BF16 <= 2e-2 for the forward pass and every gradient group
# (measured: FP32 <= 5e-7, BF16 forward 4.6e-3, gradients <= 9e-3)
@pytest.mark.parametrize("mfma,tf,tg", [(False, 1e-5, 1e-5), (True, 2e-2, 2e-2)])
def test_forward_and_gradients(P, torch, case, mfma, tf, tg, errlog):
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
    prec = "BF16" if mfma else "FP32"
    errlog(f"FNO forward {prec} (per batch entry)", [rel(y[b], y_ref[b]) for b in range(B)], tf)
    L = fno.loss_grad(ud, td)
    assert abs(L - L_ref) < tf * L_ref
    g = fno.get_grad().astype(np.float64)
    names, errs = [], []
    for name, off, size in groups():
        names.append(name)
        errs.append(rel(g[off:off + size], g_ref[off:off + size]))
    errlog(f"FNO gradients {prec} ({' '.join(names)})", errs, tg)


@pytest.mark.parametrize("mfma", [False, True])
def test_adam_reduces_loss(P, torch, case, mfma):
    theta, u, tgt, *_ = case
    fno = P.FNO(batch=B, mfma=mfma, **CFG)
    fno.set_params(theta)
    ud = torch.from_numpy(u).float().cuda()
    td = torch.from_numpy(tgt).float().cuda()
    losses = [fno.train_step(ud, td, 1e-3) for _ in range(8)]
    assert losses[-1] < 0.9 * losses[0] and all(np.diff(losses) < 0.02 * losses[0])


# Shapes that exercise the inference kernels' edge cases: an odd radix (24),
# odd channel counts (an unpaired last line), more than 32 channels or hidden
# units (several matrix tiles, masked rows), one row per block (96, 128), a
# single layer (lift straight into the projection), and n = 64: the
# benchmark's width and modes, and 20 channels with 16 modes.
SHAPES = [
    dict(n=24, width=5, modes=4, layers=2, hidden=40),
    dict(n=48, width=36, modes=5, layers=1, hidden=16),
    dict(n=96, width=3, modes=6, layers=2, hidden=8),
    dict(n=128, width=2, modes=4, layers=1, hidden=8),
    dict(n=64, width=32, modes=12, layers=2, hidden=16),
    dict(n=64, width=20, modes=16, layers=1, hidden=8),
]


_shape_cache = {}


def shape_case(i):
    if i not in _shape_cache:
        import oracle.fno as F
        cfg = SHAPES[i]
        theta = I.fno_init_params(seed=11, out_scale=0.5, **cfg).astype(np.float32).astype(np.float64)
        n, nb = cfg["n"], 2 if cfg["n"] <= 48 else 1
        rng = np.random.default_rng(12)
        u = rng.standard_normal((nb, 3, n, n, n)).astype(np.float32).astype(np.float64)
        _shape_cache[i] = (theta, u, F.forward(theta, u, cfg) - u)
    return _shape_cache[i]


@pytest.mark.parametrize("mfma,tf", [(False, 1e-5), (True, 2e-2)])
@pytest.mark.parametrize("i", range(len(SHAPES)),
                         ids=[f"n{c['n']}w{c['width']}l{c['layers']}h{c['hidden']}" for c in SHAPES])
def test_forward_shapes(P, torch, i, mfma, tf):
    cfg = SHAPES[i]
    theta, u, y_ref = shape_case(i)
    nb = u.shape[0]
    fno = P.FNO(batch=nb, mfma=mfma, **cfg)
    fno.set_params(theta)
    ud = torch.from_numpy(u).float().cuda()
    od = torch.empty_like(ud)
    fno.forward(ud, od)
    y = od.cpu().numpy() - u
    for b in range(nb):
        assert rel(y[b], y_ref[b]) < tf, b
    # in place (out aliases u) gives the same result
    fno.forward(ud, ud)
    assert np.array_equal(ud.cpu().numpy(), od.cpu().numpy())


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


@pytest.mark.parametrize("bad", [
    dict(n=16, width=8, modes=9, layers=2, hidden=16, batch=2),     # 2 m > n
    dict(n=40, width=8, modes=3, layers=2, hidden=16, batch=2),     # unsupported n
    dict(n=64, width=64, modes=12, layers=1, hidden=8, batch=64),   # mixing LDS bound
    dict(n=16, width=8, modes=3, layers=9, hidden=16, batch=2),     # too many layers
])
def test_invalid_configs(P, torch, bad):
    with pytest.raises(P.PstError):
        P.FNO(**bad)
