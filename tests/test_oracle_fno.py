"""Pins of the FNO oracle: the hand-derived gradient against central finite
differences, the spectral-convolution adjoint against the dot-product
identity, and the identity-weight spectral layer against an explicit numpy
low-pass filter."""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

CFG = dict(n=8, width=4, modes=2, layers=2, hidden=6)


@pytest.fixture(scope="module")
def F():
    import oracle.fno as f
    return f


def setup(F, seed=0, batch=2):
    theta = I.fno_init_params(CFG["n"], CFG["width"], CFG["modes"], CFG["layers"], CFG["hidden"], seed=seed,
                              out_scale=0.5)
    rng = np.random.default_rng(seed + 1)
    n = CFG["n"]
    u = rng.standard_normal((batch, 3, n, n, n))
    tgt = u + 0.3 * rng.standard_normal((batch, 3, n, n, n))
    return theta, u, tgt


def test_param_count_matches_layout(F):
    theta, _, _ = setup(F)
    n, w, m, L, h = CFG["n"], CFG["width"], CFG["modes"], CFG["layers"], CFG["hidden"]
    nm = (2 * m) ** 2 * m
    assert theta.size == w * 3 + w + L * (w * w + w + nm * w * w * 2) + h * w + h + 3 * h + 3
    assert theta.size == I.fno_param_count(n, w, m, L, h)


def test_gradient_finite_differences(F):
    theta, u, tgt = setup(F)
    L0, g = F.loss_and_grad(theta, u, tgt, CFG)
    assert abs(L0 - F.loss(F.forward(theta, u, CFG), tgt)) < 1e-14
    rng = np.random.default_rng(5)
    # coordinates from every parameter group
    offs, off = [], 0
    for name, shape in F.param_shapes(CFG["width"], CFG["modes"], CFG["layers"], CFG["hidden"], CFG["n"]):
        size = int(np.prod(shape))
        offs += list(off + rng.choice(size, size=min(size, 6), replace=False))
        off += size
    h = 1e-6
    for i in offs:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (F.loss(F.forward(tp, u, CFG), tgt) - F.loss(F.forward(tm, u, CFG), tgt)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_spectral_conv_adjoint(F):
    """<K x, y> = <x, K^T y> with K^T y = c2r(conj(R)^T n^3 r2c(y)) / n^3."""
    n, m, c = 8, 3, 3
    rng = np.random.default_rng(2)
    nm = (2 * m) ** 2 * m
    R = rng.standard_normal((nm, c, c)) + 1j * rng.standard_normal((nm, c, c))
    x = rng.standard_normal((1, c, n, n, n))
    y = rng.standard_normal((1, c, n, n, n))
    Kx, _ = F.spectral_conv(x, R, n, m)
    kz, ky, kx = F.mode_index(n, m)
    Gh = n ** 3 * F._r2c_b(y)[:, :, kz, ky, kx]
    gV = np.einsum("mco,bom->bcm", np.conj(R), Gh)
    H = np.zeros((1, c, n, n, n // 2 + 1), complex)
    H[:, :, kz, ky, kx] = gV
    KTy = F._c2r_b(H, n) / n ** 3
    lhs, rhs = np.sum(Kx * y), np.sum(x * KTy)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_identity_weights_are_a_low_pass_filter(F):
    n, m, c = 12, 3, 2
    nm = (2 * m) ** 2 * m
    R = np.zeros((nm, c, c), complex)
    R[:, np.arange(c), np.arange(c)] = 1.0
    rng = np.random.default_rng(3)
    v = rng.standard_normal((1, c, n, n, n))
    got, _ = F.spectral_conv(v, R, n, m)
    kzz = np.fft.fftfreq(n, 1.0 / n)
    keep = (np.abs(kzz) < m) | (kzz == -m)        # index sets [0, m) and [n - m, n)
    mask = keep[:, None, None] & keep[None, :, None] & (np.arange(n // 2 + 1) < m)[None, None, :]
    ref = np.stack([np.fft.irfftn(np.fft.rfftn(v[0, i]) * mask, s=(n, n, n), axes=(0, 1, 2)) for i in range(c)])
    # irfftn keeps the imaginary parts on kx = 0 the c2r drops: compare real parts of a real field
    assert np.abs(got[0] - ref).max() < 1e-13


def test_gelu_and_grad(F):
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    assert np.abs((F.gelu(x + h) - F.gelu(x - h)) / (2 * h) - F.gelu_grad(x)).max() < 1e-8
    assert abs(F.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # 1 * Phi(1)
