"""Pins of the oracle's transforms against the DFT definition (eq. fftsum and
its backward counterpart, Sec. 2), brute force on tiny grids, Parseval,
single-mode transforms and a library FFT (numpy) as a third opinion."""
import numpy as np
import pytest

rng = np.random.default_rng(1234)


def dft_matrix(n, sign):
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


@pytest.mark.parametrize("n", list(range(1, 17)) + [18, 24, 27, 48, 5 * 7])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_brute_force(O, n, sign):
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n, sign) @ x
    got = O.fft1d(x, sign)
    tol = 1e-14 * max(1.0, np.log2(n)) * np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= tol
    assert np.linalg.norm(O.dft_naive(x, sign) - ref) <= tol


@pytest.mark.parametrize("n", [64, 96, 512])
def test_fft1d_numpy(O, n):
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.allclose(O.fft1d(x, -1), np.fft.fft(x), rtol=0, atol=1e-12 * np.sqrt(n))
    assert np.allclose(O.fft1d(x, 1), np.fft.ifft(x) * n, rtol=0, atol=1e-12 * np.sqrt(n))


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 8), (6, 6, 6), (2, 3, 4)])
def test_r2c3_brute_force(O, shape):
    nz, ny, nx = shape
    a = rng.standard_normal(shape)
    full = np.einsum("zyx,az,by,cx->abc", a, dft_matrix(nz, -1), dft_matrix(ny, -1),
                     dft_matrix(nx, -1)) / a.size
    got = O.r2c3(a)
    assert got.shape == (nz, ny, nx // 2 + 1)
    assert np.abs(got - full[:, :, : nx // 2 + 1]).max() < 1e-15 * 10 * np.log2(a.size)


@pytest.mark.parametrize("shape", [(4, 6, 8), (6, 6, 6), (8, 8, 8), (12, 12, 12), (24, 24, 24)])
def test_c2r3_round_trip_and_numpy(O, shape):
    a = rng.standard_normal(shape)
    h = O.r2c3(a)
    assert np.abs(h - np.fft.rfftn(a) / a.size).max() < 1e-15 * 10
    b = O.c2r3(h, shape[2])
    assert np.abs(b - a).max() < 1e-13


@pytest.mark.parametrize("n", [8, 12, 32])
def test_parseval(O, n):
    a = rng.standard_normal((n, n, n))
    h = O.r2c3(a)
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    lhs = np.mean(a * a)
    rhs = np.sum(w[None, None, :] * np.abs(h) ** 2)
    assert abs(lhs - rhs) < 1e-14 * lhs


@pytest.mark.parametrize("n", [8, 12, 16])
@pytest.mark.parametrize("k0", [(1, 2, 3), (0, 2, -1), (0, 0, 3), (3, -2, 0)])
def test_single_mode(O, n, k0):
    """u = cos(k0.x + phi) has uhat(k0) = e^{i phi}/2 and its conjugate at -k0."""
    phi = 0.7
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    kx, ky, kz = k0
    u = np.cos(kx * X + ky * Y + kz * Z + phi)
    h = O.r2c3(u)
    exp = np.zeros_like(h)
    exp[kz % n, ky % n, kx] += np.exp(1j * phi) / 2
    if kx == 0:
        exp[(-kz) % n, (-ky) % n, 0] += np.exp(-1j * phi) / 2
    assert np.abs(h - exp).max() < 1e-15 * 4


def test_shift_theorem(O):
    n = 12
    a = rng.standard_normal((n, n, n))
    s = (2, 5, 1)  # shift in (z, y, x)
    b = np.roll(a, s, axis=(0, 1, 2))
    kz = np.fft.fftfreq(n, 1.0 / n)[:, None, None]
    ky = np.fft.fftfreq(n, 1.0 / n)[None, :, None]
    kx = np.arange(n // 2 + 1)[None, None, :]
    phase = np.exp(-2j * np.pi * (kz * s[0] + ky * s[1] + kx * s[2]) / n)
    assert np.abs(O.r2c3(b) - phase * O.r2c3(a)).max() < 1e-15 * 20


def test_linearity(O):
    n = 16
    a = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    assert np.abs(O.r2c3(2 * a - 3 * b) - (2 * O.r2c3(a) - 3 * O.r2c3(b))).max() < 1e-14


def test_c2c3_brute_force(O):
    shape = (3, 4, 6)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = np.einsum("zyx,az,by,cx->abc", a, dft_matrix(3, 1), dft_matrix(4, 1), dft_matrix(6, 1))
    assert np.abs(O.c2c3(a, 1) - ref).max() < 1e-13
