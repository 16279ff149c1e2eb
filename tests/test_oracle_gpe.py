"""Pins of the oracle's Gross-Pitaevskii operator and time stepping (eq. gpe
divided by i hbar: d psi/dt = i alpha Lap psi - i beta |psi|^2 psi with
alpha = hbar / 2m, beta = g / hbar), on a complex field whose coefficients
fill the whole spectrum.  The cubic product is alias-free when every axis
keeps |k_i| <= K_i with 4 K_i < n_i (K_i = ceil(n_i/4) - 1).

Pins: the plane wave (an exact solution: |psi|^2 is constant, so the
nonlinear term is a phase rotation) in closed form, brute-force Galerkin
triple sums on tiny grids with a 2/3-rule negative control, conservation of
the particle number and of the Hamiltonian by the semi-discrete operator
(the latter with the quartic term computed by numpy's FFT), the exact
integrating factor, and the RK stability polynomial on a uniform condensate."""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

TWO_PI = 2 * np.pi


def kgrid(shape, box=(TWO_PI,) * 3):
    nx, ny, nz = shape
    f = [np.fft.fftfreq(m, 1.0 / m) * TWO_PI / L for m, L in zip(shape, box)]
    KZ, KY, KX = np.meshgrid(f[2], f[1], f[0], indexing="ij")
    return KX, KY, KZ


def kcut_mask(shape, kc):
    nx, ny, nz = shape
    w = [np.where(np.arange(m) < m // 2, np.arange(m), np.arange(m) - m) for m in shape]
    KZ, KY, KX = np.meshgrid(w[2], w[1], w[0], indexing="ij")
    return (np.abs(KX) <= kc[0]) & (np.abs(KY) <= kc[1]) & (np.abs(KZ) <= kc[2])


def to_phys(psih):
    return np.fft.ifftn(psih) * psih.size        # unnormalised backward


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("k", [(0, 0, 0), (1, 0, 0), (1, -2, 1)])
def test_plane_wave_operator(O, k):
    """psi = A exp(i k.x): -i beta D F[|psi|^2 psi] = -i beta |A|^2 A at k."""
    shape, A, beta = (16, 12, 8), 0.8 * np.exp(0.3j), 1.7
    psi = I.plane_wave(shape, k, A)
    got = O.gpe_rhs(psi, beta)
    ref = -1j * beta * abs(A) ** 2 * psi
    assert np.abs(got - ref).max() < 1e-15 * 10


@pytest.mark.parametrize("rk,tol", [(2, 2e-8), (4, 1e-13)])
def test_plane_wave_evolution(O, rk, tol):
    """The exact solution psi = A exp(i (k.x - w t)), w = alpha |k|^2 + beta |A|^2
    (the dispersion relation of eq. gpe), reached to the RK error
    (|A|^2 beta h)^(rk+1) per step: the linear part is exact."""
    shape, box = (16, 8, 12), (TWO_PI, 3.0, 5.0)
    k, A, alpha, beta = (2, 1, -1), 0.6, 0.5, 1.3
    dt, ns = 1e-3, 50
    psi0 = I.plane_wave(shape, k, A)
    got = O.gpe_step(psi0, ns, dt=dt, alpha=alpha, beta=beta, rk=rk, box=box)
    kp = np.array([TWO_PI * k[i] / box[i] for i in range(3)])
    w = alpha * kp @ kp + beta * A * A
    ref = psi0 * np.exp(-1j * w * dt * ns)
    assert np.abs(got - ref).max() < tol


# ------------------------------------------------------- Galerkin brute force
def galerkin_gpe(psih, kc, beta):
    """-i beta sum_{p - q + r = k} psi(p) conj(psi(q)) psi(r) over the kept
    cuboid, kept k only (brute force over all kept p, r)."""
    nz, ny, nx = psih.shape
    modes = np.array([(a, b, c) for a in range(-kc[0], kc[0] + 1) for b in range(-kc[1], kc[1] + 1)
                      for c in range(-kc[2], kc[2] + 1)])
    val = np.array([psih[c % nz, b % ny, a % nx] for a, b, c in modes])
    index = {tuple(m): i for i, m in enumerate(modes)}
    out = np.zeros_like(psih)
    for k in modes:
        acc = 0j
        for i, p in enumerate(modes):
            for j, r in enumerate(modes):
                q = tuple(p + r - k)
                if q in index:
                    acc += val[i] * np.conj(val[index[q]]) * val[j]
        out[k[2] % nz, k[1] % ny, k[0] % nx] = -1j * beta * acc
    return out


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 12, 8)])
def test_operator_equals_galerkin_sum(O, shape):
    kc = tuple(O.kcut_14(m) for m in shape)
    psi = I.random_wavefunction(shape, 11, spectrum=lambda k: np.exp(-0.1 * k), condensate=0.3)
    ref = galerkin_gpe(psi, kc, 0.9)
    got = O.gpe_rhs(psi, 0.9)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_two_thirds_rule_aliases_the_cubic_product(O):
    """Negative control: the 2/3-rule cutoff (3K < n, enough for quadratic
    products) is not alias-free for |psi|^2 psi."""
    shape = (8, 8, 8)
    kc = (2, 2, 2)
    psi = I.random_wavefunction(shape, 12, spectrum=lambda k: np.exp(-0.1 * k), kcut=kc)
    ref = galerkin_gpe(psi, kc, 1.0)
    got = O.gpe_rhs(psi, 1.0, kcut=kc)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("shape,box", [((16, 16, 16), (TWO_PI,) * 3), ((24, 16, 12), (4.0, TWO_PI, 3.0))])
def test_number_and_hamiltonian_conserved_by_operator(O, shape, box):
    """d/dt sum |psihat|^2 = 2 Re sum conj(psihat) N = 0, and
    dH/dt = 2 alpha Re sum |k|^2 conj(psihat) psihat_t + 2 beta Re <|psi|^2 conj(psi) psi_t> = 0
    (psihat_t = -i alpha |k|^2 psihat + N), the grid average of the quartic
    term taken with numpy's FFT: exact because 4 K_i < n_i."""
    alpha, beta = 0.7, 1.9
    psi = I.random_wavefunction(shape, 13, condensate=0.5, box=box)
    N = O.gpe_rhs(psi, beta, box=box)
    scale = np.sqrt(np.sum(np.abs(psi) ** 2) * np.sum(np.abs(N) ** 2))
    assert abs(np.real(np.sum(np.conj(psi) * N))) < 1e-14 * scale
    KX, KY, KZ = kgrid(shape, box)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    pt = -1j * alpha * k2 * psi + N
    x, xt = to_phys(psi), to_phys(pt)
    dkin = 2 * alpha * np.real(np.sum(k2 * np.conj(psi) * pt))
    dint = 2 * beta * np.real(np.mean(np.abs(x) ** 2 * np.conj(x) * xt))
    assert abs(dkin + dint) < 1e-12 * (abs(dkin) + abs(dint))
    assert abs(dkin) > 1e-6   # the test is not vacuous
    # and the oracle's invariants match numpy's
    n0, ek, ei = O.gpe_invariants(psi, alpha, beta, box=box)
    assert abs(n0 - np.sum(np.abs(psi) ** 2)) < 1e-14 * n0
    assert abs(ek - alpha * np.sum(k2 * np.abs(psi) ** 2)) < 1e-13 * ek
    assert abs(ei - 0.5 * beta * np.mean(np.abs(x) ** 4)) < 1e-13 * ei


@pytest.mark.parametrize("rk", [2, 4])
def test_integrating_factor_exact(O, rk):
    shape, box = (12, 8, 16), (3.0, TWO_PI, 9.0)
    alpha, dt, ns = 0.4, 0.01, 7
    psi0 = I.random_wavefunction(shape, 14, box=box)
    got = O.gpe_step(psi0, ns, dt=dt, alpha=alpha, beta=3.0, rk=rk, box=box, linear_only=True)
    KX, KY, KZ = kgrid(shape, box)
    ref = np.exp(-1j * alpha * (KX ** 2 + KY ** 2 + KZ ** 2) * dt * ns) * psi0
    assert np.abs(got - ref).max() < 1e-15 * 10


def taylor(z, order):
    out, fact = 0, 1.0
    for j in range(order + 1):
        if j > 0:
            fact *= j
        out = out + z ** j / fact
    return out


@pytest.mark.parametrize("rk", [2, 4])
def test_condensate_rk_polynomial(O, rk):
    """A uniform condensate psi = a stays uniform, and every stage's
    right-hand side is -i beta |z|^2 z of the current amplitude z (the
    integrating factor is 1 at k = 0): the oracle's steps equal the scalar
    Heun / classical RK stages evaluated here, and approach the exact phase
    rotation a exp(-i beta |a|^2 t) at the order of the scheme."""
    shape, a, beta, h = (8, 8, 8), 0.9 + 0.2j, 1.4, 0.05
    psi0 = np.zeros((8, 8, 8), complex)
    psi0[0, 0, 0] = a
    got = O.gpe_step(psi0, 3, dt=h, alpha=0.3, beta=beta, rk=rk)

    def f(z):
        return -1j * beta * abs(z) ** 2 * z
    z = a
    for _ in range(3):
        if rk == 2:
            k1 = f(z)
            k2 = f(z + h * k1)
            z = z + h / 2 * (k1 + k2)
        else:
            k1 = f(z)
            k2 = f(z + h / 2 * k1)
            k3 = f(z + h / 2 * k2)
            k4 = f(z + h * k3)
            z = z + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert abs(got[0, 0, 0] - z) < 1e-15 * 10
    assert np.abs(got.ravel()[1:]).max() < 1e-16 * 100
    # and close to the exact rotation a exp(-i beta |a|^2 t)
    assert abs(z - a * np.exp(-1j * beta * abs(a) ** 2 * 3 * h)) < (1e-3 if rk == 2 else 1e-6)


@pytest.mark.parametrize("rk,expect", [(2, 4.0), (4, 16.0)])
def test_rk_order(O, rk, expect):
    shape = (16, 16, 16)
    psi0 = I.random_wavefunction(shape, 15, condensate=0.6, number=2.0)
    T, alpha, beta = 0.2, 0.5, 2.0
    ref = O.gpe_step(psi0, 256, dt=T / 256, alpha=alpha, beta=beta, rk=4)
    e1 = np.abs(O.gpe_step(psi0, 8, dt=T / 8, alpha=alpha, beta=beta, rk=rk) - ref).max()
    e2 = np.abs(O.gpe_step(psi0, 16, dt=T / 16, alpha=alpha, beta=beta, rk=rk) - ref).max()
    assert abs(e1 / e2 / expect - 1) < 0.15
