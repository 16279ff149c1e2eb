"""Pins of the oracle's Navier-Stokes and MHD operators and time stepping.

Each test checks the oracle against something it does not compute itself:
closed forms (Taylor-Green curl and projected nonlinear term, exact Beltrami,
shear and Alfven solutions, the textbook RK stability polynomials), brute-force
Galerkin convolution sums on tiny grids, exact invariants of the truncated
system, and the early-time energy decay of the Taylor-Green vortex.
"""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

rng = np.random.default_rng(7)


def wvec(n):
    kx, ky, kz = I.wavenumbers(n)
    shape = (n, n, n // 2 + 1)
    return (np.broadcast_to(kx, shape).astype(float), np.broadcast_to(ky, shape).astype(float),
            np.broadcast_to(kz, shape).astype(float))


def hweights(n):
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w[None, None, :]


def inner(a, b, n):
    """<a, b> = sum_k w Re(a* . b) (real inner product of the physical fields)."""
    return np.sum(hweights(n) * np.real(np.conj(a) * b))


def grid(n):
    x = 2 * np.pi * np.arange(n) / n
    return np.meshgrid(x, x, x, indexing="ij")  # Z, Y, X


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [8, 16, 32])
def test_taylor_green_projected_nonlinear_term(O, n):
    """D P F[u x w] for Taylor-Green equals the transform of
    N_TG = (-sin2x cos2z / 8, -sin2y cos2z / 8, (cos2x + cos2y) sin2z / 8)."""
    Z, Y, X = grid(n)
    N = np.stack([-np.sin(2 * X) * np.cos(2 * Z) / 8, -np.sin(2 * Y) * np.cos(2 * Z) / 8,
                  (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8])
    ref = np.stack([np.fft.rfftn(N[c]) / n ** 3 for c in range(3)])
    got = O.ns_rhs(I.taylor_green_spec(n))
    assert np.abs(got - ref).max() < 1e-15 * 10


def test_taylor_green_vorticity_via_beltrami_identity(O):
    """For the ABC flow curl u = u, so u x w = 0 and the operator vanishes."""
    n = 16
    got = O.ns_rhs(I.abc_spec(n, 1.0, 0.7, 0.4))
    assert np.abs(got).max() < 1e-15 * 10


@pytest.mark.parametrize("n", [16, 24])
def test_output_solenoidal_and_hermitian(O, n):
    u = I.random_solenoidal(n, 3)
    r = O.ns_rhs(u)
    kx, ky, kz = wvec(n)
    div = kx * r[0] + ky * r[1] + kz * r[2]
    assert np.abs(div).max() < 1e-14 * np.abs(r).max()
    # real field: kx = 0 plane is Hermitian, r(0,-ky,-kz) = conj r(0,ky,kz)
    p = r[:, :, :, 0]
    idx = (-np.arange(n)) % n
    pz = p[:, idx][:, :, idx]
    assert np.abs(p - np.conj(pz)).max() < 1e-14 * np.abs(r).max()
    # dealiased: nothing outside the cube
    assert np.abs(r[:, ~I.cube_mask(n)]).max() == 0.0


# ------------------------------------------------------- Galerkin brute force
def full_spectrum(h, n):
    """Extend a half spectrum [c][n][n][n/2+1] to the full [c][n][n][n] cube."""
    f = np.zeros(h.shape[:3] + (n,), complex)
    f[..., : n // 2 + 1] = h
    for kx in range(n // 2 + 1, n):
        f[..., kx] = np.conj(h[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n][..., n - kx])
    return f


def galerkin_ns(h, n, kcut):
    """D P sum_{p+q=k} uhat(p) x (i q x uhat(q)) over kept p, q (brute force)."""
    f = full_spectrum(h, n)
    ks = np.arange(-kcut, kcut + 1)
    modes = np.array([(a, b, c) for a in ks for b in ks for c in ks])  # (kx, ky, kz)
    uh = np.array([f[:, kz % n, ky % n, kx % n] for kx, ky, kz in modes])  # [M][3]
    wh = 1j * np.cross(modes, uh)                                            # i q x u(q)
    out = np.zeros((3, n, n, n // 2 + 1), complex)
    index = {tuple(m): i for i, m in enumerate(modes)}
    for i, k in enumerate(modes):
        if k[0] < 0:
            continue
        acc = np.zeros(3, complex)
        for j, p in enumerate(modes):
            q = tuple(k - p)
            if q in index:
                acc += np.cross(uh[j], wh[index[q]])
        k2 = float(k @ k)
        if k2 > 0:
            acc = acc - k * (k @ acc) / k2
        else:
            acc[:] = 0
        out[:, k[2] % n, k[1] % n, k[0]] = acc
    return out


@pytest.mark.parametrize("n", [8, 9, 12])
def test_dealiased_operator_equals_galerkin_sum(O, n):
    K = I.kcut_23(n)
    u = I.random_solenoidal(n, 11, spectrum=lambda k: np.exp(-0.1 * k), kcut=K)
    ref = galerkin_ns(u, n, K)
    got = O.ns_rhs(u, kcut=K)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def galerkin_ns_sets(h, n, r_in, r_out):
    """D P sum_{p+q=k} uhat(p) x (i q x uhat(q)) by brute force, with p, q over
    the modes of the input ball |p|^2 <= r_in^2 and the result kept on the
    ball |k|^2 <= r_out^2 (spherical truncation of radius r_out)."""
    f = full_spectrum(h, n)
    ks = np.arange(-(n // 2), n // 2 + 1)
    ball = np.array([(a, b, c) for a in ks for b in ks for c in ks if a * a + b * b + c * c <= r_in * r_in])
    uh = np.array([f[:, kz % n, ky % n, kx % n] for kx, ky, kz in ball])
    wh = 1j * np.cross(ball, uh)
    index = {tuple(m): i for i, m in enumerate(ball)}
    out = np.zeros((3, n, n, n // 2 + 1), complex)
    for a in range(0, r_out + 1):
        for b in range(-r_out, r_out + 1):
            for c in range(-r_out, r_out + 1):
                k = np.array([a, b, c])
                k2 = int(k @ k)
                if k2 > r_out * r_out or k2 == 0:
                    continue
                acc = np.zeros(3, complex)
                for j, p in enumerate(ball):
                    q = tuple(k - p)
                    if q in index:
                        acc += np.cross(uh[j], wh[index[q]])
                acc = acc - k * (k @ acc) / k2
                out[:, c % n, b % n, a] = acc
    return out


def ball_mask(n, r):
    kx, ky, kz = I.wavenumbers(n)
    return (kx ** 2 + ky ** 2 + kz ** 2) <= r * r


@pytest.mark.parametrize("n", [9, 12])
def test_spherical_truncation_equals_galerkin_sum(O, n):
    """Spherical truncation |k|^2 <= K^2, K = ceil(n/3) - 1 (the ball lies in
    the alias-free cube, so the pseudospectral operator is exact): for a field
    on the ball and for a field on the whole cube, the operator equals the
    brute-force Galerkin sum over the input's modes, kept on the ball.  The
    ball's surface |k|^2 = K^2 is populated and must be kept (<= not <)."""
    K = I.kcut_23(n)
    u_cube = I.random_solenoidal(n, 21, spectrum=lambda k: np.exp(-0.1 * k), kcut=K)
    u_ball = u_cube * ball_mask(n, K)[None]
    for u, r_in in ((u_ball, K), (u_cube, int(np.ceil(np.sqrt(3) * K)))):
        ref = galerkin_ns_sets(u, n, r_in, K)
        got = O.ns_rhs(u, kcut=K, sphere=True)
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
        # nothing outside the ball; the surface modes carry a nonzero term
        assert np.abs(got[:, ~ball_mask(n, K)]).max() == 0.0
        kx, ky, kz = I.wavenumbers(n)
        surf = (kx ** 2 + ky ** 2 + kz ** 2) == K * K
        assert np.abs(got[:, surf]).max() > 1e-3 * np.abs(ref).max()
    # the strict-inequality misreading drops the populated surface
    ref = galerkin_ns_sets(u_ball, n, K, K)
    strict = ref * (~surf)[None]
    assert np.abs(strict - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("n,r", [(9, 4), (12, 5)])
def test_spherical_radius_that_aliases(O, n, r):
    """Negative control: a ball of radius r with 3r >= n (here larger than the
    cube's cutoff) is not alias-free: the pseudospectral result departs from
    the Galerkin sum."""
    u = I.random_solenoidal(n, 22, spectrum=lambda k: np.exp(-0.1 * k), kcut=n // 2 - 1)
    u = u * ball_mask(n, r)[None]
    ref = galerkin_ns_sets(u, n, r, r)
    got = O.ns_rhs(u, kcut=r, sphere=True)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("n", [9, 12])
def test_third_rule_reading_aliases(O, n):
    """Negative control: keeping |k_i| <= n/3 (3K = n) is not alias-free."""
    K = n // 3
    u = I.random_solenoidal(n, 12, spectrum=lambda k: np.exp(-0.1 * k), kcut=K)
    ref = galerkin_ns(u, n, K)
    got = O.ns_rhs(u, kcut=K)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("n,kcut", [(16, None), (24, None), (16, -1)])
def test_inviscid_energy_conservation(O, n, kcut):
    """sum_k w Re(uhat* . N) = <u . (u x w)> = 0 (with or without dealiasing)."""
    u = I.random_solenoidal(n, 5, kcut=I.kcut_23(n))
    r = O.ns_rhs(u, kcut=kcut)
    assert abs(inner(u, r, n)) < 1e-14 * np.sqrt(inner(u, u, n) * inner(r, r, n))


@pytest.mark.parametrize("n", [16, 24])
def test_mhd_ideal_invariants(O, n):
    u = I.random_solenoidal(n, 5)
    b = I.random_solenoidal(n, 6, field=1)
    nu_, nb_ = O.mhd_rhs(u, b)
    scale = np.sqrt((inner(u, u, n) + inner(b, b, n)) * (inner(nu_, nu_, n) + inner(nb_, nb_, n)))
    assert abs(inner(u, nu_, n) + inner(b, nb_, n)) < 1e-14 * scale   # total energy
    assert abs(inner(b, nu_, n) + inner(u, nb_, n)) < 1e-14 * scale   # cross helicity
    kx, ky, kz = wvec(n)
    for r in (nu_, nb_):
        assert np.abs(kx * r[0] + ky * r[1] + kz * r[2]).max() < 1e-14 * np.abs(r).max()


def test_mhd_reduces_to_ns_without_field(O):
    n = 16
    u = I.random_solenoidal(n, 5)
    nu_, nb_ = O.mhd_rhs(u, np.zeros_like(u))
    assert np.abs(nu_ - O.ns_rhs(u)).max() < 1e-15 * 10
    assert np.abs(nb_).max() == 0.0


# ------------------------------------------------------------- time stepping
@pytest.mark.parametrize("rk", [2, 4])
def test_integrating_factor_exact(O, rk):
    """With the nonlinear term off the scheme is exact: u(t) = e^{-nu k^2 t} u0."""
    n = 16
    nu, dt, ns = 0.05, 0.01, 7
    u0 = I.random_solenoidal(n, 2)
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk, linear_only=True)
    kx, ky, kz = wvec(n)
    ref = np.exp(-nu * (kx ** 2 + ky ** 2 + kz ** 2) * dt * ns) * u0
    assert np.abs(u - ref).max() < 1e-15 * 10


@pytest.mark.parametrize("rk", [2, 4])
def test_beltrami_exact_decay(O, rk):
    n = 16
    nu, dt, ns = 0.1, 0.01, 10
    u0 = I.abc_spec(n, 1.0, 0.8, 0.6)
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk)
    assert np.abs(u - np.exp(-nu * dt * ns) * u0).max() < 1e-14


@pytest.mark.parametrize("rk", [2, 4])
def test_shear_wave_exact_decay(O, rk):
    n, k = 16, 3
    nu, dt, ns = 0.02, 0.01, 10
    u0 = I.shear_wave_spec(n, k=k, amp=0.9)
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk)
    assert np.abs(u - np.exp(-nu * k * k * dt * ns) * u0).max() < 1e-15 * 10


def taylor(z, order):
    out = 0
    fact = 1.0
    for j in range(order + 1):
        if j > 0:
            fact *= j
        out = out + z ** j / fact
    return out


@pytest.mark.parametrize("rk", [2, 4])
@pytest.mark.parametrize("nu", [0.0, 0.03])
def test_alfven_wave_amplification(O, rk, nu):
    """Alfven wave on b0 zhat: the nonlinear terms reduce to the linear coupling
    +-i k b0, so a Lawson step multiplies uhat(k) by e^{-nu k^2 h} T_rk(-i k b0 h)
    with T_rk the degree-rk Taylor polynomial of exp (the RK stability function)."""
    n, k, b0, amp = 16, 2, 1.3, 0.2
    dt, ns = 0.02, 9
    u0, b0f = I.alfven_spec(n, k=k, amp=amp, b0=b0)
    u, b = O.step(u0, ns, dt=dt, nu=nu, eta=nu, rk=rk, bhat=b0f)
    kz = wvec(n)[2]
    g = np.exp(-nu * kz * kz * dt) * taylor(-1j * kz * b0 * dt, rk)
    ref_u = u0 * g ** ns
    ref_b = -ref_u.copy()
    ref_b[2, 0, 0, 0] = b0
    assert np.abs(u - ref_u).max() < 1e-14
    assert np.abs(b - ref_b).max() < 1e-14
    # and close to the exact travelling wave
    exact = u0 * np.exp((-nu * kz * kz - 1j * kz * b0) * dt * ns)
    assert np.abs(u - exact).max() < (5e-4 if rk == 2 else 5e-6) * amp


@pytest.mark.parametrize("rk,expect", [(2, 4.0), (4, 16.0)])
def test_rk_order(O, rk, expect):
    n = 16
    u0 = I.random_solenoidal(n, 9)
    T, nu = 0.16, 0.01
    ref = O.step(u0, 256, dt=T / 256, nu=nu, rk=4)
    e1 = np.abs(O.step(u0, 8, dt=T / 8, nu=nu, rk=rk) - ref).max()
    e2 = np.abs(O.step(u0, 16, dt=T / 16, nu=nu, rk=rk) - ref).max()
    assert abs(e1 / e2 / expect - 1) < 0.15


@pytest.mark.parametrize("rk,tol", [(2, 1e-10), (4, 1e-10)])
def test_taylor_green_early_energy(O, rk, tol):
    """Taylor-Green, n = 32, nu = 0.01, dt = 1e-3, 10 steps: at early times
    E(t) = E0 exp(-6 nu t) - 10 nu t^3 / 384 + O(nu t^4), E0 = 1/8
    (all energy at |k|^2 = 3; the nonlinear term feeds E8 = t^2/128 into
    |k|^2 = 8 modes, whose extra dissipation is 10 nu E8)."""
    n, nu, dt, ns = 32, 0.01, 1e-3, 10
    u = O.step(I.taylor_green_spec(n), ns, dt=dt, nu=nu, rk=rk)
    t = dt * ns
    e = O.energy(u)
    ref = 0.125 * np.exp(-6 * nu * t) - 10 * nu * t ** 3 / 384
    assert abs(e - ref) < tol * ref
    # the t^3 term is resolved: dropping it misses by far more than the tolerance
    assert abs(e - 0.125 * np.exp(-6 * nu * t)) > 10 * tol * ref


# ---------------------------------------------------------------- diagnostics
def test_energy_parseval_and_spectrum(O):
    n = 16
    u = I.random_solenoidal(n, 4, energy=0.37)
    e = O.energy(u)
    ur = O.c2r_vec(u)
    assert abs(e - 0.37) < 1e-14
    assert abs(0.5 * np.mean(np.sum(ur ** 2, axis=0)) - e) < 1e-14
    nsh = int(np.floor(np.sqrt(3) * (n // 2) + 0.5)) + 1
    s = O.spectrum(u, nsh)
    assert abs(s.sum() - e) < 1e-14
    # a single mode at |k| = sqrt(5) lands in shell floor(2.236 + .5) = 2
    v = np.zeros_like(u)
    v[0, 0, 1, 2] = 0.5  # (kx, ky, kz) = (2, 1, 0)
    sv = O.spectrum(v, nsh)
    assert sv[2] == pytest.approx(0.25, abs=1e-16) and abs(sv.sum() - 0.25) < 1e-16


def test_enstrophy_closed_forms(O):
    """Z = 1/2 sum w |k|^2 |vhat|^2: Taylor-Green (every mode at |k|^2 = 3,
    E = 1/8) gives 3/8; one mode at (2, 1, 0) of amplitude 1/2 gives
    1/2 * 2 * 5 * 1/4; a random field matches 1/2 <|curl u|^2> with the curl
    taken by numpy's FFT in physical space."""
    n = 16
    assert abs(O.enstrophy(I.taylor_green_spec(n)) - 3.0 / 8.0) < 1e-15
    v = np.zeros((3, n, n, n // 2 + 1), np.complex128)
    v[0, 0, 1, 2] = 0.5
    assert O.enstrophy(v) == pytest.approx(1.25, abs=1e-15)
    u = I.random_solenoidal(n, 6)
    ur = O.c2r_vec(u)
    k = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")

    def d(f, kk):
        return np.real(np.fft.ifftn(1j * kk * np.fft.fftn(f)))

    w = np.stack([d(ur[2], ky) - d(ur[1], kz), d(ur[0], kz) - d(ur[2], kx), d(ur[1], kx) - d(ur[0], ky)])
    assert abs(O.enstrophy(u) - 0.5 * np.mean(np.sum(w ** 2, axis=0))) < 1e-13 * O.enstrophy(u)


def test_random_field_is_solenoidal_and_real(O):
    n = 24
    u = I.random_solenoidal(n, 8)
    kx, ky, kz = wvec(n)
    assert np.abs(kx * u[0] + ky * u[1] + kz * u[2]).max() < 1e-15
    ur = O.c2r_vec(u)
    # round trip through the real field recovers the coefficients (they are Hermitian)
    assert np.abs(O.r2c_vec(ur) - u).max() < 1e-15 * 10
