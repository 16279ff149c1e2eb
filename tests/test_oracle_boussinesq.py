"""Pins of the oracle's Boussinesq operators (eq. mom with the buoyancy term,
eq. temp, eq. divv) and their time stepping.

Checked against what the oracle does not compute itself: the internal gravity
wave (a single mode transverse to its wavevector, for which the nonlinear terms
vanish and the buoyancy coupling rotates (u, theta) at N k_h/|k|) through the
textbook RK stability polynomials; brute-force Galerkin sums of the scalar
advection term on tiny grids; the exact conservation of kinetic plus scalar
energy by the truncated inviscid operators; the coupling terms alone in closed
form; and the scalar's own integrating factor.
"""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I


def wvec(n):
    kx, ky, kz = I.wavenumbers(n)
    shape = (n, n, n // 2 + 1)
    return (np.broadcast_to(kx, shape).astype(float), np.broadcast_to(ky, shape).astype(float),
            np.broadcast_to(kz, shape).astype(float))


def hweights(n):
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w


def inner(a, b, n):
    return float(np.sum(hweights(n) * np.real(np.conj(a) * b)))


def taylor(z, order):
    out, fact = 0, 1.0
    for j in range(order + 1):
        if j > 0:
            fact *= j
        out = out + z ** j / fact
    return out


@pytest.mark.parametrize("rk", [2, 4])
@pytest.mark.parametrize("nu", [0.0, 0.02])
def test_gravity_wave_amplification(O, rk, nu):
    """u = A e exp(i k.x) + c.c. with e perpendicular to k and theta = T exp(i k.x)
    + c.c.: u . grad u is a gradient and u . grad theta = 0, so only the
    buoyancy terms act: dA/dt = -w T, dT/dt = w A with w = N |k_h| / |k|.  A
    Lawson step with nu = kappa is e^{-nu k^2 h} times the RK stability
    function of that rotation: with a + i b = T_rk(i w h),
    (A, T) -> e^{-nu k^2 h} (a A - b T, b A + a T)."""
    n, k, nbv = 16, (1, 1, 2), 2.5
    dt, ns = 0.02, 11
    u0, t0 = I.gravity_wave_spec(n, k=k, amp_u=0.1, amp_t=0.07)
    u, t = O.step(u0, ns, dt=dt, nu=nu, kappa=nu, rk=rk, theta=t0, nbv=nbv)
    kv = np.array(k, float)
    k2 = float(kv @ kv)
    w = nbv * np.sqrt(kv[0] ** 2 + kv[1] ** 2) / np.sqrt(k2)
    g = taylor(1j * w * dt, rk)
    A, T = 0.1, 0.07
    for _ in range(ns):
        A, T = np.exp(-nu * k2 * dt) * (g.real * A - g.imag * T), np.exp(-nu * k2 * dt) * (g.imag * A + g.real * T)
    e = u0[:, k[2], k[1], k[0]] / 0.1
    ref_u = np.zeros_like(u0)
    ref_u[:, k[2], k[1], k[0]] = A * e
    ref_t = np.zeros_like(t0)
    ref_t[k[2], k[1], k[0]] = T
    assert np.abs(u - ref_u).max() < 1e-14
    assert np.abs(t - ref_t).max() < 1e-14
    # and close to the exact oscillation
    c, s = np.cos(w * dt * ns), np.sin(w * dt * ns)
    d = np.exp(-nu * k2 * dt * ns)
    assert abs(A - d * (0.1 * c - 0.07 * s)) < (2e-3 if rk == 2 else 2e-6)
    assert abs(T - d * (0.07 * c + 0.1 * s)) < (2e-3 if rk == 2 else 2e-6)


@pytest.mark.parametrize("n", [12, 16])
def test_inviscid_energy_conservation(O, n):
    """<u, N_u> + <theta, N_theta> = 0: u x w is perpendicular to u, <theta,
    u . grad theta> = 0 for solenoidal band-limited u, and the buoyancy terms
    exchange -N <u_z, theta> + N <theta, u_z> = 0.  With N = 0 the kinetic and
    scalar transfers vanish separately."""
    u = I.random_solenoidal(n, 3)
    t = I.random_scalar(n, 4)
    for nbv in (0.0, 1.7):
        ou, ot = O.bq_rhs(u, t, nbv)
        scale = np.sum(np.abs(u) * np.abs(ou)) + np.sum(np.abs(t) * np.abs(ot))
        assert scale > 0
        total = inner(u, ou, n) + inner(t, ot, n)
        assert abs(total) < 1e-13 * scale
        if nbv == 0.0:
            assert abs(inner(u, ou, n)) < 1e-13 * scale
            assert abs(inner(t, ot, n)) < 1e-13 * scale
        else:
            # the exchange term alone is not zero: it is what the two transfers trade
            assert abs(inner(t, ot, n)) > 1e-6 * scale


def test_coupling_terms_alone(O):
    """theta = 0: N_theta = N w_z on the kept modes and N_u is the Navier-Stokes
    operator.  u = 0: N_u = -N P (theta zhat) = -N theta (zhat - k k_z/|k|^2),
    zero at k = 0, and N_theta = 0."""
    n, nbv = 16, 1.9
    u = I.random_solenoidal(n, 5)
    t = I.random_scalar(n, 6)
    ou, ot = O.bq_rhs(u, np.zeros_like(t), nbv)
    assert np.abs(ot - nbv * u[2]).max() < 1e-15
    assert np.abs(ou - O.ns_rhs(u)).max() < 1e-15
    ou, ot = O.bq_rhs(np.zeros_like(u), t, nbv)
    kx, ky, kz = wvec(n)
    k2 = kx * kx + ky * ky + kz * kz
    k2s = np.where(k2 == 0, 1.0, k2)
    ref = -nbv * np.stack([-kx * kz / k2s * t, -ky * kz / k2s * t, (1 - kz * kz / k2s) * t])
    ref[:, k2 == 0] = 0
    assert np.abs(ou - ref).max() < 1e-15
    assert np.abs(ot).max() == 0.0


def full_spectrum_scalar(h, n):
    f = np.zeros(h.shape[:2] + (n,), complex)
    f[..., : n // 2 + 1] = h
    for kx in range(n // 2 + 1, n):
        f[..., kx] = np.conj(h[(-np.arange(n)) % n][:, (-np.arange(n)) % n][..., n - kx])
    return f


def full_spectrum_vec(h, n):
    return np.stack([full_spectrum_scalar(h[c], n) for c in range(3)])


@pytest.mark.parametrize("n", [8, 9])
def test_scalar_advection_equals_galerkin_sum(O, n):
    """N_theta (N = 0) = -D sum_{p+q=k} uhat(p) . (i q thetahat(q)) over kept p, q."""
    K = I.kcut_23(n)
    u = I.random_solenoidal(n, 12, spectrum=lambda k: np.exp(-0.1 * k), kcut=K)
    t = I.random_scalar(n, 13, spectrum=lambda k: np.exp(-0.1 * k), kcut=K)
    fu, ft = full_spectrum_vec(u, n), full_spectrum_scalar(t, n)
    ks = np.arange(-K, K + 1)
    modes = np.array([(a, b, c) for a in ks for b in ks for c in ks])
    uh = np.array([fu[:, kz % n, ky % n, kx % n] for kx, ky, kz in modes])
    gh = np.array([1j * np.array([kx, ky, kz]) * ft[kz % n, ky % n, kx % n] for kx, ky, kz in modes])
    index = {tuple(m): i for i, m in enumerate(modes)}
    ref = np.zeros((n, n, n // 2 + 1), complex)
    for k in modes:
        if k[0] < 0:
            continue
        acc = 0j
        for j, p in enumerate(modes):
            q = tuple(k - p)
            if q in index:
                acc += uh[j] @ gh[index[q]]
        ref[k[2] % n, k[1] % n, k[0]] = -acc
    _, got = O.bq_rhs(u, t, 0.0, kcut=K)
    assert np.abs(got - ref).max() < 1e-14 * max(np.abs(ref).max(), 1e-300)


@pytest.mark.parametrize("rk", [2, 4])
def test_scalar_integrating_factor_exact(O, rk):
    """Without the nonlinear operator each mode decays exactly: u by
    exp(-nu k^2 t), theta by exp(-kappa k^2 t) with its own diffusivity."""
    n, nu, kappa, dt, ns = 16, 0.03, 0.011, 0.05, 7
    u = I.random_solenoidal(n, 14)
    t = I.random_scalar(n, 15)
    su, st = O.step(u, ns, dt=dt, nu=nu, kappa=kappa, rk=rk, theta=t, nbv=3.0, linear_only=True)
    kx, ky, kz = wvec(n)
    k2 = kx * kx + ky * ky + kz * kz
    assert np.abs(su - u * np.exp(-nu * k2 * dt * ns)).max() < 1e-15
    assert np.abs(st - t * np.exp(-kappa * k2 * dt * ns)).max() < 1e-15


def test_random_scalar_is_real_and_normalised(O):
    n = 16
    t = I.random_scalar(n, 2, energy=0.3)
    phys = O.c2r3(t)
    back = O.r2c3(phys)
    assert np.abs(back - t).max() < 1e-15
    assert abs(O.energy(t) - 0.3) < 1e-13
    assert abs(0.5 * np.mean(phys ** 2) - 0.3) < 1e-13
