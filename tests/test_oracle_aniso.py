"""Pins of the oracle on anisotropic grids: independent point counts N_i and
box lengths L_i per direction (eq. fftsum and the paragraph after it), so
physical wavenumbers 2 pi p / L_i and cube cutoffs K_i = ceil(N_i/3) - 1 per
axis.  Closed forms (generalised Taylor-Green term, Beltrami and shear
solutions on a non-cubic box), brute-force Galerkin sums on tiny uneven
grids, the inviscid invariant, the exact integrating factor and the
diagnostics against numpy's FFT in physical space."""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

TWO_PI = 2 * np.pi


def alphas(box):
    return [TWO_PI / L for L in box]


def kphys(shape, box):
    """Physical wavenumbers of the half spectrum [nz][ny][nx//2+1]."""
    nx, ny, nz = shape
    ax, ay, az = alphas(box)
    fy = np.where(np.arange(ny) < ny // 2, np.arange(ny), np.arange(ny) - ny)
    fz = np.where(np.arange(nz) < nz // 2, np.arange(nz), np.arange(nz) - nz)
    full = (nz, ny, nx // 2 + 1)
    return (np.broadcast_to(ax * np.arange(nx // 2 + 1)[None, None, :], full),
            np.broadcast_to(ay * fy[None, :, None], full), np.broadcast_to(az * fz[:, None, None], full))


def coords(shape, box):
    nx, ny, nz = shape
    z = box[2] * np.arange(nz) / nz
    y = box[1] * np.arange(ny) / ny
    x = box[0] * np.arange(nx) / nx
    return np.meshgrid(z, y, x, indexing="ij")  # Z, Y, X


def hw(nx):
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[nx // 2] = 1.0
    return w[None, None, :]


def inner(a, b, nx):
    return np.sum(hw(nx) * np.real(np.conj(a) * b))


def spec(O, phys):
    return np.stack([O.r2c3(phys[c]) for c in range(phys.shape[0])])


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("shape,box,pqr", [((8, 8, 16), (TWO_PI, np.pi, 4 * np.pi), (1, 1, 2)),
                                           ((16, 16, 12), (np.pi, TWO_PI, 3 * np.pi), (1, 2, 1))])
def test_generalised_taylor_green_term(O, shape, box, pqr):
    """u = (A sin ax cos by cos cz, B cos ax sin by cos cz, 0) with A a + B b = 0
    (a, b, c the physical wavenumbers): D P F[u x w] equals the transform of
    -(A^2 a/4) P[sin 2ax cos 2cz xhat] - (B^2 b/4) P[sin 2by cos 2cz yhat], with
    P[sin 2ax cos 2cz xhat] = (c^2 sin 2ax cos 2cz, 0, -a c cos 2ax sin 2cz)/(a^2+c^2)
    (and likewise in y); on a 2 pi cube it is the familiar Taylor-Green term."""
    ax, ay, az = alphas(box)
    a, b, c = ax * pqr[0], ay * pqr[1], az * pqr[2]
    A = 0.7
    B = -A * a / b
    Z, Y, X = coords(shape, box)
    u = np.stack([A * np.sin(a * X) * np.cos(b * Y) * np.cos(c * Z),
                  B * np.cos(a * X) * np.sin(b * Y) * np.cos(c * Z), np.zeros_like(X)])
    ka, kb = A * A * a / 4, B * B * b / 4
    N = np.stack([-ka * c * c / (a * a + c * c) * np.sin(2 * a * X) * np.cos(2 * c * Z),
                  -kb * c * c / (b * b + c * c) * np.sin(2 * b * Y) * np.cos(2 * c * Z),
                  ka * a * c / (a * a + c * c) * np.cos(2 * a * X) * np.sin(2 * c * Z)
                  + kb * b * c / (b * b + c * c) * np.cos(2 * b * Y) * np.sin(2 * c * Z)])
    got = O.ns_rhs(spec(O, u), box=box, nx=shape[0])
    ref = spec(O, N)
    assert np.abs(got - ref).max() < 1e-15 * 20


def abc_phys(shape, box, pqr, A=1.0, B=0.8, C=0.6):
    """ABC flow with one physical wavenumber kappa on every axis:
    u = (A sin kz + C cos ky, B sin kx + A cos kz, C sin ky + B cos kx),
    curl u = kappa u (pqr: the integer wavenumbers giving kappa on each axis)."""
    ax, ay, az = alphas(box)
    kx, ky, kz = ax * pqr[0], ay * pqr[1], az * pqr[2]
    assert np.isclose(kx, ky) and np.isclose(ky, kz)
    Z, Y, X = coords(shape, box)
    return np.stack([A * np.sin(kz * Z) + C * np.cos(ky * Y), B * np.sin(kx * X) + A * np.cos(kz * Z),
                     C * np.sin(ky * Y) + B * np.cos(kx * X)]), kx


@pytest.mark.parametrize("rk", [2, 4])
def test_beltrami_on_anisotropic_box(O, rk):
    """curl u = kappa u makes u x w vanish: the operator is zero and the flow
    decays as exp(-nu kappa^2 t) exactly on a 16 x 16 x 8 grid of a
    2 pi x 2 pi x pi box (kappa = 2: integer wavenumbers 2, 2, 1)."""
    shape, box = (16, 16, 8), (TWO_PI, TWO_PI, np.pi)
    up, kappa = abc_phys(shape, box, (2, 2, 1))
    u0 = spec(O, up)
    assert np.abs(O.ns_rhs(u0, box=box, nx=16)).max() < 1e-15 * 10
    nu, dt, ns = 0.05, 0.01, 10
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk, box=box, nx=16)
    assert np.abs(u - np.exp(-nu * kappa ** 2 * dt * ns) * u0).max() < 1e-14


@pytest.mark.parametrize("rk", [2, 4])
def test_shear_wave_on_anisotropic_box(O, rk):
    """u = sin(c z) xhat, c = 2 pi r / Lz: exact decay exp(-nu c^2 t)."""
    shape, box = (8, 12, 16), (TWO_PI, 3 * np.pi, 5.0)
    c = TWO_PI * 3 / box[2]
    Z, Y, X = coords(shape, box)
    u0 = spec(O, np.stack([0.9 * np.sin(c * Z), 0 * Z, 0 * Z]))
    nu, dt, ns = 0.02, 0.01, 10
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk, box=box, nx=8)
    assert np.abs(u - np.exp(-nu * c * c * dt * ns) * u0).max() < 1e-15 * 20


@pytest.mark.parametrize("rk", [2, 4])
def test_integrating_factor_exact_anisotropic(O, rk):
    shape, box = (12, 8, 16), (3.0, TWO_PI, 9.0)
    nu, dt, ns = 0.05, 0.01, 7
    u0 = I.random_solenoidal(0, 2, shape=shape, box=box)
    u = O.step(u0, ns, dt=dt, nu=nu, rk=rk, linear_only=True, box=box, nx=12)
    kx, ky, kz = kphys(shape, box)
    assert np.abs(u - np.exp(-nu * (kx ** 2 + ky ** 2 + kz ** 2) * dt * ns) * u0).max() < 1e-15 * 10


# ------------------------------------------------------- Galerkin brute force
def full_modes(h, shape):
    """Coefficient of integer wavenumber (kx, ky, kz) from a half spectrum,
    through the Hermitian symmetry for kx < 0."""
    nx, ny, nz = shape

    def get(kx, ky, kz):
        if kx >= 0:
            return h[:, kz % nz, ky % ny, kx]
        return np.conj(h[:, (-kz) % nz, (-ky) % ny, -kx])
    return get


def galerkin_ns(h, shape, box, kc):
    """D P sum_{p+q=k} uhat(p) x (i q x uhat(q)) over the cuboid |p_i| <= kc_i
    (physical wavenumbers in the curl and the projection)."""
    nx, ny, nz = shape
    al = np.array(alphas(box))
    get = full_modes(h, shape)
    modes = np.array([(a, b, c) for a in range(-kc[0], kc[0] + 1) for b in range(-kc[1], kc[1] + 1)
                      for c in range(-kc[2], kc[2] + 1)])
    uh = np.array([get(*m) for m in modes])
    wh = 1j * np.cross(modes * al, uh)
    index = {tuple(m): i for i, m in enumerate(modes)}
    out = np.zeros((3, nz, ny, nx // 2 + 1), complex)
    for i, k in enumerate(modes):
        if k[0] < 0:
            continue
        acc = np.zeros(3, complex)
        for j, p in enumerate(modes):
            q = tuple(k - p)
            if q in index:
                acc += np.cross(uh[j], wh[index[q]])
        kp = k * al
        k2 = float(kp @ kp)
        acc = acc - kp * (kp @ acc) / k2 if k2 > 0 else 0 * acc
        out[:, k[2] % nz, k[1] % ny, k[0]] = acc
    return out


@pytest.mark.parametrize("shape,box", [((8, 9, 12), (TWO_PI, np.pi, 4 * np.pi)),
                                       ((12, 8, 9), (5.0, TWO_PI, 2.5))])
def test_anisotropic_operator_equals_galerkin_sum(O, shape, box):
    kc = tuple(I.kcut_23(m) for m in shape)
    u = I.random_solenoidal(0, 31, spectrum=lambda k: np.exp(-0.1 * k), shape=shape, box=box)
    ref = galerkin_ns(u, shape, box, kc)
    got = O.ns_rhs(u, box=box, nx=shape[0])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_anisotropic_third_rule_aliases(O):
    """Negative control: per-axis cutoffs n_i // 3 (3K_i = n_i on the 9 and 12
    axes) are not alias-free."""
    shape, box = (8, 9, 12), (TWO_PI, np.pi, 4 * np.pi)
    kc = (2, 3, 4)
    u = I.random_solenoidal(0, 32, spectrum=lambda k: np.exp(-0.1 * k), kcut=kc, shape=shape, box=box)
    ref = galerkin_ns(u, shape, box, kc)
    got = O.ns_rhs(u, kcut=kc, box=box, nx=shape[0])
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("shape,box", [((16, 12, 8), (TWO_PI, 3.0, 9.0)), ((24, 16, 32), (4.0, 4.0, 1.0))])
def test_anisotropic_invariants(O, shape, box):
    """Inviscid energy conservation of the operator, a solenoidal Hermitian
    output on the physical wavenumbers, and MHD energy / cross helicity."""
    nx = shape[0]
    u = I.random_solenoidal(0, 5, shape=shape, box=box)
    r = O.ns_rhs(u, box=box, nx=nx)
    assert abs(inner(u, r, nx)) < 1e-14 * np.sqrt(inner(u, u, nx) * inner(r, r, nx))
    kx, ky, kz = kphys(shape, box)
    assert np.abs(kx * r[0] + ky * r[1] + kz * r[2]).max() < 1e-14 * np.abs(kx).max() * np.abs(r).max()
    b = I.random_solenoidal(0, 6, field=1, shape=shape, box=box)
    nu_, nb_ = O.mhd_rhs(u, b, box=box, nx=nx)
    scale = np.sqrt((inner(u, u, nx) + inner(b, b, nx)) * (inner(nu_, nu_, nx) + inner(nb_, nb_, nx)))
    assert abs(inner(u, nu_, nx) + inner(b, nb_, nx)) < 1e-14 * scale
    assert abs(inner(b, nu_, nx) + inner(u, nb_, nx)) < 1e-14 * scale


# ---------------------------------------------------------------- diagnostics
def test_anisotropic_diagnostics(O):
    """Energy = <|u|^2>/2 on the grid, enstrophy = <|curl u|^2>/2 with the
    curl taken by numpy's FFT in physical space on the physical wavenumbers,
    and a single mode in shell floor(|k| / dk + 1/2), dk = min_i 2 pi / L_i."""
    shape, box = (16, 12, 8), (TWO_PI, np.pi, 4 * np.pi)
    nx, ny, nz = shape
    u = I.random_solenoidal(0, 4, energy=0.37, shape=shape, box=box)
    ur = np.stack([O.c2r3(u[c], nx=nx) for c in range(3)])
    e = O.energy(u, box=box, nx=nx)
    assert abs(e - 0.37) < 1e-14 and abs(0.5 * np.mean(np.sum(ur ** 2, axis=0)) - e) < 1e-14
    ax, ay, az = alphas(box)
    KZ, KY, KX = np.meshgrid(az * np.fft.fftfreq(nz, 1.0 / nz), ay * np.fft.fftfreq(ny, 1.0 / ny),
                             ax * np.fft.fftfreq(nx, 1.0 / nx), indexing="ij")

    def d(f, kk):
        return np.real(np.fft.ifftn(1j * kk * np.fft.fftn(f)))

    w = np.stack([d(ur[2], KY) - d(ur[1], KZ), d(ur[0], KZ) - d(ur[2], KX), d(ur[1], KX) - d(ur[0], KY)])
    z = O.enstrophy(u, box=box, nx=nx)
    assert abs(z - 0.5 * np.mean(np.sum(w ** 2, axis=0))) < 1e-13 * z
    dk = min(ax, ay, az)                      # 0.5 here
    nsh = 40
    s = O.spectrum(u, nsh, box=box, nx=nx)
    assert abs(s.sum() - e) < 1e-14
    v = np.zeros_like(u)
    v[0, 1, 1, 2] = 0.5                       # k = (2 ax, ay, az) = (2, 2, 0.5): |k| = 2.872
    sv = O.spectrum(v, nsh, box=box, nx=nx)
    shell = int(np.floor(np.sqrt(4 + 4 + 0.25) / dk + 0.5))
    assert shell == 6 and sv[shell] == pytest.approx(0.25, abs=1e-16) and abs(sv.sum() - 0.25) < 1e-16


def test_isotropic_box_scaling(O):
    """On a cube of side L the operator is the 2 pi one with every wavenumber
    times 2 pi / L: N scales by that factor for the same coefficients."""
    n = 16
    u = I.random_solenoidal(n, 8)
    r1 = O.ns_rhs(u)
    r2 = O.ns_rhs(u, box=(np.pi, np.pi, np.pi))
    assert np.abs(r2 - 2.0 * r1).max() < 1e-14 * np.abs(r1).max()
