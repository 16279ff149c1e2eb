"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds input recipes only (initial fields and forcing, given
directly by their Fourier coefficients or by their physical-space formula); it
contains no transform, operator, time step or diagnostic of the method.

Spectral arrays use the library layout: complex [3][n][n][n//2+1] (kz, ky, kx;
kx fastest), coefficients normalised so that u(x) = sum_k uhat(k) exp(i k.x).
Index p on a full axis is the wavenumber p for p < n/2 and p - n otherwise.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw j of mode (kx, ky, kz) of field f under seed s is
mix64(key(s, f, kx, ky, kz) + (j + 1) * GOLDEN), so a field is the same
whatever order the modes are visited in.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def kcut_23(n: int) -> int:
    """Cube-truncation cutoff K = ceil(n/3) - 1 (the largest K with 3K < n)."""
    return -(-n // 3) - 1


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed, field, kx, ky, kz):
    m = np.uint64(0x100000001B3)  # odd multiplier (FNV prime) to chain the counters
    k = np.uint64(seed) * m + np.uint64(field)
    for c in (kx, ky, kz):
        k = k * m + (np.asarray(c, np.int64).astype(np.uint64) & np.uint64(0xFFFF))
    return k


def uniform(seed, field, kx, ky, kz, j):
    """Counter-based uniform draw in [0, 1) (53-bit)."""
    with np.errstate(over="ignore"):
        z = _mix64(_key(seed, field, kx, ky, kz) + np.uint64(j + 1) * GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def wavenumbers(n):
    """Integer wavenumbers of the stored half spectrum, shaped for broadcasting
    against [n][n][n//2+1] (kz, ky, kx)."""
    full = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    kz = full[:, None, None]
    ky = full[None, :, None]
    kx = np.arange(n // 2 + 1)[None, None, :]
    return kx, ky, kz


def cube_mask(n, kcut=None):
    if kcut is None:
        kcut = kcut_23(n)
    kx, ky, kz = wavenumbers(n)
    return (np.abs(kx) <= kcut) & (np.abs(ky) <= kcut) & (np.abs(kz) <= kcut)


def spectrum_c2(k):
    """E(k) proportional to k^4 exp(-2 (k/4)^2) (peak at k = 4)."""
    return k ** 4 * np.exp(-2.0 * (k / 4.0) ** 2)


def spectrum_c3(k):
    """E(k) proportional to k^2 exp(-(k/3)^2)."""
    return k ** 2 * np.exp(-((k / 3.0) ** 2))


def flat_shells(lo, hi):
    """Flat amplitude on shells lo <= floor(|k| + 1/2) <= hi (forcing recipe)."""
    def e(k):
        s = np.floor(k + 0.5)
        return np.where((s >= lo) & (s <= hi), 4.0 * np.pi * k ** 2, 0.0)
    return e


def random_solenoidal(n, seed, field=0, spectrum=spectrum_c2, energy=1.0, kcut=None,
                      dtype=np.complex128, shape=None, box=None):
    """Random-phase solenoidal field in the library's spectral layout.

    For every stored mode k != 0 inside the cube |k_i| <= kcut_i:
        uhat = A(|k|) (exp(i t1) cos(phi) e1 + exp(i t2) sin(phi) e2),
        e1 = k x z / |k x z|  (x if k is parallel to z),  e2 = k x e1 / |k x e1|,
        A = sqrt(E(|k|) / (4 pi |k|^2)),
    with t1, t2, phi uniform in [0, 2 pi) from the counter-based generator
    (keyed by the integer wavenumbers) and k the physical wavenumber
    2 pi (p / Lx, q / Ly, r / Lz).  On the kx = 0 plane the half with ky > 0
    (or ky = 0, kz > 0) is drawn and the other half is its complex conjugate,
    so the field is real.  |uhat| = A whatever the phases, so the amplitudes
    are rescaled to the requested energy 1/2 sum_k w |uhat|^2 (w = 1 on
    kx = 0, else 2) before the phases are applied.  Built one kx plane at a
    time.  shape = (nx, ny, nz) and box = (Lx, Ly, Lz) give an anisotropic
    grid (layout [3][nz][ny][nx//2+1]); kcut is then None or a per-axis tuple.
    """
    nx, ny, nz = (n, n, n) if shape is None else shape
    al = np.array([1.0, 1.0, 1.0]) if box is None else 2.0 * np.pi / np.asarray(box, float)
    if kcut is None:
        kc = (kcut_23(nx), kcut_23(ny), kcut_23(nz))
    elif np.isscalar(kcut):
        kc = (kcut,) * 3
    else:
        kc = tuple(kcut)
    nxh = nx // 2 + 1
    kxmax = min(kc[0], nx // 2)
    out = np.zeros((3, nz, ny, nxh), dtype)
    kz2, ky2 = np.meshgrid(np.arange(-kc[2], kc[2] + 1), np.arange(-kc[1], kc[1] + 1), indexing="ij")
    kz2, ky2 = kz2.ravel(), ky2.ravel()

    def plane(kx):
        if kx == 0:
            keep = (ky2 > 0) | ((ky2 == 0) & (kz2 > 0))
            return ky2[keep], kz2[keep]
        return ky2, kz2

    def phys(kx, ky, kz):
        return al[0] * kx, al[1] * ky, al[2] * kz

    def amp2_of(kx, ky, kz):
        px, py, pz = phys(kx, ky, kz)
        k2 = (px * px + py * py + pz * pz).astype(np.float64)
        return spectrum(np.sqrt(k2)) / (4.0 * np.pi * k2)

    # a canonical kx > 0 mode has weight 2; a canonical kx = 0 mode stands for
    # itself and its mirror, weight 1 each: every canonical mode counts twice
    e_tot = 0.0
    for kx in range(kxmax + 1):
        ky, kz = plane(kx)
        e_tot += float(np.sum(amp2_of(kx, ky, kz)))
    scale = energy / e_tot if e_tot > 0 else 0.0
    for kx in range(kxmax + 1):
        ky, kz = plane(kx)
        kxa = np.full_like(ky, kx)
        amp = np.sqrt(amp2_of(kx, ky, kz) * scale)
        t1 = 2.0 * np.pi * uniform(seed, field, kxa, ky, kz, 0)
        t2 = 2.0 * np.pi * uniform(seed, field, kxa, ky, kz, 1)
        ph = 2.0 * np.pi * uniform(seed, field, kxa, ky, kz, 2)
        kvec = np.stack(phys(kxa, ky, kz)).astype(np.float64)
        # e1 = k x zhat = (ky, -kx, 0), or xhat when k is parallel to zhat
        e1 = np.stack([kvec[1], -kvec[0], np.zeros(ky.shape)])
        par = (kxa == 0) & (ky == 0)
        e1[:, par] = np.array([1.0, 0.0, 0.0])[:, None]
        e1 /= np.sqrt(np.sum(e1 * e1, axis=0))
        e2 = np.stack([kvec[1] * e1[2] - kvec[2] * e1[1], kvec[2] * e1[0] - kvec[0] * e1[2],
                       kvec[0] * e1[1] - kvec[1] * e1[0]])
        e2 /= np.sqrt(np.sum(e2 * e2, axis=0))
        coef = (np.exp(1j * t1) * np.cos(ph))[None] * e1 + (np.exp(1j * t2) * np.sin(ph))[None] * e2
        coef *= amp[None]
        iy, iz = np.mod(ky, ny), np.mod(kz, nz)
        for c in range(3):
            out[c, iz, iy, kx] = coef[c]
            if kx == 0:
                out[c, np.mod(-kz, nz), np.mod(-ky, ny), 0] = np.conj(coef[c])
    return out


def random_wavefunction(shape, seed, field=5, spectrum=spectrum_c3, number=1.0, condensate=0.0, kcut=None,
                        box=None, dtype=np.complex128):
    """Random-phase complex field psi for the Gross-Pitaevskii solver, full
    spectrum layout [nz][ny][nx] (c2c; no Hermitian symmetry).

    For every mode k != 0 inside the cube |k_i| <= kcut_i (default
    ceil(n_i / 4) - 1, the cutoff of a cubic product):
        psihat = A(|k|) exp(i t),  A = sqrt(E(|k|) / (4 pi |k|^2)),
    k the physical wavenumber, t uniform in [0, 2 pi) from the counter-based
    generator (draw 0 of the given field id, keyed by the integer
    wavenumbers); amplitudes scaled so that the fluctuation carries
    (1 - condensate) of the particle number sum_k |psihat|^2 = number, and the
    k = 0 mode (the condensate, real and positive) the rest."""
    nx, ny, nz = shape
    al = np.array([1.0, 1.0, 1.0]) if box is None else 2.0 * np.pi / np.asarray(box, float)
    if kcut is None:
        kc = tuple(-(-m // 4) - 1 for m in shape)
    elif np.isscalar(kcut):
        kc = (kcut,) * 3
    else:
        kc = tuple(kcut)
    kz, ky, kx = np.meshgrid(np.arange(-kc[2], kc[2] + 1), np.arange(-kc[1], kc[1] + 1),
                             np.arange(-kc[0], kc[0] + 1), indexing="ij")
    kz, ky, kx = kz.ravel(), ky.ravel(), kx.ravel()
    nz0 = (kx != 0) | (ky != 0) | (kz != 0)
    kx, ky, kz = kx[nz0], ky[nz0], kz[nz0]
    k2 = (al[0] * kx) ** 2 + (al[1] * ky) ** 2 + (al[2] * kz) ** 2
    a2 = spectrum(np.sqrt(k2)) / (4.0 * np.pi * k2)
    tot = float(np.sum(a2))
    a2 = a2 * ((1.0 - condensate) * number / tot if tot > 0 else 0.0)
    t = 2.0 * np.pi * uniform(seed, field, kx, ky, kz, 0)
    out = np.zeros((nz, ny, nx), dtype)
    out[np.mod(kz, nz), np.mod(ky, ny), np.mod(kx, nx)] = np.sqrt(a2) * np.exp(1j * t)
    out[0, 0, 0] = np.sqrt(condensate * number)
    return out


def plane_wave(shape, k=(1, 0, 0), amp=1.0, dtype=np.complex128):
    """psi = amp exp(i k . x) (integer wavenumber k), full spectrum [nz][ny][nx]."""
    nx, ny, nz = shape
    out = np.zeros((nz, ny, nx), dtype)
    out[k[2] % nz, k[1] % ny, k[0] % nx] = amp
    return out


def random_scalar(n, seed, field=3, spectrum=spectrum_c2, energy=1.0, kcut=None, dtype=np.complex128,
                  shape=None, box=None):
    """Random-phase real scalar field (temperature), spectral layout [n][n][n//2+1].

    For every stored mode k != 0 inside the cube |k_i| <= kcut:
        thetahat = A(|k|) exp(i t),  A = sqrt(E(|k|) / (4 pi |k|^2)),
    t uniform in [0, 2 pi) from the counter-based generator (draw 0 of the
    given field id), the kx = 0 plane Hermitian as in random_solenoidal, and
    the amplitudes scaled to the variance 1/2 sum_k w |thetahat|^2 = energy.
    shape = (nx, ny, nz), box = (Lx, Ly, Lz): anisotropic grid (layout
    [nz][ny][nx//2+1], k the physical wavenumber, kcut None or per axis).
    """
    nx, ny, nz = (n, n, n) if shape is None else shape
    al = np.array([1.0, 1.0, 1.0]) if box is None else 2.0 * np.pi / np.asarray(box, float)
    if kcut is None:
        kc = (kcut_23(nx), kcut_23(ny), kcut_23(nz))
    elif np.isscalar(kcut):
        kc = (kcut,) * 3
    else:
        kc = tuple(kcut)
    nxh = nx // 2 + 1
    out = np.zeros((nz, ny, nxh), dtype)
    kz2, ky2 = np.meshgrid(np.arange(-kc[2], kc[2] + 1), np.arange(-kc[1], kc[1] + 1), indexing="ij")
    kz2, ky2 = kz2.ravel(), ky2.ravel()
    planes = []
    e_tot = 0.0
    for kx in range(min(kc[0], nx // 2) + 1):
        keep = ((ky2 > 0) | ((ky2 == 0) & (kz2 > 0))) if kx == 0 else np.ones(ky2.shape, bool)
        ky, kz = ky2[keep], kz2[keep]
        k2 = ((al[0] * kx) ** 2 + (al[1] * ky) ** 2 + (al[2] * kz) ** 2).astype(np.float64)
        a2 = spectrum(np.sqrt(k2)) / (4.0 * np.pi * k2)
        e_tot += float(np.sum(a2))
        planes.append((kx, ky, kz, a2))
    scale = energy / e_tot if e_tot > 0 else 0.0
    for kx, ky, kz, a2 in planes:
        t = 2.0 * np.pi * uniform(seed, field, np.full_like(ky, kx), ky, kz, 0)
        coef = np.sqrt(a2 * scale) * np.exp(1j * t)
        iy, iz = np.mod(ky, ny), np.mod(kz, nz)
        out[iz, iy, kx] = coef
        if kx == 0:
            out[np.mod(-kz, nz), np.mod(-ky, ny), 0] = np.conj(coef)
    return out


def gravity_wave_spec(n, k=(1, 1, 2), amp_u=0.1, amp_t=0.05, dtype=np.complex128):
    """One internal-gravity-wave mode k (kx > 0) and its implicit conjugate:
    uhat(k) = amp_u e, thetahat(k) = amp_t, with e the unit vector along the
    part of zhat perpendicular to k (the only velocity direction buoyancy
    forces).  Returns (u [3][n][n][n//2+1], theta [n][n][n//2+1])."""
    kx, ky, kz = k
    kv = np.array(k, float)
    e = np.array([0.0, 0.0, 1.0]) - kv * kv[2] / (kv @ kv)
    e /= np.linalg.norm(e)
    u = np.zeros((3, n, n, n // 2 + 1), dtype)
    t = np.zeros((n, n, n // 2 + 1), dtype)
    u[:, kz % n, ky % n, kx] = amp_u * e
    t[kz % n, ky % n, kx] = amp_t
    return u, t


def forcing_shells(n, seed, lo=2, hi=3, energy=1.0, kcut=None, dtype=np.complex128, shape=None, box=None):
    """Constant solenoidal random-phase forcing on shells lo..hi (seed + 1).
    Only the box |k_i| <= hi + 1 can hold those shells, so only it is drawn
    (the draws are keyed by mode, so the result does not depend on the box).
    shape / box: anisotropic grid; the drawn box is then |a_i k_i| <= hi + 1
    on each axis (a_i = 2 pi / L_i), within the axis cutoffs."""
    if shape is None:
        if kcut is None:
            kcut = kcut_23(n)
        return random_solenoidal(n, seed + 1, field=7, spectrum=flat_shells(lo, hi),
                                 energy=energy, kcut=min(kcut, hi + 1), dtype=dtype)
    al = [1.0, 1.0, 1.0] if box is None else [2.0 * np.pi / L for L in box]
    kc = [kcut_23(m) for m in shape] if kcut is None else list(kcut)
    kc = tuple(min(kc[i], int(np.ceil((hi + 1) / al[i]))) for i in range(3))
    return random_solenoidal(0, seed + 1, field=7, spectrum=flat_shells(lo, hi), energy=energy, kcut=kc,
                             dtype=dtype, shape=shape, box=box)


# ------------------------------------------------------------ analytic fields
def taylor_green_phys(n, dtype=np.float64):
    """u = (sin x cos y cos z, -cos x sin y cos z, 0) on the grid x_j = 2 pi j / n."""
    x = 2.0 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)])
    return u.astype(dtype)


def taylor_green_spec(n, dtype=np.complex128):
    """Fourier coefficients of the Taylor-Green field: on kx = 1,
    uhat_x(1, sy, sz) = -i/8 and uhat_y(1, sy, sz) = i sy / 8 for sy, sz = +-1."""
    out = np.zeros((3, n, n, n // 2 + 1), dtype)
    for sy in (1, -1):
        for sz in (1, -1):
            out[0, sz % n, sy % n, 1] = -1j / 8
            out[1, sz % n, sy % n, 1] = 1j * sy / 8
    return out


def abc_spec(n, A=1.0, B=1.0, C=1.0, dtype=np.complex128):
    """Arnold-Beltrami-Childress flow u = (A sin z + C cos y, B sin x + A cos z,
    C sin y + B cos x) by its Fourier coefficients (curl u = u)."""
    out = np.zeros((3, n, n, n // 2 + 1), dtype)
    # sin z = (e^{iz} - e^{-iz}) / 2i ; cos y = (e^{iy} + e^{-iy}) / 2 (kx = 0 plane: both)
    out[0, 1, 0, 0] += A / 2j
    out[0, n - 1, 0, 0] += -A / 2j
    out[0, 0, 1, 0] += C / 2
    out[0, 0, n - 1, 0] += C / 2
    out[1, 0, 0, 1] += B / 2j            # sin x, kx = 1 only in the half spectrum
    out[1, 1, 0, 0] += A / 2
    out[1, n - 1, 0, 0] += A / 2
    out[2, 0, 1, 0] += C / 2j
    out[2, 0, n - 1, 0] += -C / 2j
    out[2, 0, 0, 1] += B / 2             # cos x
    return out


def shear_wave_spec(n, k=1, amp=1.0, dtype=np.complex128):
    """u = amp sin(k z) xhat."""
    out = np.zeros((3, n, n, n // 2 + 1), dtype)
    out[0, k % n, 0, 0] = amp / 2j
    out[0, (-k) % n, 0, 0] = -amp / 2j
    return out


def alfven_spec(n, k=1, amp=0.1, b0=1.0, dtype=np.complex128):
    """Alfven wave on a mean field b0 zhat: u = amp cos(k z) xhat,
    b = b0 zhat - amp cos(k z) xhat.  Returns (uhat, bhat)."""
    u = np.zeros((3, n, n, n // 2 + 1), dtype)
    u[0, k % n, 0, 0] = amp / 2
    u[0, (-k) % n, 0, 0] = amp / 2
    b = -u.copy()
    b[2, 0, 0, 0] = b0
    return u, b


# ------------------------------------------------------------ surrogate weights
def fno_param_count(n, width, modes, layers, hidden):
    """Length of the flat parameter vector of the Fourier neural operator:
    lift W [width][3], b [width]; per layer Wc [width][width], bc [width],
    R [(2 modes)^2 modes][width in][width out][re, im]; projection
    Wq1 [hidden][width], bq1 [hidden], Wq2 [3][hidden], bq2 [3]."""
    nm = (2 * modes) ** 2 * modes
    return width * 3 + width + layers * (width * width + width + nm * width * width * 2) + \
        hidden * width + hidden + 3 * hidden + 3


def fno_init_params(n, width, modes, layers, hidden, seed=0, out_scale=0.01):
    """Seeded initial parameters (numpy generator, float64), flat layout above:
    dense weights N(0, 1/fan_in) (the last one times out_scale, so the
    residual output starts close to the identity), biases 0, spectral weights
    uniform in [0, 1) + i [0, 1) over width^2."""
    rng = np.random.default_rng(seed)
    nm = (2 * modes) ** 2 * modes
    parts = [rng.standard_normal((width, 3)) / np.sqrt(3.0), np.zeros(width)]
    for _ in range(layers):
        parts += [rng.standard_normal((width, width)) / np.sqrt(width), np.zeros(width),
                  rng.random((nm, width, width, 2)) / (width * width)]
    parts += [rng.standard_normal((hidden, width)) / np.sqrt(width), np.zeros(hidden),
              out_scale * rng.standard_normal((3, hidden)) / np.sqrt(hidden), np.zeros(3)]
    theta = np.concatenate([p.reshape(-1) for p in parts])
    assert theta.size == fno_param_count(n, width, modes, layers, hidden)
    return theta
