"""Plain FP64 CPU oracle for the pseudospectral Navier-Stokes / MHD / Boussinesq hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.  The arithmetic lives in ``pst_oracle.c``
(plain C, FP64, OpenMP over independent lines); this module only marshals
numpy arrays.

Layouts (both sides of every parity test use the same ones):
  physical  real    [3][n][n][n]       (z, y, x; x fastest)
  spectral  complex [3][n][n][n//2+1]  (kz, ky, kx; kx fastest), coefficients
            normalised so that u(x) = sum_k uhat(k) exp(i k.x).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build as _build

_lib = None


class OraGrid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double), ("az", ctypes.c_double),
        ("kcx", ctypes.c_int), ("kcy", ctypes.c_int), ("kcz", ctypes.c_int),
        ("sphere", ctypes.c_int),
    ]


class OraParams(ctypes.Structure):
    _fields_ = [
        ("g", OraGrid),
        ("solver", ctypes.c_int),
        ("rk_order", ctypes.c_int),
        ("linear_only", ctypes.c_int),
        ("nu", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nbv", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i = ctypes.c_int
        L.ora_dft_naive.argtypes = [i, P, P, i]
        L.ora_fft1d.argtypes = [i, P, i]
        L.ora_r2c3.argtypes = [i, i, i, P, P]
        L.ora_c2r3.argtypes = [i, i, i, P, P]
        L.ora_c2c3.argtypes = [i, i, i, P, i]
        G = ctypes.POINTER(OraGrid)
        d = ctypes.c_double
        L.ora_ns_rhs.argtypes = [G, P, P, P]
        L.ora_mhd_rhs.argtypes = [G, P, P, P, P]
        L.ora_bq_rhs.argtypes = [G, d, P, P, P, P, P]
        L.ora_gpe_rhs.argtypes = [G, d, P, P]
        L.ora_step.argtypes = [ctypes.POINTER(OraParams), P, P, P, i]
        L.ora_step.restype = i
        L.ora_quad.argtypes = [G, i, P, i]
        L.ora_quad.restype = d
        L.ora_spectrum.argtypes = [G, i, P, P, i]
        L.ora_gpe_invariants.argtypes = [G, d, d, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def kcut_23(n: int) -> int:
    """Strict 2/3-rule cutoff K = ceil(n/3) - 1 (alias-free: 3K < n)."""
    return -(-n // 3) - 1


# ---------------------------------------------------------------- transforms
def dft_naive(x, sign=-1):
    x = _c128(x)
    out = np.empty_like(x)
    lib().ora_dft_naive(x.size, _ptr(x), _ptr(out), sign)
    return out


def fft1d(x, sign=-1):
    y = _c128(x).copy()
    lib().ora_fft1d(y.size, _ptr(y), sign)
    return y


def r2c3(a):
    """Forward 3D transform of real [nz][ny][nx] data, scaled by 1/(nx ny nz)."""
    a = _f64(a)
    nz, ny, nx = a.shape
    out = np.empty((nz, ny, nx // 2 + 1), np.complex128)
    lib().ora_r2c3(nz, ny, nx, _ptr(a), _ptr(out))
    return out


def c2r3(a, nx=None):
    """Backward (unscaled) 3D transform of a [nz][ny][nx/2+1] half spectrum."""
    a = _c128(a)
    nz, ny, nxh = a.shape
    if nx is None:
        nx = 2 * (nxh - 1)
    out = np.empty((nz, ny, nx), np.float64)
    lib().ora_c2r3(nz, ny, nx, _ptr(a), _ptr(out))
    return out


def c2c3(a, sign=-1):
    y = _c128(a).copy()
    nz, ny, nx = y.shape
    lib().ora_c2c3(nz, ny, nx, _ptr(y), sign)
    return y


def r2c_vec(u):
    return np.stack([r2c3(u[c]) for c in range(u.shape[0])])


def c2r_vec(uh):
    return np.stack([c2r3(uh[c]) for c in range(uh.shape[0])])


# ------------------------------------------------------------------- grids
TWO_PI = 2.0 * np.pi


def kcut_14(n: int) -> int:
    """Cutoff for a cubic product, K = ceil(n/4) - 1 (alias-free: 4K < n)."""
    return -(-n // 4) - 1


def grid(shape, nx=None, box=None, kcut=None, sphere=False, rule=kcut_23):
    """Grid of a half spectrum [..., nz, ny, nx//2+1] (or, rule=kcut_14 for a
    full complex spectrum, [..., nz, ny, nx]).  box: (Lx, Ly, Lz), default
    2 pi each.  kcut: None (the rule per axis), an int (every axis) or a
    tuple (kx, ky, kz); a negative value removes nothing on that axis."""
    nz, ny, last = shape[-3], shape[-2], shape[-1]
    if nx is None:
        if rule is kcut_14:
            nx = last
        else:
            nx = nz if (nz == ny and last == nz // 2 + 1) else 2 * (last - 1)
    L = (TWO_PI, TWO_PI, TWO_PI) if box is None else box
    if kcut is None:
        kc = (rule(nx), rule(ny), rule(nz))
    elif np.isscalar(kcut):
        kc = (int(kcut),) * 3
    else:
        kc = tuple(int(k) for k in kcut)
    return OraGrid(nx=nx, ny=ny, nz=nz, ax=TWO_PI / L[0], ay=TWO_PI / L[1], az=TWO_PI / L[2],
                   kcx=kc[0], kcy=kc[1], kcz=kc[2], sphere=int(sphere))


# ------------------------------------------------------------------- solvers
def ns_rhs(uhat, fhat=None, kcut=None, sphere=False, box=None, nx=None):
    uhat = _c128(uhat)
    g = grid(uhat.shape, nx, box, kcut, sphere)
    out = np.empty_like(uhat)
    f = _c128(fhat) if fhat is not None else None
    lib().ora_ns_rhs(ctypes.byref(g), _ptr(uhat), _ptr(f) if f is not None else None, _ptr(out))
    return out


def mhd_rhs(uhat, bhat, kcut=None, sphere=False, box=None, nx=None):
    uhat = _c128(uhat)
    bhat = _c128(bhat)
    g = grid(uhat.shape, nx, box, kcut, sphere)
    ou = np.empty_like(uhat)
    ob = np.empty_like(bhat)
    lib().ora_mhd_rhs(ctypes.byref(g), _ptr(uhat), _ptr(bhat), _ptr(ou), _ptr(ob))
    return ou, ob


def bq_rhs(uhat, thhat, nbv, fhat=None, kcut=None, sphere=False, box=None, nx=None):
    """Boussinesq operators (N_u, N_theta); thhat is [nz][ny][nx//2+1] (or [1][...])."""
    uhat = _c128(uhat)
    th = _c128(thhat).reshape(uhat.shape[1:])
    g = grid(uhat.shape, nx, box, kcut, sphere)
    ou = np.empty_like(uhat)
    ot = np.empty_like(th)
    f = _c128(fhat) if fhat is not None else None
    lib().ora_bq_rhs(ctypes.byref(g), float(nbv), _ptr(uhat), _ptr(th),
                     _ptr(f) if f is not None else None, _ptr(ou), _ptr(ot))
    return ou, ot


def gpe_rhs(psihat, beta, kcut=None, box=None):
    """Gross-Pitaevskii nonlinear operator -i beta D F[|psi|^2 psi] of a full
    complex spectrum [nz][ny][nx]; default cutoff ceil(n_i/4) - 1 per axis."""
    psi = _c128(psihat)
    g = grid(psi.shape, None, box, kcut, False, rule=kcut_14)
    out = np.empty_like(psi)
    lib().ora_gpe_rhs(ctypes.byref(g), float(beta), _ptr(psi), _ptr(out))
    return out


def step(uhat, nsteps, *, dt, nu, rk=4, bhat=None, eta=None, fhat=None, kcut=None,
         sphere=False, linear_only=False, theta=None, kappa=None, nbv=0.0, box=None, nx=None):
    """Advance (u, b) or (u, theta) by nsteps Lawson IF-RK steps; returns new
    arrays.  theta (Boussinesq): [nz][ny][nx//2+1], diffusivity kappa (default nu)."""
    u = _c128(uhat).copy()
    if theta is not None:
        b = _c128(theta).reshape(u.shape[1:]).copy()
        solver, e2 = 2, nu if kappa is None else kappa
    else:
        b = _c128(bhat).copy() if bhat is not None else None
        solver, e2 = (1 if b is not None else 0), nu if eta is None else eta
    g = grid(u.shape, nx, box, kcut, sphere)
    p = OraParams(g=g, solver=solver, rk_order=rk, linear_only=int(linear_only), nu=nu, eta=e2, dt=dt,
                  nbv=float(nbv))
    f = _c128(fhat) if fhat is not None else None
    lib().ora_step(ctypes.byref(p), _ptr(u), _ptr(b) if b is not None else None,
                   _ptr(f) if f is not None else None, nsteps)
    return (u, b) if b is not None else u


def gpe_step(psihat, nsteps, *, dt, alpha, beta, rk=4, kcut=None, box=None, linear_only=False):
    """Advance psi (full complex spectrum [nz][ny][nx]) by nsteps Lawson IF-RK
    steps of d psi/dt = i alpha Lap psi - i beta |psi|^2 psi."""
    psi = _c128(psihat).copy()
    g = grid(psi.shape, None, box, kcut, False, rule=kcut_14)
    p = OraParams(g=g, solver=3, rk_order=rk, linear_only=int(linear_only), nu=alpha, eta=0.0, dt=dt,
                  nbv=float(beta))
    lib().ora_step(ctypes.byref(p), _ptr(psi), None, None, nsteps)
    return psi


def gpe_invariants(psihat, alpha, beta, box=None):
    """(particle number, kinetic energy, interaction energy) of psi."""
    psi = _c128(psihat)
    g = grid(psi.shape, None, box, None, False, rule=kcut_14)
    out = np.zeros(3, np.float64)
    lib().ora_gpe_invariants(ctypes.byref(g), float(alpha), float(beta), _ptr(psi), _ptr(out))
    return tuple(out)


def _as_comps(vhat):
    vhat = _c128(vhat)
    return vhat[None] if vhat.ndim == 3 else vhat


def energy(vhat, box=None, nx=None):
    """1/2 sum_k w |vhat|^2 over the components of a [c][nz][ny][nx//2+1] field,
    or of a scalar field given as [nz][ny][nx//2+1]."""
    v = _as_comps(vhat)
    g = grid(v.shape, nx, box)
    return lib().ora_quad(ctypes.byref(g), v.shape[0], _ptr(v), 0)


def enstrophy(vhat, box=None, nx=None):
    """Z = 1/2 sum_k w |k|^2 |vhat|^2 (w = 1 on kx = 0 and kx = nx/2, else 2)."""
    v = _as_comps(vhat)
    g = grid(v.shape, nx, box)
    return lib().ora_quad(ctypes.byref(g), v.shape[0], _ptr(v), 1)


def spectrum(vhat, nshells, box=None, nx=None):
    v = _as_comps(vhat)
    g = grid(v.shape, nx, box)
    out = np.zeros(nshells, np.float64)
    lib().ora_spectrum(ctypes.byref(g), v.shape[0], _ptr(v), _ptr(out), nshells)
    return out
