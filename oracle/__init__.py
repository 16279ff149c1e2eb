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


class OraParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("solver", ctypes.c_int),
        ("rk_order", ctypes.c_int),
        ("kcut", ctypes.c_int),
        ("sphere", ctypes.c_int),
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
        L.ora_ns_rhs.argtypes = [i, i, i, P, P, P]
        L.ora_mhd_rhs.argtypes = [i, i, i, P, P, P, P]
        L.ora_bq_rhs.argtypes = [i, i, i, ctypes.c_double, P, P, P, P, P]
        L.ora_energy_nc.argtypes = [i, i, P]
        L.ora_energy_nc.restype = ctypes.c_double
        L.ora_step.argtypes = [ctypes.POINTER(OraParams), P, P, P, i]
        L.ora_step.restype = i
        L.ora_energy.argtypes = [i, P]
        L.ora_energy.restype = ctypes.c_double
        L.ora_enstrophy.argtypes = [i, P]
        L.ora_enstrophy.restype = ctypes.c_double
        L.ora_spectrum.argtypes = [i, P, P, i]
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


# ------------------------------------------------------------------- solvers
def ns_rhs(uhat, fhat=None, kcut=None, sphere=False):
    uhat = _c128(uhat)
    n = uhat.shape[1]
    if kcut is None:
        kcut = kcut_23(n)
    out = np.empty_like(uhat)
    f = _c128(fhat) if fhat is not None else None
    lib().ora_ns_rhs(n, kcut, int(sphere), _ptr(uhat), _ptr(f) if f is not None else None, _ptr(out))
    return out


def mhd_rhs(uhat, bhat, kcut=None, sphere=False):
    uhat = _c128(uhat)
    bhat = _c128(bhat)
    n = uhat.shape[1]
    if kcut is None:
        kcut = kcut_23(n)
    ou = np.empty_like(uhat)
    ob = np.empty_like(bhat)
    lib().ora_mhd_rhs(n, kcut, int(sphere), _ptr(uhat), _ptr(bhat), _ptr(ou), _ptr(ob))
    return ou, ob


def bq_rhs(uhat, thhat, nbv, fhat=None, kcut=None, sphere=False):
    """Boussinesq operators (N_u, N_theta); thhat is [n][n][n//2+1] (or [1][...])."""
    uhat = _c128(uhat)
    th = _c128(thhat).reshape(uhat.shape[1:])
    n = uhat.shape[1]
    if kcut is None:
        kcut = kcut_23(n)
    ou = np.empty_like(uhat)
    ot = np.empty_like(th)
    f = _c128(fhat) if fhat is not None else None
    lib().ora_bq_rhs(n, kcut, int(sphere), float(nbv), _ptr(uhat), _ptr(th),
                     _ptr(f) if f is not None else None, _ptr(ou), _ptr(ot))
    return ou, ot


def step(uhat, nsteps, *, dt, nu, rk=4, bhat=None, eta=None, fhat=None, kcut=None,
         sphere=False, linear_only=False, theta=None, kappa=None, nbv=0.0):
    """Advance (u, b) or (u, theta) by nsteps Lawson IF-RK steps; returns new
    arrays.  theta (Boussinesq): [n][n][n//2+1], diffusivity kappa (default nu)."""
    u = _c128(uhat).copy()
    n = u.shape[1]
    if theta is not None:
        b = _c128(theta).reshape(u.shape[1:]).copy()
        solver, e2 = 2, nu if kappa is None else kappa
    else:
        b = _c128(bhat).copy() if bhat is not None else None
        solver, e2 = (1 if b is not None else 0), nu if eta is None else eta
    p = OraParams(n=n, solver=solver, rk_order=rk,
                  kcut=kcut_23(n) if kcut is None else kcut, sphere=int(sphere),
                  linear_only=int(linear_only), nu=nu, eta=e2, dt=dt, nbv=float(nbv))
    f = _c128(fhat) if fhat is not None else None
    lib().ora_step(ctypes.byref(p), _ptr(u), _ptr(b) if b is not None else None,
                   _ptr(f) if f is not None else None, nsteps)
    return (u, b) if b is not None else u


def energy(vhat):
    """1/2 sum_k w |vhat|^2 over the components of a [3][n][n][n//2+1] field, or
    of a scalar field given as [n][n][n//2+1] or [1][n][n][n//2+1]."""
    vhat = _c128(vhat)
    if vhat.ndim == 3:
        vhat = vhat[None]
    return lib().ora_energy_nc(vhat.shape[1], vhat.shape[0], _ptr(vhat))


def enstrophy(vhat):
    """Z = 1/2 sum_k w |k|^2 |vhat|^2 (w = 1 on kx = 0 and kx = n/2, else 2)."""
    vhat = _c128(vhat)
    return lib().ora_enstrophy(vhat.shape[1], _ptr(vhat))


def spectrum(vhat, nshells):
    vhat = _c128(vhat)
    out = np.zeros(nshells, np.float64)
    lib().ora_spectrum(vhat.shape[1], _ptr(vhat), _ptr(out), nshells)
    return out
