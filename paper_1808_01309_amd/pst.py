"""ctypes binding over the C ABI of libpst.so (include/pst.h).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module loads libpst.so and raises ImportError if it is missing
(build it with ``python -m paper_1808_01309_amd.build``); there is no fallback.

Device buffers are passed as torch tensors (PyTorch provides device memory and
the current HIP stream); host buffers as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# PyTorch ships its own HIP runtime (same soname as the system one).  Loading
# torch first makes libpst.so bind to that runtime, so the process holds a
# single HIP runtime and device pointers / streams from torch are valid here.
import torch  # noqa: E402,F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpst.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: the HIP library has not been built")
lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ ABI types
PST_OK, PST_ERR_INVALID_ARG, PST_ERR_UNSUPPORTED_N, PST_ERR_OOM, PST_ERR_HIP, PST_ERR_NONFINITE, \
    PST_ERR_UNSUPPORTED = range(7)
PST_NS, PST_MHD, PST_BOUSSINESQ, PST_GPE = 0, 1, 2, 3
PST_FP32, PST_FP64 = 0, 1
PST_FIELD_U, PST_FIELD_B, PST_FIELD_THETA, PST_FIELD_PSI = 0, 1, 2, 3
_FIELDS = {"u": PST_FIELD_U, "b": PST_FIELD_B, "theta": PST_FIELD_THETA, "psi": PST_FIELD_PSI}
_SOLVERS = {"ns": PST_NS, "mhd": PST_MHD, "boussinesq": PST_BOUSSINESQ, "gpe": PST_GPE}
PST_SPACE_PHYS, PST_SPACE_SPEC = 0, 1
PST_MEM_HOST, PST_MEM_DEVICE = 0, 1
PST_FLAG_LINEAR_ONLY, PST_FLAG_TIMERS = 1, 2
KERNEL_KINDS = ["zinv", "yinv", "xpass", "yfwd", "zfwd", "fftx", "ffty", "fftz", "other"]


class pst_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("solver", ctypes.c_int), ("precision", ctypes.c_int),
                ("rk_order", ctypes.c_int), ("nu", ctypes.c_double), ("eta", ctypes.c_double),
                ("dt", ctypes.c_double), ("dealias", ctypes.c_int), ("flags", ctypes.c_uint),
                ("nbv", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class pst_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("kcut", ctypes.c_int), ("ncomp", ctypes.c_int),
                ("modes_per_comp", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("radices", ctypes.c_int * 4), ("tile_lines", ctypes.c_int),
                ("steps_done", ctypes.c_longlong), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("kcut_x", ctypes.c_int), ("kcut_y", ctypes.c_int),
                ("nshells", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_S = ctypes.c_int  # pst_status
lib.pst_status_str.argtypes = [_S]
lib.pst_status_str.restype = ctypes.c_char_p
lib.pst_last_error.argtypes = [_P]
lib.pst_last_error.restype = ctypes.c_char_p
lib.pst_supported_n.argtypes = [_I]
lib.pst_supported_n.restype = _I
lib.pst_plan_create.argtypes = [ctypes.POINTER(pst_params), _P, ctypes.POINTER(_P)]
lib.pst_plan_create.restype = _S
lib.pst_plan_destroy.argtypes = [_P]
lib.pst_plan_destroy.restype = None
for _name, _args in [("pst_set_state", [_P, _I, _I, _P, _I]), ("pst_get_state", [_P, _I, _I, _P, _I]),
                     ("pst_set_forcing", [_P, _P, _I]), ("pst_rhs", [_P, _P, _P]), ("pst_step", [_P, _I]),
                     ("pst_energy", [_P, _P]), ("pst_enstrophy", [_P, _P]), ("pst_spectrum", [_P, _I, _P, _I]),
                     ("pst_fft_r2c", [_P, _P, _P, _I]), ("pst_fft_c2r", [_P, _P, _P, _I]),
                     ("pst_query", [_P, ctypes.POINTER(pst_info)]),
                     ("pst_timer_read", [_P, _P, _P, _I])]:
    getattr(lib, _name).argtypes = _args
    getattr(lib, _name).restype = _S

lib.pst_project.argtypes = [_P, _P, _I, _P, _P]
lib.pst_project.restype = _S
lib.pst_fft_c2r_noalloc.argtypes = [_I, _I, _P, _P, _I, _P]
lib.pst_fft_c2r_noalloc.restype = _S
lib.pst_fft_c2r_noalloc_bytes.argtypes = [_I, _I, _I]
lib.pst_fft_c2r_noalloc_bytes.restype = ctypes.c_size_t

_ens_sigs = [("pst_ensemble_create", [_I, _P, ctypes.POINTER(pst_params), _P, ctypes.POINTER(_P)]),
             ("pst_ensemble_set_state", [_P, _I, _P, _I]), ("pst_ensemble_get_state", [_P, _I, _P, _I]),
             ("pst_ensemble_step", [_P, _I]), ("pst_ensemble_set_mode", [_P, _I]),
             ("pst_ensemble_get_mode", [_P, _P]),
             ("pst_ensemble_energy", [_P, _P]), ("pst_ensemble_autotune", [_P, ctypes.c_char_p, _I, _P]),
             ("pst_ensemble_set_schedule", [_P, _I]), ("pst_ensemble_query", [_P, _P, _P, _P, _P, _P]),
             ("pst_ensemble_set_class_schedule", [_P, _I, _I]), ("pst_ensemble_class_schedules", [_P, _P]),
             ("pst_ensemble_project", [_P]), ("pst_ensemble_diagnostics", [_P, _P, _P]),
             ("pst_ensemble_rel_l2", [_P, _P, _P]),
             ("pst_ensemble_set_spin_limit", [_P, ctypes.c_longlong])]
for _name, _args in _ens_sigs:
    getattr(lib, _name).argtypes = _args
    getattr(lib, _name).restype = _S
lib.pst_ensemble_destroy.argtypes = [_P]
lib.pst_ensemble_destroy.restype = None
lib.pst_ensemble_last_error.argtypes = [_P]
lib.pst_ensemble_last_error.restype = ctypes.c_char_p

class pst_fno_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("width", ctypes.c_int), ("modes", ctypes.c_int), ("layers", ctypes.c_int),
                ("hidden", ctypes.c_int), ("batch", ctypes.c_int), ("mfma", ctypes.c_int)]


for _name, _args in [("pst_fno_create", [ctypes.POINTER(pst_fno_params), _P, ctypes.POINTER(_P)]),
                     ("pst_fno_param_count", [_P, ctypes.POINTER(ctypes.c_longlong)]),
                     ("pst_fno_set_params", [_P, _P, _I]), ("pst_fno_get_params", [_P, _P, _I]),
                     ("pst_fno_get_grad", [_P, _P, _I]), ("pst_fno_forward", [_P, _P, _P, _I]),
                     ("pst_fno_loss_grad", [_P, _P, _P, _I, ctypes.POINTER(ctypes.c_double)]),
                     ("pst_fno_adam", [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
                     ("pst_fno_train_step", [_P, _P, _P, _I, ctypes.c_float, ctypes.POINTER(ctypes.c_double)])]:
    getattr(lib, _name).argtypes = _args
    getattr(lib, _name).restype = _S
lib.pst_fno_destroy.argtypes = [_P]
lib.pst_fno_destroy.restype = None
lib.pst_fno_last_error.argtypes = [_P]
lib.pst_fno_last_error.restype = ctypes.c_char_p

EXPORTED = ["pst_fno_create", "pst_fno_destroy", "pst_fno_last_error", "pst_fno_param_count", "pst_fno_set_params",
            "pst_fno_get_params", "pst_fno_get_grad", "pst_fno_forward", "pst_fno_loss_grad", "pst_fno_adam",
            "pst_fno_train_step",
            "pst_ensemble_create", "pst_ensemble_destroy", "pst_ensemble_last_error", "pst_ensemble_set_state",
            "pst_ensemble_get_state", "pst_ensemble_step", "pst_ensemble_set_mode", "pst_ensemble_get_mode",
            "pst_ensemble_energy",
            "pst_ensemble_autotune", "pst_ensemble_set_schedule", "pst_ensemble_query", "pst_ensemble_project",
            "pst_ensemble_set_class_schedule", "pst_ensemble_class_schedules",
            "pst_ensemble_diagnostics", "pst_ensemble_rel_l2", "pst_ensemble_set_spin_limit",
            "pst_status_str", "pst_last_error", "pst_supported_n", "pst_plan_create", "pst_plan_destroy",
            "pst_set_state", "pst_get_state", "pst_set_forcing", "pst_rhs", "pst_step", "pst_energy", "pst_enstrophy",
            "pst_spectrum", "pst_fft_r2c", "pst_fft_c2r", "pst_query", "pst_timer_read",
            "pst_fft_c2r_noalloc", "pst_fft_c2r_noalloc_bytes", "pst_project"]


class PstError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib.pst_status_str(status).decode()}: {msg}")
        self.status = status


def kcut_23(n):
    return -(-n // 3) - 1


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(x):
    """Device pointer of a torch tensor, or host pointer of a numpy array."""
    if x is None:
        return None, PST_MEM_HOST
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("host array must be C-contiguous")
        return ctypes.c_void_p(x.ctypes.data), PST_MEM_HOST
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(x.data_ptr()), (PST_MEM_DEVICE if x.is_cuda else PST_MEM_HOST)


def _check_buf(x, dtype, numel, what, device=None):
    """Validate a buffer handed to a C call that reads or writes a fixed byte
    count: element type, element count, contiguity and (device=True) that a
    torch tensor lives on the GPU.  Raises ValueError on a mismatch."""
    if isinstance(x, np.ndarray):
        if device:
            raise ValueError(f"{what}: expected a device tensor, got a numpy array")
        if x.dtype != np.dtype(dtype):
            raise ValueError(f"{what}: dtype {x.dtype}, expected {np.dtype(dtype)}")
        n = x.size
    else:
        if device is not None and bool(x.is_cuda) != bool(device):
            raise ValueError(f"{what}: tensor on {x.device}, expected {'a GPU' if device else 'the host'}")
        if _np_dtype(x) != np.dtype(dtype):
            raise ValueError(f"{what}: dtype {x.dtype}, expected {np.dtype(dtype)}")
        n = x.numel()
    if n != numel:
        raise ValueError(f"{what}: {n} elements, expected {numel}")


class Plan:
    """One solver plan (pst_plan_create ... pst_plan_destroy)."""

    def __init__(self, n, solver="ns", precision="fp32", rk_order=4, nu=0.0, eta=None, dt=1e-3,
                 linear_only=False, timers=False, stream=None, dealias="cube", kappa=None, nbv=0.0,
                 alpha=0.0, beta=0.0, shape=None, box=None):
        """solver: "ns", "mhd" (eta: magnetic diffusivity), "boussinesq"
        (kappa: scalar diffusivity, default nu; nbv: Brunt-Vaisala frequency)
        or "gpe" (d psi/dt = i alpha Lap psi - i beta |psi|^2 psi).
        shape = (nx, ny, nz) and box = (Lx, Ly, Lz) give an anisotropic grid
        (n is then ignored where shape is given); default n^3 on [0, 2 pi)^3."""
        nx, ny, nz = (n, n, n) if shape is None else shape
        lx, ly, lz = (0.0, 0.0, 0.0) if box is None else box
        second = kappa if solver == "boussinesq" else eta
        p = pst_params(n=n, solver=_SOLVERS[solver],
                       precision=PST_FP64 if precision == "fp64" else PST_FP32, rk_order=rk_order,
                       nu=nu, eta=nu if second is None else second, dt=dt,
                       dealias={"cube": 0, "sphere": 1, "none": 2}[dealias],
                       flags=(PST_FLAG_LINEAR_ONLY if linear_only else 0) | (PST_FLAG_TIMERS if timers else 0),
                       nbv=nbv, alpha=alpha, beta=beta, nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz)
        self.params = p
        self.n = nz
        self.shape = (nx, ny, nz)
        self.fp64 = precision == "fp64"
        self.mhd = solver == "mhd"
        self.solver = solver
        self.ncomp = {"ns": 3, "mhd": 6, "boussinesq": 4, "gpe": 1}[solver]
        self.gpe = solver == "gpe"
        self.real_np = np.float64 if self.fp64 else np.float32
        self.cplx_np = np.complex128 if self.fp64 else np.complex64
        h = _P()
        s = lib.pst_plan_create(ctypes.byref(p), _P(_stream_handle(stream)), ctypes.byref(h))
        if s != PST_OK:
            raise PstError(s, lib.pst_last_error(None).decode())
        self._h = h

    # --------------------------------------------------------------- helpers
    def _check(self, s):
        if s != PST_OK:
            raise PstError(s, lib.pst_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.pst_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def spec_shape(self, ncomp=3):
        # GPE: the whole spectrum of a complex field
        nx, ny, nz = self.shape
        return (ncomp, nz, ny, nx if self.gpe else nx // 2 + 1)

    def phys_shape(self, ncomp=3):
        nx, ny, nz = self.shape
        return (ncomp, nz, ny, nx)

    def _phys_np(self):
        return self.cplx_np if self.gpe else self.real_np

    def _field_nc(self, field):
        return 1 if field in ("theta", "psi") else 3

    # --------------------------------------------------------------- ABI calls
    def set_state(self, data, field=None, space=None):
        """data: numpy (host) or torch (device) array, spectral complex
        [nc][n][n][n/2+1] or physical real [nc][n][n][n] (nc = 3 for u and b,
        1 for theta, which may also be given without the leading axis).  GPE
        (field psi): spectral complex [1][n][n][n], physical complex
        [1][n][n][n]; space must then be given for physical data."""
        if field is None:
            field = "psi" if self.gpe else "u"
        f = _FIELDS[field]
        if space is None:
            space = "spec" if (self.gpe or np.iscomplexobj(np.empty(0, dtype=_np_dtype(data)))) else "phys"
        pdt = self.cplx_np if space == "spec" else self._phys_np()
        if isinstance(data, np.ndarray):
            data = np.ascontiguousarray(data, pdt)
        nc = self._field_nc(field)
        shape = self.spec_shape(nc) if space == "spec" else self.phys_shape(nc)
        _check_buf(data, pdt, int(np.prod(shape)), "set_state")
        ptr, mem = _ptr(data)
        self._check(lib.pst_set_state(self._h, f, PST_SPACE_SPEC if space == "spec" else PST_SPACE_PHYS,
                                      ptr, mem))

    def get_state(self, field=None, space="spec", out=None):
        if field is None:
            field = "psi" if self.gpe else "u"
        f = _FIELDS[field]
        sp = PST_SPACE_SPEC if space == "spec" else PST_SPACE_PHYS
        nc = self._field_nc(field)
        pdt = self.cplx_np if space == "spec" else self._phys_np()
        shape = self.spec_shape(nc) if space == "spec" else self.phys_shape(nc)
        if out is None:
            out = np.empty(shape, pdt)
        _check_buf(out, pdt, int(np.prod(shape)), "get_state")
        ptr, mem = _ptr(out)
        self._check(lib.pst_get_state(self._h, f, sp, ptr, mem))
        return out

    def set_forcing(self, fhat):
        if fhat is None:
            self._check(lib.pst_set_forcing(self._h, None, PST_MEM_HOST))
            return
        if isinstance(fhat, np.ndarray):
            fhat = np.ascontiguousarray(fhat, self.cplx_np)
        _check_buf(fhat, self.cplx_np, int(np.prod(self.spec_shape(3))), "set_forcing")
        ptr, mem = _ptr(fhat)
        self._check(lib.pst_set_forcing(self._h, ptr, mem))

    def rhs(self, state_dev, rhs_dev):
        m = int(np.prod(self.spec_shape(self.ncomp)))
        _check_buf(state_dev, self.cplx_np, m, "rhs state", device=True)
        _check_buf(rhs_dev, self.cplx_np, m, "rhs output", device=True)
        a, _ = _ptr(state_dev)
        b, _ = _ptr(rhs_dev)
        self._check(lib.pst_rhs(self._h, a, b))

    def step(self, nsteps=1):
        self._check(lib.pst_step(self._h, nsteps))

    def energy(self):
        out = np.zeros(2, np.float64)
        self._check(lib.pst_energy(self._h, out.ctypes.data_as(_P)))
        return float(out[0]), float(out[1])

    def enstrophy(self):
        out = np.zeros(2, np.float64)
        self._check(lib.pst_enstrophy(self._h, out.ctypes.data_as(_P)))
        return float(out[0]), float(out[1])

    def spectrum(self, field=None, nshells=None):
        if field is None:
            field = "psi" if self.gpe else "u"
        if nshells is None:
            nshells = self.query()["nshells"]
        out = np.zeros(nshells, np.float64)
        self._check(lib.pst_spectrum(self._h, _FIELDS[field], out.ctypes.data_as(_P), nshells))
        return out

    def fft_r2c(self, x, out, nfields):
        _check_buf(x, self.real_np, nfields * int(np.prod(self.phys_shape(1))), "fft_r2c input", device=True)
        _check_buf(out, self.cplx_np, nfields * int(np.prod(self.spec_shape(1))), "fft_r2c output", device=True)
        a, _ = _ptr(x)
        b, _ = _ptr(out)
        self._check(lib.pst_fft_r2c(self._h, a, b, nfields))

    def fft_c2r(self, x, out, nfields):
        _check_buf(x, self.cplx_np, nfields * int(np.prod(self.spec_shape(1))), "fft_c2r input", device=True)
        _check_buf(out, self.real_np, nfields * int(np.prod(self.phys_shape(1))), "fft_c2r output", device=True)
        a, _ = _ptr(x)
        b, _ = _ptr(out)
        self._check(lib.pst_fft_c2r(self._h, a, b, nfields))

    def project(self, spec_dev, ngroups, diagnostics=True):
        """Dealias and project ngroups 3-component spectral fields in place
        (device [ngroups][3][nz][ny][nx/2+1]); with diagnostics, returns the
        energy and enstrophy of every group (numpy arrays)."""
        _check_buf(spec_dev, self.cplx_np, ngroups * int(np.prod(self.spec_shape(3))), "project", device=True)
        if not diagnostics:
            self._check(lib.pst_project(self._h, _ptr(spec_dev)[0], ngroups, None, None))
            return None
        e = np.zeros(ngroups, np.float64)
        z = np.zeros(ngroups, np.float64)
        self._check(lib.pst_project(self._h, _ptr(spec_dev)[0], ngroups, e.ctypes.data_as(_P), z.ctypes.data_as(_P)))
        return e, z

    def query(self):
        info = pst_info()
        self._check(lib.pst_query(self._h, ctypes.byref(info)))
        return {"n": info.n, "kcut": info.kcut, "ncomp": info.ncomp,
                "modes_per_comp": info.modes_per_comp, "workspace_bytes": info.workspace_bytes,
                "radices": [r for r in info.radices if r], "tile_lines": info.tile_lines,
                "steps_done": info.steps_done, "shape": (info.nx, info.ny, info.nz),
                "kcuts": (info.kcut_x, info.kcut_y, info.kcut), "nshells": info.nshells}

    def timers(self, reset=True):
        ms = np.zeros(len(KERNEL_KINDS), np.float64)
        cnt = np.zeros(len(KERNEL_KINDS), np.int64)
        self._check(lib.pst_timer_read(self._h, ms.ctypes.data_as(_P), cnt.ctypes.data_as(_P), int(reset)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}


def fft_c2r_noalloc(n, x, out, nfields, precision="fp32", stream=None):
    """pst_fft_c2r_noalloc: the unpruned 3D c2r transform of nfields fields
    without a plan or any device allocation (its workspace is the library's
    static per-GPU scratch array; calls overlapping on one GPU race)."""
    fp64 = precision == "fp64"
    cn, rn = (np.complex128, np.float64) if fp64 else (np.complex64, np.float32)
    _check_buf(x, cn, nfields * n * n * (n // 2 + 1), "fft_c2r_noalloc input", device=True)
    _check_buf(out, rn, nfields * n * n * n, "fft_c2r_noalloc output", device=True)
    s = lib.pst_fft_c2r_noalloc(n, PST_FP64 if fp64 else PST_FP32, _ptr(x)[0], _ptr(out)[0], nfields,
                                _P(_stream_handle(stream)))
    if s != PST_OK:
        raise PstError(s, lib.pst_last_error(None).decode())


def fft_c2r_noalloc_bytes(n, nfields, precision="fp32"):
    return int(lib.pst_fft_c2r_noalloc_bytes(n, PST_FP64 if precision == "fp64" else PST_FP32, nfields))


def _np_dtype(x):
    if isinstance(x, np.ndarray):
        return x.dtype
    import torch
    return {torch.complex64: np.complex64, torch.complex128: np.complex128,
            torch.float32: np.float32, torch.float64: np.float64}[x.dtype]


ENS_MODES = {"graph": 0, "persistent": 1, "batched": 2, "sequential": 3, "batched_graph": 4}


class Ensemble:
    """Independent Navier-Stokes runs of uneven n (pst_ensemble_*), FP32."""

    def __init__(self, sizes, rk_order=4, nu=1e-2, dt=1e-3, stream=None):
        self.sizes = list(sizes)
        p = pst_params(n=0, solver=PST_NS, precision=PST_FP32, rk_order=rk_order, nu=nu, eta=nu, dt=dt,
                       dealias=0, flags=0)
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        h = _P()
        s = lib.pst_ensemble_create(len(self.sizes), arr, ctypes.byref(p), _P(_stream_handle(stream)),
                                    ctypes.byref(h))
        if s != PST_OK:
            raise PstError(s, lib.pst_ensemble_last_error(None).decode())
        self._h = h

    def _check(self, s):
        if s != PST_OK:
            raise PstError(s, lib.pst_ensemble_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.pst_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_run_buf(self, run, buf, what):
        # an out-of-range run is left to the library, which reports it
        if 0 <= run < len(self.sizes):
            n = self.sizes[run]
            _check_buf(buf, np.complex64, 3 * n * n * (n // 2 + 1), what)

    def set_state(self, run, uhat):
        if isinstance(uhat, np.ndarray):
            uhat = np.ascontiguousarray(uhat, np.complex64)
        self._check_run_buf(run, uhat, "ensemble set_state")
        ptr, mem = _ptr(uhat)
        self._check(lib.pst_ensemble_set_state(self._h, run, ptr, mem))

    def get_state(self, run, out=None):
        n = self.sizes[run]
        if out is None:
            out = np.empty((3, n, n, n // 2 + 1), np.complex64)
        self._check_run_buf(run, out, "ensemble get_state")
        ptr, mem = _ptr(out)
        self._check(lib.pst_ensemble_get_state(self._h, run, ptr, mem))
        return out

    def set_mode(self, mode):
        self._check(lib.pst_ensemble_set_mode(self._h, ENS_MODES.get(mode, mode)))

    def step(self, nsteps=1):
        self._check(lib.pst_ensemble_step(self._h, nsteps))

    def energy(self):
        out = np.zeros(len(self.sizes), np.float64)
        self._check(lib.pst_ensemble_energy(self._h, out.ctypes.data_as(_P)))
        return out

    def project(self):
        self._check(lib.pst_ensemble_project(self._h))

    def diagnostics(self):
        e = np.zeros(len(self.sizes), np.float64)
        z = np.zeros(len(self.sizes), np.float64)
        self._check(lib.pst_ensemble_diagnostics(self._h, e.ctypes.data_as(_P), z.ctypes.data_as(_P)))
        return e, z

    def rel_l2(self, other):
        out = np.zeros(len(self.sizes), np.float64)
        self._check(lib.pst_ensemble_rel_l2(self._h, other._h, out.ctypes.data_as(_P)))
        return out

    def autotune(self, cache_path=None, force=False):
        v = ctypes.c_int(-1)
        self._check(lib.pst_ensemble_autotune(self._h, cache_path.encode() if cache_path else None, int(force),
                                              ctypes.byref(v)))
        return v.value

    def set_schedule(self, variant):
        self._check(lib.pst_ensemble_set_schedule(self._h, variant))

    def set_class_schedule(self, cls, variant):
        """Variant of one size class's batched / sequential launches."""
        self._check(lib.pst_ensemble_set_class_schedule(self._h, int(cls), int(variant)))

    def class_schedules(self):
        nc = self.query()["sizes"]
        out = (ctypes.c_int * max(len(nc), 1))()
        self._check(lib.pst_ensemble_class_schedules(self._h, out))
        return list(out[:len(nc)])

    def set_spin_limit(self, polls):
        """Test only: polls of a device-wide barrier before it reports a timeout."""
        self._check(lib.pst_ensemble_set_spin_limit(self._h, int(polls)))

    def get_mode(self):
        m = ctypes.c_int(-1)
        self._check(lib.pst_ensemble_get_mode(self._h, ctypes.byref(m)))
        return {v: k for k, v in ENS_MODES.items()}.get(m.value, m.value)

    def query(self):
        nc = ctypes.c_int()
        cn = (ctypes.c_int * 4)()
        cr = (ctypes.c_int * 4)()
        var = ctypes.c_int()
        grid = ctypes.c_int()
        self._check(lib.pst_ensemble_query(self._h, ctypes.byref(nc), cn, cr, ctypes.byref(var), ctypes.byref(grid)))
        return {"sizes": list(cn[:nc.value]), "runs": list(cr[:nc.value]), "variant": var.value, "grid": grid.value}


class FNO:
    """Fourier-neural-operator surrogate (pst_fno_*); tensors are torch CUDA float32."""

    def __init__(self, n, width=32, modes=12, layers=4, hidden=128, batch=8, mfma=True, stream=None):
        self.cfg = dict(n=n, width=width, modes=modes, layers=layers, hidden=hidden)
        self.batch = batch
        p = pst_fno_params(n=n, width=width, modes=modes, layers=layers, hidden=hidden, batch=batch, mfma=int(mfma))
        h = _P()
        s = lib.pst_fno_create(ctypes.byref(p), _P(_stream_handle(stream)), ctypes.byref(h))
        if s != PST_OK:
            raise PstError(s, lib.pst_fno_last_error(None).decode())
        self._h = h
        c = ctypes.c_longlong()
        self._check(lib.pst_fno_param_count(h, ctypes.byref(c)))
        self.nparam = c.value

    def _check(self, s):
        if s != PST_OK:
            raise PstError(s, lib.pst_fno_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.pst_fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        assert theta.size == self.nparam
        self._check(lib.pst_fno_set_params(self._h, theta.ctypes.data_as(_P), PST_MEM_HOST))

    def get_params(self):
        out = np.empty(self.nparam, np.float32)
        self._check(lib.pst_fno_get_params(self._h, out.ctypes.data_as(_P), PST_MEM_HOST))
        return out

    def get_grad(self):
        out = np.empty(self.nparam, np.float32)
        self._check(lib.pst_fno_get_grad(self._h, out.ctypes.data_as(_P), PST_MEM_HOST))
        return out

    def _check_io(self, u, other, what):
        b = u.shape[0] if u.dim() >= 1 else 0
        if not 1 <= b <= self.batch:
            raise ValueError(f"batch {b} outside 1..{self.batch}")
        n = self.cfg["n"]
        numel = b * 3 * n ** 3
        _check_buf(u, np.float32, numel, "fno input", device=True)
        _check_buf(other, np.float32, numel, what, device=True)
        return b

    def forward(self, u, out):
        b = self._check_io(u, out, "fno output")
        self._check(lib.pst_fno_forward(self._h, _ptr(u)[0], _ptr(out)[0], b))

    def loss_grad(self, u, tgt):
        self._check_io(u, tgt, "fno target")
        L = ctypes.c_double()
        self._check(lib.pst_fno_loss_grad(self._h, _ptr(u)[0], _ptr(tgt)[0], u.shape[0], ctypes.byref(L)))
        return L.value

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib.pst_fno_adam(self._h, lr, beta1, beta2, eps))

    def train_step(self, u, tgt, lr):
        self._check_io(u, tgt, "fno target")
        L = ctypes.c_double()
        self._check(lib.pst_fno_train_step(self._h, _ptr(u)[0], _ptr(tgt)[0], u.shape[0], lr, ctypes.byref(L)))
        return L.value
