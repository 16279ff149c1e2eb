"""Surrogate pipeline around the library's FNO and ensemble solver.

Host-side orchestration only (which kernels to launch, when to trust the
surrogate); every transform, network layer, solver step, projection and
diagnostic runs in the HIP library.  PyTorch holds the device buffers.

  generate()  trajectories of the Navier-Stokes solver (ensemble of seeded
              runs) stored as physical FP32 fields on the device;
  train()     Adam on random (state, state + horizon steps) pairs;
  rollout()   hybrid rollout: the surrogate advances `horizon` solver steps per
              application; an energy-budget guard checks every application and
              a solver audit every `audit_every` applications, and the solver
              takes over (for the next window) when the relative L2 error of
              an audit exceeds `tol`.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import pst


class Converter:
    """Spectral (library layout) <-> physical fields with the library's FFTs,
    for batches of `batch` 3-component fields in one transform call."""

    def __init__(self, n, batch=1):
        import torch
        self.n = n
        self.plan = pst.Plan(n, precision="fp32")
        self.spec = torch.empty((batch, 3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")

    def to_phys(self, spec, out, nfields=3):
        self.plan.fft_c2r(spec, out, nfields)

    def to_spec(self, phys, out, nfields=3):
        self.plan.fft_r2c(phys, out, nfields)


def generate(nseeds, n=64, steps=510, seed0=1000, nu=1e-2, dt=1e-3, rk=4, spectrum=I.spectrum_c2, log=None):
    """Solver trajectories: float32 device tensor [nseeds][steps + 1][3][n][n][n]."""
    import torch
    ens = pst.Ensemble([n] * nseeds, rk_order=rk, nu=nu, dt=dt)
    ens.set_mode("batched")
    for s in range(nseeds):
        ens.set_state(s, I.random_solenoidal(n, seed0 + s, spectrum=spectrum, dtype=np.complex64))
    conv = Converter(n)
    data = torch.empty((nseeds, steps + 1, 3, n, n, n), dtype=torch.float32, device="cuda")

    def grab(t):
        for s in range(nseeds):
            ens.get_state(s, conv.spec[0])
            conv.to_phys(conv.spec[0], data[s, t])

    grab(0)
    for t in range(1, steps + 1):
        ens.step(1)
        grab(t)
        if log and t % 100 == 0:
            log(f"generate: step {t}/{steps}")
    torch.cuda.synchronize()
    ens.close()
    return data


def train(fno, data, iters=2000, batch=8, lr=1e-3, decay_every=500, gamma=0.5, horizon=10, seed=0, log=None):
    """Adam on random pairs (data[s, t], data[s, t + horizon]); returns the loss history."""
    import torch
    rng = np.random.default_rng(seed)
    S, T = data.shape[0], data.shape[1]
    n = data.shape[-1]
    u = torch.empty((batch, 3, n, n, n), dtype=torch.float32, device="cuda")
    tgt = torch.empty_like(u)
    hist = []
    for it in range(iters):
        s = rng.integers(0, S, batch)
        t = rng.integers(0, T - horizon, batch)
        for b in range(batch):
            u[b].copy_(data[s[b], t[b]])
            tgt[b].copy_(data[s[b], t[b] + horizon])
        cur = lr * gamma ** (it // decay_every)
        hist.append(fno.train_step(u, tgt, cur))
        if log and (it % 100 == 0 or it == iters - 1):
            log(f"train: iter {it} loss {hist[-1]:.4e} lr {cur:.2e}")
    return np.array(hist)


class _Stage:
    """An ensemble plus the buffers to move its states to and from physical space
    (one transform call for all runs)."""

    def __init__(self, sizes, nu, dt, rk, conv, mode="batched"):
        self.ens = pst.Ensemble(sizes, rk_order=rk, nu=nu, dt=dt)
        self.ens.set_mode(mode)   # the fastest execution mode of the solver
        self.conv = conv
        self.nb = len(sizes)

    def load(self, phys, project=False):
        self.conv.to_spec(phys, self.conv.spec, 3 * self.nb)
        for b in range(self.nb):
            self.ens.set_state(b, self.conv.spec[b])
        if project:
            self.ens.project()

    def store(self, phys):
        for b in range(self.nb):
            self.ens.get_state(b, self.conv.spec[b])
        self.conv.to_phys(self.conv.spec, phys, 3 * self.nb)


def rollout(fno, init_phys, apps=50, horizon=10, nu=1e-2, dt=1e-3, rk=4, tol=1e-2, tau_e=2e-3,
            audit_every=5, reference=True):
    """Hybrid rollout of a batch of states [B][3][n][n][n] (device float32).

    Per application: surrogate output -> dealias + projection (solver kernels)
    -> energy guard |E_sur - E_pred| / E_pred <= tau_e with
    E_pred = E exp(-2 nu Z / E * horizon dt) from the input's energy E and
    enstrophy Z; every audit_every applications the solver advances the input
    by `horizon` steps and the surrogate result is replaced by the solver's if
    its relative L2 error exceeds tol; a failed guard or audit hands the next
    window to the solver.  Returns timings and errors; with reference=True the
    plain solver rollout of the same states is timed and used to measure the
    true error of every window (outside the hybrid timing).  Both timings
    start with the state uploaded and every kernel's first-call set-up done
    (one untimed pass through the operations of a window)."""
    import torch
    B, n = init_phys.shape[0], init_phys.shape[-1]
    conv = Converter(n, B)
    sizes = [n] * B
    sur = _Stage(sizes, nu, dt, rk, conv)     # holds the surrogate's (projected) state
    sol = _Stage(sizes, nu, dt, rk, conv)     # solver windows and audits
    x = init_phys.clone()
    y = torch.empty_like(x)
    spec_sur = torch.empty_like(conv.spec)   # the surrogate's output, projected, in spectral space
    stats = {"apps": apps, "horizon": horizon, "guard_fail": 0, "audits": 0, "audit_fail": 0,
             "solver_windows": 0, "audit_err": []}
    # per window: wall time since the start, who advanced it, and the state
    # (kept on the device, in a buffer allocated before the timing, for the
    # untimed comparison with the plain rollout)
    t_win, by_sur = [], []
    states = torch.empty((apps,) + tuple(x.shape), dtype=x.dtype, device=x.device) if reference else None
    # every operation of a window once, untimed (first-call set-up: workspace
    # allocations, code loading), on scratch copies
    fno.forward(x, y)
    conv.to_spec(y, spec_sur, 3 * B)
    conv.plan.project(spec_sur, B)
    conv.to_phys(spec_sur, y, 3 * B)
    for b in range(B):
        sur.ens.set_state(b, spec_sur[b])
    sol.load(x)
    sol.ens.step(1)
    sur.ens.rel_l2(sol.ens)
    sol.store(y)
    # the starting state as the plain rollout has it (uploaded before its
    # timing), with the guard's inputs
    sol.load(x)
    sol_has_x = True                      # sol holds the current state
    e_in, z_in = sol.ens.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver_next = False
    for a in range(apps):
        if solver_next:
            if not sol_has_x:
                sol.load(x)
            sol.ens.step(horizon)
            sol.store(x)
            e_in, z_in = sol.ens.diagnostics()
            sol_has_x = True
            stats["solver_windows"] += 1
            solver_next = False
            torch.cuda.synchronize()
            t_win.append(time.perf_counter() - t0)
            by_sur.append(False)
            if reference:
                states[a].copy_(x)
            continue
        fno.forward(x, y)
        # dealias + projection of all runs in one call, with their energy and
        # enstrophy (the guard's inputs)
        conv.to_spec(y, spec_sur, 3 * B)
        e1, z1 = conv.plan.project(spec_sur, B)
        e_pred = e_in * np.exp(-2.0 * nu * z_in / e_in * horizon * dt)
        guard_ok = bool(np.all(np.abs(e1 - e_pred) <= tau_e * e_pred))
        audit = (a % audit_every) == audit_every - 1
        if not guard_ok or audit:
            if not sol_has_x:
                sol.load(x)
            sol.ens.step(horizon)
            for b in range(B):
                sur.ens.set_state(b, spec_sur[b])
            err = sur.ens.rel_l2(sol.ens)
            if audit:
                stats["audits"] += 1
                stats["audit_err"].append(float(err.max()))
            if not guard_ok:
                stats["guard_fail"] += 1
            if not guard_ok or err.max() > tol:
                if audit and guard_ok:
                    stats["audit_fail"] += 1
                sol.store(x)              # the solver's state replaces the surrogate's
                e_in, z_in = sol.ens.diagnostics()
                sol_has_x = True
                solver_next = True
                torch.cuda.synchronize()
                t_win.append(time.perf_counter() - t0)
                by_sur.append(False)
                if reference:
                    states[a].copy_(x)
                continue
        conv.to_phys(spec_sur, x, 3 * B)
        e_in, z_in = e1, z1
        sol_has_x = False
        torch.cuda.synchronize()
        t_win.append(time.perf_counter() - t0)
        by_sur.append(True)
        if reference:
            states[a].copy_(x)
    torch.cuda.synchronize()
    stats["t_hybrid_s"] = time.perf_counter() - t0
    if reference:
        ref = _Stage(sizes, nu, dt, rk, conv)
        ref.load(init_phys)
        ref.ens.step(1)
        torch.cuda.synchronize()
        ref.load(init_phys)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ref.ens.step(apps * horizon)
        torch.cuda.synchronize()
        stats["t_plain_s"] = time.perf_counter() - t1
        # true error of the hybrid end state against the plain rollout
        chk = _Stage(sizes, nu, dt, rk, conv)
        chk.load(x)
        stats["final_rel_l2"] = chk.ens.rel_l2(ref.ens).tolist()
        stats["speedup"] = stats["t_plain_s"] / stats["t_hybrid_s"]
        # untimed: the hybrid's error against the plain rollout after every window
        ref.load(init_phys)
        win_err = []
        for w in range(apps):
            ref.ens.step(horizon)
            chk.load(states[w])
            win_err.append(float(chk.ens.rel_l2(ref.ens).max()))
        stats["window_err_vs_plain"] = win_err
        stats["window_time_s"] = t_win
        stats["window_by_surrogate"] = by_sur
        stats.update(matched_horizon(stats, tol))
    return stats


def matched_horizon(stats, tol):
    """Speed-up over the horizon in which the hybrid stays within `tol` of the
    plain rollout: the first w windows whose errors (against the plain solver
    at the same time) are all <= tol; plain time of those w windows (its mean
    time per step) over the hybrid's wall time for them."""
    err = stats["window_err_vs_plain"]
    w = 0
    while w < len(err) and err[w] <= tol:
        w += 1
    out = {"tol": tol, "matched_windows": w, "matched_steps": w * stats["horizon"]}
    if w > 0:
        t_plain = stats["t_plain_s"] * w / stats["apps"]
        out["matched_speedup"] = t_plain / stats["window_time_s"][w - 1]
        out["matched_max_err"] = max(err[:w])
        out["matched_surrogate_windows"] = int(sum(stats["window_by_surrogate"][:w]))
    else:
        out["matched_speedup"] = None
    return out


def window_errors(fno, init_phys, apps=50, horizon=10, nu=1e-2, dt=1e-3, rk=4):
    """Untimed evaluation: relative L2 error of each surrogate application
    started from the plain solver's state, and of the free surrogate rollout,
    against the plain solver at every window."""
    import torch
    B, n = init_phys.shape[0], init_phys.shape[-1]
    conv = Converter(n, B)
    sizes = [n] * B
    ref = _Stage(sizes, nu, dt, rk, conv)
    sur = _Stage(sizes, nu, dt, rk, conv)
    ref.load(init_phys)
    xr = init_phys.clone()
    xf = init_phys.clone()
    y = torch.empty_like(xr)
    one, free = [], []
    for a in range(apps):
        fno.forward(xr, y)                # one application from the true state
        ref.ens.step(horizon)
        ref.store(xr)
        sur.load(y, project=True)
        one.append(float(sur.ens.rel_l2(ref.ens).max()))
        fno.forward(xf, y)                # free rollout
        sur.load(y, project=True)
        sur.store(xf)
        free.append(float(sur.ens.rel_l2(ref.ens).max()))
    return {"one_step_err": one, "free_rollout_err": free}
