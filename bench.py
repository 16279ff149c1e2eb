"""Benchmark: ms per RK4 step and per-pass HBM bandwidth of the pseudospectral
Navier-Stokes hot path at 512^3, FP32 (headline) and FP64, on one GPU.

Workload (Navier-Stokes 512^3): solenoidal random-phase initial velocity with
E(k) ~ k^4 exp(-2 (k/4)^2), seed 1, unit energy; constant random-phase
forcing on shells 2..3 (seed 2, unit forcing energy); nu = 2e-3; classical
RK4 with the viscous integrating factor; dt = 5e-4.  The state is resident in
HBM before the timed region; each timed step is one full pass of the hot path
(4 right-hand sides of 5 kernels each, with the RK update fused).

Defaults: 2 warm-up + 18 timed steps (the workload's 20 steps); `value` is
the mean over the timed steps, the per-step median is reported too.

Prints one JSON line.  Also reported (under "extra"): a plain device copy's
bandwidth; the standalone 3D r2c / c2r transforms of 3 fields at 512^3 per pass
in GB/s; the MHD 1024^3 RK2 step; the 96-run ensemble in every execution mode;
the FNO's forward pass and training step at 64^3; the surrogate pipeline run
live (its speed-up over the whole rollout and over the horizon in which it
stays within 1e-2 of the plain solver); the Boussinesq 512^3, Gross-Pitaevskii
512^3 and anisotropic 1024 x 1024 x 256 legs; the roofline of the dominant
kernel (algorithmic bytes per launch / HIP-event-timed launch duration, as a
fraction of 8 TB/s and of the copy bandwidth) and the FP64 CPU oracle timed on
one step on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "ms/RK step + FFT HBM GB/s at 512^3, FP32 vs FP64; surrogate speed-up @1e-2 err"
KINDS = ["zinv", "yinv", "xpass", "yfwd", "zfwd"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fft", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-fno", action="store_true")
    ap.add_argument("--no-mhd", action="store_true")
    ap.add_argument("--no-bq", action="store_true")
    ap.add_argument("--no-gpe", action="store_true")
    ap.add_argument("--no-aniso", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="report the surrogate's committed summary instead of running its pipeline (data, "
                         "about 20 s of training, evaluation, timed hybrid rollout) live")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counter scaling)")
    return ap.parse_args()


def kernel_bytes(n, esz, rk, mhd=False, bq=False, gpe=False, shape=None):
    """Algorithmic HBM bytes per launch of each solver kernel: every array
    element a pass must read or write, once.  State components / backward
    fields / forward fields: 3 / 6 / 3 (Navier-Stokes), 6 / 12 / 6 (MHD),
    4 / 10 / 4 (Boussinesq: u, theta; v, i k x v, grad theta, theta), 1 / 1 / 1
    (Gross-Pitaevskii: psi on the whole spectrum, cutoff ceil(n/4) - 1).
    shape = (nx, ny, nz): per-axis sizes and cutoffs."""
    nx, ny, nz = (n, n, n) if shape is None else shape
    cut = (lambda m: -(-m // 4) - 1) if gpe else (lambda m: -(-m // 3) - 1)
    Kx, Ky, Kz = cut(nx), cut(ny), cut(nz)
    My, Mz = 2 * Ky + 1, 2 * Kz + 1
    nxk = 2 * Kx + 1 if gpe else Kx + 1
    sc, sa, sb = nxk * My * Mz, nxk * My * nz, nxk * ny * nz
    rk_arrays = 13.0 / 4.0 if rk == 4 else 5.0 / 2.0  # state-sized arrays touched per stage update
    ns, nb, nf = (6, 12, 6) if mhd else (4, 10, 4) if bq else (1, 1, 1) if gpe else (3, 6, 3)
    return {
        "zinv": (ns * sc + nb * sa) * esz,
        "yinv": (nb * sa + nb * sb) * esz,
        "xpass": (nb * sb + nf * sb) * esz,
        "yfwd": (nf * sb + nf * sa) * esz,
        "zfwd": (nf * sa + rk_arrays * ns * sc) * esz,
    }


def fft_bytes(n, nf, esz_c):
    """Algorithmic bytes per pass of the standalone unpruned 3D transforms."""
    nxh = n // 2 + 1
    real = nf * n ** 3 * (esz_c // 2)
    cplx = nf * n * n * nxh * esz_c
    return {"fftx": real + cplx, "ffty": 2 * cplx, "fftz": 2 * cplx}


def timed_steps(plan, torch, steps):
    """Runs `steps` steps between two device synchronisations; returns the wall
    ms per step and the per-step durations from events on the plan's stream
    (torch's current stream)."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        plan.step(1)
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return (t1 - t0) * 1e3 / steps, per


def run_solver(pst, torch, I, n, prec, steps, warmup):
    plan = pst.Plan(n, precision=prec, rk_order=4, nu=2e-3, dt=5e-4, timers=True)
    cdt = np.complex128 if prec == "fp64" else np.complex64
    plan.set_state(I.random_solenoidal(n, 1, dtype=cdt))
    plan.set_forcing(I.forcing_shells(n, 1, dtype=cdt))
    plan.step(warmup)
    torch.cuda.synchronize()
    plan.timers(reset=True)
    ms, per = timed_steps(plan, torch, steps)
    tm = plan.timers(reset=True)
    e = plan.energy()[0]
    info = plan.query()
    info["median_step_ms"] = float(np.median(per))
    plan.close()
    return ms, tm, e, info


def band_limited_field(torch, I, n, seed, field, spectrum, energy, kb=24):
    """Random-phase solenoidal field whose spectrum is negligible beyond |k_i| = kb
    (E ~ k^2 exp(-(k/3)^2) is below 1e-25 there): generated on a 64^3 grid with
    the cube cut at kb and placed into the n^3 layout on the device (the
    counter-based generator gives every mode the same value on any grid)."""
    m = 64
    small = torch.from_numpy(I.random_solenoidal(m, seed, field=field, spectrum=spectrum, energy=energy,
                                                 kcut=kb, dtype=np.complex64)).cuda()
    big = torch.zeros((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    for bz, sz in ((slice(0, kb + 1), slice(0, kb + 1)), (slice(n - kb, n), slice(m - kb, m))):
        for by, sy in ((slice(0, kb + 1), slice(0, kb + 1)), (slice(n - kb, n), slice(m - kb, m))):
            big[:, bz, by, :kb + 1] = small[:, sz, sy, :kb + 1]
    return big


def run_mhd(pst, torch, I, n=1024, steps=5, warmup=1):
    """MHD 1024^3 FP32, random-phase u and b with E(k) ~ k^2 exp(-(k/3)^2),
    E_u = E_b = 1/2, nu = eta = 1e-3, RK2, dt = 2.5e-4: ms per step and per pass."""
    plan = pst.Plan(n, solver="mhd", precision="fp32", rk_order=2, nu=1e-3, eta=1e-3, dt=2.5e-4, timers=True)
    for f, name in ((0, "u"), (1, "b")):
        st = band_limited_field(torch, I, n, 3, f, I.spectrum_c3, 0.5)
        plan.set_state(st, field=name)
        del st
    torch.cuda.empty_cache()
    plan.step(warmup)
    torch.cuda.synchronize()
    plan.timers(reset=True)
    ms, per = timed_steps(plan, torch, steps)
    tm = plan.timers(reset=True)
    kb = kernel_bytes(n, 8, 2, mhd=True)
    kern = {k: {"ms": tm[k][0] / max(tm[k][1], 1), "launches": tm[k][1]} for k in KINDS}
    for k in KINDS:
        kern[k]["GB_s"] = kb[k] / kern[k]["ms"] / 1e6
    res = {"n": n, "precision": "fp32", "rk_order": 2, "steps": steps, "ms_per_step": ms,
           "median_step_ms": float(np.median(per)), "kernels": kern,
           "effective_GB_s": 2 * sum(kb.values()) / ms / 1e6, "energy_end": plan.energy()}
    plan.close()
    torch.cuda.empty_cache()
    return res


def run_boussinesq(pst, torch, I, n=512, steps=10, warmup=2):
    """Boussinesq 512^3 FP32 RK4 (the paper's reference equations), nu = kappa
    = 2e-3, N = 2, dt = 5e-4: the Navier-Stokes workload's u and forcing plus a
    random-phase theta of the same spectrum (variance 1/2): ms per step and per pass."""
    plan = pst.Plan(n, solver="boussinesq", precision="fp32", rk_order=4, nu=2e-3, kappa=2e-3, dt=5e-4,
                    nbv=2.0, timers=True)
    plan.set_state(I.random_solenoidal(n, 1, dtype=np.complex64), field="u")
    plan.set_state(I.random_scalar(n, 2, energy=0.5, dtype=np.complex64), field="theta")
    plan.set_forcing(I.forcing_shells(n, 1, dtype=np.complex64))
    plan.step(warmup)
    torch.cuda.synchronize()
    plan.timers(reset=True)
    ms, per = timed_steps(plan, torch, steps)
    tm = plan.timers(reset=True)
    kb = kernel_bytes(n, 8, 4, bq=True)
    kern = {k: {"ms": tm[k][0] / max(tm[k][1], 1), "launches": tm[k][1]} for k in KINDS}
    for k in KINDS:
        kern[k]["GB_s"] = kb[k] / kern[k]["ms"] / 1e6
    res = {"n": n, "precision": "fp32", "rk_order": 4, "nbv": 2.0, "steps": steps, "ms_per_step": ms,
           "median_step_ms": float(np.median(per)), "kernels": kern,
           "effective_GB_s": 4 * sum(kb.values()) / ms / 1e6, "energy_end": plan.energy()}
    plan.close()
    torch.cuda.empty_cache()
    return res


def run_leg(plan, torch, kb, nstage, steps, warmup):
    """Time `steps` steps of a prepared plan: ms per step and per pass."""
    plan.step(warmup)
    torch.cuda.synchronize()
    plan.timers(reset=True)
    ms, per = timed_steps(plan, torch, steps)
    tm = plan.timers(reset=True)
    kern = {k: {"ms": tm[k][0] / max(tm[k][1], 1), "launches": tm[k][1]} for k in KINDS}
    for k in KINDS:
        kern[k]["GB_s"] = kb[k] / kern[k]["ms"] / 1e6
    return {"steps": steps, "ms_per_step": ms, "median_step_ms": float(np.median(per)), "kernels": kern,
            "effective_GB_s": nstage * sum(kb.values()) / ms / 1e6, "energy_end": plan.energy()}


def run_gpe(pst, torch, I, n=512, steps=10, warmup=2):
    """Gross-Pitaevskii 512^3 FP32 RK4 (the paper's fourth solver, eq. gpe):
    alpha = 0.5, beta = 1, dt = 1e-3, random-phase psi with E(k) ~ k^2
    exp(-(k/3)^2), half the particles in the k = 0 condensate."""
    plan = pst.Plan(n, solver="gpe", precision="fp32", rk_order=4, dt=1e-3, alpha=0.5, beta=1.0, timers=True)
    psi = I.random_wavefunction((n, n, n), 1, condensate=0.5, kcut=24, dtype=np.complex64)
    plan.set_state(psi[None])
    del psi
    res = run_leg(plan, torch, kernel_bytes(n, 8, 4, gpe=True), 4, steps, warmup)
    res.update({"n": n, "precision": "fp32", "rk_order": 4, "alpha": 0.5, "beta": 1.0})
    plan.close()
    torch.cuda.empty_cache()
    return res


ANISO_SHAPE, ANISO_BOX = (1024, 1024, 256), (2 * np.pi, 2 * np.pi, np.pi / 2)


def run_aniso(pst, torch, I, steps=5, warmup=1):
    """Navier-Stokes on the paper's 4:4:1 grid 1024 x 1024 x 256 (box 2 pi x 2 pi
    x pi/2, so the grid spacing is the same in every direction), FP32 RK4,
    nu = 1e-3, dt = 2.5e-4: the 512^3 workload's spectrum (seed 1, unit
    energy; the modes |a_i k_i| <= 24 carry it) and shell 2-3 forcing."""
    plan = pst.Plan(0, precision="fp32", rk_order=4, nu=1e-3, dt=2.5e-4, timers=True, shape=ANISO_SHAPE,
                    box=ANISO_BOX)
    kc = (24, 24, 6)
    plan.set_state(I.random_solenoidal(0, 1, kcut=kc, dtype=np.complex64, shape=ANISO_SHAPE, box=ANISO_BOX))
    plan.set_forcing(I.forcing_shells(0, 1, dtype=np.complex64, shape=ANISO_SHAPE, box=ANISO_BOX))
    res = run_leg(plan, torch, kernel_bytes(0, 8, 4, shape=ANISO_SHAPE), 4, steps, warmup)
    res.update({"shape": list(ANISO_SHAPE), "box": [float(b) for b in ANISO_BOX], "precision": "fp32",
                "rk_order": 4})
    plan.close()
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(torch, gib=4, reps=5):
    """A plain device-to-device copy of `gib` GiB: read + write bytes per second."""
    src = torch.empty(gib << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) / ms / 1e6


def mall_copy_bandwidth(torch, sizes_mb=(32, 64, 100, 128, 200), reps=50):
    """Device copies whose source + destination (2x the size) stay within or
    cross the 256 MB last-level cache (MALL): read + write bytes per second,
    the practical ceiling of the ensemble's and the FNO's working sets."""
    out = {}
    for mb in sizes_mb:
        src = torch.empty(mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        out[f"{mb}MB"] = 2.0 * (mb << 20) / (a.elapsed_time(b) / reps) / 1e6
        del src, dst
    torch.cuda.empty_cache()
    return out


def run_fft(pst, torch, n, prec, reps=5, nf=3):
    plan = pst.Plan(n, precision=prec, timers=True)
    rt = torch.float64 if prec == "fp64" else torch.float32
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.randn((nf, n, n, n), dtype=rt, device="cuda")
    y = torch.empty((nf, n, n, n // 2 + 1), dtype=ct, device="cuda")
    z = torch.empty_like(x)
    plan.fft_r2c(x, y, nf)
    plan.fft_c2r(y, z, nf)
    torch.cuda.synchronize()
    plan.timers(reset=True)
    res = {}
    for name, fn in (("r2c", lambda: plan.fft_r2c(x, y, nf)), ("c2r", lambda: plan.fft_c2r(y, z, nf))):
        for _ in range(reps):
            fn()
        tm = plan.timers(reset=True)
        res[name] = {k: tm[k][0] / max(tm[k][1], 1) for k in ("fftx", "ffty", "fftz")}
    plan.close()
    del x, y, z
    torch.cuda.empty_cache()
    return res


def run_ensemble(pst, torch, I, steps=200, seq_steps=10):
    """96 Navier-Stokes runs of uneven size (32 x 48^3, 48 x 64^3, 16 x 96^3), FP32,
    RK4, dt = 1e-3, nu = 1e-2, random-phase initial fields (seeds 0..95):
    `steps` steps in each graph mode (the persistent kernel, or the batched
    launches, replayed from a HIP graph; the autotuner picks the faster one),
    and a shorter timing of the direct persistent, batched and per-run
    sequential launches of the same kernels."""
    sizes = [48] * 32 + [64] * 48 + [96] * 16
    ens = pst.Ensemble(sizes, rk_order=4, nu=1e-2, dt=1e-3)
    init = [I.random_solenoidal(n, r, dtype=np.complex64) for r, n in enumerate(sizes)]
    for r, u in enumerate(init):
        ens.set_state(r, u)
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "pst_ensemble_autotune.json")
    variant = ens.autotune(cache)
    tuned = ens.get_mode()
    q = ens.query()
    res = {"runs": len(sizes), "sizes": {"48": 32, "64": 48, "96": 16}, "variant": variant,
           "class_variants": {str(n): v for n, v in zip(q["sizes"], ens.class_schedules())},
           "tuned_mode": tuned, "grid_blocks": q["grid"]}
    timings = {}
    for mode, nst in (("graph", steps), ("batched_graph", steps), ("persistent", seq_steps),
                      ("batched", seq_steps), ("sequential", seq_steps)):
        for r, u in enumerate(init):
            ens.set_state(r, u)
        ens.set_mode(mode)
        ens.step(1)                      # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.step(nst)
        torch.cuda.synchronize()
        timings[mode] = (time.perf_counter() - t0) * 1e3 / nst
    pts = sum(n ** 3 for n in sizes)
    # algorithmic pass traffic of one RK4 step of all runs (every run's five
    # passes per stage, as for a single plan)
    step_bytes = sum(4 * sum(kernel_bytes(n, 8, 4).values()) for n in sizes)
    res["algorithmic_GB_per_step"] = step_bytes / 1e9
    res["ms_per_step"] = timings
    res["wall_s_200_steps_tuned"] = timings[tuned] * steps / 1e3
    res["point_steps_per_s"] = pts / (timings[tuned] / 1e3)
    res["speedup_vs_sequential"] = timings["sequential"] / timings[tuned]
    res["speedup_vs_batched"] = timings["batched"] / timings[tuned]
    res["effective_GB_s_tuned"] = step_bytes / timings[tuned] / 1e6
    e = ens.energy()
    res["energy_range_end"] = [float(e.min()), float(e.max())]
    ens.close()
    return res


def traffic_from_profiles(kernel, n, prec):
    """HBM bytes per launch from committed rocprofv3 counter summaries, valid
    only while the kernel sources are unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_n{n}_{prec}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha") != kernel_source_sha():
        return None
    return rec.get("bytes_per_launch")


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1808_01309_amd", "csrc")
    for f in ("fft_engine.h", "kernels.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n):
    """The FP64 oracle (untuned) on this host: one whole RK4 step (four
    right-hand sides of 9 textbook 3D FFTs each, products, projection, Lawson
    updates) of the same 512^3 workload."""
    import oracle as O
    from paper_1808_01309_amd import inputs as I
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    u = I.random_solenoidal(n, 1)
    f = I.forcing_shells(n, 1)
    t0 = time.perf_counter()
    O.step(u, 1, dt=5e-4, nu=2e-3, rk=4, fhat=f)
    dt = time.perf_counter() - t0
    return {"value": dt * 1e3, "unit": "ms/RK4 step", "cores": threads, "kind": "oracle",
            "sample": f"one FP64 RK4 step of the {n}^3 forced Navier-Stokes workload (4 right-hand sides) "
                      f"took {dt:.2f} s on {threads} threads of {cpu_model()}"}


FNO_CFG = dict(n=64, width=32, modes=12, layers=4, hidden=128)


def run_fno(pst, torch, I, batch=8, reps=20, train_reps=5):
    """FNO surrogate at 64^3 (4 spectral layers, 12 modes, width 32, hidden 128,
    BF16 matrix-core channel mixing), batch 8, seeded random weights and
    inputs: forward (fused inference kernels) and one training step (forward,
    loss, backward, Adam)."""
    fno = pst.FNO(batch=batch, mfma=True, **FNO_CFG)
    fno.set_params(I.fno_init_params(seed=1, out_scale=0.5, **FNO_CFG).astype(np.float32))
    n = FNO_CFG["n"]
    gen = torch.Generator(device="cuda").manual_seed(5)
    u = torch.randn((batch, 3, n, n, n), device="cuda", generator=gen)
    tgt = u + 0.1 * torch.randn((batch, 3, n, n, n), device="cuda", generator=gen)
    out = torch.empty_like(u)
    for _ in range(3):
        fno.forward(u, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fno.forward(u, out)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) * 1e3 / reps
    fno.train_step(u, tgt, 1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(train_reps):
        fno.train_step(u, tgt, 1e-5)
    torch.cuda.synchronize()
    trn = (time.perf_counter() - t0) * 1e3 / train_reps
    fno.close()
    return {"config": dict(FNO_CFG, batch=batch, mfma=True), "forward_ms": fwd, "train_step_ms": trn}


def surrogate_summary(live):
    """Surrogate speed-up: the pipeline run live, or the committed summary of its
    last full run (which trains for about 70 s)."""
    if live:
        from paper_1808_01309_amd import run_surrogate
        res = run_surrogate.run([])
        return dict(res["summary"], source="live run (python -m paper_1808_01309_amd.run_surrogate)")
    path = os.path.join(ROOT, "profiles", "surrogate_c5_fno64.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return dict(rec["summary"], source="profiles/surrogate_c5_fno64.json (not re-measured in this run)")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": a.gpus}))
        sys.exit(2)
    import torch

    from paper_1808_01309_amd import inputs as I
    from paper_1808_01309_amd import pst

    n = a.n
    print("[bench] device copy bandwidth (4 GiB)", file=sys.stderr, flush=True)
    copy_gbs = copy_bandwidth(torch)
    mall = mall_copy_bandwidth(torch)
    if a.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] n={n} fp32 solver: warmup {a.warmup}, timed {a.steps}", file=sys.stderr, flush=True)
    ms32, tm32, e32, info = run_solver(pst, torch, I, n, "fp32", a.steps, a.warmup)
    out_extra = {"copy_GB_s": copy_gbs, "mall_copy_GB_s": mall,
                 "fp32": {"ms_per_step": ms32, "median_step_ms": info["median_step_ms"], "energy_end": e32}}
    per32 = {k: tm32[k][0] / max(tm32[k][1], 1) for k in KINDS}
    kb32 = kernel_bytes(n, 8, 4)
    out_extra["fp32"]["kernels"] = {k: {"ms": per32[k], "GB_s": kb32[k] / per32[k] / 1e6,
                                        "launches": tm32[k][1]} for k in KINDS}
    step_bytes32 = 4 * sum(kb32.values())
    out_extra["fp32"]["effective_GB_s"] = step_bytes32 / ms32 / 1e6
    out_extra["fp32"]["algorithmic_GB_per_step"] = step_bytes32 / 1e9
    if not a.no_fp64:
        print(f"[bench] n={n} fp64 solver", file=sys.stderr, flush=True)
        ms64, tm64, e64, info64 = run_solver(pst, torch, I, n, "fp64", a.steps, a.warmup)
        per64 = {k: tm64[k][0] / max(tm64[k][1], 1) for k in KINDS}
        kb64 = kernel_bytes(n, 16, 4)
        out_extra["fp64"] = {"ms_per_step": ms64, "median_step_ms": info64["median_step_ms"], "energy_end": e64,
                             "kernels": {k: {"ms": per64[k], "GB_s": kb64[k] / per64[k] / 1e6,
                                             "launches": tm64[k][1]} for k in KINDS},
                             "effective_GB_s": 4 * sum(kb64.values()) / ms64 / 1e6}
    if not a.no_fft:
        print(f"[bench] n={n} standalone FFTs", file=sys.stderr, flush=True)
        ffts = {}
        for prec, esz in (("fp32", 8), ("fp64", 16)):
            if prec == "fp64" and a.no_fp64:
                continue
            r = run_fft(pst, torch, n, prec)
            fb = fft_bytes(n, 3, esz)
            ffts[prec] = {d: {k: {"ms": r[d][k], "GB_s": fb[k] / r[d][k] / 1e6} for k in fb} for d in r}
        out_extra["fft_3fields"] = ffts
    if not a.no_ensemble:
        print("[bench] ensemble: 96 runs (48^3, 64^3, 96^3), 200 RK4 steps", file=sys.stderr, flush=True)
        out_extra["ensemble"] = run_ensemble(pst, torch, I)
    if not a.no_mhd:
        print("[bench] MHD 1024^3 FP32 RK2 (5 steps)", file=sys.stderr, flush=True)
        out_extra["mhd1024"] = run_mhd(pst, torch, I)
    if not a.no_bq and n == 512:
        print("[bench] Boussinesq 512^3 FP32 RK4 (10 steps)", file=sys.stderr, flush=True)
        out_extra["boussinesq512"] = run_boussinesq(pst, torch, I)
    if not a.no_gpe and n == 512:
        print("[bench] Gross-Pitaevskii 512^3 FP32 RK4 (10 steps)", file=sys.stderr, flush=True)
        out_extra["gpe512"] = run_gpe(pst, torch, I)
    if not a.no_aniso:
        print("[bench] Navier-Stokes 1024x1024x256 FP32 RK4 (5 steps)", file=sys.stderr, flush=True)
        out_extra["aniso_1024x1024x256"] = run_aniso(pst, torch, I)
    if not a.no_fno:
        print("[bench] FNO surrogate forward / training step (64^3, batch 8)", file=sys.stderr, flush=True)
        out_extra["fno"] = run_fno(pst, torch, I)
    if not a.no_surrogate:
        print("[bench] surrogate pipeline: data, training, evaluation, hybrid rollout", file=sys.stderr,
              flush=True)
    out_extra["surrogate"] = surrogate_summary(not a.no_surrogate)
    # dominant kernel of the headline (FP32) step
    dom = max(KINDS, key=lambda k: tm32[k][0])
    ach = kb32[dom] / per32[dom] / 1e6
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "frac_of_copy": round(ach / copy_gbs, 4),
            "traffic": traffic_from_profiles(dom, n, "fp32"),
            "algorithmic_bytes_per_launch": kb32[dom], "avg_launch_ms": per32[dom]}
    cpu = None
    if not a.no_cpu:
        print(f"[bench] cpu baseline (oracle, {n}^3 FP64 rhs)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(n)
    line = {
        "metric": METRIC, "value": round(ms32, 4), "unit": "ms/RK4 step", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms32, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Navier-Stokes {n}^3 periodic, RK4 dt=5e-4, nu=2e-3, random-phase "
                               f"E(k)~k^4 exp(-2(k/4)^2) unit energy, shell 2-3 forcing, 2/3-rule cube "
                               f"dealiasing", "n": n, "precision": "fp32", "rk_order": 4,
                   "radices": info["radices"], "tile_lines": info["tile_lines"]},
        "roofline": roof, "cpu_baseline": cpu, "extra": out_extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
