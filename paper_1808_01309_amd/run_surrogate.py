"""Train and evaluate the FNO surrogate at 64^3 (library entry point).

    python -m paper_1808_01309_amd.run_surrogate [--iters 2000] [--seeds 40] ...

1. Trajectories: `seeds` Navier-Stokes runs at 64^3 (random-phase initial
   fields, E(k) ~ k^4 exp(-2 (k/4)^2), unit energy, nu = 1e-2, dt = 1e-3, RK4)
   advanced `steps` steps by the ensemble solver; every state is kept.
2. Training: `iters` Adam steps on random (state, state + 10 steps) pairs,
   batch 8, width 32, 12 modes, 4 layers, BF16 matrix-core channel mixing.
3. Evaluation on 8 held-out seeds: one-application and free-rollout errors
   against the plain solver, then the timed hybrid rollout (50 applications x
   10 steps with guard, audits and solver takeover) against the plain FP32
   solver's 500 steps.
Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def run(argv=None):
    """Runs the pipeline; returns the result dictionary."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--seeds", type=int, default=40)
    ap.add_argument("--steps", type=int, default=510)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--apps", type=int, default=50)
    ap.add_argument("--eval-seeds", type=int, default=8)
    a = ap.parse_args(argv)
    import torch

    from . import inputs as I
    from . import pst
    from . import surrogate as S

    def log(msg):
        print(f"[surrogate] {msg}", file=sys.stderr, flush=True)

    res = {"config": vars(a)}
    t0 = time.perf_counter()
    data = S.generate(a.seeds, n=a.n, steps=a.steps, seed0=1000, log=log)
    res["generate_s"] = time.perf_counter() - t0
    cfg = dict(n=a.n, width=a.width, modes=a.modes, layers=a.layers, hidden=a.hidden)
    fno = pst.FNO(batch=a.batch, mfma=True, **cfg)
    fno.set_params(I.fno_init_params(seed=0, **cfg))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = S.train(fno, data, iters=a.iters, batch=a.batch, lr=a.lr, log=log)
    torch.cuda.synchronize()
    res["train_s"] = time.perf_counter() - t0
    res["train_ms_per_iter"] = res["train_s"] * 1e3 / a.iters
    res["loss_first_100"] = float(hist[:100].mean())
    res["loss_last_100"] = float(hist[-100:].mean())
    del data
    torch.cuda.empty_cache()
    # held-out initial states (physical)
    conv = S.Converter(a.n)
    x0 = torch.empty((a.eval_seeds, 3, a.n, a.n, a.n), dtype=torch.float32, device="cuda")
    for b in range(a.eval_seeds):
        spec = torch.from_numpy(I.random_solenoidal(a.n, 2000 + b, dtype=np.complex64)).cuda()
        conv.to_phys(spec, x0[b])  # one run at a time: spec is [3][n][n][n/2+1]
    fwd = torch.empty_like(x0)
    fno.forward(x0, fwd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        fno.forward(x0, fwd)
    torch.cuda.synchronize()
    res["fno_forward_ms_batch"] = (time.perf_counter() - t0) * 1e2
    log("window errors")
    res["windows"] = S.window_errors(fno, x0, apps=a.apps)
    log("hybrid rollout")
    res["hybrid"] = S.rollout(fno, x0, apps=a.apps)
    h = res["hybrid"]
    res["summary"] = {
        "speedup": h.get("speedup"),
        "fno_forward_ms_batch": res["fno_forward_ms_batch"],
        "plain_solver_ms_per_10_steps": h["t_plain_s"] * 1e3 / h["apps"] if "t_plain_s" in h else None,
        "max_audited_window_err": max(h["audit_err"]) if h["audit_err"] else None,
        "accepted_windows": h["apps"] - h["solver_windows"] - h["audit_fail"] - h["guard_fail"],
        "solver_windows": h["solver_windows"], "audit_fail": h["audit_fail"], "guard_fail": h["guard_fail"],
        "max_one_application_err": max(res["windows"]["one_step_err"]),
        "final_rel_l2_vs_plain_max": max(h["final_rel_l2"]) if "final_rel_l2" in h else None,
        # the horizon reading: speed-up while the hybrid stays within 1e-2 of the plain rollout
        "matched_windows": h.get("matched_windows"), "matched_steps": h.get("matched_steps"),
        "matched_speedup": h.get("matched_speedup"), "matched_max_err": h.get("matched_max_err"),
        "matched_surrogate_windows": h.get("matched_surrogate_windows"),
    }
    fno.close()
    return res


def main(argv=None):
    print(json.dumps(run(argv)))


if __name__ == "__main__":
    main()
