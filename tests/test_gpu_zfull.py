"""Parity at the full workload sizes, in the launch configurations the
benchmark times (collected after the other GPU tests: these are the slow ones).

* Navier-Stokes 512^3, RK4, dt = 5e-4, nu = 2e-3, shell forcing: one right-hand
  side and one RK4 step of the FP32 and FP64 paths against the FP64 oracle,
  every coefficient (the oracle needs seconds per right-hand side on the host
  cores).
* MHD 1024^3, RK2, dt = 2.5e-4, nu = eta = 1e-3, FP32: properties that hold at
  any size (the oracle would need ~100 GB of host memory there).  The
  dealiased nonlinear terms conserve total energy and cross-helicity exactly,
  so their transfers must vanish to rounding; over 5 steps the total energy
  must fall by the dissipation alone.
* MHD at 128^3 and 256^3 (the sizes below 1024^3 where the oracle still fits
  in host memory): right-hand side of the FP32 and FP64 paths against the
  oracle, and one RK2 step of the 1024^3 benchmark's parameters at 128^3; the
  Navier-Stokes right-hand side at 256^3 (its own radix schedule).
* Boussinesq 512^3, RK4, dt = 5e-4, nu = kappa = 2e-3, N = 2, shell forcing
  (the benchmark's Boussinesq leg): one right-hand side and one RK4 step of
  the FP32 and FP64 paths against the FP64 oracle, every coefficient; the
  right-hand side at 256^3; at 1024^3 the internal gravity wave in closed form.
* The 96-run ensemble (32 x 48^3, 48 x 64^3, 16 x 96^3) with its autotuned
  schedule: the graph-replayed persistent step equals the batched launches
  bitwise for every run, and one run of each size equals the oracle.
* The FNO at 64^3 (width 32, 12 modes, 4 layers, hidden 128) created for
  batch 8: the last sample's output against the FP64 oracle, BF16 and FP32.
"""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def P():
    from paper_1808_01309_amd import pst
    return pst


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ------------------------------------------------------------ NS 512^3
N512, NU512, DT512 = 512, 2e-3, 5e-4


@pytest.fixture(scope="module")
def ns512(O):
    u0 = I.random_solenoidal(N512, 1)
    f = I.forcing_shells(N512, 1)
    rhs = O.ns_rhs(u0, f)
    step = O.step(u0, 1, dt=DT512, nu=NU512, rk=4, fhat=f)
    return u0, f, rhs, step


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ns512_rhs_and_step(P, torch, ns512, prec, errlog):
    u0, f, rhs_ref, step_ref = ns512
    plan = P.Plan(N512, precision=prec, rk_order=4, nu=NU512, dt=DT512)
    plan.set_forcing(f)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    sd = torch.from_numpy(u0).to(ct).cuda()
    rd = torch.empty_like(sd)
    plan.rhs(sd, rd)
    got = rd.cpu().numpy()
    errlog(f"NS 512^3 {prec} rhs vs oracle (u_x, u_y, u_z)", [rel(got[c], rhs_ref[c]) for c in range(3)], TOL[prec])
    del rd
    plan.set_state(sd)
    del sd
    plan.step(1)
    got = plan.get_state()
    errlog(f"NS 512^3 {prec} 1 RK4 step vs oracle", [rel(got[c], step_ref[c]) for c in range(3)], TOL[prec])
    plan.close()
    torch.cuda.empty_cache()


# ------------------------------------------------------------ C2 over 20 steps
C2_STEPS = 20


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_c2_fp32_vs_fp64_20_steps(P, torch, seed, errlog):
    """The 512^3 workload over its 20 RK4 steps, FP32 and FP64 from the same
    FP64 initial condition and forcing (seed, seed + 1): the FP32 path against
    the plain FP64 GPU solver, per component, after the last step."""
    u0 = I.random_solenoidal(N512, seed)
    f = I.forcing_shells(N512, seed)
    out = {}
    for prec in ("fp64", "fp32"):
        plan = P.Plan(N512, precision=prec, rk_order=4, nu=NU512, dt=DT512)
        plan.set_forcing(f)
        plan.set_state(u0)
        plan.step(C2_STEPS)
        out[prec] = plan.get_state().astype(np.complex128)
        e = plan.energy()[0]
        assert np.isfinite(e) and 0.5 < e < 2.0
        plan.close()
        torch.cuda.empty_cache()
    errlog(f"NS 512^3 seed {seed} 20 RK4 steps: FP32 vs FP64 GPU",
           [rel(out["fp32"][c], out["fp64"][c]) for c in range(3)], TOL["fp32"])


@pytest.fixture(scope="module")
def ns256_20(O):
    n = 256
    u0 = I.random_solenoidal(n, 1)
    f = I.forcing_shells(n, 1)
    return u0, f, O.step(u0, C2_STEPS, dt=DT512, nu=NU512, rk=4, fhat=f)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ns256_20_steps_vs_oracle(P, torch, ns256_20, prec, errlog):
    """20 RK4 steps with the 512^3 workload's nu, dt and forcing at 256^3 (the
    largest grid where 20 oracle steps take about a minute on the host cores),
    every coefficient against the FP64 oracle."""
    u0, f, ref = ns256_20
    plan = P.Plan(256, precision=prec, rk_order=4, nu=NU512, dt=DT512)
    plan.set_forcing(f)
    plan.set_state(u0)
    plan.step(C2_STEPS)
    got = plan.get_state()
    errlog(f"NS 256^3 {prec} 20 RK4 steps vs oracle", [rel(got[c], ref[c]) for c in range(3)], TOL[prec])
    plan.close()


# ------------------------------------------------------------ MHD 1024^3
N1024, KB = 1024, 24   # the E(k) ~ k^2 exp(-(k/3)^2) fields are below 1e-25 beyond |k_i| = 24


def embed(torch, small, n, kb):
    """Modes |k_i| <= kb of a field generated on a small grid, placed in the
    n^3 layout (the counter-based generator gives every mode the same value
    on any grid)."""
    m = small.shape[1]
    s = torch.from_numpy(small).cuda()
    big = torch.zeros((small.shape[0], n, n, n // 2 + 1), dtype=s.dtype, device="cuda")
    for bz, sz in ((slice(0, kb + 1), slice(0, kb + 1)), (slice(n - kb, n), slice(m - kb, m))):
        for by, sy in ((slice(0, kb + 1), slice(0, kb + 1)), (slice(n - kb, n), slice(m - kb, m))):
            big[:, bz, by, :kb + 1] = s[:, sz, sy, :kb + 1]
    return big


def wsum(torch, t):
    """sum over a half spectrum with weight 1 on kx = 0, 2 elsewhere (FP64)."""
    return 2.0 * t.sum(dtype=torch.float64).item() - t[..., 0].sum(dtype=torch.float64).item()


def re_dot(a, b):
    return a.real * b.real + a.imag * b.imag


def test_mhd1024_invariants_and_dissipation(P, torch):
    n, nu, eta, dt = N1024, 1e-3, 1e-3, 2.5e-4
    kw = dict(spectrum=I.spectrum_c3, energy=0.5, kcut=KB, dtype=np.complex64)
    st = torch.empty((6, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    st[:3] = embed(torch, I.random_solenoidal(64, 3, field=0, **kw), n, KB)
    st[3:] = embed(torch, I.random_solenoidal(64, 3, field=1, **kw), n, KB)
    plan = P.Plan(n, solver="mhd", precision="fp32", rk_order=2, nu=nu, eta=eta, dt=dt)
    rhs = torch.empty_like(st)
    plan.rhs(st, rhs)
    torch.cuda.synchronize()
    te = sum(wsum(torch, re_dot(st[c], rhs[c])) for c in range(6))
    th = sum(wsum(torch, re_dot(st[c], rhs[c + 3]) + re_dot(st[c + 3], rhs[c])) for c in range(3))
    se = sum(wsum(torch, st[c].abs() * rhs[c].abs()) for c in range(6))
    sh = sum(wsum(torch, st[c].abs() * rhs[c + 3].abs() + st[c + 3].abs() * rhs[c].abs()) for c in range(3))
    assert se > 0 and sh > 0
    assert abs(te) < 1e-5 * se, (te, se)
    assert abs(th) < 1e-5 * sh, (th, sh)
    del rhs
    # 5 steps of the benchmark configuration: dE = -int 2 (nu Z_u + eta Z_b) dt
    plan.set_state(st[:3], field="u")
    plan.set_state(st[3:], field="b")
    ks = torch.fft.fftfreq(n, d=1.0 / n, device="cuda").to(torch.float32)
    k2 = ks[:, None, None] ** 2 + ks[None, :, None] ** 2 + ks[None, None, : n // 2 + 1] ** 2

    def dissipation():
        plan.get_state("u", out=st[:3])
        plan.get_state("b", out=st[3:])
        zu = sum(wsum(torch, k2 * st[c].abs() ** 2) for c in range(3))
        zb = sum(wsum(torch, k2 * st[c + 3].abs() ** 2) for c in range(3))
        pz = plan.enstrophy()   # 1/2 sum w |k|^2 |.|^2, from the library
        assert abs(pz[0] - 0.5 * zu) < 1e-5 * pz[0] and abs(pz[1] - 0.5 * zb) < 1e-5 * pz[1]
        return nu * zu + eta * zb   # = -dE/dt with E = 1/2 sum w |.|^2

    e = [sum(plan.energy())]
    d = [dissipation()]
    for _ in range(5):
        plan.step(1)
        e.append(sum(plan.energy()))
        d.append(dissipation())
    pred = -sum(dt * 0.5 * (d[i] + d[i + 1]) for i in range(5))
    de = e[-1] - e[0]
    assert pred < 0 and abs(de - pred) < 0.05 * abs(pred), (de, pred)
    plan.close()
    del st, k2
    torch.cuda.empty_cache()


def test_1024_taylor_green_closed_form(P, torch):
    """Right-hand sides at 1024^3 (where the x pass of MHD and the z passes have
    their own radix schedules): MHD for u = Taylor-Green, b = 0 and for u = 0,
    b = Taylor-Green, where the projected u x w (resp. j x b = -(b x curl b))
    has a closed form and the induction term vanishes; Navier-Stokes (FP32,
    FP64) for u = Taylor-Green."""
    n = N1024
    m = 16
    x = 2 * np.pi * np.arange(m) / m
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    Nx = np.stack([-np.sin(2 * X) * np.cos(2 * Z) / 8, -np.sin(2 * Y) * np.cos(2 * Z) / 8,
                   (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8])
    ref = embed(torch, np.stack([np.fft.rfftn(Nx[c], axes=(0, 1, 2)) / m ** 3 for c in range(3)]).astype(np.complex64),
                n, 2)
    tg = embed(torch, I.taylor_green_spec(m).astype(np.complex64), n, 1)
    plan = P.Plan(n, solver="mhd", precision="fp32")
    st = torch.zeros((6, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    rhs = torch.empty_like(st)
    scale = ref.abs().max().item()
    for part, sign in ((slice(0, 3), 1.0), (slice(3, 6), -1.0)):
        st.zero_()
        st[part] = tg
        plan.rhs(st, rhs)
        err_u = (rhs[:3] - sign * ref).abs().max().item()
        err_b = rhs[3:].abs().max().item()
        assert err_u < 1e-5 * scale and err_b < 1e-5 * scale, (part, err_u, err_b, scale)
    plan.close()
    del st, rhs
    torch.cuda.empty_cache()
    # the Navier-Stokes path at the same size (its z passes share the schedule)
    for prec, ct in (("fp32", torch.complex64), ("fp64", torch.complex128)):
        plan = P.Plan(n, precision=prec)
        su = tg.to(ct)
        rhs = torch.empty_like(su)
        plan.rhs(su, rhs)
        err = (rhs - ref.to(ct)).abs().max().item()
        assert err < (1e-5 if prec == "fp32" else 1e-12) * scale, (prec, err, scale)
        plan.close()
        del su, rhs
        torch.cuda.empty_cache()
    del ref, tg


# ------------------------------------------------------------ 128^3, 256^3
_mid = {}


def mhd_case(O, n):
    """Inputs and oracle right-hand side of the MHD case at n (cached per n)."""
    if ("mhd", n) not in _mid:
        kw = dict(spectrum=I.spectrum_c3, energy=0.5)
        u = I.random_solenoidal(n, 40 + n, **kw)
        b = I.random_solenoidal(n, 40 + n, field=1, **kw)
        _mid[("mhd", n)] = (u, b) + tuple(O.mhd_rhs(u, b))
    return _mid[("mhd", n)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [128, 256])
def test_mhd_rhs_mid_sizes(O, P, torch, n, prec, errlog):
    u, b, ru, rb = mhd_case(O, n)
    plan = P.Plan(n, solver="mhd", precision=prec)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    sd = torch.from_numpy(np.concatenate([u, b])).to(ct).cuda()
    rd = torch.empty_like(sd)
    plan.rhs(sd, rd)
    got = rd.cpu().numpy()
    errlog(f"MHD {n}^3 {prec} rhs vs oracle (u_x, u_y, u_z, b_x, b_y, b_z)",
           [rel(got[c], ru[c]) for c in range(3)] + [rel(got[3 + c], rb[c]) for c in range(3)], TOL[prec])
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mhd_step_128(O, P, torch, prec, errlog):
    n, nu, dt = 128, 1e-3, 2.5e-4
    u, b = mhd_case(O, n)[:2]
    if ("mhd_step", n) not in _mid:
        _mid[("mhd_step", n)] = O.step(u, 1, dt=dt, nu=nu, eta=nu, rk=2, bhat=b)
    su, sb = _mid[("mhd_step", n)]
    plan = P.Plan(n, solver="mhd", precision=prec, rk_order=2, nu=nu, eta=nu, dt=dt)
    plan.set_state(u, field="u")
    plan.set_state(b, field="b")
    plan.step(1)
    gu, gb = plan.get_state("u"), plan.get_state("b")
    errlog(f"MHD 128^3 {prec} 1 RK2 step vs oracle (u, b components)",
           [rel(gu[c], su[c]) for c in range(3)] + [rel(gb[c], sb[c]) for c in range(3)], TOL[prec])
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ns_rhs_256(O, P, torch, prec, errlog):
    n = 256
    if ("ns", n) not in _mid:
        u = I.random_solenoidal(n, 10 + n)
        f = I.forcing_shells(n, 10 + n)
        _mid[("ns", n)] = (u, f, O.ns_rhs(u, f))
    u, f, ref = _mid[("ns", n)]
    plan = P.Plan(n, precision=prec)
    plan.set_forcing(f)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    sd = torch.from_numpy(u).to(ct).cuda()
    rd = torch.empty_like(sd)
    plan.rhs(sd, rd)
    got = rd.cpu().numpy()
    errlog(f"NS 256^3 {prec} rhs vs oracle", [rel(got[c], ref[c]) for c in range(3)], TOL[prec])
    plan.close()


# ------------------------------------------------------------ Boussinesq 512^3
@pytest.fixture(scope="module")
def bq512(O):
    u = I.random_solenoidal(N512, 1)
    t = I.random_scalar(N512, 2, energy=0.5)
    f = I.forcing_shells(N512, 1)
    rhs = O.bq_rhs(u, t, 2.0, fhat=f)
    step = O.step(u, 1, dt=DT512, nu=NU512, rk=4, fhat=f, theta=t, kappa=NU512, nbv=2.0)
    return u, t, f, rhs, step


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_bq512_rhs_and_step(P, torch, bq512, prec, errlog):
    u, t, f, (ru, rt), (su, stt) = bq512
    plan = P.Plan(N512, solver="boussinesq", precision=prec, rk_order=4, nu=NU512, kappa=NU512, dt=DT512, nbv=2.0)
    plan.set_forcing(f)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    sd = torch.from_numpy(np.concatenate([u, t[None]])).to(ct).cuda()
    rd = torch.empty_like(sd)
    plan.rhs(sd, rd)
    got = rd.cpu().numpy()
    errlog(f"Boussinesq 512^3 {prec} rhs vs oracle (u_x, u_y, u_z, theta)",
           [rel(got[c], ru[c]) for c in range(3)] + [rel(got[3], rt)], TOL[prec])
    del rd
    plan.set_state(sd[:3], field="u")
    plan.set_state(sd[3:], field="theta")
    del sd
    plan.step(1)
    gu = plan.get_state("u")
    errlog(f"Boussinesq 512^3 {prec} 1 RK4 step vs oracle (u_x, u_y, u_z, theta)",
           [rel(gu[c], su[c]) for c in range(3)] + [rel(plan.get_state("theta")[0], stt)], TOL[prec])
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_bq_rhs_256(O, P, torch, prec, errlog):
    n = 256
    if ("bq", n) not in _mid:
        u = I.random_solenoidal(n, 50)
        t = I.random_scalar(n, 51, energy=0.5)
        f = I.forcing_shells(n, 50)
        _mid[("bq", n)] = (u, t, f) + tuple(O.bq_rhs(u, t, 2.0, fhat=f))
    u, t, f, ru, rt = _mid[("bq", n)]
    plan = P.Plan(n, solver="boussinesq", precision=prec, nbv=2.0)
    plan.set_forcing(f)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    sd = torch.from_numpy(np.concatenate([u, t[None]])).to(ct).cuda()
    rd = torch.empty_like(sd)
    plan.rhs(sd, rd)
    got = rd.cpu().numpy()
    errlog(f"Boussinesq 256^3 {prec} rhs vs oracle (u_x, u_y, u_z, theta)",
           [rel(got[c], ru[c]) for c in range(3)] + [rel(got[3], rt)], TOL[prec])
    plan.close()


def test_bq_1024_gravity_wave(P, torch):
    """Boussinesq at 1024^3 (its own radix schedules and tiles): two RK4 steps
    of the internal gravity wave follow the RK4 stability function of the
    buoyancy rotation, and every other coefficient stays zero."""
    n, k, nbv, nu, dt, ns = N1024, (1, 1, 2), 2.5, 1e-3, 0.02, 2
    u0, t0 = I.gravity_wave_spec(16, k=k, amp_u=0.1, amp_t=0.07)
    plan = P.Plan(n, solver="boussinesq", precision="fp32", rk_order=4, nu=nu, kappa=nu, dt=dt, nbv=nbv)
    plan.set_state(embed(torch, u0.astype(np.complex64), n, 2), field="u")
    th = embed(torch, t0[None].astype(np.complex64), n, 2)
    plan.set_state(th, field="theta")
    plan.step(ns)
    kv = np.array(k, float)
    k2 = float(kv @ kv)
    w = nbv * np.sqrt(kv[0] ** 2 + kv[1] ** 2) / np.sqrt(k2)
    z = 1j * w * dt
    g = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    A, T = 0.1, 0.07
    d = np.exp(-nu * k2 * dt)
    for _ in range(ns):
        A, T = d * (g.real * A - g.imag * T), d * (g.imag * A + g.real * T)
    e = u0[:, k[2], k[1], k[0]] / 0.1
    su = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    plan.get_state("u", out=su)
    got_u = su[:, k[2], k[1], k[0]].cpu().numpy()
    assert np.abs(got_u - A * e).max() < 1e-6
    su[:, k[2], k[1], k[0]] = 0
    assert su.abs().max().item() < 1e-6
    del su
    plan.get_state("theta", out=th)
    assert abs(th[0, k[2], k[1], k[0]].item() - T) < 1e-6
    th[0, k[2], k[1], k[0]] = 0
    assert th.abs().max().item() < 1e-6
    plan.close()
    del th
    torch.cuda.empty_cache()


# ------------------------------------------------------------ ensemble, 96 runs
def test_ensemble_96_runs(O, P, torch, tmp_path):
    sizes = [48] * 32 + [64] * 48 + [96] * 16
    nu, dt, ns = 1e-2, 1e-3, 3
    init = [I.random_solenoidal(n, r, dtype=np.complex64) for r, n in enumerate(sizes)]
    outs = {}
    for mode in ("graph", "batched"):
        ens = P.Ensemble(sizes, rk_order=4, nu=nu, dt=dt)
        ens.autotune(str(tmp_path / "tune.json"))
        for r, u in enumerate(init):
            ens.set_state(r, u)
        ens.set_mode(mode)
        ens.step(ns)
        outs[mode] = [ens.get_state(r) for r in range(len(sizes))]
        ens.close()
    for r in range(len(sizes)):
        assert np.array_equal(outs["graph"][r], outs["batched"][r]), r
    for r in (0, 32, 80):   # one run of each size
        ref = O.step(init[r].astype(np.complex128), ns, dt=dt, nu=nu, rk=4)
        assert rel(outs["graph"][r], ref) < 1e-5, (r, sizes[r])


# ------------------------------------------------------------ FNO, batch 8
def test_fno_full_config(P, torch):
    import oracle.fno as F
    cfg = dict(n=64, width=32, modes=12, layers=4, hidden=128)
    theta = I.fno_init_params(seed=1, out_scale=0.5, **cfg).astype(np.float32).astype(np.float64)
    x = np.random.default_rng(21).standard_normal((8, 3, 64, 64, 64)).astype(np.float32)
    y_ref = F.forward(theta, x[7:].astype(np.float64), cfg)[0] - x[7]
    xd = torch.from_numpy(x).cuda()
    for mfma, tol in ((True, 2e-2), (False, 1e-5)):
        fno = P.FNO(batch=8, mfma=mfma, **cfg)
        fno.set_params(theta)
        od = torch.empty_like(xd)
        fno.forward(xd, od)
        y = od[7].cpu().numpy().astype(np.float64) - x[7]
        assert rel(y, y_ref) < tol, mfma
        fno.close()
