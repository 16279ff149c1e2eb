"""GPU parity of the Boussinesq solver (eq. mom with buoyancy, eq. temp,
eq. divv) through the C ABI against the FP64 oracle, on the same seeded
inputs: right-hand sides at sizes spanning several tiles and ragged tails,
RK2 and RK4 steps with forcing and kappa != nu, the internal gravity wave in
closed form, the scalar's diagnostics and state I/O, and field errors.

Tolerances as for the other solvers: relative L2 per field <= 1e-12 (FP64),
<= 1e-5 (FP32).
"""
import numpy as np
import pytest

from paper_1808_01309_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
NBV = 1.3


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
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def fields(n, seed):
    u = I.random_solenoidal(n, seed)
    t = I.random_scalar(n, seed + 1, energy=0.4)
    return u, t


def gpu_rhs(P, torch, plan, u, t):
    ct = torch.complex128 if plan.fp64 else torch.complex64
    st = torch.from_numpy(np.concatenate([u, t[None]])).to(ct).cuda()
    out = torch.empty_like(st)
    plan.rhs(st, out)
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [16, 24, 48, 64, 128])
def test_bq_rhs(O, P, torch, n, prec):
    u, t = fields(n, 30 + n)
    f = I.forcing_shells(n, 30 + n)
    plan = P.Plan(n, solver="boussinesq", precision=prec, nbv=NBV)
    plan.set_forcing(f)
    got = gpu_rhs(P, torch, plan, u, t)
    ru, rt = O.bq_rhs(u, t, NBV, fhat=f)
    assert max(rel(got[c], ru[c]) for c in range(3)) < TOL[prec]
    assert rel(got[3], rt) < TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("rk", [2, 4])
def test_bq_steps(O, P, torch, prec, rk):
    n, nu, kappa, dt, ns = 48, 8e-3, 5e-3, 2e-3, 3
    u, t = fields(n, 7)
    f = I.forcing_shells(n, 7)
    plan = P.Plan(n, solver="boussinesq", precision=prec, rk_order=rk, nu=nu, kappa=kappa, dt=dt, nbv=NBV)
    plan.set_forcing(f)
    plan.set_state(u, field="u")
    plan.set_state(t, field="theta")
    plan.step(ns)
    ru, rt = O.step(u, ns, dt=dt, nu=nu, rk=rk, fhat=f, theta=t, kappa=kappa, nbv=NBV)
    assert max(rel(plan.get_state("u")[c], ru[c]) for c in range(3)) < TOL[prec]
    assert rel(plan.get_state("theta")[0], rt) < TOL[prec]
    eu, et = plan.energy()
    assert abs(eu - O.energy(ru)) < 1e-6 * O.energy(ru)
    assert abs(et - O.energy(rt)) < 1e-6 * O.energy(rt)
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bq_rhs_sphere(O, P, torch, prec):
    """Spherical truncation: the nonlinear and coupling terms of u and theta are
    kept for |k|^2 <= K^2 only (inputs inside the sphere on both sides)."""
    n = 48
    u, t = fields(n, 9)
    kx, ky, kz = I.wavenumbers(n)
    K = I.kcut_23(n)
    inside = (kx ** 2 + ky ** 2 + kz ** 2) <= K * K
    u, t = u * inside[None], t * inside
    plan = P.Plan(n, solver="boussinesq", precision=prec, nbv=NBV, dealias="sphere")
    got = gpu_rhs(P, torch, plan, u, t)
    ru, rt = O.bq_rhs(u, t, NBV, sphere=True)
    assert max(rel(got[c], ru[c]) for c in range(3)) < TOL[prec]
    assert rel(got[3], rt) < TOL[prec]
    plan.close()


def test_gravity_wave_gpu(P, torch):
    """The internal gravity wave's amplitudes follow the RK4 stability
    function of the buoyancy rotation (FP64, closed form)."""
    n, k, nbv, nu, dt, ns = 32, (1, 1, 2), 2.5, 0.02, 0.02, 11
    u0, t0 = I.gravity_wave_spec(n, k=k, amp_u=0.1, amp_t=0.07)
    plan = P.Plan(n, solver="boussinesq", precision="fp64", rk_order=4, nu=nu, kappa=nu, dt=dt, nbv=nbv)
    plan.set_state(u0, field="u")
    plan.set_state(t0, field="theta")
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
    ref_u = u0 * (A / 0.1)
    ref_t = t0 * (T / 0.07)
    assert np.abs(plan.get_state("u") - ref_u).max() < 1e-13
    assert np.abs(plan.get_state("theta")[0] - ref_t).max() < 1e-13
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bq_state_io_and_diagnostics(O, P, torch, prec):
    n = 32
    u, t = fields(n, 3)
    plan = P.Plan(n, solver="boussinesq", precision=prec, nbv=NBV)
    plan.set_state(u, field="u")
    plan.set_state(t, field="theta")
    tol = TOL[prec]
    assert rel(plan.get_state("theta")[0], t) < tol
    phys = plan.get_state("theta", space="phys")
    assert phys.shape == (1, n, n, n)
    assert rel(phys[0], O.c2r3(t)) < tol
    plan.set_state(phys, field="theta", space="phys")          # physical round trip
    assert rel(plan.get_state("theta")[0], t) < tol
    eu, et = plan.energy()
    assert abs(eu - O.energy(u)) < 1e-6 * O.energy(u)
    assert abs(et - O.energy(t)) < 1e-6 * O.energy(t)
    zu, zt = plan.enstrophy()
    kx, ky, kz = I.wavenumbers(n)
    k2 = (kx * kx + ky * ky + kz * kz).astype(float)
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    zref = 0.5 * float(np.sum(w * k2 * np.abs(t) ** 2))
    assert abs(zt - zref) < 1e-6 * zref
    spec = plan.spectrum("theta")
    assert abs(spec.sum() - O.energy(t)) < 1e-6 * O.energy(t)
    plan.close()


def test_bq_field_errors(P, torch):
    plan = P.Plan(16, solver="boussinesq", nbv=NBV)
    with pytest.raises(P.PstError):
        plan.get_state("b")
    plan.close()
    plan = P.Plan(16)
    with pytest.raises(P.PstError):
        plan.get_state("theta")
    plan.close()
    plan = P.Plan(16, solver="mhd")
    with pytest.raises(P.PstError):
        plan.set_forcing(I.forcing_shells(16, 1))
    plan.close()
