"""GPU parity of the Navier-Stokes (BR1) path against the FP64 oracle: residual (both
forms, isolated, periodic/wall/far-field, mixed orders with mortars, FP64 and FP32),
RK3 steps and the tau-estimate on box elements (the curved vortex workload is covered
with the curved elements)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import residual_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

MU, PR = 0.01, 0.72
A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)


def rk3_ns_reference(mesh, orders, u, dt, nsteps):
    """Williamson RK3 stages composed from the oracle's NS residual (coefficients as in
    the oracle's pinned Euler stepper)."""
    u = u.copy()
    for _ in range(nsteps):
        G = np.zeros_like(u)
        for k in range(3):
            r = oracle.residual_ns(mesh, orders, u, mesh["mu"], mesh["Pr"])
            G = -dt * r if k == 0 else A[k] * G - dt * r
            u = u + B[k] * G
    return u


CASES = [((3, 2, 2), (1, 6), 70, (0,) * 6, wl.ROE),
         ((2, 3, 1), (2, 5), 71, (1, 2, 0, 0, 0, 0), wl.ROE),
         ((2, 2, 2), (1, 4), 72, (0, 0, 2, 2, 0, 0), wl.LF)]


def _case(shape, orng, seed, bc, flux):
    rng = np.random.default_rng(seed)
    qinf = tuple(wl.conserved(np.array(1.0), np.array(0.3), np.array(0.2), np.array(0.1), np.array(1.0)))
    mesh = wl.ns_mesh(wl.box_mesh(shape, bc=bc, flux=flux, qfar=qinf), MU, PR)
    orders = wl.random_orders(int(np.prod(shape)), *orng, rng)
    u = wl.random_state(orders, rng)
    return mesh, orders, u, rng


@pytest.mark.parametrize("shape,orng,seed,bc,flux", CASES)
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True)])
def test_ns_residual_fp64(shape, orng, seed, bc, flux, form, isolated):
    mesh, orders, u, _ = _case(shape, orng, seed, bc, flux)
    plan = dg.Plan(mesh, orders)
    ref = oracle.residual_ns(mesh, orders, u, MU, PR, form=form, isolated=isolated)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u), form=form, isolated=isolated))
    s = residual_scale(mesh, orders, u)
    if form == 1:
        s *= np.prod(1.0 / np.asarray(mesh["n"])) / 8
    assert np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), s) < 1e-12


@pytest.mark.parametrize("shape,orng,seed,bc,flux", CASES[:2])
def test_ns_residual_fp32(shape, orng, seed, bc, flux):
    mesh, orders, u, _ = _case(shape, orng, seed, bc, flux)
    plan = dg.Plan(mesh, orders)
    ref = oracle.residual_ns(mesh, orders, u, MU, PR)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u, dtype=torch.float32))).astype(np.float64)
    assert np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), residual_scale(mesh, orders, u)) < 1e-5


def test_ns_rk3():
    mesh, orders, _, rng = _case((2, 2, 2), (2, 4), 73, (0,) * 6, wl.ROE)
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.2)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    g = torch.empty_like(ud)
    dg.rk3_step(plan, ud, g, 1e-3, 3)
    ref = rk3_ns_reference(mesh, orders, u, 1e-3, 3)
    assert np.max(np.abs(plan.to_natural(ud) - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("isolated", [False, True])
def test_ns_tau(isolated):
    mesh, fo, u, rng = _case((3, 2, 1), (2, 6), 74, (0,) * 6, wl.ROE)
    co = np.minimum(fo, wl.random_orders(6, 1, 5, rng))
    dudt = oracle.residual_ns(mesh, fo, u, MU, PR)
    rc = oracle.residual_ns(mesh, co, oracle.restrict(fo, co, u), MU, PR, isolated=isolated)
    ref = rc - oracle.restrict(fo, co, dudt)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    tn, _, _ = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated)
    s = np.max(np.abs(rc))  # the coarse residual of which tau is a difference
    assert np.max(np.abs(coarse.to_natural(tn) - ref)) / max(np.max(np.abs(ref)), s) < 1e-12
