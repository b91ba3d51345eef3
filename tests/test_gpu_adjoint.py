"""GPU adjoint path against the oracle: the hand-written VJP of the residual
checked by central differences of the FP64 oracle residual (dot tests and a
brute-force Jacobian on a tiny mesh), the autograd wrapper, the wall-force
functional and its gradient, and the adjoint-weighted tau (eta).

Finite-difference tolerance: central differences at eps = 1e-6 carry a truncation
error O(eps^2 |r'''|) and a rounding error O(1e-16 |r| / eps) ~ 1e-10 |r|; the
checks allow 1e-7 of the scale |v| |r| (dot tests) or of max |J| (Jacobian)."""
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

EPS = 1e-6


def _setup(shape, lo, hi, seed, bc=(0,) * 6, flux=wl.ROE):
    rng = np.random.default_rng(seed)
    qinf = tuple(wl.conserved(np.array(1.0), np.array(0.3), np.array(0.4), np.array(0.5), np.array(1.0)))
    mesh = wl.box_mesh(shape, bc=bc, flux=flux, qfar=qinf)
    orders = wl.random_orders(int(np.prod(shape)), lo, hi, rng)
    u = wl.random_state(orders, rng)
    return mesh, orders, u, rng


CASES = [((2, 2, 2), 1, 5, 50, (0,) * 6, wl.ROE),
         ((3, 2, 1), 2, 4, 51, (1, 2, 0, 0, 0, 0), wl.ROE),
         ((2, 1, 2), 1, 3, 52, (0, 0, 1, 2, 0, 0), wl.LF)]


@pytest.mark.parametrize("shape,lo,hi,seed,bc,flux", CASES)
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True)])
def test_vjp_dot_against_oracle_differences(shape, lo, hi, seed, bc, flux, form, isolated):
    mesh, orders, u, rng = _setup(shape, lo, hi, seed, bc, flux)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    r0 = oracle.residual(mesh, orders, u, form=form, isolated=isolated)
    for _ in range(8):
        v = rng.normal(size=u.size)
        d = rng.normal(size=u.size) * np.abs(u) * 1e-2
        g = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v), form=form, isolated=isolated))
        fd = (oracle.residual(mesh, orders, u + EPS * d, form, isolated)
              - oracle.residual(mesh, orders, u - EPS * d, form, isolated)) / (2 * EPS)
        lhs, rhs = g @ d, v @ fd
        scale = np.linalg.norm(v) * np.linalg.norm(r0) * 1e-2
        assert abs(lhs - rhs) < 1e-7 * scale + 1e-9 * abs(rhs), (lhs, rhs)


def test_vjp_full_jacobian_tiny_mesh():
    mesh, orders, u, rng = _setup((2, 1, 2), 1, 2, 53, bc=(1, 2, 0, 0, 0, 0))
    plan = dg.Plan(mesh, orders)
    n = u.size
    J = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = EPS * max(abs(u[i]), 1.0)
        J[:, i] = (oracle.residual(mesh, orders, u + e) - oracle.residual(mesh, orders, u - e)) / (2 * e[i])
    v = rng.normal(size=n)
    g = plan.to_natural(dg.residual_vjp(plan, plan.to_plan(u), plan.to_plan(v)))
    ref = J.T @ v
    assert np.max(np.abs(g - ref)) < 1e-6 * np.max(np.abs(ref))


def test_autograd_function():
    mesh, orders, u, rng = _setup((2, 2, 1), 1, 4, 54)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u).requires_grad_(True)
    r = dg.ResidualFn.apply(plan, ud)
    w = torch.from_numpy(rng.normal(size=u.size)).cuda()
    (r * w).sum().backward()
    ref = dg.residual_vjp(plan, ud.detach(), w)
    assert torch.equal(ud.grad, ref)
    assert torch.equal(r.detach(), dg.residual(plan, ud.detach()))


def test_functional_and_gradient():
    mesh, orders, u, rng = _setup((3, 2, 2), 1, 6, 55, bc=(1, 2, 0, 0, 0, 0))
    plan = dg.Plan(mesh, orders)
    J, g = dg.functional(plan, plan.to_plan(u))
    Jr, gr = oracle.functional(mesh, orders, u)
    assert abs(float(J) - Jr) < 1e-13 * abs(Jr)
    assert np.max(np.abs(plan.to_natural(g) - gr)) < 1e-13 * np.max(np.abs(gr))


@pytest.mark.parametrize("isolated", [False, True])
def test_adjoint_weighted_tau(isolated):
    mesh, fo, u, rng = _setup((2, 2, 2), 2, 6, 56, bc=(1, 2, 0, 0, 0, 0))
    co = np.minimum(fo, wl.random_orders(8, 1, 5, rng))
    psi = rng.normal(size=u.size)
    dudt = oracle.residual(mesh, fo, u)
    eta_r = oracle.tau_eta(mesh, fo, co, u, dudt, psi, isolated=isolated)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    tn, tt, norms, eta = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated, psi=fine.to_plan(psi))
    _, tt_r, _, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=isolated)
    scale = np.abs(tt_r).sum() * np.max(np.abs(psi)) + 1e-300
    got = coarse.elem_to_natural(eta.cpu().numpy())
    assert np.max(np.abs(got - eta_r)) < 1e-12 * scale


@pytest.mark.slow
def test_c4_workload():
    """24^3, N = 5 (3.0M nodes), slip wall at x = 0: VJP checked by central differences of
    the oracle residual at eps = 1e-6 on 64 seeded random directions; functional and its
    gradient; coupled tau at Nc = 4 weighted by dJ/du."""
    mesh, orders = wl.c4()
    u = wl.c4_state(oracle.node_coords(mesh, orders), orders)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    rng = np.random.default_rng(4)
    J, g = dg.functional(plan, ud)
    Jr, gr = oracle.functional(mesh, orders, u)
    assert abs(float(J) - Jr) < 1e-12 * abs(Jr)
    assert np.max(np.abs(plan.to_natural(g) - gr)) < 1e-13 * np.max(np.abs(gr))
    v = rng.normal(size=u.size)
    vjp = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v)))
    r0 = oracle.residual(mesh, orders, u)
    worst = 0.0
    for _ in range(64):
        d = rng.normal(size=u.size)
        d /= np.max(np.abs(d))
        fd = (oracle.residual(mesh, orders, u + EPS * d) - oracle.residual(mesh, orders, u - EPS * d)) / (2 * EPS)
        worst = max(worst, abs(vjp @ d - v @ fd) / (np.linalg.norm(v) * np.linalg.norm(r0)))
    assert worst < 1e-7
    co = wl.uniform_orders(len(orders), 4)
    coarse = plan.coarse(co)
    _, _, _, eta = dg.tau_estimate(plan, coarse, ud, psi=g)
    eta_r = oracle.tau_eta(mesh, orders, co, u, r0, gr)
    assert np.max(np.abs(coarse.elem_to_natural(eta.cpu().numpy()) - eta_r)) < 1e-12 * (np.abs(eta_r).sum() + 1e-300)
