"""GPU adjoint path against the oracle: the hand-written VJP of the residual compared
element by element with the oracle's hand-transposed VJP (itself pinned by complex-step
dot tests and discrete conservation, tests/test_oracle_vjp.py) on random mixed-order
meshes with periodic, slip-wall and far-field faces, on periodic chains covering every
ordered mortar pair of orders 1..7 in each direction, on a tiny mesh against the whole
complex-step Jacobian, and at the full 24^3, N = 5 adjoint workload; the autograd
wrapper, the wall-force functional and its gradient, and the adjoint-weighted tau
(eta) with the adjoint in either form.

Bar: FP64 fields within 1e-12 of max |out_oracle| (the transposed operator has no
cancellation beyond that of its inputs' scale)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import mortar_chain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

TOL = 1e-12
QINF = tuple(wl.conserved(np.array(1.0), np.array(0.3), np.array(0.4), np.array(0.5), np.array(1.0)))


def _setup(shape, lo, hi, seed, bc=(0,) * 6, flux=wl.ROE):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh(shape, bc=bc, flux=flux, qfar=QINF)
    orders = wl.random_orders(int(np.prod(shape)), lo, hi, rng)
    u = wl.random_state(orders, rng)
    return mesh, orders, u, rng


def _rel(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


CASES = [((2, 2, 2), 1, 5, 50, (0,) * 6, wl.ROE),
         ((3, 2, 1), 2, 4, 51, (1, 2, 0, 0, 0, 0), wl.ROE),
         ((2, 1, 2), 1, 3, 52, (0, 0, 1, 2, 0, 0), wl.LF),
         ((2, 2, 1), 1, 9, 57, (2, 1, 1, 2, 0, 0), wl.ROE),
         ((1, 2, 3), 1, 7, 58, (0, 0, 0, 0, 1, 2), wl.LF)]


@pytest.mark.parametrize("shape,lo,hi,seed,bc,flux", CASES)
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True), (1, True)])
def test_vjp_against_oracle(shape, lo, hi, seed, bc, flux, form, isolated):
    mesh, orders, u, rng = _setup(shape, lo, hi, seed, bc, flux)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    for _ in range(2):
        v = rng.normal(size=u.size)
        got = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v), form=form, isolated=isolated))
        ref = oracle.residual_vjp(mesh, orders, u, v, form, isolated)
        assert _rel(got, ref) < TOL


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_vjp_every_mortar_pair(d, flux):
    rng = np.random.default_rng(60 + d + 3 * flux)
    mesh, orders = mortar_chain(d, rng)
    mesh["flux"] = flux
    u = wl.random_state(orders, rng)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    for form in (0, 1):
        v = rng.normal(size=u.size)
        got = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v), form=form))
        assert _rel(got, oracle.residual_vjp(mesh, orders, u, v, form)) < TOL


def test_vjp_whole_jacobian_tiny_mesh():
    """Rows of the GPU's transposed product against the oracle's complex-step Jacobian."""
    from oracle import adjoint
    mesh, orders, u, rng = _setup((2, 1, 2), 1, 2, 53, bc=(1, 2, 0, 0, 0, 0))
    plan = dg.Plan(mesh, orders)
    Jac = adjoint.cs_jacobian(mesh, orders, u)
    ud = plan.to_plan(u)
    for _ in range(4):
        v = rng.normal(size=u.size)
        got = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v)))
        assert _rel(got, Jac.T @ v) < TOL


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
    assert _rel(plan.to_natural(ud.grad), oracle.residual_vjp(mesh, orders, u, plan.to_natural(w))) < TOL


def test_functional_and_gradient():
    mesh, orders, u, rng = _setup((3, 2, 2), 1, 6, 55, bc=(1, 2, 0, 0, 0, 0))
    plan = dg.Plan(mesh, orders)
    J, g = dg.functional(plan, plan.to_plan(u))
    Jr, gr = oracle.functional(mesh, orders, u)
    assert abs(float(J) - Jr) < 1e-13 * abs(Jr)
    assert np.max(np.abs(plan.to_natural(g) - gr)) < 1e-13 * np.max(np.abs(gr))


def _mass(mesh, orders):
    h = (np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / np.asarray(mesh["n"])
    J = np.prod(h) / 8.0
    out = []
    for o in np.asarray(orders).reshape(-1, 3):
        w = [oracle.lgl(int(N))[1] for N in o]
        out.append(np.tile(J * np.einsum("k,j,i->kji", w[2], w[1], w[0]).ravel(), 5))
    return np.concatenate(out)


@pytest.mark.parametrize("isolated", [False, True])
@pytest.mark.parametrize("psi_form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_adjoint_weighted_tau(isolated, psi_form):
    mesh, fo, u, rng = _setup((2, 2, 2), 2, 6, 56, bc=(1, 2, 0, 0, 0, 0))
    co = np.minimum(fo, wl.random_orders(8, 1, 5, rng))
    psi_t = rng.normal(size=u.size)
    # the new-form adjoint of the same functional is M times the traditional one
    psi = psi_t if psi_form == dg.FORM_TRAD else _mass(mesh, fo) * psi_t
    dudt = oracle.residual(mesh, fo, u)
    eta_r = oracle.tau_eta(mesh, fo, co, u, dudt, psi, isolated=isolated, psi_form=psi_form)
    eta_t = oracle.tau_eta(mesh, fo, co, u, dudt, psi_t, isolated=isolated, psi_form=dg.FORM_TRAD)
    assert np.max(np.abs(eta_r - eta_t)) < 1e-12 * np.abs(eta_t).sum()
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    tn, tt, norms, eta = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated, psi=fine.to_plan(psi),
                                         psi_form=psi_form)
    _, tt_r, _, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=isolated)
    scale = np.abs(tt_r).sum() * np.max(np.abs(psi_t)) + 1e-300
    got = coarse.elem_to_natural(eta.cpu().numpy())
    assert np.max(np.abs(got - eta_r)) < 1e-12 * scale


@pytest.mark.slow
def test_c4_workload():
    """24^3, N = 5 (3.0M nodes), slip wall at x = 0, far field at x = 1: the VJP against the
    oracle's over the whole field (both forms), the functional and its gradient, and the
    coupled tau at Nc = 4 weighted by dJ/du."""
    mesh, orders = wl.c4()
    u = wl.c4_state(oracle.node_coords(mesh, orders), orders)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    rng = np.random.default_rng(4)
    J, g = dg.functional(plan, ud)
    Jr, gr = oracle.functional(mesh, orders, u)
    assert abs(float(J) - Jr) < 1e-12 * abs(Jr)
    assert np.max(np.abs(plan.to_natural(g) - gr)) < 1e-13 * np.max(np.abs(gr))
    for form in (0, 1):
        v = rng.normal(size=u.size)
        got = plan.to_natural(dg.residual_vjp(plan, ud, plan.to_plan(v), form=form))
        assert _rel(got, oracle.residual_vjp(mesh, orders, u, v, form)) < TOL
    co = wl.uniform_orders(len(orders), 4)
    coarse = plan.coarse(co)
    r0 = oracle.residual(mesh, orders, u)
    _, _, _, eta = dg.tau_estimate(plan, coarse, ud, psi=g)
    eta_r = oracle.tau_eta(mesh, orders, co, u, r0, gr)
    assert np.max(np.abs(coarse.elem_to_natural(eta.cpu().numpy()) - eta_r)) < 1e-12 * (np.abs(eta_r).sum() + 1e-300)
