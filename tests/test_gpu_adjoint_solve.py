"""GPU adjoint solve (dg_adjoint_solve: restarted GMRES on the residual VJP) against the
oracle's dense adjoint (finite-difference Jacobian of the oracle residual, numpy solve):
the x-force adjoint at a smooth state on a box with a slip wall and a far field,
traditional and new forms; the residual the solver reports is checked with an
independent VJP."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402


@pytest.mark.parametrize("form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_adjoint_matches_dense(form):
    rng = np.random.default_rng(40 + form)
    mesh = wl.box_mesh((2, 2, 2), bc=(1, 2, 0, 0, 0, 0), qfar=wl.conserved(*(np.array(x) for x in
                                                                           (1.0, 0.3, 0.0, 0.0, 1.0))))
    orders = wl.random_orders(8, 1, 2, rng)
    # a smooth state (the density pulse of the adjoint workload): its Jacobian has
    # eigenvalues of positive real part, which unpreconditioned restarted GMRES needs
    # (at a random state it stagnates, as scipy's GMRES does on the same matrix)
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.3, amp=0.2)
    u = wl.add_rho_noise(u, orders, rng, 1e-3)
    _, g = oracle.functional(mesh, orders, u)
    psi_ref, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=form)
    plan = dg.Plan(mesh, orders)
    ud, gd = plan.to_plan(u), plan.to_plan(g)
    psi, iters, relres = dg.adjoint_solve(plan, ud, gd, restart=200, max_iter=4000, rtol=1e-11, form=form)
    assert relres <= 1e-11 and iters > 0
    # the reported residual, recomputed with an independent VJP call
    r = dg.residual_vjp(plan, ud, psi, form=form) - gd
    assert float(torch.linalg.vector_norm(r)) <= 2e-11 * float(torch.linalg.vector_norm(gd))
    # the oracle's adjoint equation (finite-difference Jacobian, error ~1e-9 relative)
    psi_n = plan.to_natural(psi)
    assert np.linalg.norm(Jac.T @ psi_n - g) <= 1e-6 * np.linalg.norm(g)
    cond = np.linalg.cond(Jac)
    assert np.linalg.norm(psi_n - psi_ref) <= 1e-9 * cond * np.linalg.norm(psi_ref)


def test_zero_right_hand_side_and_errors():
    mesh = wl.box_mesh((2, 2, 2), bc=(1, 2, 0, 0, 0, 0))
    plan = dg.Plan(mesh, np.full((8, 3), 2, dtype=np.int32))
    rng = np.random.default_rng(5)
    u = plan.to_plan(wl.random_state(plan.orders_natural, rng))
    g = torch.zeros_like(u)
    psi, iters, relres = dg.adjoint_solve(plan, u, g)
    assert iters == 0 and relres == 0.0 and float(psi.abs().max()) == 0.0
    with pytest.raises(dg.DGError):
        dg.adjoint_solve(plan, u, u, restart=0)
    with pytest.raises(dg.DGError):
        dg.adjoint_solve(plan, u, u, restart=201)
