"""GPU adjoint solve (dg_adjoint_solve: restarted GMRES on the residual VJP) against the
oracle's dense adjoint (complex-step Jacobian of the oracle residual, numpy solve):
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
    # the oracle's adjoint equation (complex-step Jacobian, exact to rounding) holds to the
    # solver's tolerance, and the solutions agree to it times the condition number
    psi_n = plan.to_natural(psi)
    assert np.linalg.norm(Jac.T @ psi_n - g) <= 3e-11 * np.linalg.norm(g)
    cond = np.linalg.cond(Jac)
    assert np.linalg.norm(psi_n - psi_ref) <= 3e-11 * cond * np.linalg.norm(psi_ref)


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


def test_adjoint_weighted_estimate_from_the_solved_adjoint():
    """The chain the adjoint serves: the x-force adjoint of the traditional form solved on
    the GPU, then eta = sum over coarse nodes of (I psi) tau_trad per element, against the
    oracle's dense adjoint and its adjoint-weighted estimate."""
    rng = np.random.default_rng(42)
    mesh = wl.box_mesh((2, 2, 2), bc=(1, 2, 0, 0, 0, 0), qfar=wl.conserved(*(np.array(x) for x in
                                                                           (1.0, 0.3, 0.0, 0.0, 1.0))))
    fo = wl.random_orders(8, 1, 2, rng)
    co = np.ones_like(fo)
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.3, amp=0.2)
    u = wl.add_rho_noise(u, fo, rng, 1e-3)
    _, g = oracle.functional(mesh, fo, u)
    psi_ref, Jac = adjoint.adjoint_solve(mesh, fo, u, g, form=dg.FORM_TRAD)
    dudt = oracle.residual(mesh, fo, u)
    eta_ref = oracle.tau_eta(mesh, fo, co, u, dudt, psi_ref)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    ud = fine.to_plan(u)
    psi, _, relres = dg.adjoint_solve(fine, ud, fine.to_plan(g), restart=200, max_iter=4000, rtol=1e-11,
                                      form=dg.FORM_TRAD)
    assert relres <= 1e-11
    _, tt, _, eta = dg.tau_estimate(fine, coarse, ud, None, False, psi, psi_form=dg.FORM_TRAD)
    got = coarse.elem_to_natural(eta.cpu().numpy())
    # error budget: the solver's tolerance times the condition number, carried through the
    # sum of |I psi| |tau_trad|
    scale = np.sum(np.abs(oracle.restrict(fo, co, psi_ref)) * np.abs(coarse.to_natural(tt)))
    assert np.max(np.abs(got - eta_ref)) <= 3e-11 * np.linalg.cond(Jac) * scale


@pytest.mark.parametrize("restart", [7, 8, 9, 17])
def test_restart_lengths_and_determinism(restart):
    """Krylov bases around the eight-vector width of one inner-product pass: two solves
    agree bitwise (fixed partition and summation order of every reduction), and the
    reported relative residual is that of the returned psi, recomputed with a separate
    VJP."""
    rng = np.random.default_rng(50 + restart)
    mesh = wl.box_mesh((2, 2, 2), bc=(1, 2, 0, 0, 0, 0), qfar=wl.conserved(*(np.array(x) for x in
                                                                           (1.0, 0.3, 0.0, 0.0, 1.0))))
    orders = wl.random_orders(8, 1, 3, rng)
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.3, amp=0.2)
    u = wl.add_rho_noise(u, orders, rng, 1e-3)
    _, g = oracle.functional(mesh, orders, u)
    plan = dg.Plan(mesh, orders)
    ud, gd = plan.to_plan(u), plan.to_plan(g)
    form = dg.FORM_NEW
    psi1, it1, rr1 = dg.adjoint_solve(plan, ud, gd, restart=restart, max_iter=400, rtol=1e-10, form=form)
    psi2, it2, rr2 = dg.adjoint_solve(plan, ud, gd, restart=restart, max_iter=400, rtol=1e-10, form=form)
    assert torch.equal(psi1, psi2) and it1 == it2 and rr1 == rr2
    assert it1 > restart  # at least one restart
    r = dg.residual_vjp(plan, ud, psi1, form=form) - gd
    true_rel = float(torch.linalg.vector_norm(r)) / float(torch.linalg.vector_norm(gd))
    assert abs(true_rel - rr1) <= 1e-8 * rr1 + 1e-14
