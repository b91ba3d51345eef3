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


def _wall_case(shape, N, seed):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh(shape, bc=(1, 2, 0, 0, 0, 0), qfar=wl.conserved(*(np.array(x) for x in
                                                                       (1.0, 0.3, 0.0, 0.0, 1.0))))
    E = int(np.prod(shape))
    orders = wl.uniform_orders(E, N)
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.3, amp=0.2)
    u = wl.add_rho_noise(u, orders, rng, 1e-3)
    return mesh, orders, u, rng


# (2, 2, 2): two colours (even periodic directions); (2, 3, 2): a third colour for the odd
# periodic y direction (12 colours in all)
@pytest.mark.parametrize("shape,N", [((2, 2, 2), 2), ((2, 3, 2), 1)])
@pytest.mark.parametrize("form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_precond_is_the_inverse_of_the_diagonal_blocks(shape, N, form):
    """The element-block Jacobi preconditioner, assembled on the GPU from probing VJPs and
    inverted in FP32, applied to a vector, against the inverse diagonal blocks of the
    oracle's dense adjoint operator (complex-step Jacobian, transposed)."""
    mesh, orders, u, rng = _wall_case(shape, N, 50 + form)
    _, g = oracle.functional(mesh, orders, u)
    _, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=form)
    A = Jac.T
    nd = 5 * (N + 1) ** 3
    E = len(orders)
    x = rng.normal(size=E * nd)
    ref = np.concatenate([np.linalg.solve(A[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd], x[e * nd:(e + 1) * nd])
                          for e in range(E)])
    plan = dg.Plan(mesh, orders)
    pc = dg.adjoint_precond(plan, plan.to_plan(u), form=form)
    z = plan.to_natural(dg.adjoint_precond_apply(plan, pc, plan.to_plan(x)))
    conds = [np.linalg.cond(A[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd]) for e in range(E)]
    # FP32 blocks and inverse: within a few units of 2^-24 times the block condition number
    assert np.max(np.abs(z - ref)) <= 1e-6 * max(conds) * np.max(np.abs(ref))


@pytest.mark.parametrize("form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_preconditioned_solve_matches_dense(form):
    """The right-preconditioned solve converges to the dense oracle adjoint, to the same
    bar as the plain solve, in fewer products."""
    mesh, orders, u, _ = _wall_case((2, 2, 2), 2, 60 + form)
    _, g = oracle.functional(mesh, orders, u)
    psi_ref, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=form)
    plan = dg.Plan(mesh, orders)
    ud, gd = plan.to_plan(u), plan.to_plan(g)
    pc = dg.adjoint_precond(plan, ud, form=form)
    psi, iters, relres = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form, precond=pc)
    _, iters0, _ = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form)
    assert relres <= 1e-11 and 0 < iters < iters0
    r = dg.residual_vjp(plan, ud, psi, form=form) - gd
    assert float(torch.linalg.vector_norm(r)) <= 2e-11 * float(torch.linalg.vector_norm(gd))
    psi_n = plan.to_natural(psi)
    assert np.linalg.norm(Jac.T @ psi_n - g) <= 3e-11 * np.linalg.norm(g)
    assert np.linalg.norm(psi_n - psi_ref) <= 3e-11 * np.linalg.cond(Jac) * np.linalg.norm(psi_ref)


def test_precond_refuses_mixed_orders_and_foreign_plans():
    mesh, orders, u, rng = _wall_case((2, 2, 2), 2, 70)
    plan = dg.Plan(mesh, orders)
    pc = dg.adjoint_precond(plan, plan.to_plan(u))
    other = dg.Plan(mesh, orders)
    with pytest.raises(dg.DGError, match="another plan"):
        dg.adjoint_precond_apply(other, pc, other.to_plan(u))
    mixed = dg.Plan(mesh, wl.random_orders(8, 1, 3, rng))
    with pytest.raises(dg.DGError, match="one order triple"):
        dg.adjoint_precond(mixed, mixed.to_plan(wl.random_state(mixed.orders_natural, rng)))


def test_preconditioned_solve_converges_where_plain_gmres_stalls():
    """The adjoint workload's boundaries and state on 8^3 elements of order 5: plain
    GMRES(30) is still above 1e-2 after 300 products; with the element-block Jacobi
    preconditioner it reaches 1e-8 (about 350 products; the oracle's scipy GMRES with the
    same preconditioner needs 346), the reported residual checked with an independent VJP."""
    mesh, orders = wl.c4(8, 5)
    plan = dg.Plan(mesh, orders)
    u = plan.to_plan(wl.c4_state(plan.to_natural(plan.node_coords(), nv=3), orders))
    _, g = dg.functional(plan, u)
    _, it0, rr0 = dg.adjoint_solve(plan, u, g, restart=30, max_iter=300, rtol=1e-8, form=dg.FORM_TRAD)
    assert rr0 > 1e-2
    pc = dg.adjoint_precond(plan, u, form=dg.FORM_TRAD)
    psi, it, rr = dg.adjoint_solve(plan, u, g, restart=30, max_iter=1500, rtol=1e-8, form=dg.FORM_TRAD, precond=pc)
    assert rr <= 1e-8 and it < 1000
    r = dg.residual_vjp(plan, u, psi, form=dg.FORM_TRAD) - g
    assert float(torch.linalg.vector_norm(r)) <= 2e-8 * float(torch.linalg.vector_norm(g))


@pytest.mark.parametrize("shape,N", [((2, 2, 2), 2), ((2, 3, 2), 1)])
def test_compact_precond_against_dense_blocks(shape, N):
    """The compact form (FP16 blocks over per-column scales) applied to a vector, against
    the inverse diagonal blocks of the oracle's dense adjoint operator: within the FP32
    form's bar plus the FP16 rounding of every block entry, 2^-11 of its column's largest
    (the scales taken from the exact inverse)."""
    mesh, orders, u, rng = _wall_case(shape, N, 80)
    _, g = oracle.functional(mesh, orders, u)
    _, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=dg.FORM_TRAD)
    A = Jac.T
    nd = 5 * (N + 1) ** 3
    E = len(orders)
    x = rng.normal(size=E * nd)
    blocks = [np.linalg.inv(A[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd]) for e in range(E)]
    ref = np.concatenate([blocks[e] @ x[e * nd:(e + 1) * nd] for e in range(E)])
    conds = [np.linalg.cond(A[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd]) for e in range(E)]
    fp16 = max(float(np.abs(blocks[e]).max(axis=0) @ np.abs(x[e * nd:(e + 1) * nd])) for e in range(E))
    plan = dg.Plan(mesh, orders)
    pc = dg.adjoint_precond(plan, plan.to_plan(u))
    pc16 = dg.adjoint_precond_compact(plan, pc)
    assert pc16.numel() < 0.6 * pc.numel()
    z = plan.to_natural(dg.adjoint_precond_apply(plan, pc16, plan.to_plan(x)))
    err = np.max(np.abs(z - ref))
    assert err <= 1e-6 * max(conds) * np.max(np.abs(ref)) + 1.01 * 2.0 ** -11 * fp16
    # and not merely within that bound: the FP16 form does differ from the FP32 one
    z32 = plan.to_natural(dg.adjoint_precond_apply(plan, pc, plan.to_plan(x)))
    assert np.max(np.abs(z - z32)) > 0
    with pytest.raises(dg.DGError, match="already compact"):
        dg.adjoint_precond_compact(plan, pc16)
    other = dg.Plan(mesh, orders)
    with pytest.raises(dg.DGError, match="another plan"):
        dg.adjoint_precond_compact(other, pc)


@pytest.mark.parametrize("form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_compact_preconditioned_solve_matches_dense(form):
    """With the compact preconditioner the solve reaches the same FP64 bar and the dense
    oracle adjoint; its product count stays within a few of the FP32 form's."""
    mesh, orders, u, _ = _wall_case((2, 2, 2), 2, 90 + form)
    _, g = oracle.functional(mesh, orders, u)
    psi_ref, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=form)
    plan = dg.Plan(mesh, orders)
    ud, gd = plan.to_plan(u), plan.to_plan(g)
    pc = dg.adjoint_precond(plan, ud, form=form)
    pc16 = dg.adjoint_precond_compact(plan, pc)
    _, it32, _ = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form, precond=pc)
    psi, it, relres = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form, precond=pc16)
    assert relres <= 1e-11 and it <= it32 + max(3, it32 // 10)
    r = dg.residual_vjp(plan, ud, psi, form=form) - gd
    assert float(torch.linalg.vector_norm(r)) <= 2e-11 * float(torch.linalg.vector_norm(gd))
    psi_n = plan.to_natural(psi)
    assert np.linalg.norm(psi_n - psi_ref) <= 3e-11 * np.linalg.cond(Jac) * np.linalg.norm(psi_ref)


@pytest.mark.parametrize("shape,N", [((2, 2, 2), 2), ((2, 3, 2), 1)])
def test_gauss_seidel_sweep_against_dense(shape, N):
    """The colour-ordered block Gauss-Seidel sweep z = (D + L)^-1 x against forward block
    substitution with the oracle's dense adjoint operator, the colours in the order the
    library reports (two colours, and twelve for the odd periodic y direction)."""
    mesh, orders, u, rng = _wall_case(shape, N, 100)
    _, g = oracle.functional(mesh, orders, u)
    _, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=dg.FORM_TRAD)
    A = Jac.T
    nd = 5 * (N + 1) ** 3
    E = len(orders)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    pc = dg.adjoint_precond(plan, ud)
    colour = dg.adjoint_precond_colours(plan, pc)
    # face neighbours differ in colour: no coupling block between two elements of a colour
    for e in range(E):
        for f in range(E):
            if e != f and colour[e] == colour[f]:
                assert not np.any(A[e * nd:(e + 1) * nd, f * nd:(f + 1) * nd])
    x = rng.normal(size=E * nd)
    ref = np.zeros(E * nd)
    for c in range(int(colour.max()) + 1):
        for e in np.where(colour == c)[0]:
            s = slice(e * nd, (e + 1) * nd)
            ref[s] = np.linalg.solve(A[s, s], x[s] - A[s, :] @ ref)
    z = plan.to_natural(dg.adjoint_precond_apply_gs(plan, pc, ud, plan.to_plan(x)))
    conds = [np.linalg.cond(A[e * nd:(e + 1) * nd, e * nd:(e + 1) * nd]) for e in range(E)]
    assert np.max(np.abs(z - ref)) <= 1e-5 * max(conds) * np.max(np.abs(ref))


@pytest.mark.parametrize("form", [dg.FORM_TRAD, dg.FORM_NEW])
def test_gauss_seidel_solve_matches_dense(form):
    """The solve with the Gauss-Seidel sweep reaches the dense oracle adjoint at the same
    FP64 bar, in fewer products than with block Jacobi."""
    mesh, orders, u, _ = _wall_case((2, 2, 2), 2, 110 + form)
    _, g = oracle.functional(mesh, orders, u)
    psi_ref, Jac = adjoint.adjoint_solve(mesh, orders, u, g, form=form)
    plan = dg.Plan(mesh, orders)
    ud, gd = plan.to_plan(u), plan.to_plan(g)
    pc = dg.adjoint_precond(plan, ud, form=form)
    _, itj, _ = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form, precond=pc)
    psi, it, relres = dg.adjoint_solve(plan, ud, gd, restart=30, max_iter=4000, rtol=1e-11, form=form, precond=pc,
                                       sweep=dg.PRECOND_GAUSS_SEIDEL)
    assert relres <= 1e-11 and it < itj
    r = dg.residual_vjp(plan, ud, psi, form=form) - gd
    assert float(torch.linalg.vector_norm(r)) <= 2e-11 * float(torch.linalg.vector_norm(gd))
    psi_n = plan.to_natural(psi)
    assert np.linalg.norm(psi_n - psi_ref) <= 3e-11 * np.linalg.cond(Jac) * np.linalg.norm(psi_ref)
    with pytest.raises(dg.DGError, match="unknown preconditioner sweep"):
        dg.adjoint_solve(plan, ud, gd, precond=pc, sweep=7)


def test_gauss_seidel_on_the_adjoint_workload():
    """8^3 elements of order 5 with the adjoint workload's boundaries and state: the
    compact preconditioner applied as the Gauss-Seidel sweep reaches 1e-8 in well under
    the block-Jacobi product count, the residual checked with an independent VJP."""
    mesh, orders = wl.c4(8, 5)
    plan = dg.Plan(mesh, orders)
    u = plan.to_plan(wl.c4_state(plan.to_natural(plan.node_coords(), nv=3), orders))
    _, g = dg.functional(plan, u)
    pc = dg.adjoint_precond_compact(plan, dg.adjoint_precond(plan, u, form=dg.FORM_TRAD))
    _, itj, rrj = dg.adjoint_solve(plan, u, g, restart=30, max_iter=1500, rtol=1e-8, form=dg.FORM_TRAD, precond=pc)
    psi, it, rr = dg.adjoint_solve(plan, u, g, restart=30, max_iter=1500, rtol=1e-8, form=dg.FORM_TRAD, precond=pc,
                                   sweep=dg.PRECOND_GAUSS_SEIDEL)
    assert rrj <= 1e-8 and rr <= 1e-8 and it < 0.7 * itj
    r = dg.residual_vjp(plan, u, psi, form=dg.FORM_TRAD) - g
    assert float(torch.linalg.vector_norm(r)) <= 2e-8 * float(torch.linalg.vector_norm(g))
