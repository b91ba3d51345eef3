"""The adaptation loops of Section 2.4 as library entry points (dg_adapt_dynamic,
dg_adapt_static) against the same loops composed from the oracle: RK3 steps, the
isolated truncation-error map, the degree selection (oracle/select.py: decrease limit
and jump condition (b) for the dynamic loop, approach 1 or 2 over the stored maps for
the static one), the projection onto the selected degrees.  Degrees are compared bit
for bit at every stage, the final state at 1e-11 of its size, and the step-weighted
number of degrees of freedom of Section 3.2 exactly.

The threshold tau_max is picked by running the oracle loop: the first candidate that
changes the degrees and keeps every map value of every stage at least 1e-6 (relative)
away from it, so that rounding differences between the two sides cannot move a
combination across it."""
import numpy as np
import pytest

import oracle
from oracle import select as sel
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

DT, K = 2e-3, 4


def _setup(seed):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh((4, 3, 2), hi=(1.0, 0.75, 0.5))
    orders = np.full((24, 3), 5, dtype=np.int32)
    orders[rng.random(24) < 0.3, 0] = 4
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.15)
    return mesh, orders, wl.add_rho_noise(u, orders, rng, 1e-3)


def _margin(m, t):
    m = m[np.isfinite(m)]
    return float(np.min(np.abs(m - t)) / t)


def _oracle_dynamic(mesh, orders, u, nstages, t, nmin, nmax, form):
    stages, margin, ndof = [], np.inf, 0
    for _ in range(nstages):
        u = oracle.rk3(mesh, orders, u, DT, K)
        ndof += int(wl.node_offsets(orders)[-1]) * K
        ten, tet, _ = oracle.sweep(mesh, orders, u, oracle.residual(mesh, orders, u))
        m = ten if form == dg.FORM_NEW else tet
        margin = min(margin, _margin(m, t))
        new = sel.select_orders(orders, [m], t, nmin, nmax, 1)
        new = sel.apply_jump(mesh, sel.limit_decrease(new, orders, 1, nmax), 2)
        u = oracle.project(orders, new, u)
        orders = new
        stages.append(new)
    return stages, u, margin, ndof / (nstages * K)


def _oracle_static(mesh, orders, u, nstages, after, t, nmin, nmax, approach, form):
    maps, margin = [], np.inf
    for _ in range(nstages):
        u = oracle.rk3(mesh, orders, u, DT, K)
        ten, tet, _ = oracle.sweep(mesh, orders, u, oracle.residual(mesh, orders, u))
        maps.append(ten if form == dg.FORM_NEW else tet)
        margin = min(margin, _margin(maps[-1], t))
    if approach == 2:
        margin = min(margin, _margin(np.max(np.stack(maps), axis=0), t))
    new = sel.apply_jump(mesh, sel.select_orders(orders, maps, t, nmin, nmax, approach), 2)
    ndof = (int(wl.node_offsets(orders)[-1]) * nstages * K + int(wl.node_offsets(new)[-1]) * after)
    u = oracle.project(orders, new, u)
    u = oracle.rk3(mesh, new, u, DT, after)
    return new, u, margin, ndof / (nstages * K + after)


def _pick(run, orders, first_map):
    v = np.sort(first_map[np.isfinite(first_map) & (first_map > 0)])
    for q in (0.5, 0.35, 0.65, 0.2, 0.8, 0.1, 0.9):
        lo, hi = v[int(q * (len(v) - 1))], v[min(len(v) - 1, int(q * (len(v) - 1)) + 1)]
        t = float(np.sqrt(lo * hi)) if lo > 0 else float(hi / 2)
        res = run(t)
        changed = not np.array_equal(np.asarray(res[0][-1] if isinstance(res[0], list) else res[0]), orders)
        if res[2] > 1e-6 and changed:
            return t, res
    pytest.fail("no threshold with a safe margin")


@pytest.mark.parametrize("form", [dg.FORM_NEW, dg.FORM_TRAD])
def test_dynamic_loop(form):
    mesh, orders, u0 = _setup(11)
    nstages, nmin, nmax = 3, 2, 7
    u1 = oracle.rk3(mesh, orders, u0, DT, K)
    ten, tet, _ = oracle.sweep(mesh, orders, u1, oracle.residual(mesh, orders, u1))
    t, (stages, u_ref, _, ndof_ref) = _pick(
        lambda t: _oracle_dynamic(mesh, orders, u0, nstages, t, nmin, nmax, form), orders,
        ten if form == dg.FORM_NEW else tet)
    plan = dg.Plan(mesh, orders)
    new_plan, u, got, rep = dg.adapt_dynamic(plan, plan.to_plan(u0), DT, K, nstages, t, nmin=nmin, nmax=nmax,
                                             jump=2, max_decrease=1, form=form)
    for s in range(nstages):
        assert np.array_equal(got[s], stages[s]), s
    assert np.array_equal(new_plan.orders_natural, stages[-1])
    assert np.max(np.abs(new_plan.to_natural(u) - u_ref)) < 1e-11 * np.max(np.abs(u_ref))
    assert rep["steps"] == nstages * K and rep["ndof_final"] == int(wl.node_offsets(stages[-1])[-1])
    assert rep["ndof_dyn"] == ndof_ref


@pytest.mark.parametrize("approach", [1, 2])
def test_static_loop(approach):
    mesh, orders, u0 = _setup(12)
    nstages, after, nmin, nmax = 3, 5, 1, 8
    u1 = oracle.rk3(mesh, orders, u0, DT, K)
    ten, _, _ = oracle.sweep(mesh, orders, u1, oracle.residual(mesh, orders, u1))
    t, (new, u_ref, _, ndof_ref) = _pick(
        lambda t: _oracle_static(mesh, orders, u0, nstages, after, t, nmin, nmax, approach, dg.FORM_NEW),
        orders, ten)
    plan = dg.Plan(mesh, orders)
    new_plan, u, got, rep = dg.adapt_static(plan, plan.to_plan(u0), DT, K, nstages, after, t, nmin=nmin,
                                            nmax=nmax, jump=2, approach=approach)
    assert np.array_equal(got[0], new) and np.array_equal(new_plan.orders_natural, new)
    assert np.max(np.abs(new_plan.to_natural(u) - u_ref)) < 1e-11 * np.max(np.abs(u_ref))
    assert rep["steps"] == nstages * K + after
    assert abs(rep["ndof_dyn"] - ndof_ref) <= 1e-12 * ndof_ref


def test_loop_arguments_refused():
    mesh, orders, u0 = _setup(13)
    plan = dg.Plan(mesh, orders)
    u = plan.to_plan(u0)
    with pytest.raises(dg.DGError, match="nstages"):
        dg.adapt_dynamic(plan, u, DT, K, 0, 1e-2)
    ns = dg.Plan(wl.ns_mesh(mesh, 0.01, 0.72), orders)
    with pytest.raises(dg.DGError, match="orders <= 7"):
        dg.adapt_dynamic(ns, ns.to_plan(u0), DT, K, 1, 1e-2, nmax=8)
    with pytest.raises(dg.DGError, match="approach"):
        dg.adapt_static(plan, u, DT, K, 1, 1, 1e-2, approach=3)
