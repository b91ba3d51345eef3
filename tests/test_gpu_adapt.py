"""GPU solution transfer between order maps (dg_project) and the per-stage decrease
limit of the selection against the oracle; two stages of dynamic p-adaptation
(advance, isolated sweep, selection with the decrease limit and jump condition (b),
re-planning, projection) run on the GPU and in the oracle side by side."""
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


def _rel(x, ref):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


@pytest.mark.parametrize("seed", [1, 2])
def test_project_random_orders(seed):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh((4, 3, 3))
    fo = wl.random_orders(36, 1, 9, rng)
    to = wl.random_orders(36, 1, 9, rng)
    to[:6] = fo[:6]                       # unchanged elements
    to[6:12] = np.minimum(9, fo[6:12] + 1)  # raised in every direction
    u = wl.random_state(fo, rng)
    src, dst = dg.Plan(mesh, fo), dg.Plan(mesh, to)
    got = dst.to_natural(dg.project(src, dst, src.to_plan(u)))
    assert _rel(got, oracle.project(fo, to, u)) < 1e-12
    # coarse plans are valid sources and targets
    co = np.minimum(fo, rng.integers(1, 10, fo.shape)).astype(np.int32)
    cplan = src.coarse(co)
    got = dst.to_natural(dg.project(cplan, dst, cplan.to_plan(oracle.restrict(fo, co, u))))
    assert _rel(got, oracle.project(co, to, oracle.restrict(fo, co, u))) < 1e-12


def test_project_sweep_workload_size():
    """16^3 elements of order 7 onto orders drawn in 1..9, checked on 512 sampled elements."""
    rng = np.random.default_rng(3)
    mesh = wl.box_mesh(16)
    fo = wl.uniform_orders(4096, 7)
    to = wl.random_orders(4096, 1, 9, rng)
    src, dst = dg.Plan(mesh, fo), dg.Plan(mesh, to)
    u = wl.random_state(fo, rng)
    got = dst.to_natural(dg.project(src, dst, src.to_plan(u)))
    sample = np.sort(rng.choice(4096, 512, replace=False))
    offs_f, offs_t = wl.node_offsets(fo), wl.node_offsets(to)
    u_s = np.concatenate([u[5 * offs_f[e]:5 * offs_f[e + 1]] for e in sample])
    g_s = np.concatenate([got[5 * offs_t[e]:5 * offs_t[e + 1]] for e in sample])
    assert _rel(g_s, oracle.project(fo[sample], to[sample], u_s)) < 1e-12


def test_decrease_limit():
    rng = np.random.default_rng(4)
    mesh = wl.box_mesh((5, 4, 3), bc=(0, 0, 1, 1, 0, 0))
    orders = rng.integers(2, 9, (60, 3)).astype(np.int32)
    offs = sel.combo_offsets(orders)
    maps = [rng.integers(0, 10, int(offs[-1])) / 8.0]
    plan = dg.Plan(mesh, orders)
    prev = torch.from_numpy(orders.copy()).cuda()
    for dec, jump in ((1, 0), (1, 2), (2, 1), (0, 0)):
        got = dg.select_orders(plan, [plan.map_to_plan(maps[0])], tau_max=0.5, nmin=1, nmax=8, approach=2,
                               jump=jump, prev=prev, max_decrease=dec).cpu().numpy()
        exp = sel.select_orders(orders, maps, 0.5, 1, 8, 2)
        exp = sel.apply_jump(mesh, sel.limit_decrease(exp, orders, dec, 8), jump)
        assert np.array_equal(got, exp)


def _gap_threshold(v):
    """tau_max at the middle of the widest relative gap between consecutive sorted map
    values in the central half: no rounding can move a value across it."""
    v = np.sort(v[v > 0])
    lo, hi = len(v) // 4, 3 * len(v) // 4
    k = lo + int(np.argmax(v[lo + 1:hi + 1] / v[lo:hi]))
    assert v[k + 1] / v[k] > 1 + 1e-6
    return 0.5 * (v[k] + v[k + 1])


def test_dynamic_adaptation_two_stages():
    rng = np.random.default_rng(6)
    mesh = wl.box_mesh((4, 3, 2), hi=(1.0, 0.75, 0.5))
    orders = np.full((24, 3), 5, dtype=np.int32)
    u_ref = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.15)
    u_ref = wl.add_rho_noise(u_ref, orders, rng, 1e-3)
    plan = dg.Plan(mesh, orders)
    u = plan.to_plan(u_ref)
    g = torch.empty_like(u)
    dt, nsteps = 2e-3, 5
    for stage in range(2):
        # advance
        dg.rk3_step(plan, u, g, dt, nsteps)
        u_ref = oracle.rk3(mesh, orders, u_ref, dt, nsteps)
        assert _rel(plan.to_natural(u), u_ref) < 1e-11
        # estimate: isolated truncation-error map (new form)
        dudt_ref = oracle.residual(mesh, orders, u_ref)
        ten_ref, _, _ = oracle.sweep(mesh, orders, u_ref, dudt_ref)
        ten, _ = dg.tau_sweep(plan, u)
        tau_max = _gap_threshold(ten_ref)
        # select: one order down at most per stage, jump condition (b)
        prev = torch.from_numpy(orders.copy()).cuda()
        new = dg.select_orders(plan, [ten], tau_max=tau_max, nmin=1, nmax=7, approach=2, jump=2, prev=prev,
                               max_decrease=1).cpu().numpy()
        exp = sel.select_orders(orders, [ten_ref], tau_max, 1, 7, 2)
        exp = sel.apply_jump(mesh, sel.limit_decrease(exp, orders, 1, 7), 2)
        assert np.array_equal(new, exp)
        assert not np.array_equal(new, orders)
        # adapt: new plan, solution projected onto it
        new_plan = dg.Plan(mesh, new)
        u = dg.project(plan, new_plan, u)
        u_ref = oracle.project(orders, new, u_ref)
        plan, orders = new_plan, new
        g = torch.empty_like(u)
        assert _rel(plan.to_natural(u), u_ref) < 1e-11


def test_total_map_fmax():
    """Static adaptation: the F_max total map accumulated on the GPU equals numpy's
    NaN-propagating maximum, and selecting from it equals approach 2 over the stages."""
    rng = np.random.default_rng(7)
    mesh = wl.box_mesh((5, 4, 3))
    orders = rng.integers(1, 10, (60, 3)).astype(np.int32)
    plan = dg.Plan(mesh, orders)
    n = int(plan.combo_offsets()[-1])
    maps = []
    for _ in range(4):
        m = rng.integers(0, 12, n) / 8.0
        m[rng.random(n) < 0.005] = np.nan
        maps.append(m)
    dev = [torch.from_numpy(m).cuda() for m in maps]
    acc = dev[0].clone()
    for m in dev[1:]:
        dg.map_fmax(plan, acc, m)
    exp = maps[0]
    for m in maps[1:]:
        exp = np.maximum(exp, m)
    got = acc.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(exp))
    assert np.array_equal(got[~np.isnan(got)], exp[~np.isnan(exp)])
    for jump in (0, 2):
        a = dg.select_orders(plan, [acc], tau_max=0.7, nmin=1, nmax=9, approach=2, jump=jump)
        b = dg.select_orders(plan, dev, tau_max=0.7, nmin=1, nmax=9, approach=2, jump=jump)
        assert torch.equal(a, b)
