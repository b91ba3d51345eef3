"""GPU degree selection (dg_select_orders) against the oracle, bit-exact: the two-stage
example of Section 2.4.2, random maps with many ties and NaNs over fine orders 1..9 on
a box with periodic, wall and far-field faces (approaches 1 and 2, jump conditions
none, (a) and (b)), the 16 x 16 x 16 order-7 mesh of the isotropic sweep workload,
and argument validation."""
import json
import os

import numpy as np
import pytest

from oracle import select as sel
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "select_two_stage_table.json")


def _gpu(plan, maps_nat, **kw):
    got = dg.select_orders(plan, [plan.map_to_plan(m) for m in maps_nat], **kw)
    return got.cpu().numpy()


def _ref(mesh, orders, maps_nat, tau_max, nmin, nmax, approach, jump):
    o = sel.select_orders(orders, maps_nat, tau_max, nmin, nmax, approach)
    return sel.apply_jump(mesh, o, jump)


def test_table_example():
    with open(GOLD) as f:
        t = json.load(f)
    mesh = wl.box_mesh((1, 1, 1))
    P = (4, 4, 2)
    orders = np.array([P], dtype=np.int32)
    maps = []
    for st in ("stage1", "stage2"):
        ok = {tuple(c) for c in t["passing"][st]}
        maps.append(np.array([0.25 if (N[0], N[1]) in ok else 4.0 for N in sel.combos(P)]))
    plan = dg.Plan(mesh, orders)
    for approach in (1, 2):
        got = _gpu(plan, maps, tau_max=1.0, nmin=t["nmin"], nmax=t["nmax"], approach=approach)
        assert tuple(got[0]) == tuple(t["approach%d" % approach]["degrees"]) + (1,)


CASES = [(a, j, nmin, nmax) for a in (1, 2) for j in (0, 1, 2) for (nmin, nmax) in ((1, 9), (2, 6))]


@pytest.mark.parametrize("approach,jump,nmin,nmax", CASES)
def test_random_maps(approach, jump, nmin, nmax):
    rng = np.random.default_rng(100 + 10 * approach + jump + nmin)
    mesh = wl.box_mesh((6, 5, 4), bc=(0, 0, 1, 1, 2, 2))
    orders = rng.integers(1, 10, (120, 3)).astype(np.int32)
    offs = sel.combo_offsets(orders)
    n = int(offs[-1])
    maps = []
    for _ in range(3):
        m = rng.integers(0, 10, n) / 8.0  # coarse values: ties in both the value and NDOF
        m[rng.random(n) < 0.01] = np.nan
        maps.append(m)
    plan = dg.Plan(mesh, orders)
    got = _gpu(plan, maps, tau_max=0.5, nmin=nmin, nmax=nmax, approach=approach, jump=jump)
    exp = _ref(mesh, orders, maps, 0.5, nmin, nmax, approach, jump)
    assert np.array_equal(got, exp)


def _decaying_maps(orders, nstages, rng):
    """Maps shaped like truncation-error maps in the asymptotic range: per element a
    level A_e and decay rates a_d, value A_e exp(-sum_d a_d N_d) times lognormal noise."""
    offs = sel.combo_offsets(orders)
    maps = [np.empty(int(offs[-1])) for _ in range(nstages)]
    for e, P in enumerate(orders):
        N = np.array(sel.combos(P), dtype=np.float64)
        a = rng.uniform(0.3, 2.0, 3)
        A = np.exp(rng.normal(0.0, 1.0))
        for m in maps:
            m[offs[e]:offs[e + 1]] = A * np.exp(-N @ a + rng.normal(0.0, 0.3, len(N)))
    return maps


@pytest.mark.slow
def test_sweep_workload_size():
    """16 x 16 x 16 elements of order 7 (216 combinations each), two stages of decaying
    maps, approach 2 with jump (b) and approach 1 with jump (a)."""
    rng = np.random.default_rng(7)
    mesh = wl.box_mesh((16, 16, 16))
    orders = np.full((4096, 3), 7, dtype=np.int32)
    maps = _decaying_maps(orders, 2, rng)
    plan = dg.Plan(mesh, orders)
    for approach, jump in ((2, 2), (1, 1)):
        got = _gpu(plan, maps, tau_max=1e-3, nmin=1, nmax=8, approach=approach, jump=jump)
        exp = _ref(mesh, orders, maps, 1e-3, 1, 8, approach, jump)
        assert np.array_equal(got, exp)
        assert len(np.unique(got)) >= 4  # a spread of degrees, not one fallback


def test_sweep_maps_end_to_end():
    """GPU sweep then GPU selection against oracle sweep then oracle selection, on a
    random (asymmetric) state, with tau_max in a wide gap of the oracle's map values so
    that rounding of the two sweeps cannot move a combination across the threshold."""
    import oracle
    rng = np.random.default_rng(8)
    mesh = wl.box_mesh((3, 3, 2))
    orders = wl.random_orders(18, 2, 6, rng)
    u = wl.random_state(orders, rng)
    dudt = oracle.residual(mesh, orders, u)
    ten_r, tet_r, _ = oracle.sweep(mesh, orders, u, dudt)
    plan = dg.Plan(mesh, orders)
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u))
    for m_gpu, m_ref in ((ten, ten_r), (tet, tet_r)):
        v = np.sort(m_ref)
        k = len(v) // 4 + int(np.argmax(v[len(v) // 4 + 1: len(v) // 2] / v[len(v) // 4: len(v) // 2 - 1]))
        tau_max = 0.5 * (v[k] + v[k + 1])
        assert v[k + 1] / v[k] > 1 + 1e-9
        got = dg.select_orders(plan, [m_gpu], tau_max=tau_max, nmin=1, nmax=7, approach=2, jump=2).cpu().numpy()
        exp = _ref(mesh, orders, [m_ref], tau_max, 1, 7, 2, 2)
        assert np.array_equal(got, exp)


def test_invalid_arguments():
    mesh = wl.box_mesh((2, 2, 2))
    plan = dg.Plan(mesh, np.full((8, 3), 3, dtype=np.int32))
    m = torch.zeros(int(plan.combo_offsets()[-1]), dtype=torch.float64, device="cuda")
    for kw in (dict(approach=3), dict(jump=3), dict(nmin=0), dict(nmin=5, nmax=4), dict(nmax=10),
               dict(tau_max=float("nan"))):
        args = dict(tau_max=1.0, nmin=1, nmax=9, approach=2, jump=0)
        args.update(kw)
        with pytest.raises(dg.DGError):
            dg.select_orders(plan, [m], **args)
    with pytest.raises(dg.DGError):
        dg.select_orders(plan, [], tau_max=1.0)
    with pytest.raises(dg.DGError):
        dg.select_orders(plan, [m] * 33, tau_max=1.0)
