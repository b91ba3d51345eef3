"""GPU parity on curved elements (the sine-mapped box of the Navier-Stokes workload)
against the FP64 oracle: node coordinates and metric terms; the Euler and
Navier-Stokes residuals (both forms, isolated, periodic and far-field boxes, mortars on
the x and y faces) in FP64 and FP32; RK3 steps; the isolated and coupled
tau-estimates (sampling and L2 restriction) and the coupled one's refusal below the
geometry order; the isolated sweep (Euler and Navier-Stokes, curved and box);
the 32 x 32 x 2 vortex workload on the curved mesh."""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import residual_scale, sweep_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

MU, PR = 0.01, 0.72
TOL64, TOL32 = 1e-12, 1e-5
A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
QINF = tuple(float(v) for v in wl.conserved(*(np.array(x) for x in (1.0, 0.3, 0.2, 0.0, 1.0))))


def _mesh(n, bc=(0,) * 6, flux=wl.ROE, ns=False):
    m = wl.sine_mapped(wl.box_mesh(n, hi=(1.0, 1.0, n[2] / n[0]), bc=bc, flux=flux, qfar=QINF))
    return wl.ns_mesh(m, MU, PR) if ns else m


def err(x, ref, s):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), s))


def _case(n, orng, seed, bc=(0,) * 6, flux=wl.ROE, ns=False, state="random", per_element=False):
    """per_element: (Nx, Ny) drawn per element and Nz in 1..2, so faces between the
    layers are non-conforming too; otherwise per element column with Nz = 1."""
    rng = np.random.default_rng(seed)
    mesh = _mesh(n, bc, flux, ns)
    if per_element:
        orders = wl.element_orders(mesh, *orng, rng, nz_range=(1, 2))
    else:
        orders = wl.column_orders(mesh, *orng, rng)
    if state == "random":
        u = wl.random_state(orders, rng)
    else:
        u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.15)
        u = wl.add_rho_noise(u, orders, rng, 1e-3)
    return mesh, orders, u, rng


def _resid(mesh, orders, u, **kw):
    if mesh.get("mu") is not None:
        return oracle.residual_ns(mesh, orders, u, mesh["mu"], mesh["Pr"], **kw)
    return oracle.residual(mesh, orders, u, **kw)


def test_coordinates_and_metrics():
    mesh, orders, u, _ = _case((4, 3, 2), (2, 6), 90)
    plan = dg.Plan(mesh, orders)
    xyz = plan.to_natural(plan.node_coords(), nv=3)
    assert np.max(np.abs(xyz - oracle.node_coords(mesh, orders))) < 1e-14
    met = plan.to_natural(plan.metrics(), nv=10)
    ref = oracle.metrics(mesh, orders)
    assert np.max(np.abs(met - ref)) < 1e-13 * np.max(np.abs(ref))
    # coarse plans sample the fine geometry at their nodes
    co = orders.copy()
    co[:, :2] = np.minimum(orders[:, :2], np.random.default_rng(1).integers(1, 6, (len(orders), 2)))
    cplan = plan.coarse(co)
    metc = cplan.to_natural(cplan.metrics(), nv=10)
    refc = oracle.metrics(mesh, co)
    assert np.max(np.abs(metc - refc)) < 1e-13 * np.max(np.abs(refc))


CASES = [((3, 3, 2), (2, 6), 91, (0,) * 6, wl.ROE, False),
         ((3, 2, 2), (2, 5), 92, (2, 2, 0, 0, 0, 0), wl.ROE, False),
         ((2, 3, 2), (2, 4), 93, (0, 0, 1, 1, 0, 0), wl.LF, False),
         ((3, 3, 2), (2, 6), 191, (0,) * 6, wl.ROE, True),
         ((3, 2, 3), (2, 5), 192, (2, 2, 0, 0, 0, 0), wl.LF, True)]


@pytest.mark.parametrize("n,orng,seed,bc,flux,per_element", CASES)
@pytest.mark.parametrize("ns", [False, True])
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True)])
def test_residual_fp64(n, orng, seed, bc, flux, per_element, ns, form, isolated):
    mesh, orders, u, _ = _case(n, orng, seed, bc, flux, ns, per_element=per_element)
    plan = dg.Plan(mesh, orders)
    ref = _resid(mesh, orders, u, form=form, isolated=isolated)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u), form=form, isolated=isolated))
    s = residual_scale(mesh, orders, u)
    if form == 1:
        s *= np.prod(1.0 / np.asarray(mesh["n"])) / 8
    assert err(got, ref, s) < TOL64


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("ns", [False, True])
def test_residual_fp32(ns, per_element):
    mesh, orders, u, _ = _case((3, 3, 2), (2, 6), 94, ns=ns, per_element=per_element)
    plan = dg.Plan(mesh, orders)
    ref = _resid(mesh, orders, u)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u, dtype=torch.float32))).astype(np.float64)
    assert err(got, ref, residual_scale(mesh, orders, u)) < TOL32


@pytest.mark.parametrize("per_element", [False, True])
def test_free_stream_on_the_gpu(per_element):
    mesh, orders, _, _ = _case((3, 3, 2), (2, 6), 95, bc=(2, 2, 0, 0, 0, 0), ns=True, per_element=per_element)
    u = wl.uniform_state(orders, np.array(QINF))
    plan = dg.Plan(mesh, orders)
    r = dg.residual(plan, plan.to_plan(u)).cpu().numpy()
    assert np.max(np.abs(r)) < 1e-13 * residual_scale(mesh, orders, u)


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_rk3_ns(dtype, tol, per_element):
    mesh, orders, u, _ = _case((3, 3, 2), (2, 5), 96, ns=True, state="pulse", per_element=per_element)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u, dtype=dtype)
    g = torch.empty_like(ud)
    dt = 2e-4
    dg.rk3_step(plan, ud, g, dt, 3)
    ref = u.copy()
    for _ in range(3):
        G = np.zeros_like(ref)
        for k in range(3):
            r = _resid(mesh, orders, ref)
            G = -dt * r if k == 0 else A[k] * G - dt * r
            ref = ref + B[k] * G
    assert np.max(np.abs(plan.to_natural(ud).astype(np.float64) - ref)) < tol * np.max(np.abs(ref))


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("ns,isolated,restriction", [(False, True, 0), (True, True, 0), (False, False, 0),
                                                     (True, False, 0), (False, False, 1), (True, True, 1)])
def test_tau(ns, isolated, restriction, per_element):
    """Isolated estimates at any coarse order; coupled ones with coarse orders at or
    above the geometry order (2, 2, 1), mortars between the coarse orders."""
    mesh, fo, u, rng = _case((3, 3, 2), (2, 6), 97, ns=ns, state="pulse", per_element=per_element)
    co = fo.copy()
    lo = 1 if isolated else 2
    co[:, :2] = np.maximum(lo, np.minimum(fo[:, :2], rng.integers(1, 6, (len(fo), 2))))
    dudt = _resid(mesh, fo, u)
    R = oracle.project if restriction else oracle.restrict
    rc = _resid(mesh, co, R(fo, co, u), isolated=isolated)
    ref = rc - R(fo, co, dudt)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    tn, tt, norms = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated, restriction=restriction)
    s = np.max(np.abs(rc))  # the coarse residual of which tau is a difference
    assert err(coarse.to_natural(tn), ref, s) < TOL64
    Jc = oracle.metrics(mesh, co).reshape(-1)
    # traditional form: J w w w tau_new with the coarse J of every node
    offs = wl.node_offsets(co)
    www = []
    for e, o in enumerate(co):
        w = [oracle.lgl(int(N))[1] for N in o]
        ne = int(offs[e + 1] - offs[e])
        J = Jc[10 * offs[e] + 9 * ne: 10 * offs[e] + 10 * ne]
        www.append(np.tile(J * np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1), 5))
    jw = np.concatenate(www)
    assert err(coarse.to_natural(tt), ref * jw, np.max(np.abs(rc * jw))) < TOL64
    nrm = coarse.elem_to_natural(norms.cpu().numpy())
    mx = np.array([np.max(np.abs(ref[5 * offs[e]:5 * offs[e + 1]])) for e in range(len(co))])
    assert err(nrm[:, 0], mx, s) < TOL64


def test_coupled_tau_below_the_geometry_order_refused():
    mesh, fo, u, _ = _case((2, 2, 2), (2, 4), 96)
    co = fo.copy()
    co[0, 0] = 1
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    with pytest.raises(dg.DGError):
        dg.tau_estimate(fine, coarse, fine.to_plan(u), None, False)
    dg.tau_estimate(fine, coarse, fine.to_plan(u), None, True)  # the isolated one is defined


@pytest.mark.parametrize("curved,ns", [(True, False), (True, True), (False, True)])
def test_sweep(curved, ns):
    rng = np.random.default_rng(98)
    n = (2, 2, 2)
    base = wl.box_mesh(n, hi=(1.0, 1.0, 1.0))
    mesh = wl.sine_mapped(base) if curved else base
    if ns:
        mesh = wl.ns_mesh(mesh, MU, PR)
    orders = wl.element_orders(mesh, 2, 5, rng, nz_range=(1, 3)) if curved else wl.random_orders(8, 1, 5, rng)
    u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.2)
    u = wl.add_rho_noise(u, orders, rng, 1e-3)
    dudt = _resid(mesh, orders, u)
    if ns:
        ten_r, tet_r, offs = oracle.sweep_ns(mesh, orders, u, dudt, MU, PR)
    else:
        ten_r, tet_r, offs = oracle.sweep(mesh, orders, u, dudt)
    plan = dg.Plan(mesh, orders)
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u), plan.to_plan(dudt))
    off = plan.combo_offsets()
    nat = lambda t: np.concatenate([t.cpu().numpy()[off[p]:off[p + 1]] for p in np.argsort(plan.perm)])
    sn, st = sweep_scale(mesh, orders, u, ns=(MU, PR) if ns else None)
    assert err(nat(ten), ten_r, sn) < TOL64
    assert err(nat(tet), tet_r, st) < TOL64


@pytest.mark.slow
def test_c3_workload_curved():
    """The vortex workload on the sine-mapped 32 x 32 x 2 mesh: 10 FP32 RK3 steps at
    dt = 1e-5 against the FP64 oracle composition, the isolated FP64 estimate on a drawn
    coarse map, and the sweep of a sample of elements."""
    mesh, orders, rng = wl.c3()
    u = wl.c3_state(oracle.node_coords(mesh, orders), orders, mesh, rng)
    plan = dg.Plan(mesh, orders)
    u32 = plan.to_plan(u, dtype=torch.float32)
    g = torch.empty_like(u32)
    dg.rk3_step(plan, u32, g, 1e-5, 10)
    ref = u.copy()
    for _ in range(10):
        G = np.zeros_like(ref)
        for k in range(3):
            r = _resid(mesh, orders, ref)
            G = -1e-5 * r if k == 0 else A[k] * G - 1e-5 * r
            ref = ref + B[k] * G
    e32 = np.max(np.abs(plan.to_natural(u32).astype(np.float64) - ref)) / np.max(np.abs(ref))
    assert e32 < 1e-5
    dudt = _resid(mesh, orders, u)
    co = orders.copy()
    co[:, :2] = np.minimum(orders[:, :2], rng.integers(1, 6, (len(orders), 2)))
    tref = _resid(mesh, co, oracle.restrict(orders, co, u), isolated=True) - oracle.restrict(orders, co, dudt)
    coarse = plan.coarse(co)
    tn, _, _ = dg.tau_estimate(plan, coarse, plan.to_plan(u), None, True)
    # At p = 1/(gamma Ma^2) = 17.9 on curved elements the residuals' own rounding exceeds
    # 1e-12 of max |r^Nc(Q^c)| (about 85 here): the oracle's residual of the exact free
    # stream on this mesh, zero in exact arithmetic, is 2.7e-8 (fine) and 9.5e-9 (coarse,
    # isolated).  The estimate is measured against the cancelling-term scale s instead.
    s = residual_scale(mesh, orders, u)
    assert err(coarse.to_natural(tn), tref, s) < TOL64
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u), plan.to_plan(dudt))
    sample = np.sort(rng.choice(len(orders), 48, replace=False))
    ten_r, _, offs = oracle.sweep_ns(mesh, orders, u, dudt, mesh["mu"], mesh["Pr"], elems=sample)
    off = plan.combo_offsets()
    inv = plan.inv_perm()
    got = np.concatenate([ten.cpu().numpy()[off[inv[e]]:off[inv[e] + 1]] for e in sample])
    assert err(got, ten_r, s) < TOL64
