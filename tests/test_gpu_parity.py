"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Tolerance (FP64): max |x - x_oracle| <= 1e-12 * max(max |x_oracle|, s).  For residuals s
is the scale of their cancelling terms (largest |f| * |Ja| * ||D|| / J); for tau-estimates
and the sweep's maps s is max |r^Nc(Q^c)|, the size of the coarse residual of the
restricted state, of which the estimate is a difference (same form as the output).  FP32
state and arithmetic: 1e-5 on the same measure.  Integer layout data must match exactly.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import residual_scale, sweep_scale, tau_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

TOL64 = 1e-12
TOL32 = 1e-5


def err(x, ref, s):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), s)) if x.size else 0.0


def _case(shape, lo, hi, seed, bc=(0,) * 6, flux=wl.ROE, hi_len=(1.0, 1.0, 1.0), state="random"):
    rng = np.random.default_rng(seed)
    qfar = (1.1, 0.3, -0.1, 0.2, 2.4)
    mesh = wl.box_mesh(shape, hi=hi_len, bc=bc, flux=flux, qfar=qfar)
    E = int(np.prod(shape))
    orders = wl.random_orders(E, lo, hi, rng)
    if state == "random":
        u = wl.random_state(orders, rng)
    else:
        u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, sigma=0.2)
    return mesh, orders, u, rng


CASES = [
    # (shape, order range, seed, bc, flux, box)
    ((3, 3, 3), (1, 7), 1, (0,) * 6, wl.ROE, (1.0, 1.0, 1.0)),
    ((4, 2, 3), (1, 9), 2, (0,) * 6, wl.LF, (2.0, 1.0, 0.5)),
    ((3, 2, 2), (2, 5), 3, (1, 2, 0, 0, 1, 1), wl.ROE, (1.0, 1.0, 1.0)),
    ((1, 1, 1), (3, 6), 4, (0,) * 6, wl.ROE, (1.0, 1.0, 1.0)),
    ((5, 1, 2), (1, 3), 5, (2, 1, 0, 0, 0, 0), wl.LF, (1.0, 0.3, 1.0)),
    ((2, 2, 2), (9, 9), 6, (0,) * 6, wl.ROE, (1.0, 1.0, 1.0)),
    ((4, 4, 4), (1, 1), 7, (0,) * 6, wl.ROE, (1.0, 1.0, 1.0)),
]


@pytest.mark.parametrize("shape,orng,seed,bc,flux,box", CASES)
def test_layout_is_stable_bucket_sort(shape, orng, seed, bc, flux, box):
    mesh, orders, u, _ = _case(shape, *orng, seed, bc, flux, box)
    plan = dg.Plan(mesh, orders)
    npe = np.prod(orders.astype(np.int64) + 1, axis=1)
    cls = np.where(npe <= 256, 1, np.where(npe <= 512, 2, 4))
    keys = [(cls[e], *orders[e], e) for e in range(len(orders))]
    expect = np.array([k[-1] for k in sorted(keys)])
    assert np.array_equal(plan.perm, expect)
    assert np.array_equal(plan.orders, orders[expect])
    assert np.array_equal(plan.node_offset, np.concatenate([[0], np.cumsum(npe[expect])]))
    # the layout round trip is exact
    assert np.array_equal(plan.to_natural(plan.to_plan(u)), u)


@pytest.mark.parametrize("shape,orng,seed,bc,flux,box", CASES)
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("isolated", [False, True])
def test_residual_fp64(shape, orng, seed, bc, flux, box, form, isolated):
    mesh, orders, u, _ = _case(shape, *orng, seed, bc, flux, box)
    plan = dg.Plan(mesh, orders)
    ref = oracle.residual(mesh, orders, u, form=form, isolated=isolated)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u), form=form, isolated=isolated))
    s = residual_scale(mesh, orders, u)
    if form == 1:
        s *= np.prod((np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / np.asarray(mesh["n"])) / 8
    assert err(got, ref, s) < TOL64


@pytest.mark.parametrize("shape,orng,seed,bc,flux,box", CASES[:3])
def test_residual_fp32(shape, orng, seed, bc, flux, box):
    mesh, orders, u, _ = _case(shape, *orng, seed, bc, flux, box)
    plan = dg.Plan(mesh, orders)
    ref = oracle.residual(mesh, orders, u)
    got = plan.to_natural(dg.residual(plan, plan.to_plan(u, dtype=torch.float32)))
    assert err(got.astype(np.float64), ref, residual_scale(mesh, orders, u)) < TOL32


@pytest.mark.parametrize("N", [1, 4, 7])
@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_fp32_free_stream_exact(N, flux):
    """FP32 keeps a uniform state exactly steady on a conforming periodic box: every
    derivative subtracts the flux at its line's first node (the rows of D sum to zero),
    and the Riemann flux of equal states is the physical flux, so the residual is a
    bitwise zero (the FP32 tables' rounded row sums would leave about 1e-7 of |f| ||D||
    otherwise).  Mixed orders interpolate on the mortars and keep it within rounding."""
    rng = np.random.default_rng(40 + N)
    mesh = wl.box_mesh((3, 2, 2), hi=(1.0, 0.7, 1.3), flux=flux)
    q = (1.2, 0.3, -0.2, 0.25, 2.7)
    orders = wl.uniform_orders(12, N)
    plan = dg.Plan(mesh, orders)
    r = dg.residual(plan, plan.to_plan(wl.uniform_state(orders, q), dtype=torch.float32))
    assert float(r.abs().max()) == 0.0
    mixed = wl.random_orders(12, 1, 7, rng)
    plan = dg.Plan(mesh, mixed)
    u = wl.uniform_state(mixed, q)
    r = dg.residual(plan, plan.to_plan(u, dtype=torch.float32))
    assert float(r.abs().max()) < 1e-5 * residual_scale(mesh, mixed, u)


def test_residual_deterministic():
    mesh, orders, u, _ = _case((3, 3, 3), 1, 7, 11)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u)
    a = dg.residual(plan, ud)
    b = dg.residual(plan, ud)
    assert torch.equal(a, b)


@pytest.mark.parametrize("shape,orng,seed,bc,flux,box", CASES[:5])
@pytest.mark.parametrize("isolated", [False, True])
def test_tau_estimate(shape, orng, seed, bc, flux, box, isolated):
    mesh, fo, u, rng = _case(shape, *orng, seed, bc, flux, box, state="pulse")
    co = np.minimum(fo, wl.random_orders(len(fo), 1, 6, rng))
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    dudt = oracle.residual(mesh, fo, u)
    tn_r, tt_r, n_r, vn_r = oracle.tau(mesh, fo, co, u, dudt, isolated=isolated)
    sn, st = tau_scale(mesh, fo, co, u, isolated=isolated)
    ud = fine.to_plan(u)
    for pass_dudt in (False, True):
        tn, tt, norms, vn = dg.tau_estimate(fine, coarse, ud, fine.to_plan(dudt) if pass_dudt else None,
                                            isolated=isolated, varnorms=True)
        assert err(coarse.to_natural(tn), tn_r, sn) < TOL64
        assert err(coarse.to_natural(tt), tt_r, st) < TOL64
        nrm = coarse.elem_to_natural(norms.cpu().numpy())
        assert err(nrm[:, 0], n_r[:, 0], sn) < TOL64 and err(nrm[:, 1], n_r[:, 1], st) < TOL64
        # per-variable maxima: their maximum over the variables is the element norm
        vnn = coarse.elem_to_natural(vn.cpu().numpy())
        assert err(vnn[:, 0], vn_r[:, 0], sn) < TOL64 and err(vnn[:, 1], vn_r[:, 1], st) < TOL64
        assert np.array_equal(vnn.max(axis=2), nrm)


def test_tau_vanishes_at_fine_orders():
    mesh, fo, u, _ = _case((3, 2, 2), 1, 7, 12)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(fo)
    ud = fine.to_plan(u)
    dudt = dg.residual(fine, ud)
    tn, tt, norms = dg.tau_estimate(fine, coarse, ud, dudt)
    # same kernels on identical coarse inputs: exact zero
    assert float(norms.abs().max()) == 0.0


def _sweep_natural(plan, t):
    off = plan.combo_offsets()
    a = t.cpu().numpy()
    return np.concatenate([a[off[p]:off[p + 1]] for p in np.argsort(plan.perm)])


@pytest.mark.parametrize("shape,orng,seed", [((3, 2, 2), (1, 8), 21), ((2, 2, 2), (7, 7), 22),
                                             ((4, 3, 1), (1, 4), 23), ((2, 2, 1), (7, 9), 25)])
def test_sweep(shape, orng, seed):
    mesh, fo, u, _ = _case(shape, *orng, seed, state="pulse")
    plan = dg.Plan(mesh, fo)
    dudt = oracle.residual(mesh, fo, u)
    ten_r, tet_r, offs = oracle.sweep(mesh, fo, u, dudt)
    ud = plan.to_plan(u)
    ten, tet = dg.tau_sweep(plan, ud, plan.to_plan(dudt))
    sn, st = sweep_scale(mesh, fo, u)
    assert err(_sweep_natural(plan, ten), ten_r, sn) < TOL64
    assert err(_sweep_natural(plan, tet), tet_r, st) < TOL64
    # dudt computed inside the call gives the same map
    ten2, _ = dg.tau_sweep(plan, ud)
    assert err(_sweep_natural(plan, ten2), ten_r, sn) < TOL64


def test_sweep_isotropic_fast_path():
    """Elements with equal fine orders in every direction (N = 1..7) take the
    isotropic sweep kernel; mixed with anisotropic elements in one call."""
    rng = np.random.default_rng(24)
    mesh = wl.box_mesh((3, 3, 2))
    N = rng.permutation(np.resize(np.arange(1, 8), 18))  # every order 1..7 at least twice
    fo = np.stack([N, N, N], axis=1).astype(np.int32)
    fo[[2, 11]] = [[3, 5, 2], [7, 6, 7]]
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.2)
    dudt = oracle.residual(mesh, fo, u)
    ten_r, tet_r, offs = oracle.sweep(mesh, fo, u, dudt)
    plan = dg.Plan(mesh, fo)
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u), plan.to_plan(dudt))
    sn, st = sweep_scale(mesh, fo, u)
    assert err(_sweep_natural(plan, ten), ten_r, sn) < TOL64
    assert err(_sweep_natural(plan, tet), tet_r, st) < TOL64


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_rk3_graph_replays(dtype, tol):
    mesh, orders = wl.c1()
    u0 = wl.pulse_state(oracle.node_coords(mesh, orders), orders)
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(u0, dtype=dtype)
    g = torch.empty_like(ud)
    ref = u0.copy()
    # several replays of the captured step, with eager work and syncs in between
    for chunk in (1, 4, 5):
        dg.rk3_step(plan, ud, g, 1e-3, chunk)
        _ = dg.residual(plan, ud)
        torch.cuda.synchronize()
        ref = oracle.rk3(mesh, orders, ref, 1e-3, chunk)
        e = np.max(np.abs(plan.to_natural(ud).astype(np.float64) - ref)) / np.max(np.abs(ref))
        assert e < tol


def test_c1_workload():
    """C1: 4^3 periodic cube, N = 3, pulse; residual both forms, tau on the 8 uniform
    coarse maps {1,2}^3 (coupled and isolated), 10 RK3 steps at dt = 1e-3."""
    mesh, fo = wl.c1()
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo)
    plan = dg.Plan(mesh, fo)
    ud = plan.to_plan(u)
    s = residual_scale(mesh, fo, u)
    dudt = oracle.residual(mesh, fo, u)
    assert err(plan.to_natural(dg.residual(plan, ud)), dudt, s) < TOL64
    for c in [(a, b, c) for c in (1, 2) for b in (1, 2) for a in (1, 2)]:
        co = wl.uniform_orders(64, c)
        cp = plan.coarse(co)
        for iso in (False, True):
            tn, _, norms = dg.tau_estimate(plan, cp, ud, isolated=iso)
            tn_r, _, n_r, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=iso)
            sn, _ = tau_scale(mesh, fo, co, u, isolated=iso)
            assert err(cp.to_natural(tn), tn_r, sn) < TOL64
            assert err(cp.elem_to_natural(norms.cpu().numpy())[:, 0], n_r[:, 0], sn) < TOL64
    g = torch.empty_like(ud)
    dg.rk3_step(plan, ud, g, 1e-3, 10)
    ref = oracle.rk3(mesh, fo, u, 1e-3, 10)
    assert np.max(np.abs(plan.to_natural(ud) - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.slow
def test_c2_workload_sampled():
    """C2 at full size (16^3, N = 7, 2.1M nodes): the fine residual and the coupled
    tau-estimate on the drawn coarse map against the full oracle; the isolated sweep
    on 24 sampled elements."""
    mesh, fo, crange = wl.c2()
    xyz = oracle.node_coords(mesh, fo)
    u, co = wl.c2_state_and_coarse(xyz, mesh, fo)
    plan = dg.Plan(mesh, fo)
    ud = plan.to_plan(u)
    s = residual_scale(mesh, fo, u)
    dudt = oracle.residual(mesh, fo, u)
    r = dg.residual(plan, ud)
    assert err(plan.to_natural(r), dudt, s) < TOL64
    cp = plan.coarse(co)
    tn, tt, norms = dg.tau_estimate(plan, cp, ud, r)
    tn_r, tt_r, n_r, _ = oracle.tau(mesh, fo, co, u, dudt)
    sn, st = tau_scale(mesh, fo, co, u)
    assert err(cp.to_natural(tn), tn_r, sn) < TOL64
    assert err(cp.to_natural(tt), tt_r, st) < TOL64
    assert err(cp.elem_to_natural(norms.cpu().numpy())[:, 0], n_r[:, 0], sn) < TOL64
    ten, tet = dg.tau_sweep(plan, ud, r)
    rng = np.random.default_rng(99)
    sample = np.sort(rng.choice(4096, 24, replace=False))
    ten_r, tet_r, offs = oracle.sweep(mesh, fo, u, dudt, elems=sample)
    sn, st = sweep_scale(mesh, fo, u, elems=sample)
    full = _sweep_natural(plan, ten)
    got = np.concatenate([full[216 * e:216 * (e + 1)] for e in sample])
    assert err(got, ten_r, sn) < TOL64
    full = _sweep_natural(plan, tet)
    got = np.concatenate([full[216 * e:216 * (e + 1)] for e in sample])
    assert err(got, tet_r, st) < TOL64


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_check_state(dtype):
    """Admissibility check: a valid state passes; negative density, negative pressure and
    a NaN are each counted once."""
    mesh, orders, u, _ = _case((3, 2, 2), 1, 5, 11, (0,) * 6, wl.ROE, (1.0, 1.0, 1.0))
    plan = dg.Plan(mesh, orders)
    assert dg.check_state(plan, plan.to_plan(u, dtype=dtype)) == 0
    offs = wl.node_offsets(orders)
    bad = u.copy()
    ne0 = int(offs[1] - offs[0])
    bad[0] = -1.0                              # density of node 0, element 0
    e3 = 5 * offs[3]
    ne3 = int(offs[4] - offs[3])
    bad[e3 + 4 * ne3 + 1] = 0.0                # rho E = 0: negative pressure at node 1
    e7 = 5 * offs[7]
    bad[e7 + 2 * int(offs[8] - offs[7])] = np.nan
    with pytest.raises(dg.DGError, match="non-physical state: 3 nodes"):
        dg.check_state(plan, plan.to_plan(bad, dtype=dtype))


def test_misaligned_pointers_rejected():
    """Device arrays off a 16-byte boundary are refused before any launch."""
    import ctypes
    mesh, orders, u, _ = _case((2, 2, 2), 1, 3, 12)
    plan = dg.Plan(mesh, orders)
    n = 5 * plan.n_nodes
    buf = torch.zeros(n + 2, dtype=torch.float64, device="cuda")
    good = torch.zeros(n, dtype=torch.float64, device="cuda")
    off = ctypes.c_void_p(buf.data_ptr() + 8)
    L = dg.lib()
    st = L.dg_residual(plan.handle, off, ctypes.c_void_p(good.data_ptr()), 0, 0, 0, None)
    assert st == -1 and b"aligned" in L.dg_last_error()
    m = torch.zeros(int(plan.combo_offsets()[-1]) + 2, dtype=torch.float64, device="cuda")
    st = L.dg_tau_sweep(plan.handle, ctypes.c_void_p(good.data_ptr()), None, 0, ctypes.c_void_p(m.data_ptr() + 8),
                        ctypes.c_void_p(m.data_ptr()), None)
    assert st == -1
    st = L.dg_check_state(plan.handle, off, 0, None, None)
    assert st == -1
