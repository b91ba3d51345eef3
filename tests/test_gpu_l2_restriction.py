"""GPU parity of the tau-estimate with the L2-projection restriction (Section 2.3, the
restriction operator I^N taken as the exact L2 projection onto the coarse space) against
the oracle: coupled and isolated estimates with mortars and walls, the adjoint-weighted
sum, the sweep on its anisotropic and isotropic kernels, the curved and Navier-Stokes
sweep, the full-size 16^3 N = 7 workload on sampled elements, and argument checks."""
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
L2 = dg.RESTRICT_L2


def err(x, ref, s):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), s))


def _sweep_natural(plan, t):
    off = plan.combo_offsets()
    a = t.cpu().numpy()
    return np.concatenate([a[off[p]:off[p + 1]] for p in np.argsort(plan.perm)])


@pytest.mark.parametrize("shape,orng,seed,bc,isolated", [
    ((3, 3, 2), (1, 7), 41, (0,) * 6, False),
    ((3, 2, 3), (2, 8), 42, (1, 1, 0, 0, 2, 2), False),
    ((3, 3, 2), (1, 7), 43, (0,) * 6, True),
])
def test_tau_estimate_l2(shape, orng, seed, bc, isolated):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh(shape, bc=bc, qfar=(1.1, 0.3, -0.1, 0.2, 2.4))
    E = int(np.prod(shape))
    fo = wl.random_orders(E, *orng, rng)
    co = np.minimum(fo, wl.random_orders(E, 1, 6, rng))
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.2)
    dudt = oracle.residual(mesh, fo, u)
    psi = rng.normal(size=u.shape)
    tn_r, tt_r, n_r, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=isolated, restriction=oracle.L2)
    eta_r = oracle.tau_eta(mesh, fo, co, u, dudt, psi, isolated=isolated, restriction=oracle.L2)
    fine = dg.Plan(mesh, fo)
    coarse = fine.coarse(co)
    sn, st = tau_scale(mesh, fo, co, u, isolated=isolated, restriction=oracle.L2)
    tn, tt, norms, eta = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated, fine.to_plan(psi),
                                         restriction=L2)
    assert err(coarse.to_natural(tn), tn_r, sn) < TOL64
    assert err(coarse.to_natural(tt), tt_r, st) < TOL64
    nrm = coarse.elem_to_natural(norms.cpu().numpy())
    assert err(nrm[:, 0], n_r[:, 0], sn) < TOL64 and err(nrm[:, 1], n_r[:, 1], st) < TOL64
    # eta_e sums (I psi) * tau over the element: its rounding scale is the same sum of
    # |I psi| * |r^Nc| (traditional form)
    rct = np.abs(oracle.tau(mesh, fo, co, u, np.zeros_like(u), isolated=isolated, restriction=oracle.L2)[1])
    ip = np.abs(oracle.project(fo, co, psi))
    offs = wl.node_offsets(co)
    s_eta = max(float(np.sum(ip[5 * offs[k]:5 * offs[k + 1]] * rct[5 * offs[k]:5 * offs[k + 1]]))
                for k in range(E))
    e = coarse.elem_to_natural(eta.cpu().numpy())
    assert np.max(np.abs(e - eta_r)) < 1e-12 * max(np.max(np.abs(eta_r)), s_eta)
    # the sampling estimate on the same inputs is a different result
    tn_s = dg.tau_estimate(fine, coarse, fine.to_plan(u), None, isolated)[0]
    assert float((tn_s - tn).abs().max()) > 1e-6 * float(tn.abs().max())


@pytest.mark.parametrize("iso", [False, True])
def test_sweep_l2(iso):
    rng = np.random.default_rng(44 + iso)
    mesh = wl.box_mesh((3, 3, 2))
    if iso:  # equal fine orders: the isotropic kernel, one anisotropic element per call
        N = rng.integers(1, 8, 18)
        fo = np.stack([N, N, N], axis=1).astype(np.int32)
        fo[4] = [2, 6, 4]
    else:
        fo = wl.random_orders(18, 1, 8, rng)
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.2)
    dudt = oracle.residual(mesh, fo, u)
    ten_r, tet_r, _ = oracle.sweep(mesh, fo, u, dudt, restriction=oracle.L2)
    plan = dg.Plan(mesh, fo)
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u), None, restriction=L2)
    sn, st = sweep_scale(mesh, fo, u, restriction=oracle.L2)
    assert err(_sweep_natural(plan, ten), ten_r, sn) < TOL64
    assert err(_sweep_natural(plan, tet), tet_r, st) < TOL64


@pytest.mark.parametrize("ns", [False, True])
def test_sweep_l2_curved(ns):
    rng = np.random.default_rng(46 + ns)
    mesh = wl.sine_mapped(wl.box_mesh((2, 2, 2)))
    if ns:
        mesh = wl.ns_mesh(mesh, 0.01, 0.72)
    fo = wl.column_orders(mesh, 2, 5, rng, nz_order=2)
    u = wl.add_rho_noise(wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.2), fo, rng, 1e-3)
    if ns:
        dudt = oracle.residual_ns(mesh, fo, u, 0.01, 0.72)
        ten_r, tet_r, _ = oracle.sweep_ns(mesh, fo, u, dudt, 0.01, 0.72, restriction=oracle.L2)
    else:
        dudt = oracle.residual(mesh, fo, u)
        ten_r, tet_r, _ = oracle.sweep(mesh, fo, u, dudt, restriction=oracle.L2)
    plan = dg.Plan(mesh, fo)
    ten, tet = dg.tau_sweep(plan, plan.to_plan(u), plan.to_plan(dudt), restriction=L2)
    sn, st = sweep_scale(mesh, fo, u, restriction=oracle.L2, ns=(0.01, 0.72) if ns else None)
    assert err(_sweep_natural(plan, ten), ten_r, sn) < TOL64
    assert err(_sweep_natural(plan, tet), tet_r, st) < TOL64


@pytest.mark.slow
def test_c2_workload_l2_sampled():
    """16^3 elements at N = 7 (2.1M nodes): the coupled estimate on the drawn coarse map
    against the full oracle, the sweep on 16 sampled elements, both with the L2
    restriction."""
    mesh, fo, _ = wl.c2()
    u, co = wl.c2_state_and_coarse(oracle.node_coords(mesh, fo), mesh, fo)
    plan = dg.Plan(mesh, fo)
    ud = plan.to_plan(u)
    dudt = oracle.residual(mesh, fo, u)
    r = dg.residual(plan, ud)
    cp = plan.coarse(co)
    tn, _, norms = dg.tau_estimate(plan, cp, ud, r, restriction=L2)
    tn_r, _, n_r, _ = oracle.tau(mesh, fo, co, u, dudt, restriction=oracle.L2)
    sn, _ = tau_scale(mesh, fo, co, u, restriction=oracle.L2)
    assert err(cp.to_natural(tn), tn_r, sn) < TOL64
    assert err(cp.elem_to_natural(norms.cpu().numpy())[:, 0], n_r[:, 0], sn) < TOL64
    ten, _ = dg.tau_sweep(plan, ud, r, restriction=L2)
    sample = np.sort(np.random.default_rng(100).choice(4096, 16, replace=False))
    ten_r, _, _ = oracle.sweep(mesh, fo, u, dudt, elems=sample, restriction=oracle.L2)
    sn, _ = sweep_scale(mesh, fo, u, elems=sample, restriction=oracle.L2)
    full = _sweep_natural(plan, ten)
    got = np.concatenate([full[216 * e:216 * (e + 1)] for e in sample])
    assert err(got, ten_r, sn) < TOL64


def test_invalid_restriction():
    mesh = wl.box_mesh((2, 2, 2))
    fo = np.full((8, 3), 3, dtype=np.int32)
    plan = dg.Plan(mesh, fo)
    u = plan.to_plan(wl.pulse_state(oracle.node_coords(mesh, fo), fo))
    with pytest.raises(dg.DGError):
        dg.tau_sweep(plan, u, restriction=2)
    with pytest.raises(dg.DGError):
        dg.tau_estimate(plan, plan.coarse(np.full((8, 3), 2, dtype=np.int32)), u, restriction=-1)
