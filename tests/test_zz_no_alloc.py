"""The allocation-free residual (dg_residual_noalloc) through the C ABI against the
residual with the plan's own scratch (dg_residual): two calls in a row, the second on
a smaller mesh (so the static scratch holds the first call's larger contents), for box
Euler meshes with mortars and every boundary kind, box Navier-Stokes (gradients in the
scratch too) and curved Navier-Stokes plans, FP64 and FP32.  The kernels are the same
and deterministic, so the results must be identical bit for bit; FP64 results are also
checked against the oracle at 1e-12 of the cancelling-term scale."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import residual_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402

QF = tuple(float(v) for v in wl.conserved(*(np.array(x) for x in (1.05, 0.3, -0.1, 0.2, 1.1))))


def _abi(name, plan, u, r, form, iso):
    L = dg.lib()
    code = 0 if u.dtype == torch.float64 else 1
    st = getattr(L, name)(plan.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(r.data_ptr()), code,
                          int(form), int(iso), dg._stream())
    assert st == 0, L.dg_last_error()


def _meshes(kind):
    rng = np.random.default_rng(61)
    if kind == "euler":
        big = wl.box_mesh((5, 4, 4), bc=(1, 2, 0, 0, 0, 0), qfar=QF)
        small = wl.box_mesh((2, 3, 2), bc=(0, 0, 1, 2, 0, 0), qfar=QF)
        return [(big, wl.random_orders(80, 1, 8, rng)), (small, wl.random_orders(12, 1, 5, rng))]
    if kind == "ns":
        big = wl.ns_mesh(wl.box_mesh((4, 4, 3)), 0.01, 0.72)
        small = wl.ns_mesh(wl.box_mesh((2, 2, 2)), 0.01, 0.72)
        return [(big, wl.random_orders(48, 1, 6, rng)), (small, wl.random_orders(8, 1, 4, rng))]
    big = wl.ns_mesh(wl.sine_mapped(wl.box_mesh((4, 4, 2), hi=(1.0, 1.0, 0.5))), 0.01, 0.72)
    small = wl.ns_mesh(wl.sine_mapped(wl.box_mesh((2, 2, 2), hi=(1.0, 1.0, 1.0))), 0.01, 0.72)
    return [(big, wl.element_orders(big, 2, 6, rng, nz_range=(1, 2))),
            (small, wl.element_orders(small, 2, 4, rng, nz_range=(1, 2)))]


def _oracle(mesh, orders, u, form, iso):
    if mesh.get("mu") is not None:
        return oracle.residual_ns(mesh, orders, u, mesh["mu"], mesh["Pr"], form=form, isolated=iso)
    return oracle.residual(mesh, orders, u, form=form, isolated=iso)


@pytest.mark.parametrize("kind", ["euler", "ns", "curved"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_calls_larger_then_smaller(kind, dtype):
    rng = np.random.default_rng(62)
    for form, iso in ((0, 0), (1, 0)):
        for mesh, orders in _meshes(kind):
            plan = dg.Plan(mesh, orders)
            u = wl.random_state(orders, rng)
            ud = plan.to_plan(u, dtype=dtype)
            want = torch.empty_like(ud)
            got = torch.full_like(ud, float("nan"))
            _abi("dg_residual", plan, ud, want, form, iso)
            _abi("dg_residual_noalloc", plan, ud, got, form, iso)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (kind, form, mesh["n"])
            if dtype == torch.float64:
                ref = _oracle(mesh, orders, u, form, iso)
                s = residual_scale(mesh, orders, u)
                if form == 1:
                    s *= np.prod((np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / np.asarray(mesh["n"])) / 8
                e = np.max(np.abs(plan.to_natural(got) - ref)) / max(np.max(np.abs(ref)), s)
                assert e < 1e-12


def test_binding_and_isolated():
    rng = np.random.default_rng(63)
    mesh, orders = _meshes("euler")[1]
    plan = dg.Plan(mesh, orders)
    ud = plan.to_plan(wl.random_state(orders, rng))
    out = torch.empty_like(ud)
    assert torch.equal(dg.residual_noalloc(plan, ud, out, isolated=True), dg.residual(plan, ud, isolated=True))


def test_refuses_plans_beyond_the_scratch():
    """16^3 elements of order 8 need 6 x 5 x 81 x 4096 = 9.95 Mi doubles of face
    fluxes, more than the 8 Mi the static scratch holds."""
    plan = dg.Plan(wl.box_mesh((16, 16, 16)), wl.uniform_orders(4096, (8, 8, 8)))
    u = torch.ones(5 * plan.n_nodes, dtype=torch.float64, device="cuda")
    r = torch.empty_like(u)
    with pytest.raises(dg.DGError, match="at most 8388608"):
        dg.residual_noalloc(plan, u, r)
