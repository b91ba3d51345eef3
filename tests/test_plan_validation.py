"""Plan creation refuses invalid meshes and order maps before it touches the device
(the checks of dg_plan_create run on the host, so this runs without a GPU)."""
import os

import numpy as np
import pytest

import paper_2210_03523_amd as dg
import workloads as wl

pytestmark = pytest.mark.skipif(not os.path.exists(dg.LIB_PATH), reason="library not built")


def _orders(E, N=3):
    return np.full((E, 3), N, dtype=np.int32)


@pytest.mark.parametrize("bad", [0, 10, -1])
def test_orders_outside_1_to_9(bad):
    o = _orders(8)
    o[3, 1] = bad
    with pytest.raises(dg.DGError, match="orders must be in 1..9"):
        dg.Plan(wl.box_mesh((2, 2, 2)), o)


def test_order_count_must_match_the_mesh():
    with pytest.raises(dg.DGError, match="order triples"):
        dg.Plan(wl.box_mesh((2, 2, 2)), _orders(7))


@pytest.mark.parametrize("change,msg", [
    (lambda m: m.update(bc=(0, 1, 0, 0, 0, 0)), "periodic faces must come in pairs"),
    (lambda m: m.update(bc=(3, 3, 0, 0, 0, 0)), "unknown boundary condition"),
    (lambda m: m.update(flux=2), "unknown flux"),
    (lambda m: m.update(gamma=1.0), "gamma must exceed 1"),
    (lambda m: m.update(hi=(1.0, 0.0, 1.0)), "mesh extent must be positive"),
    (lambda m: m.update(n=(2, 0, 2)), "at least one element"),
])
def test_invalid_mesh(change, msg):
    m = wl.box_mesh((2, 2, 2))
    change(m)
    with pytest.raises(dg.DGError, match=msg):
        dg.Plan(m, _orders(int(np.prod(m["n"]))))


def test_navier_stokes_needs_a_prandtl_number():
    m = wl.ns_mesh(wl.box_mesh((2, 2, 2)), 0.01, 0.0)
    with pytest.raises(dg.DGError, match="Navier-Stokes"):
        dg.Plan(m, _orders(8))


def test_curved_orders_below_the_geometry_order():
    m = wl.sine_mapped(wl.box_mesh((2, 2, 2)))
    o = _orders(8, 2)
    o[5, 0] = 1  # geometry order (2, 2, 1)
    with pytest.raises(dg.DGError, match="geometry order"):
        dg.Plan(m, o)


def test_batch_refuses_a_repeated_plan_handle():
    """Two problems of a batch may not share a plan (its face-flux scratch would be
    written by both): the handles are compared before any plan is read, so two copies
    of one (never dereferenced) handle value are refused on the host."""
    import ctypes
    fake = ctypes.c_void_p(0x1000)
    arr = (ctypes.c_void_p * 2)(fake.value, fake.value)
    out = ctypes.c_void_p()
    st = dg.lib().dg_batch_create(arr, 2, dg.DG_F32, ctypes.byref(out))
    assert st == -1
    assert b"appears twice" in dg.lib().dg_last_error()
