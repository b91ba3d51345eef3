"""Pins of the oracle's force functional, its gradient and the adjoint-weighted
truncation error eta (used with the adjoint of a force functional).

The functional is the x-pressure force on slip walls: its value for a pressure
field the wall quadrature integrates exactly is a closed form; its gradient is
checked against central differences of the value; eta with a constant weight is
the plain sum of the traditional-form estimate.
"""
import numpy as np

import oracle
import workloads as wl
from helpers import elem_view


def _wall_mesh(n=(2, 3, 2)):
    return wl.box_mesh(n, bc=(wl.WALL, wl.FARFIELD, 0, 0, 0, 0), qfar=(1.0, 0.3, 0.0, 0.0, 2.545))


def test_functional_closed_form():
    mesh = _wall_mesh()
    rng = np.random.default_rng(40)
    orders = wl.random_orders(12, 2, 5, rng)
    xyz = oracle.node_coords(mesh, orders)

    def fn(x, y, z):
        p = 1.0 + 0.3 * y + 0.2 * z * z
        one = np.ones_like(x)
        return wl.conserved(one, 0.1 * one, 0.0 * one, 0.0 * one, p)
    u = wl._ragged_apply(xyz, orders, fn)
    J, _ = oracle.functional(mesh, orders, u)
    # wall x = 0 with outward normal -e_x: J = -int_0^1 int_0^1 p dy dz
    assert abs(J - (-(1.0 + 0.15 + 0.2 / 3.0))) < 1e-13
    # a wall on the other side flips the sign; no wall gives zero
    mesh2 = wl.box_mesh((2, 3, 2), bc=(wl.FARFIELD, wl.WALL, 0, 0, 0, 0))
    assert abs(oracle.functional(mesh2, orders, u)[0] - (1.0 + 0.15 + 0.2 / 3.0)) < 1e-13
    assert oracle.functional(wl.box_mesh((2, 3, 2)), orders, u)[0] == 0.0


def test_functional_gradient_matches_differences():
    mesh = _wall_mesh()
    rng = np.random.default_rng(41)
    orders = wl.random_orders(12, 1, 5, rng)
    u = wl.random_state(orders, rng)
    J, g = oracle.functional(mesh, orders, u)
    for _ in range(8):
        d = rng.normal(size=u.size)
        eps = 1e-6
        fd = (oracle.functional(mesh, orders, u + eps * d, grad=False)
              - oracle.functional(mesh, orders, u - eps * d, grad=False)) / (2 * eps)
        # central differences: truncation O(eps^2), rounding O(1e-16 |J| / eps)
        assert abs(fd - g @ d) < 1e-8 * (abs(J) + abs(fd))
    # the gradient lives only on the wall face nodes
    nz_elems = {e for e in range(12) if np.any(elem_view(g, orders, e) != 0.0)}
    assert nz_elems == {e for e in range(12) if e % 2 == 0}


def test_eta_with_constant_weight_sums_traditional_tau():
    mesh = wl.box_mesh((2, 2, 2))
    rng = np.random.default_rng(42)
    fo = wl.random_orders(8, 2, 6, rng)
    co = np.minimum(fo, wl.random_orders(8, 1, 5, rng))
    u = wl.random_state(fo, rng)
    dudt = oracle.residual(mesh, fo, u)
    psi = np.full_like(u, 0.75)
    for iso in (False, True):
        eta = oracle.tau_eta(mesh, fo, co, u, dudt, psi, isolated=iso)
        _, tt, _, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=iso)
        ref = np.array([0.75 * elem_view(tt, co, e).sum() for e in range(8)])
        assert np.allclose(eta, ref, rtol=1e-12, atol=1e-15 * np.abs(tt).sum())
