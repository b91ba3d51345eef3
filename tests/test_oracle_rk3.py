"""Pins of the oracle's Williamson low-storage RK3 (set-up at the start of Section 3).

Third-order convergence in dt, conservation of sum(J w U) and free-stream
preservation; together they fix the three (A_k, B_k) coefficient pairs.
"""
import numpy as np

import oracle
import workloads as wl
from helpers import per_var
from test_oracle_residual import _mass_weights


def _setup():
    mesh = wl.box_mesh(2)
    orders = wl.uniform_orders(8, 4)
    xyz = oracle.node_coords(mesh, orders)
    u = wl.pulse_state(xyz, orders, sigma=0.15)
    return mesh, orders, u


def test_third_order_in_time():
    mesh, orders, u = _setup()
    T = 0.04
    ref = oracle.rk3(mesh, orders, u, T / 256, 256)
    errs = [np.max(np.abs(oracle.rk3(mesh, orders, u, T / n, n) - ref)) for n in (4, 8, 16)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.8) and np.all(rates < 3.3), rates


def test_conservation_and_free_stream():
    mesh, orders, u = _setup()
    Mw = _mass_weights(mesh, orders)
    u10 = oracle.rk3(mesh, orders, u, 1e-3, 10)
    m0 = (per_var(u, orders) * Mw).sum(axis=1)
    m1 = (per_var(u10, orders) * Mw).sum(axis=1)
    assert np.all(np.abs(m1 - m0) < 1e-13 * np.abs(per_var(u, orders) * Mw).sum())
    q = wl.conserved(np.array(1.1), np.array(0.2), np.array(0.3), np.array(-0.1), np.array(1.0))
    uf = wl.uniform_state(orders, q)
    assert np.max(np.abs(oracle.rk3(mesh, orders, uf, 1e-3, 5) - uf)) < 1e-13
    # dt = 0 leaves the state untouched bitwise
    u1 = oracle.rk3(mesh, orders, u, 0.0, 3)
    assert np.array_equal(u1, u)
