"""Pins of the oracle's truncation-error pieces: the exact truncation error
(eqs. TEtildedef and TEdef), the tau-estimate (Section 2.3, variational DG form)
and the isolated sweep (TE map).

The pins use what the paper and the mathematics fix: exponential decay of the
exact truncation error for a smooth solution (Introduction and Section 2.3),
convergence of the estimate to the exact value as the fine order grows, the
identity at Nc = Nf, exactness of the isolated estimate on a state the coarse
space represents, and the pointwise relation tau = J w tau~ of the two forms.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import elem_view, per_var
from test_oracle_residual import contact_state

SIG = 0.1


def _pulse_divergence(x, y, z):
    """div f for the periodised pulse with u = (1,0,0), p = 1: (rho_x, rho_x, 0, 0, rho_x/2)."""
    rx = np.zeros_like(x)
    for kx in (-1, 0, 1):
        for ky in (-1, 0, 1):
            for kz in (-1, 0, 1):
                dx = x - 0.5 - kx
                r2 = dx ** 2 + (y - 0.5 - ky) ** 2 + (z - 0.5 - kz) ** 2
                rx += 0.5 * np.exp(-r2 / (2 * SIG * SIG)) * (-dx / (SIG * SIG))
    zero = np.zeros_like(x)
    return np.stack([rx, rx, zero, zero, 0.5 * rx])


def _sampled(mesh, orders):
    xyz = oracle.node_coords(mesh, orders)
    return wl.pulse_state(xyz, orders, images=True), wl._ragged_apply(xyz, orders, _pulse_divergence)


def exact_tau(mesh, N):
    """tau~_exact = M^-1 F^N(I q) - I F(q) on a uniform order-N mesh."""
    o = wl.uniform_orders(wl.num_elems(mesh), N)
    u, F = _sampled(mesh, o)
    return oracle.residual(mesh, o, u) - F


def test_exact_tau_decays_exponentially():
    mesh = wl.box_mesh(4)
    norms = np.array([np.max(np.abs(exact_tau(mesh, N))) for N in range(2, 13)])
    slope = np.polyfit(np.arange(2, 13), np.log10(norms), 1)[0]
    assert slope < -0.5  # more than half a decade per order
    assert norms[-1] < 1e-5 * norms[0]
    # monotone over every pair of orders two apart (odd/even effects aside)
    assert np.all(norms[2:] < norms[:-2])


def test_estimate_converges_to_exact():
    """tau_est(Nc; Nf) from q^P = I^Nf q and r^P = M^-1 F^Nf(q^P) tends to the exact
    tau(Nc) as Nf grows (the estimate of Section 2.3 is consistent)."""
    mesh = wl.box_mesh(4)
    Nc = 3
    co = wl.uniform_orders(64, Nc)
    ref = exact_tau(mesh, Nc)
    errs = []
    for Nf in (5, 7, 9, 11):
        fo = wl.uniform_orders(64, Nf)
        u, _ = _sampled(mesh, fo)
        dudt = oracle.residual(mesh, fo, u)
        tn, _, _, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=False)
        errs.append(np.max(np.abs(tn - ref)))
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0)
    assert errs[-1] < 1e-4 * np.max(np.abs(ref))


def test_coupled_tau_vanishes_at_fine_order():
    rng = np.random.default_rng(20)
    mesh = wl.box_mesh((3, 2, 2))
    fo = wl.random_orders(12, 1, 6, rng)
    u = wl.random_state(fo, rng)
    dudt = oracle.residual(mesh, fo, u)
    tn, tt, norms, vn = oracle.tau(mesh, fo, fo, u, dudt, isolated=False)
    assert np.all(tn == 0.0) and np.all(tt == 0.0) and np.all(norms == 0.0)
    # isolated at Nc = Nf keeps only the lifting: tau~ = r_iso - r = -SAT/J
    tn_i, _, _, _ = oracle.tau(mesh, fo, fo, u, dudt, isolated=True)
    assert np.array_equal(tn_i, oracle.residual(mesh, fo, u, isolated=True) - dudt)


def test_traditional_is_mass_scaled_new_form():
    rng = np.random.default_rng(21)
    mesh = wl.box_mesh((2, 2, 3), hi=(0.5, 1.0, 1.5))
    fo = wl.random_orders(12, 2, 7, rng)
    co = np.minimum(fo, wl.random_orders(12, 1, 6, rng))
    u = wl.random_state(fo, rng)
    dudt = oracle.residual(mesh, fo, u)
    for iso in (False, True):
        tn, tt, norms, vn = oracle.tau(mesh, fo, co, u, dudt, isolated=iso)
        h = np.array([0.25, 0.5, 0.5])
        J = h.prod() / 8
        for e in range(12):
            w = [oracle.lgl(int(N))[1] for N in co[e]]
            Mw = J * np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1)
            a, b = elem_view(tn, co, e), elem_view(tt, co, e)
            assert np.allclose(b, Mw * a, rtol=1e-15, atol=0)
            assert norms[e, 0] == np.max(np.abs(a)) and norms[e, 1] == np.max(np.abs(b))
            assert np.array_equal(vn[e, 0], np.max(np.abs(a), axis=1))


def test_estimate_exact_on_representable_state():
    """For the degree-2 contact state of the residual pins, every coarse space
    with orders >= 2 holds the state exactly, so both the coupled and the isolated
    estimate vanish (up to rounding); an order-1 direction makes it nonzero."""
    rng = np.random.default_rng(22)
    mesh = wl.box_mesh((3, 2, 2))
    fo = wl.random_orders(12, 4, 7, rng)
    u, _ = contact_state(mesh, fo, rng, np.array([0.4, 0.2, -0.6]))
    dudt = oracle.residual(mesh, fo, u)
    scale = np.max(np.abs(dudt))
    co = np.minimum(fo, wl.random_orders(12, 2, 6, rng))
    for iso in (False, True):
        tn, _, _, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=iso)
        assert np.max(np.abs(tn)) < 1e-12 * scale
    co1 = co.copy()
    co1[:, 1] = 1
    tn, _, _, _ = oracle.tau(mesh, fo, co1, u, dudt, isolated=True)
    assert np.max(np.abs(tn)) > 1e-4 * scale


def test_sweep_matches_per_combo_isolated_estimate():
    """The sweep's entry for combo (c1,c2,c3) (c1 fastest) equals the isolated
    estimate on the uniform coarse map (c1,c2,c3); directions of order 1 keep 1."""
    rng = np.random.default_rng(23)
    mesh = wl.box_mesh((2, 2, 1))
    fo = np.array([[4, 3, 1], [2, 5, 3], [3, 3, 3], [1, 1, 2]], dtype=np.int32)
    u = wl.random_state(fo, rng)
    dudt = oracle.residual(mesh, fo, u)
    ten, tet, offs = oracle.sweep(mesh, fo, u, dudt)
    assert list(np.diff(offs)) == [6, 8, 8, 1]
    for e in range(4):
        cmax = np.maximum(fo[e] - 1, 1)
        slot = offs[e]
        for c3 in range(1, cmax[2] + 1):
            for c2 in range(1, cmax[1] + 1):
                for c1 in range(1, cmax[0] + 1):
                    co = fo.copy()
                    co[e] = (c1, c2, c3)
                    _, _, norms, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=True)
                    assert ten[slot] == norms[e, 0] and tet[slot] == norms[e, 1]
                    slot += 1
    # a subset of elements gives the same values
    ten2, tet2, offs2 = oracle.sweep(mesh, fo, u, dudt, elems=[2, 0])
    assert np.array_equal(ten2[:8], ten[offs[2]:offs[3]]) and np.array_equal(ten2[8:], ten[:6])
