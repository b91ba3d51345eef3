"""Pins of the oracle's Navier-Stokes (BR1) operator: the first-order system of
Section 2.1 (eqs. SystemAdvDiff, DGSEMsystem:2) with the BR1 diffusive flux of the
paper's set-up (start of Section 3).

Pins: the viscous flux against the Stokes stress and Fourier heat flux built from
primitive gradients; free-stream preservation; discrete conservation; exact BR1
gradients of a continuous piecewise-quadratic state (mortars on every face); and
exactness of the full residual on a C1 piecewise-cubic shear flow with constant
total energy, where viscous stress and heat flux both contribute.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import elem_view, per_var, residual_scale
from test_oracle_residual import _mass_weights, contact_state

G_ = 1.4
MU, PR = 0.01, 0.72


def test_viscous_flux_matches_stokes_and_fourier():
    rng = np.random.default_rng(60)
    for _ in range(10):
        rho, p = rng.uniform(0.8, 1.2), rng.uniform(0.8, 1.2)
        u = rng.normal(size=3) * 0.3
        grad_u = rng.normal(size=(3, 3))   # grad_u[k, l] = d u_k / d x_l
        grad_rho = rng.normal(size=3)
        grad_p = rng.normal(size=3)
        # conserved gradients by the chain rule
        Gm = np.zeros((3, 5))
        E = p / (G_ - 1) + 0.5 * rho * u @ u
        for l in range(3):
            Gm[l, 0] = grad_rho[l]
            Gm[l, 1:4] = grad_rho[l] * u + rho * grad_u[:, l]
            Gm[l, 4] = grad_p[l] / (G_ - 1) + 0.5 * grad_rho[l] * (u @ u) + rho * (u @ grad_u[:, l])
        q = np.array([rho, *(rho * u), E])
        T = p / rho
        grad_T = (grad_p - T * grad_rho) / rho
        tau = MU * (grad_u + grad_u.T) - 2.0 / 3.0 * MU * np.trace(grad_u) * np.eye(3)
        kappa = MU * G_ / ((G_ - 1) * PR)
        for d in range(3):
            ref = np.array([0.0, *tau[:, d], u @ tau[:, d] + kappa * grad_T[d]])
            assert np.allclose(oracle.viscous_flux(q, Gm.reshape(-1), d, G_, MU, PR), ref, rtol=1e-12, atol=1e-14)


def test_free_stream_and_conservation():
    rng = np.random.default_rng(61)
    mesh = wl.box_mesh((3, 2, 2), hi=(1.0, 0.5, 1.0))
    orders = wl.random_orders(12, 1, 6, rng)
    q = wl.conserved(np.array(1.1), np.array(0.3), np.array(-0.2), np.array(0.1), np.array(0.9))
    u = wl.uniform_state(orders, q)
    assert np.max(np.abs(oracle.gradient(mesh, orders, u))) < 1e-12
    assert np.max(np.abs(oracle.residual_ns(mesh, orders, u, MU, PR))) < 1e-13 * residual_scale(mesh, orders, u)
    u = wl.random_state(orders, rng)
    for form in (0, 1):
        r = per_var(oracle.residual_ns(mesh, orders, u, MU, PR, form=form), orders)
        w = r * _mass_weights(mesh, orders) if form == 0 else r
        assert np.all(np.abs(w.sum(axis=1)) < 1e-13 * np.abs(w).sum(axis=1))


def test_br1_gradient_exact_on_continuous_quadratic():
    rng = np.random.default_rng(62)
    mesh = wl.box_mesh((3, 2, 2))
    orders = wl.random_orders(12, 2, 6, rng)
    U = np.array([0.3, -0.2, 0.4])
    u, _ = contact_state(mesh, orders, rng, U)
    g = oracle.gradient(mesh, orders, u)
    # reference: differentiate rho = 1 + 0.1 g(x) h(y) k(z) exactly; conserved vars are
    # affine in rho for constant velocity and pressure
    rng2 = np.random.default_rng(62)
    wl.random_orders(12, 2, 6, rng2)
    nx, ny, nz = mesh["n"]
    fx = (rng2.normal(size=nx), rng2.normal(size=nx))
    fy = (rng2.normal(size=ny), rng2.normal(size=ny))
    fz = (rng2.normal(size=nz), rng2.normal(size=nz))
    from test_oracle_residual import _pw_quadratic
    xyz = oracle.node_coords(mesh, orders)
    for e in range(12):
        ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
        X = elem_view(xyz, orders, e, nv=3)
        gx, dgx = _pw_quadratic(X[0], ix, 1.0 / nx, *fx)
        gy, dgy = _pw_quadratic(X[1], iy, 1.0 / ny, *fy)
        gz, dgz = _pw_quadratic(X[2], iz, 1.0 / nz, *fz)
        grad_rho = 0.1 * np.stack([dgx * gy * gz, gx * dgy * gz, gx * gy * dgz])
        dq = np.array([1.0, *U, 0.5 * U @ U])  # d(conserved)/d(rho)
        Ge = elem_view(g, orders, e, nv=15).reshape(3, 5, -1)
        ref = grad_rho[:, None, :] * dq[None, :, None]
        assert np.max(np.abs(Ge - ref)) < 1e-11 * np.max(np.abs(ref))


def _hermite(y, iy, h, vals, slopes):
    n = len(vals)
    t = (y - iy * h) / h
    v0, v1 = vals[iy], vals[(iy + 1) % n]
    s0, s1 = slopes[iy], slopes[(iy + 1) % n]
    H0, H1 = 2 * t ** 3 - 3 * t ** 2 + 1, -2 * t ** 3 + 3 * t ** 2
    G0, G1 = t ** 3 - 2 * t ** 2 + t, t ** 3 - t ** 2
    dH0, dH1, dG0, dG1 = 6 * t ** 2 - 6 * t, -6 * t ** 2 + 6 * t, 3 * t ** 2 - 4 * t + 1, 3 * t ** 2 - 2 * t
    ddH0, ddH1, ddG0, ddG1 = 12 * t - 6, -12 * t + 6, 6 * t - 4, 6 * t - 2
    U = v0 * H0 + v1 * H1 + h * (s0 * G0 + s1 * G1)
    dU = (v0 * dH0 + v1 * dH1 + h * (s0 * dG0 + s1 * dG1)) / h
    ddU = (v0 * ddH0 + v1 * ddH1 + h * (s0 * ddG0 + s1 * ddG1)) / h ** 2
    return U, dU, ddU


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_shear_flow_exact(flux):
    """rho = 1, u = (U(y), 0, 0), rho E = E0 constant (so p = (gamma-1)(E0 - U^2/2), T = p),
    U a C1 periodic piecewise cubic, N_y = 7 everywhere, random orders in x and z.  Every
    term is a polynomial the scheme differentiates exactly and every trace is continuous,
    so the NS residual equals at each node
        (0, -mu U'', p', 0, -mu (1 - gamma/Pr)(U'^2 + U U'')),  p' = -(gamma-1) U U'."""
    rng = np.random.default_rng(63)
    nx, ny, nz = 2, 3, 2
    mesh = wl.box_mesh((nx, ny, nz), flux=flux)
    orders = wl.random_orders(12, 1, 6, rng)
    orders[:, 1] = 7
    vals, slopes = rng.normal(size=ny) * 0.3, rng.normal(size=ny)
    E0 = 3.0
    xyz = oracle.node_coords(mesh, orders)
    u = np.zeros(5 * int(wl.node_offsets(orders)[-1]))
    ref = np.zeros_like(u)
    for e in range(12):
        iy = (e // nx) % ny
        X = elem_view(xyz, orders, e, nv=3)
        U, dU, ddU = _hermite(X[1], iy, 1.0 / ny, vals, slopes)
        one, zero = np.ones_like(U), np.zeros_like(U)
        elem_view(u, orders, e)[:] = np.stack([one, U, zero, zero, E0 * one])
        dp = -(G_ - 1) * U * dU
        elem_view(ref, orders, e)[:] = np.stack([zero, -MU * ddU, dp, zero,
                                                 -MU * (1 - G_ / PR) * (dU * dU + U * ddU)])
    r = oracle.residual_ns(mesh, orders, u, MU, PR)
    scale = residual_scale(mesh, orders, u)
    assert np.max(np.abs(r - ref)) < 1e-12 * scale
    # the viscous part is resolved: the inviscid residual misses it
    assert np.max(np.abs(oracle.residual(mesh, orders, u) - ref)) > 1e-4
