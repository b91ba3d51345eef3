"""Dense adjoint of the DGSEM residual for small meshes.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of
the benchmark are the only users.  The GPU library never loads it and shares no code
with it.

The Jacobian d r / d u of the oracle residual is formed column by column, either by the
oracle's complex-step directional derivative (exact to rounding; box Euler meshes) or by
central differences, and the adjoint problem (d r / d u)^T psi = g is solved with numpy's
dense solver (a library primitive).  This is the adjoint problem behind the adjoint-weighted
truncation error (the functional error estimate as the truncation error weighted by the
adjoint of the functional).  Layouts are natural (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import residual, residual_jvp


def fd_jacobian(mesh: dict, orders, u, form: int = 0, isolated: bool = False, rel_eps: float = 1e-6):
    """J[:, j] = (r(u + h e_j) - r(u - h e_j)) / (2 h), h = rel_eps max(1, |u_j|)."""
    u = np.asarray(u, dtype=np.float64)
    n = u.size
    J = np.empty((n, n))
    for j in range(n):
        h = rel_eps * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        J[:, j] = (residual(mesh, orders, up, form=form, isolated=isolated) -
                   residual(mesh, orders, um, form=form, isolated=isolated)) / (2.0 * h)
    return J


def cs_jacobian(mesh: dict, orders, u, form: int = 0, isolated: bool = False):
    """J[:, j] = (d r / d u) e_j by complex step."""
    u = np.asarray(u, dtype=np.float64)
    n = u.size
    J = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        J[:, j] = residual_jvp(mesh, orders, u, e, form=form, isolated=isolated)
        e[j] = 0.0
    return J


def adjoint_solve(mesh: dict, orders, u, g, form: int = 0, isolated: bool = False):
    """psi with (d r / d u)^T psi = g (dense, complex-step Jacobian); also returns the
    Jacobian."""
    J = cs_jacobian(mesh, orders, u, form=form, isolated=isolated)
    return np.linalg.solve(J.T, np.asarray(g, dtype=np.float64)), J
