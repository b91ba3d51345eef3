"""Pins of the dense finite-difference Jacobian behind the oracle's adjoint solve:
discrete conservation (the mass-weighted column sums of d r / d u vanish on a periodic
mesh), free-stream preservation (a uniform perturbation of a uniform state is in the
kernel of the Jacobian), and agreement of Jacobian-vector products with directional
differences at two step sizes (second-order convergence)."""
import numpy as np

import oracle
from oracle import adjoint
import workloads as wl


def _mass(mesh, orders):
    offs = wl.node_offsets(orders)
    h = [(mesh["hi"][d] - mesh["lo"][d]) / mesh["n"][d] for d in range(3)]
    J = h[0] * h[1] * h[2] / 8.0
    m = []
    for e, o in enumerate(orders):
        w = np.einsum("k,j,i->kji", *(oracle.lgl(int(N))[1] for N in o[::-1])).reshape(-1)
        m.append(np.tile(J * w, 5))
    return np.concatenate(m)


def test_conservation_and_free_stream():
    rng = np.random.default_rng(1)
    mesh = wl.box_mesh((2, 2, 1))
    orders = wl.random_orders(4, 1, 2, rng)
    u = wl.random_state(orders, rng)
    Jac = adjoint.fd_jacobian(mesh, orders, u)
    M = _mass(mesh, orders)
    # sum over nodes of M r(u) is zero for every u: the mass-weighted column sums vanish
    # variable by variable
    n = len(M) // 5
    offs = wl.node_offsets(orders)
    for v in range(5):
        sel = np.concatenate([np.arange(5 * offs[e] + v * (offs[e + 1] - offs[e]),
                                        5 * offs[e] + (v + 1) * (offs[e + 1] - offs[e])) for e in range(4)])
        col = M[sel] @ Jac[sel, :]
        assert np.max(np.abs(col)) < 1e-7 * np.max(np.abs(Jac))
    # uniform state: uniform perturbations keep the free stream
    u0 = wl.uniform_state(orders, np.array(wl.conserved(*(np.array(x) for x in (1.0, 0.3, -0.2, 0.1, 1.0)))))
    J0 = adjoint.fd_jacobian(mesh, orders, u0)
    for v in range(5):
        d = np.zeros_like(u0)
        for e in range(4):
            ne = int(offs[e + 1] - offs[e])
            d[5 * offs[e] + v * ne: 5 * offs[e] + (v + 1) * ne] = 1.0
        assert np.max(np.abs(J0 @ d)) < 1e-7 * np.max(np.abs(J0))


def test_jacobian_vector_products_converge():
    rng = np.random.default_rng(2)
    mesh = wl.box_mesh((2, 1, 1), bc=(1, 2, 0, 0, 0, 0))
    orders = wl.random_orders(2, 1, 3, rng)
    u = wl.random_state(orders, rng)
    Jac = adjoint.fd_jacobian(mesh, orders, u)
    v = rng.normal(size=u.size)
    v /= np.linalg.norm(v)
    errs = []
    for h in (1e-3, 1e-4):  # below the kinks of the Roe flux's |eigenvalue| terms
        d = (oracle.residual(mesh, orders, u + h * v) - oracle.residual(mesh, orders, u - h * v)) / (2 * h)
        errs.append(np.max(np.abs(d - Jac @ v)))
    assert errs[1] < errs[0] / 20.0  # O(h^2) directional differences approach J v


def test_complex_step_jacobian_matches_differences():
    rng = np.random.default_rng(3)
    mesh = wl.box_mesh((2, 1, 2), bc=(1, 2, 0, 0, 0, 0))
    orders = wl.random_orders(4, 1, 2, rng)
    u = wl.random_state(orders, rng)
    Jc = adjoint.cs_jacobian(mesh, orders, u, form=1)
    Jf = adjoint.fd_jacobian(mesh, orders, u, form=1)
    assert np.max(np.abs(Jc - Jf)) < 1e-8 * np.max(np.abs(Jc))


def test_eta_independent_of_the_adjoint_form():
    """The adjoint of the new form r = M^-1 F is M times the adjoint of the traditional
    form F, so the adjoint-weighted estimate of a consistent pair does not depend on the
    form the adjoint was solved in; feeding the new-form adjoint as if it were the
    traditional one does."""
    rng = np.random.default_rng(6)
    qinf = wl.conserved(*(np.array(x) for x in (1.0, 0.3, 0.0, 0.0, 1.0)))
    mesh = wl.box_mesh((2, 2, 1), bc=(1, 2, 0, 0, 0, 0), qfar=qinf)
    fo = wl.random_orders(4, 1, 3, rng)
    co = np.minimum(fo, wl.random_orders(4, 1, 2, rng))
    u = wl.pulse_state(oracle.node_coords(mesh, fo), fo, sigma=0.3, amp=0.2)
    _, g = oracle.functional(mesh, fo, u)
    dudt = oracle.residual(mesh, fo, u)
    psi_t, _ = adjoint.adjoint_solve(mesh, fo, u, g, form=1)
    psi_n, _ = adjoint.adjoint_solve(mesh, fo, u, g, form=0)
    M = _mass(mesh, fo)
    assert np.max(np.abs(psi_n - M * psi_t)) < 1e-9 * np.max(np.abs(psi_n))
    eta_t = oracle.tau_eta(mesh, fo, co, u, dudt, psi_t, psi_form=1)
    eta_n = oracle.tau_eta(mesh, fo, co, u, dudt, psi_n, psi_form=0)
    assert np.max(np.abs(eta_t - eta_n)) < 1e-9 * np.max(np.abs(eta_t))
    wrong = oracle.tau_eta(mesh, fo, co, u, dudt, psi_n, psi_form=1)
    assert np.max(np.abs(wrong - eta_t)) > 1e-3 * np.max(np.abs(eta_t))
