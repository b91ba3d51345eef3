"""Pins of the oracle's DGSEM residual (Section 2.1, eqs. DGSEMsystem and
DGMassMatrixLeft/Right) on box meshes with per-element anisotropic orders.

Each pin checks the residual against something fixed by the mathematics:
free-stream preservation, discrete conservation, exactness on a contact
discontinuity-free state whose flux is affine in the density (mortars on every
face), an independently written 1D weak-form DGSEM, bitwise translation
invariance and the placement of the surface terms.
"""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle
import workloads as wl
from helpers import elem_view, per_var, residual_scale, split

G = 1.4


def _mass_weights(mesh, orders):
    """J w_i w_j w_k per node (natural ragged, one value per node)."""
    n = np.asarray(mesh["n"], dtype=float)
    h = (np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / n
    J = h.prod() / 8.0
    out = []
    for o in np.asarray(orders).reshape(-1, 3):
        w = [oracle.lgl(int(N))[1] for N in o]
        out.append(J * np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1))
    return np.concatenate(out)


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_free_stream_mixed_orders(flux):
    rng = np.random.default_rng(10)
    q = wl.conserved(np.array(1.2), np.array(0.3), np.array(-0.2), np.array(0.5), np.array(0.9))
    mesh = wl.box_mesh((3, 3, 2), flux=flux)
    orders = wl.random_orders(18, 1, 7, rng)
    u = wl.uniform_state(orders, q)
    r = oracle.residual(mesh, orders, u)
    s = residual_scale(mesh, orders, u)
    assert np.max(np.abs(r)) < 1e-13 * s
    # boundary conditions: far field carrying the same state on x, slip walls on y
    # for a flow tangent to them
    q2 = wl.conserved(np.array(1.2), np.array(0.3), np.array(0.0), np.array(0.5), np.array(0.9))
    mesh2 = wl.box_mesh((3, 2, 2), bc=(2, 2, 1, 1, 0, 0), flux=flux, qfar=q2)
    orders2 = wl.random_orders(12, 1, 6, rng)
    u2 = wl.uniform_state(orders2, q2)
    r2 = oracle.residual(mesh2, orders2, u2)
    assert np.max(np.abs(r2)) < 1e-13 * residual_scale(mesh2, orders2, u2)


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_discrete_conservation_periodic(flux):
    rng = np.random.default_rng(11)
    mesh = wl.box_mesh((3, 2, 3), lo=(0, 0, 0), hi=(1.5, 1.0, 0.75), flux=flux)
    orders = wl.random_orders(18, 1, 7, rng)
    u = wl.random_state(orders, rng)
    for form in (0, 1):
        r = oracle.residual(mesh, orders, u, form=form)
        Mw = _mass_weights(mesh, orders)
        R = per_var(r, orders)
        weighted = R * Mw if form == 0 else R  # traditional form is already M r
        tot = weighted.sum(axis=1)
        ref = np.abs(weighted).sum(axis=1)
        assert np.all(np.abs(tot) < 1e-13 * ref), (form, tot / ref)


def _pw_quadratic(x, ie, h, vals, beta):
    """Continuous periodic piecewise quadratic: element ie carries
    c_ie (1-xi)/2 + c_{ie+1} (1+xi)/2 + beta_ie (1 - xi^2); returns value and d/dx."""
    n = len(vals)
    xi = 2.0 * (x - ie * h) / h - 1.0
    c0, c1, b = vals[ie], vals[(ie + 1) % n], beta[ie]
    g = c0 * (1 - xi) / 2 + c1 * (1 + xi) / 2 + b * (1 - xi * xi)
    dg = (2.0 / h) * (-c0 / 2 + c1 / 2 - 2.0 * b * xi)
    return g, dg


def contact_state(mesh, orders, rng, U):
    """rho = 1 + 0.1 g(x) h(y) k(z) with continuous periodic piecewise quadratics;
    returns (u, div f) in the natural ragged layout (div f evaluated element-wise)."""
    nx, ny, nz = mesh["n"]
    fx = (rng.normal(size=nx), rng.normal(size=nx))
    fy = (rng.normal(size=ny), rng.normal(size=ny))
    fz = (rng.normal(size=nz), rng.normal(size=nz))
    xyz = oracle.node_coords(mesh, orders)
    E = nx * ny * nz
    u = np.zeros(5 * int(wl.node_offsets(orders)[-1]))
    div = np.zeros_like(u)
    for e in range(E):
        ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
        X = elem_view(xyz, orders, e, nv=3)
        gx, dgx = _pw_quadratic(X[0], ix, 1.0 / nx, *fx)
        gy, dgy = _pw_quadratic(X[1], iy, 1.0 / ny, *fy)
        gz, dgz = _pw_quadratic(X[2], iz, 1.0 / nz, *fz)
        rho = 1.0 + 0.1 * gx * gy * gz
        grad = 0.1 * np.stack([dgx * gy * gz, gx * dgy * gz, gx * gy * dgz])
        one = np.ones_like(rho)
        elem_view(u, orders, e)[:] = wl.conserved(rho, U[0] * one, U[1] * one, U[2] * one, one)
        a = U @ grad
        elem_view(div, orders, e)[:] = np.stack([a, a * U[0], a * U[1], a * U[2], a * 0.5 * (U @ U)])
    return u, div


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_contact_exact_with_mortars(flux):
    """rho = 1 + 0.1 g(x) h(y) k(z) (continuous, degree 2 per direction), constant
    velocity U and pressure: every flux is affine in rho, so the DGSEM residual
    equals div f = (U . grad rho)(1, U, |U|^2/2) at the nodes for any orders >= 2,
    with non-conforming mortars on every face."""
    rng = np.random.default_rng(12)
    mesh = wl.box_mesh((3, 3, 2), flux=flux)
    orders = wl.random_orders(18, 2, 6, rng)
    u, div = contact_state(mesh, orders, rng, np.array([0.3, -0.5, 0.7]))
    r = oracle.residual(mesh, orders, u)
    s = residual_scale(mesh, orders, u)
    assert np.max(np.abs(r - div)) < 2e-13 * s
    # the check has teeth: dropping the face coupling breaks it at face nodes
    r_iso = oracle.residual(mesh, orders, u, isolated=True)
    assert np.max(np.abs(r_iso - div)) < 2e-13 * s  # continuous state: SAT vanishes too
    bad = wl.random_orders(18, 1, 6, rng)  # order-1 directions cannot hold the quadratic
    bad[:, 0] = 1
    ub, divb = contact_state(mesh, bad, np.random.default_rng(12), np.array([0.3, -0.5, 0.7]))
    assert np.max(np.abs(oracle.residual(mesh, bad, ub) - divb)) > 1e-6 * s


def _lgl_independent(N):
    """Gauss-Lobatto nodes, weights and differentiation matrix from numpy's Legendre
    module and a monomial Vandermonde matrix (independent of the oracle)."""
    dL = npleg.legder(np.eye(N + 1)[N])
    x = np.concatenate([[-1.0], np.sort(np.real(npleg.legroots(dL))), [1.0]])
    LN = npleg.legval(x, np.eye(N + 1)[N])
    w = 2.0 / (N * (N + 1) * LN ** 2)
    V = np.vander(x, N + 1, increasing=True)
    dV = np.zeros_like(V)
    for k in range(1, N + 1):
        dV[:, k] = k * x ** (k - 1)
    D = dV @ np.linalg.inv(V)
    return x, w, D


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_reduces_to_1d_weak_form(flux):
    """A state depending on x only reduces the 3D residual to a 1D DGSEM in weak
    form: (h/2) w_j dq_j/dt = sum_i w_i D_ij f_i - [f* l_j] (Section 2.1)."""
    N, nx = 4, 5
    mesh = wl.box_mesh((nx, 2, 2), lo=(0, 0, 0), hi=(2.0, 1.0, 1.0), flux=flux)
    orders = np.tile(np.array([N, 2, 3], dtype=np.int32), (nx * 4, 1))
    rng = np.random.default_rng(13)
    x, w, D = _lgl_independent(N)
    h = 2.0 / nx
    # random x-only nodal state per x-element (discontinuous across elements)
    rho = rng.uniform(0.8, 1.2, (nx, N + 1))
    vel = rng.uniform(-0.4, 0.4, (nx, N + 1))
    p = rng.uniform(0.8, 1.2, (nx, N + 1))
    q1 = np.stack([rho, rho * vel, p / (G - 1) + 0.5 * rho * vel ** 2])  # [3, nx, n]
    # 3D state
    u = np.zeros(5 * int(wl.node_offsets(orders)[-1]))
    for e in range(nx * 4):
        ix = e % nx
        blk = elem_view(u, orders, e)
        n1, n2, n3 = N + 1, 3, 4
        i = np.tile(np.arange(n1), n2 * n3)
        blk[0] = rho[ix, i]
        blk[1] = rho[ix, i] * vel[ix, i]
        blk[4] = p[ix, i] / (G - 1) + 0.5 * rho[ix, i] * vel[ix, i] ** 2
    r = oracle.residual(mesh, orders, u)

    def f1(q):
        r_, m_, E_ = q
        v_ = m_ / r_
        p_ = (G - 1) * (E_ - 0.5 * r_ * v_ ** 2)
        return np.stack([m_, m_ * v_ + p_, (E_ + p_) * v_])

    def nf(qa, qb):
        to3 = lambda q: np.array([q[0], q[1], 0.0, 0.0, q[2]])
        f = oracle.numflux(to3(qa), to3(qb), np.array([1.0, 0, 0]), G, flux)
        return f[[0, 1, 4]]

    r1 = np.zeros((3, nx, N + 1))
    for ix in range(nx):
        qe = q1[:, ix]
        fe = f1(qe)
        vol = (w[:, None] * D).T @ fe.T  # sum_i w_i D_ij f_i  -> [n, 3]
        fR = nf(qe[:, N], q1[:, (ix + 1) % nx, 0])
        fL = nf(q1[:, (ix - 1) % nx, N], qe[:, 0])
        rhs = vol.T.copy()
        rhs[:, N] -= fR
        rhs[:, 0] += fL
        dqdt = rhs / (0.5 * h * w)
        r1[:, ix] = -dqdt
    s = residual_scale(mesh, orders, u)
    for e in range(nx * 4):
        ix = e % nx
        blk = elem_view(r, orders, e)
        i = np.tile(np.arange(N + 1), 12)
        for v3, v5 in ((0, 0), (1, 1), (2, 4)):
            assert np.max(np.abs(blk[v5] - r1[v3, ix, i])) < 1e-12 * s
        assert np.max(np.abs(blk[2:4])) < 1e-12 * s


def test_translation_is_bitwise_permutation():
    rng = np.random.default_rng(14)
    nx, ny, nz = 4, 3, 2
    mesh = wl.box_mesh((nx, ny, nz))
    E = nx * ny * nz
    orders = wl.random_orders(E, 1, 5, rng)
    u = wl.random_state(orders, rng)
    r = oracle.residual(mesh, orders, u)
    # shift by one element along x
    perm = np.array([((e % nx) - 1) % nx + nx * (e // nx) for e in range(E)])  # new e <- old perm[e]
    orders_s = orders[perm]
    blocks = split(u, orders)
    u_s = np.concatenate([blocks[perm[e]].reshape(-1) for e in range(E)])
    r_s = oracle.residual(mesh, orders_s, u_s)
    rb = split(r, orders)
    for e in range(E):
        assert np.array_equal(elem_view(r_s, orders_s, e), rb[perm[e]])


def test_surface_terms_only_on_face_nodes():
    rng = np.random.default_rng(15)
    mesh = wl.box_mesh((2, 2, 2))
    orders = wl.random_orders(8, 2, 6, rng)
    u = wl.random_state(orders, rng)
    r = oracle.residual(mesh, orders, u)
    ri = oracle.residual(mesh, orders, u, isolated=True)
    for e in range(8):
        n1, n2, n3 = orders[e] + 1
        k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
        inner = ((i > 0) & (i < n1 - 1) & (j > 0) & (j < n2 - 1) & (k > 0) & (k < n3 - 1)).reshape(-1)
        a, b = elem_view(r, orders, e), elem_view(ri, orders, e)
        assert np.array_equal(a[:, inner], b[:, inner])
        assert np.max(np.abs(a[:, ~inner] - b[:, ~inner])) > 0.0


def test_forms_related_by_mass_matrix():
    """Traditional form = M times new form, M = diag(J w_i w_j w_k) (eq. TEdef)."""
    rng = np.random.default_rng(16)
    mesh = wl.box_mesh((2, 3, 2), hi=(1.0, 0.6, 2.0))
    orders = wl.random_orders(12, 1, 6, rng)
    u = wl.random_state(orders, rng)
    rn = per_var(oracle.residual(mesh, orders, u, form=0), orders)
    rt = per_var(oracle.residual(mesh, orders, u, form=1), orders)
    Mw = _mass_weights(mesh, orders)
    assert np.max(np.abs(rt - Mw * rn)) < 1e-13 * np.max(np.abs(rt))
