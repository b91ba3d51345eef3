"""Pins of the oracle's derivatives of the residual (box Euler meshes).

The oracle has two independent routes to the derivative of the residual r(u) of
Section 2.1 (the adjoint problem behind the adjoint-weighted estimate, Section 2.2's
remark on functional errors): a complex-step directional derivative (the residual in
complex arithmetic) and a hand-transposed vector-Jacobian product.  They are pinned
here to things other than themselves:

* the closed-form Jacobian of the physical flux: central differences of the real
  flux, homogeneity of degree one of the Euler flux (A(q) q = f(q)), and its
  eigenvalues u_n - c, u_n, u_n, u_n, u_n + c;
* the Riemann-flux Jacobians (complex step): central differences of the real
  numerical flux, consistency (at equal states d f*/d qL + d f*/d qR = A), and at
  equal states the textbook upwind split of the Roe flux, d f*/d qR = (A - |A|)/2
  with |A| = R |Lambda| R^-1 from numpy's eigendecomposition (Rusanov: (A - s I)/2);
* the complex residual: its real part is the oracle residual, its imaginary part
  divided by h matches central differences of the real residual;
* the VJP: the dot test <v, J d> = <J^T v, d> against the complex-step JVP on
  random meshes (periodic, slip-wall and far-field faces; Roe and Rusanov; both
  forms; isolated) and on periodic chains whose consecutive tangential orders run
  through every ordered pair in 1..7 (all mortar pairs, each direction); the whole
  Jacobian on a tiny mesh (rows by VJP, columns by JVP); and, independently of the
  JVP, discrete conservation: on a periodic mesh sum_i M_ii r_i,v does not depend on
  the state, so J^T (M e_v) = 0 (new form) and J^T e_v = 0 (traditional form).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import de_bruijn_pairs, mortar_chain

G = 1.4


def _rand_q(rng):
    rho = rng.uniform(0.6, 1.5)
    vel = rng.uniform(-0.6, 0.6, 3)
    p = rng.uniform(0.6, 1.5)
    return wl.conserved(np.array(rho), *[np.array(c) for c in vel], np.array(p))


def _rand_n(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def _fd_cols(fn, q, eps=1e-6):
    out = []
    for j in range(5):
        e = np.zeros(5)
        e[j] = eps * max(1.0, abs(q[j]))
        out.append((fn(q + e) - fn(q - e)) / (2 * e[j]))
    return np.stack(out, axis=1)


def test_flux_jacobian_closed_form():
    rng = np.random.default_rng(0)
    for _ in range(50):
        q, n = _rand_q(rng), _rand_n(rng)
        A = oracle.flux_jacobian(q, n)
        fd = _fd_cols(lambda x: oracle.flux_n(x, n), q)
        assert np.max(np.abs(A - fd)) < 1e-8 * np.max(np.abs(A))
        # homogeneous of degree one: f(q) = A(q) q
        f = oracle.flux_n(q, n)
        assert np.max(np.abs(A @ q - f)) < 1e-14 * np.max(np.abs(f)) * 10
        rho, vel = q[0], q[1:4] / q[0]
        p = (G - 1) * (q[4] - 0.5 * rho * vel @ vel)
        c, un = np.sqrt(G * p / rho), vel @ n
        ev = np.sort(np.linalg.eigvals(A).real)
        assert np.allclose(ev, np.sort([un - c, un, un, un, un + c]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [wl.ROE, wl.LF])
def test_numflux_jacobians_against_differences(kind):
    rng = np.random.default_rng(1 + kind)
    for _ in range(40):
        qL, qR, n = _rand_q(rng), _rand_q(rng), _rand_n(rng)
        AL, AR = oracle.numflux_jacobian(qL, qR, n, kind=kind)
        fdL = _fd_cols(lambda x: oracle.numflux(x, qR, n, kind=kind), qL)
        fdR = _fd_cols(lambda x: oracle.numflux(qL, x, n, kind=kind), qR)
        scale = max(np.max(np.abs(AL)), np.max(np.abs(AR)))
        assert np.max(np.abs(AL - fdL)) < 1e-7 * scale
        assert np.max(np.abs(AR - fdR)) < 1e-7 * scale


def test_numflux_jacobians_at_equal_states():
    rng = np.random.default_rng(3)
    for _ in range(40):
        q, n = _rand_q(rng), _rand_n(rng)
        A = oracle.flux_jacobian(q, n)
        # Roe: upwind split of the Jacobian, |A| = R |Lambda| R^-1
        lam, R = np.linalg.eig(A)
        absA = (R @ np.diag(np.abs(lam.real)) @ np.linalg.inv(R)).real
        AL, AR = oracle.numflux_jacobian(q, q, n, kind=wl.ROE)
        assert np.max(np.abs(AL + AR - A)) < 1e-13 * np.max(np.abs(A)) * 10
        assert np.max(np.abs(AR - 0.5 * (A - absA))) < 1e-11 * np.max(np.abs(A))
        assert np.max(np.abs(AL - 0.5 * (A + absA))) < 1e-11 * np.max(np.abs(A))
        # Rusanov: f* = (fL + fR)/2 - s (qR - qL)/2, s = |u_n| + c
        rho, vel = q[0], q[1:4] / q[0]
        p = (G - 1) * (q[4] - 0.5 * rho * vel @ vel)
        s = abs(vel @ n) + np.sqrt(G * p / rho)
        AL, AR = oracle.numflux_jacobian(q, q, n, kind=wl.LF)
        assert np.max(np.abs(AR - 0.5 * (A - s * np.eye(5)))) < 1e-13 * np.max(np.abs(A)) * 10
        assert np.max(np.abs(AL - 0.5 * (A + s * np.eye(5)))) < 1e-13 * np.max(np.abs(A)) * 10


QINF = tuple(wl.conserved(np.array(1.0), np.array(0.3), np.array(0.4), np.array(0.5), np.array(1.0)))

MESHES = [((2, 2, 2), 1, 5, (0,) * 6, wl.ROE),
          ((3, 2, 1), 1, 4, (1, 2, 0, 0, 0, 0), wl.ROE),
          ((2, 1, 2), 1, 3, (0, 0, 1, 2, 0, 0), wl.LF),
          ((1, 2, 2), 2, 6, (0, 0, 0, 0, 2, 1), wl.ROE),
          ((1, 1, 1), 1, 7, (0,) * 6, wl.ROE),
          ((2, 2, 1), 1, 9, (1, 1, 0, 0, 2, 2), wl.LF)]


def _case(shape, lo, hi, bc, flux, seed):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh(shape, lo=(0.1, -0.2, 0.0), hi=(1.1, 0.6, 1.5), bc=bc, flux=flux, qfar=QINF)
    orders = wl.random_orders(int(np.prod(shape)), lo, hi, rng)
    return mesh, orders, wl.random_state(orders, rng), rng


@pytest.mark.parametrize("i", range(len(MESHES)))
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True), (1, True)])
def test_complex_residual_and_jvp(i, form, isolated):
    mesh, orders, u, rng = _case(*MESHES[i], seed=10 + i)
    r = oracle.residual(mesh, orders, u, form, isolated)
    re, im = oracle.residual_cstep(mesh, orders, u, rng.normal(size=u.size), 1e-30, form, isolated)
    assert np.max(np.abs(re - r)) <= 1e-15 * np.max(np.abs(r))
    d = rng.normal(size=u.size) * 1e-2
    jd = oracle.residual_jvp(mesh, orders, u, d, form, isolated)
    eps = 1e-5
    fd = (oracle.residual(mesh, orders, u + eps * d, form, isolated)
          - oracle.residual(mesh, orders, u - eps * d, form, isolated)) / (2 * eps)
    assert np.max(np.abs(jd - fd)) < 1e-7 * np.max(np.abs(jd))


def _dot_err(mesh, orders, u, rng, form, isolated, ntries=4):
    worst = 0.0
    for _ in range(ntries):
        v, d = rng.normal(size=u.size), rng.normal(size=u.size)
        jd = oracle.residual_jvp(mesh, orders, u, d, form, isolated)
        jtv = oracle.residual_vjp(mesh, orders, u, v, form, isolated)
        a, b = v @ jd, jtv @ d
        worst = max(worst, abs(a - b) / (np.abs(v) @ np.abs(jd) + np.abs(jtv) @ np.abs(d)))
    return worst


@pytest.mark.parametrize("i", range(len(MESHES)))
@pytest.mark.parametrize("form,isolated", [(0, False), (1, False), (0, True), (1, True)])
def test_vjp_dot_test(i, form, isolated):
    mesh, orders, u, rng = _case(*MESHES[i], seed=20 + i)
    assert _dot_err(mesh, orders, u, rng, form, isolated) < 1e-12


def test_de_bruijn_covers_every_pair():
    seq = de_bruijn_pairs(7)
    pairs = {(seq[i], seq[(i + 1) % len(seq)]) for i in range(len(seq))}
    assert len(seq) == 49 and pairs == {(a, b) for a in range(1, 8) for b in range(1, 8)}


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_vjp_dot_test_every_mortar_pair(d, flux):
    rng = np.random.default_rng(30 + d + 3 * flux)
    mesh, orders = mortar_chain(d, rng)
    mesh["flux"] = flux
    u = wl.random_state(orders, rng)
    for form in (0, 1):
        assert _dot_err(mesh, orders, u, rng, form, False, ntries=2) < 1e-12


@pytest.mark.parametrize("bc", [(1, 2, 0, 0, 0, 0), (0, 0, 2, 1, 1, 1)])
def test_vjp_whole_jacobian_tiny_mesh(bc):
    rng = np.random.default_rng(40)
    mesh = wl.box_mesh((2, 1, 2), bc=bc, qfar=QINF)
    orders = wl.random_orders(4, 1, 2, rng)
    u = wl.random_state(orders, rng)
    n = u.size
    eye = np.eye(n)
    cols = np.stack([oracle.residual_jvp(mesh, orders, u, eye[j]) for j in range(n)], axis=1)
    rows = np.stack([oracle.residual_vjp(mesh, orders, u, eye[i]) for i in range(n)], axis=0)
    assert np.max(np.abs(rows - cols)) < 1e-12 * np.max(np.abs(cols))


def _mass(mesh, orders):
    """Diagonal of M = J w_i w_j w_k in the natural layout (box elements)."""
    h = (np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / np.asarray(mesh["n"])
    J = np.prod(h) / 8.0
    out = []
    for o in np.asarray(orders).reshape(-1, 3):
        w = [oracle.lgl(int(N))[1] for N in o]
        www = np.einsum("k,j,i->kji", w[2], w[1], w[0]).ravel()
        out.append(np.tile(J * www, 5))
    return np.concatenate(out)


@pytest.mark.parametrize("flux", [wl.ROE, wl.LF])
def test_vjp_keeps_discrete_conservation(flux):
    rng = np.random.default_rng(50 + flux)
    mesh = wl.box_mesh((3, 2, 2), hi=(1.0, 0.8, 1.2), flux=flux)
    orders = wl.random_orders(12, 1, 6, rng)
    u = wl.random_state(orders, rng)
    M = _mass(mesh, orders)
    var = np.concatenate([np.repeat(np.arange(5), int(c)) for c in wl.node_counts(orders)])
    for v in range(5):
        ev = (var == v).astype(float)
        for form, weight in ((0, M * ev), (1, ev)):
            g = oracle.residual_vjp(mesh, orders, u, weight, form)
            # scale of the terms that cancel: the same weight with random factors in
            # [0.5, 1.5] (no systematic cancellation)
            ref = oracle.residual_vjp(mesh, orders, u, weight * rng.uniform(0.5, 1.5, u.size), form)
            assert np.max(np.abs(g)) < 1e-12 * np.max(np.abs(ref)), (v, form)


def test_vjp_conservation_with_slip_walls():
    """With a slip wall the mass-weighted sum of the momentum's normal component is not
    conserved (the wall exerts the pressure force), but mass and energy are: J^T (M e_rho)
    and J^T (M e_E) vanish, J^T (M e_mx) does not."""
    rng = np.random.default_rng(52)
    mesh = wl.box_mesh((2, 2, 2), bc=(1, 1, 0, 0, 0, 0))
    orders = wl.random_orders(8, 1, 5, rng)
    u = wl.random_state(orders, rng)
    M = _mass(mesh, orders)
    var = np.concatenate([np.repeat(np.arange(5), int(c)) for c in wl.node_counts(orders)])
    g = {v: oracle.residual_vjp(mesh, orders, u, M * (var == v), 0) for v in range(5)}
    ref = oracle.residual_vjp(mesh, orders, u, M * rng.uniform(0.5, 1.5, u.size), 0)
    for v in (0, 2, 3, 4):
        assert np.max(np.abs(g[v])) < 1e-12 * np.max(np.abs(ref)), v
    assert np.max(np.abs(g[1])) > 1e-3 * np.max(np.abs(ref))
