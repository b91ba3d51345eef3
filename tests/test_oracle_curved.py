"""Pins of the oracle on curved elements: the sine-mapped box of the Navier-Stokes
workload, (x, y, z) -> (x + f, y + f, z), f = a sin(2 pi x) sin(2 pi y), each element's
geometry the order-(2, 2, 1) Gauss-Lobatto interpolant of the map (Section 2.1: the
mapping of every element onto the reference cube, the metric terms Ja^d and J, and the
contravariant fluxes).

Pins: the node coordinates against an independent numpy evaluation of the geometry
interpolant, and the metric terms against the closed forms of a quasi-2D map built from
numpy polynomial derivatives; the total volume; the discrete metric identities;
free-stream preservation with mortars on the x and y faces (Euler and Navier-Stokes,
periodic and far-field boxes); discrete conservation; exactness of the residual and of
the BR1 gradient on a density linear in the mapped coordinates; the coarse geometry
equals the restricted fine coordinates; sweep entries equal the isolated estimate
composed from the residual, both for Euler and Navier-Stokes.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import elem_view, per_var, residual_scale

AMP = 0.05
MU, PR = 0.01, 0.72


def _mesh(n=(3, 3, 2), bc=(0,) * 6, flux=wl.ROE, qfar=(1.0, 0.0, 0.0, 0.0, 2.5)):
    hz = 1.0 / n[0]
    return wl.sine_mapped(wl.box_mesh(n, hi=(1.0, 1.0, n[2] * hz), bc=bc, flux=flux, qfar=qfar), amp=AMP)


def _lagrange_eval(nodes, vals, t):
    """Value of the Lagrange interpolant through (nodes, vals) at t (numpy polyfit)."""
    c = np.polyfit(nodes, vals, len(nodes) - 1)
    return np.polyval(c, t), np.polyval(np.polyder(c), t)


def _geometry_reference(mesh, o, e):
    """Mapped coordinates X, Y and their reference derivatives at the nodes of element e,
    from an independent evaluation of the tensor-product order-2 interpolant."""
    nx, ny, nz = mesh["n"]
    ix, iy = e % nx, (e // nx) % ny
    hx, hy = 1.0 / nx, 1.0 / ny
    g = oracle.lgl(2)[0]
    xs = [oracle.lgl(int(N))[0] for N in o]
    # map values on the 3 x 3 geometry grid
    xb = hx * (ix + 0.5 * (g + 1.0))
    yb = hy * (iy + 0.5 * (g + 1.0))
    f = AMP * np.sin(2 * np.pi * xb)[:, None] * np.sin(2 * np.pi * yb)[None, :]
    PX = xb[:, None] + f
    PY = yb[None, :] + f
    out = {k: np.zeros((len(xs[1]), len(xs[0]))) for k in ("X", "Y", "Xx", "Xy", "Yx", "Yy")}
    for jj, eta in enumerate(xs[1]):
        for ii, xi in enumerate(xs[0]):
            # interpolate along xi for each geometry eta-row, then along eta
            for name, P in (("X", PX), ("Y", PY)):
                rows = np.array([_lagrange_eval(g, P[:, b], xi) for b in range(3)])  # value, d/dxi
                v, dv_eta = _lagrange_eval(g, rows[:, 0], eta)
                dv_xi, _ = _lagrange_eval(g, rows[:, 1], eta)
                out[name][jj, ii] = v
                out[name + "x"][jj, ii] = dv_xi
                out[name + "y"][jj, ii] = dv_eta
    return out


def test_coordinates_and_metrics_against_closed_forms():
    mesh = _mesh()
    rng = np.random.default_rng(80)
    orders = wl.column_orders(mesh, 2, 5, rng)
    xyz = oracle.node_coords(mesh, orders)
    met = oracle.metrics(mesh, orders)
    hz = (mesh["hi"][2] - mesh["lo"][2]) / mesh["n"][2]
    for e in (0, 4, 8, 13):
        o = orders[e]
        ref = _geometry_reference(mesh, o, e)
        X = elem_view(xyz, orders, e, nv=3).reshape(3, o[2] + 1, o[1] + 1, o[0] + 1)
        M = elem_view(met, orders, e, nv=10).reshape(10, o[2] + 1, o[1] + 1, o[0] + 1)
        for k in range(o[2] + 1):
            assert np.allclose(X[0, k], ref["X"], atol=1e-14)
            assert np.allclose(X[1, k], ref["Y"], atol=1e-14)
            Jxy = ref["Xx"] * ref["Yy"] - ref["Xy"] * ref["Yx"]
            closed = [0.5 * hz * ref["Yy"], -0.5 * hz * ref["Xy"], 0 * Jxy,
                      -0.5 * hz * ref["Yx"], 0.5 * hz * ref["Xx"], 0 * Jxy,
                      0 * Jxy, 0 * Jxy, Jxy, 0.5 * hz * Jxy]
            for c in range(10):
                assert np.allclose(M[c, k], closed[c], atol=1e-12), c


def test_volume_and_metric_identities():
    mesh = _mesh((4, 3, 2))
    rng = np.random.default_rng(81)
    orders = wl.column_orders(mesh, 2, 6, rng)
    met = oracle.metrics(mesh, orders)
    vol = 0.0
    for e in range(len(orders)):
        o = orders[e]
        n = o + 1
        M = elem_view(met, orders, e, nv=10).reshape(10, n[2], n[1], n[0])
        w = [oracle.lgl(int(N))[1] for N in o]
        assert np.all(M[9] > 0)
        vol += float(np.einsum("kji,k,j,i->", M[9], w[2], w[1], w[0]))
        D = [oracle.dmat(int(N)) for N in o]
        for comp in range(3):
            div = (np.einsum("iq,kjq->kji", D[0], M[0 * 3 + comp]) + np.einsum("jq,kqi->kji", D[1], M[1 * 3 + comp])
                   + np.einsum("kq,qji->kji", D[2], M[2 * 3 + comp]))
            assert np.max(np.abs(div)) < 1e-14 * np.max(np.abs(M[:9])) * 40
    box = np.prod(np.asarray(mesh["hi"]) - np.asarray(mesh["lo"]))
    assert abs(vol - box) < 1e-14


def _draw(mesh, lo, hi, rng, per_element):
    """Per-column orders (conforming faces between layers) or per-element orders with
    Nz in 1..2 (non-conforming faces in every direction)."""
    if per_element:
        return wl.element_orders(mesh, lo, hi, rng, nz_range=(1, 2))
    return wl.column_orders(mesh, lo, hi, rng)


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("flux,bc", [(wl.ROE, (0,) * 6), (wl.LF, (0,) * 6), (wl.ROE, (2, 2, 0, 0, 0, 0))])
def test_free_stream(flux, bc, per_element):
    q = wl.conserved(*(np.array(v) for v in (1.1, 0.3, -0.2, 0.1, 0.9)))
    mesh = _mesh((3, 3, 2), bc=bc, flux=flux, qfar=tuple(float(v) for v in q))
    rng = np.random.default_rng(82)
    orders = _draw(mesh, 2, 6, rng, per_element)
    u = wl.uniform_state(orders, q)
    s = residual_scale(mesh, orders, u)
    assert np.max(np.abs(oracle.residual(mesh, orders, u))) < 1e-13 * s
    # gradient scale: |Q| max||D|| / h
    gscale = np.max(np.abs(u)) * np.max(orders) ** 2 * mesh["n"][0]
    assert np.max(np.abs(oracle.gradient(mesh, orders, u))) < 1e-13 * gscale
    assert np.max(np.abs(oracle.residual_ns(mesh, orders, u, MU, PR))) < 1e-13 * s


@pytest.mark.parametrize("per_element", [False, True])
def test_conservation(per_element):
    mesh = _mesh((3, 3, 2))
    rng = np.random.default_rng(83)
    orders = _draw(mesh, 2, 6, rng, per_element)
    u = wl.random_state(orders, rng)
    met = oracle.metrics(mesh, orders)
    Jn = np.concatenate([elem_view(met, orders, e, nv=10)[9] for e in range(len(orders))])
    www = []
    for o in orders:
        w = [oracle.lgl(int(N))[1] for N in o]
        www.append(np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1))
    www = np.concatenate(www)
    for res in (oracle.residual(mesh, orders, u), oracle.residual_ns(mesh, orders, u, MU, PR)):
        r = per_var(res, orders)
        tot = (r * Jn * www).sum(axis=1)
        assert np.all(np.abs(tot) < 1e-13 * np.abs(r * Jn * www).sum(axis=1))
    r1 = per_var(oracle.residual(mesh, orders, u, form=1), orders)
    assert np.all(np.abs(r1.sum(axis=1)) < 1e-13 * np.abs(r1).sum(axis=1))


def test_linear_density_is_exact():
    """rho = 1 + a X + b Y (X, Y mapped coordinates), constant velocity (u, v, 0) and
    temperature T0 (p = T0 rho): every contravariant flux is a polynomial the scheme
    differentiates exactly when N_x, N_y >= 4, and the state is continuous, so away from
    the periodic seam (where the linear density jumps) the residual is the divergence of
    the flux at the nodes, for Euler and Navier-Stokes alike (zero viscous stress and
    heat flux), and the BR1 gradient is exact.  Euler and the gradient are checked on
    elements one column away from the seam, Navier-Stokes (whose face flux also reads
    the neighbours' gradients) two columns away."""
    mesh = _mesh((6, 6, 2))
    rng = np.random.default_rng(84)
    orders = wl.column_orders(mesh, 4, 6, rng)
    a, b, T0, uu, vv, g = 0.3, -0.2, 0.8, 0.4, -0.3, 1.4
    xyz = oracle.node_coords(mesh, orders)
    u = np.zeros(5 * int(wl.node_offsets(orders)[-1]))
    ref = np.zeros_like(u)
    gref = np.zeros(3 * len(u))
    for e in range(len(orders)):
        X = elem_view(xyz, orders, e, nv=3)
        rho = 1.0 + a * X[0] + b * X[1]
        p = T0 * rho
        elem_view(u, orders, e)[:] = wl.conserved(rho, uu + 0 * rho, vv + 0 * rho, 0 * rho, p)
        udr = uu * a + vv * b                    # u . grad rho
        k2 = 0.5 * (uu * uu + vv * vv)
        one = np.ones_like(rho)
        elem_view(ref, orders, e)[:] = np.stack([udr * one, (uu * udr + T0 * a) * one, (vv * udr + T0 * b) * one,
                                                 0 * one, (T0 * g / (g - 1) + k2) * udr * one])
        dq = np.array([1.0, uu, vv, 0.0, T0 / (g - 1) + k2])   # d(conserved)/d(rho)
        G = elem_view(gref, orders, e, nv=15).reshape(3, 5, -1)
        G[0] = a * dq[:, None]
        G[1] = b * dq[:, None]
    s = residual_scale(mesh, orders, u)
    r_eu = oracle.residual(mesh, orders, u)
    r_ns = oracle.residual_ns(mesh, orders, u, MU, PR)
    grad = oracle.gradient(mesh, orders, u)
    gscale = np.max(np.abs(u)) * np.max(orders) ** 2 * mesh["n"][0]   # |Q| max||D|| / h
    nx, ny, _ = mesh["n"]
    checked = 0
    for e in range(len(orders)):
        ix, iy = e % nx, (e // nx) % ny
        inner = min(ix, iy, nx - 1 - ix, ny - 1 - iy)
        if inner >= 1:
            assert np.max(np.abs(elem_view(r_eu, orders, e) - elem_view(ref, orders, e))) < 1e-12 * s
            assert np.max(np.abs(elem_view(grad, orders, e, nv=15) - elem_view(gref, orders, e, nv=15))) < 1e-13 * gscale
            checked += 1
        if inner >= 2:
            assert np.max(np.abs(elem_view(r_ns, orders, e) - elem_view(ref, orders, e))) < 1e-12 * s
    assert checked == 2 * 16
    # the seam is where the exactness stops
    assert np.max(np.abs(r_eu - ref)) > 1e-3


def test_coarse_geometry_is_the_restricted_fine_geometry():
    mesh = _mesh((3, 2, 2))
    rng = np.random.default_rng(85)
    fo = wl.column_orders(mesh, 2, 6, rng)
    co = fo.copy()
    co[:, :2] = np.minimum(fo[:, :2], rng.integers(1, 6, (len(fo), 2)))
    xf = oracle.node_coords(mesh, fo)
    xc = oracle.node_coords(mesh, co)
    # restrict the 3 coordinate fields (padded to 5 fields) with the oracle's restriction
    pad = np.concatenate([np.concatenate([elem_view(xf, fo, e, nv=3), np.zeros((2, wl.node_counts(fo)[e]))]).ravel()
                          for e in range(len(fo))])
    rc = oracle.restrict(fo, co, pad)
    got = np.concatenate([elem_view(rc, co, e)[:3].ravel() for e in range(len(co))])
    assert np.max(np.abs(got - xc)) < 1e-14


@pytest.mark.parametrize("viscous", [False, True])
def test_sweep_equals_composed_isolated_estimate(viscous):
    mesh = _mesh((2, 2, 2))
    rng = np.random.default_rng(86 + viscous)
    fo = wl.column_orders(mesh, 2, 4, rng)
    xyz = oracle.node_coords(mesh, fo)
    u = wl.pulse_state(xyz, fo, sigma=0.2)
    u = wl.add_rho_noise(u, fo, rng, 1e-3)
    if viscous:
        dudt = oracle.residual_ns(mesh, fo, u, MU, PR)
        ten, tet, offs = oracle.sweep_ns(mesh, fo, u, dudt, MU, PR)
    else:
        dudt = oracle.residual(mesh, fo, u)
        ten, tet, offs = oracle.sweep(mesh, fo, u, dudt)
    E = len(fo)
    for e in range(E):
        cm = np.maximum(fo[e] - 1, 1)
        k = 0
        for c3 in range(1, cm[2] + 1):
            for c2 in range(1, cm[1] + 1):
                for c1 in range(1, cm[0] + 1):
                    co = fo.copy()
                    co[e] = (c1, c2, c3)
                    uc = oracle.restrict(fo, co, u)
                    if viscous:
                        res = oracle.residual_ns(mesh, co, uc, MU, PR, isolated=True)
                    else:
                        res = oracle.residual(mesh, co, uc, isolated=True)
                    tn = elem_view(res - oracle.restrict(fo, co, dudt), co, e)
                    Jn = elem_view(oracle.metrics(mesh, co), co, e, nv=10)[9]
                    w = [oracle.lgl(int(N))[1] for N in (c1, c2, c3)]
                    www = np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1)
                    assert abs(ten[offs[e] + k] - np.max(np.abs(tn))) < 1e-14 * max(1.0, np.max(np.abs(tn)))
                    assert abs(tet[offs[e] + k] - np.max(np.abs(tn * Jn * www))) < 1e-16
                    k += 1
