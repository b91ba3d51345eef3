"""Pins of the solution transfer onto a new order map (oracle.project): exact on
polynomials of the target space (evaluated with numpy polynomials), the residual of a
lowering is L2-orthogonal to the target space (numpy Gauss-Legendre quadrature on the
reference cube), raising then lowering is the identity, the element integral is kept;
and the per-stage decrease limit of the selection oracle."""
import numpy as np
import pytest

import oracle
from oracle import select as sel


def _nodes(N):
    return np.asarray(oracle.lgl(int(N))[0])


def _offsets(orders):
    n = np.prod(np.asarray(orders) + 1, axis=1)
    return np.concatenate([[0], np.cumsum(n)])


def _eval_poly(coef, x, y, z):
    """sum_{abc} coef[a,b,c] x^a y^b z^c on the tensor grid (x fastest)."""
    X = np.polynomial.polynomial.polyvander(x, coef.shape[0] - 1)
    Y = np.polynomial.polynomial.polyvander(y, coef.shape[1] - 1)
    Z = np.polynomial.polynomial.polyvander(z, coef.shape[2] - 1)
    return np.einsum("ia,jb,kc,abc->kji", X, Y, Z, coef).reshape(-1)


def _nodal_to_values(vals, N, pts):
    """Evaluate the tensor-product interpolant of nodal values (order N, [k][j][i]) at the
    tensor grid pts (three 1-D arrays), through numpy Vandermonde solves."""
    out = vals.reshape(N[2] + 1, N[1] + 1, N[0] + 1)
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        x = _nodes(N[d])
        V = np.polynomial.polynomial.polyvander(x, N[d])
        C = np.linalg.solve(V, np.moveaxis(out, axis, 0).reshape(N[d] + 1, -1))
        W = np.polynomial.polynomial.polyvander(pts[d], N[d]) @ C
        out = np.moveaxis(W.reshape((len(pts[d]),) + np.moveaxis(out, axis, 0).shape[1:]), 0, axis)
    return out


def test_exact_on_target_space():
    rng = np.random.default_rng(1)
    fo = np.array([[3, 6, 2], [7, 2, 5], [4, 4, 4], [1, 8, 3]], dtype=np.int32)
    to = np.array([[6, 2, 2], [3, 5, 1], [4, 7, 2], [5, 4, 3]], dtype=np.int32)
    u = np.zeros(5 * _offsets(fo)[-1])
    exp = np.zeros(5 * _offsets(to)[-1])
    of, ot = _offsets(fo), _offsets(to)
    for e in range(len(fo)):
        deg = np.minimum(fo[e], to[e])
        nf, nt = int(of[e + 1] - of[e]), int(ot[e + 1] - ot[e])
        for v in range(5):
            coef = rng.normal(size=tuple(deg + 1))
            u[5 * of[e] + v * nf: 5 * of[e] + (v + 1) * nf] = _eval_poly(coef, *(_nodes(n) for n in fo[e]))
            exp[5 * ot[e] + v * nt: 5 * ot[e] + (v + 1) * nt] = _eval_poly(coef, *(_nodes(n) for n in to[e]))
    got = oracle.project(fo, to, u)
    assert np.max(np.abs(got - exp)) < 1e-12 * np.max(np.abs(exp))


def test_lowering_residual_is_orthogonal():
    rng = np.random.default_rng(2)
    fo = np.array([[6, 5, 4]], dtype=np.int32)
    to = np.array([[3, 5, 2]], dtype=np.int32)  # x and z lowered, y kept
    u = rng.normal(size=5 * int(np.prod(fo[0] + 1)))
    pu = oracle.project(fo, to, u)
    g, w = np.polynomial.legendre.leggauss(10)
    W = np.einsum("k,j,i->kji", w, w, w)
    nf, nt = int(np.prod(fo[0] + 1)), int(np.prod(to[0] + 1))
    for v in range(5):
        a = _nodal_to_values(u[v * nf:(v + 1) * nf], fo[0], (g, g, g))
        b = _nodal_to_values(pu[v * nt:(v + 1) * nt], to[0], (g, g, g))
        r = a - b
        for p in range(to[0, 0] + 1):
            for q in range(to[0, 1] + 1):
                for s in range(to[0, 2] + 1):
                    phi = np.einsum("k,j,i->kji", g ** s, g ** q, g ** p)
                    assert abs(np.sum(W * r * phi)) < 1e-12 * np.sqrt(np.sum(W * a * a))


def test_raise_then_lower_is_identity_and_integral_kept():
    rng = np.random.default_rng(3)
    lo = rng.integers(1, 6, (20, 3)).astype(np.int32)
    hi = (lo + rng.integers(0, 4, (20, 3))).astype(np.int32)
    u = rng.normal(size=5 * _offsets(lo)[-1])
    up = oracle.project(lo, hi, u)
    back = oracle.project(hi, lo, up)
    assert np.max(np.abs(back - u)) < 1e-12 * np.max(np.abs(u))
    # element integrals (LGL quadrature, exact on both sides) are kept by any transfer
    mixed = np.where(rng.random((20, 3)) < 0.5, lo, np.maximum(1, lo - 1)).astype(np.int32)
    for src, dst, x in ((lo, hi, u), (hi, lo, up), (lo, mixed, u)):
        y = oracle.project(src, dst, x)
        os_, od = _offsets(src), _offsets(dst)
        for e in range(20):
            ws = np.einsum("k,j,i->kji", *(oracle.lgl(int(n))[1] for n in src[e][::-1])).reshape(-1)
            wd = np.einsum("k,j,i->kji", *(oracle.lgl(int(n))[1] for n in dst[e][::-1])).reshape(-1)
            ns, nd = len(ws), len(wd)
            for v in range(5):
                I0 = ws @ x[5 * os_[e] + v * ns: 5 * os_[e] + (v + 1) * ns]
                I1 = wd @ y[5 * od[e] + v * nd: 5 * od[e] + (v + 1) * nd]
                assert abs(I0 - I1) < 1e-12 * max(1.0, abs(I0))


def test_decrease_limit():
    prev = np.array([[5, 5, 5], [2, 8, 1], [9, 9, 9]], dtype=np.int32)
    sel_ = np.array([[1, 7, 4], [1, 3, 1], [2, 2, 2]], dtype=np.int32)
    got = sel.limit_decrease(sel_, prev, 1, 8)
    assert got.tolist() == [[4, 7, 4], [1, 7, 1], [8, 8, 8]]
    assert np.array_equal(sel.limit_decrease(sel_, prev, 10, 8), sel_)
