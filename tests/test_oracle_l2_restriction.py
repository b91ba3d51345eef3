"""Pins of the tau-estimate with the L2-projection restriction (Section 2.3: the operator
I^N of the truncation-error definition maps the fine solution into the coarse space; the
paper samples, the exact L2 projection is the other choice).

The restriction of Q and of the fine time derivative is computed here independently of
the oracle's tables: Gauss-Lobatto nodes from numpy's Legendre roots, the projection
from its normal equations under numpy Gauss-Legendre quadrature on the reference cube,
the sampling from Lagrange products.  The coarse residual of the restricted state comes
from oracle.residual (pinned by its own tests)."""
import numpy as np
import pytest

import oracle
import workloads as wl


def _lgl(N):
    P = np.polynomial.legendre.Legendre.basis(N)
    return np.concatenate([[-1.0], np.sort(P.deriv().roots().real), [1.0]])


def _lgl_weights(N):
    x = _lgl(N)
    return 2.0 / (N * (N + 1) * np.polynomial.legendre.Legendre.basis(N)(x) ** 2)


def _lagrange(xn, x):
    """L[q, k] = l_k(x_q) for the Lagrange basis on the nodes xn."""
    L = np.ones((len(x), len(xn)))
    for k in range(len(xn)):
        for m in range(len(xn)):
            if m != k:
                L[:, k] *= (x - xn[m]) / (xn[k] - xn[m])
    return L


def _op_sample(c, f):
    return _lagrange(_lgl(f), _lgl(c))


def _op_l2(c, f):
    g, w = np.polynomial.legendre.leggauss(16)
    Bc, Bf = _lagrange(_lgl(c), g), _lagrange(_lgl(f), g)
    return np.linalg.solve(Bc.T @ (w[:, None] * Bc), Bc.T @ (w[:, None] * Bf))


def _apply(fo, co, u, op):
    """Element by element and variable by variable, A3 (x) A2 (x) A1 on [k][j][i] blocks."""
    nf = np.prod(fo + 1, axis=1)
    nc = np.prod(co + 1, axis=1)
    of, oc = np.concatenate([[0], np.cumsum(nf)]), np.concatenate([[0], np.cumsum(nc)])
    out = np.zeros(5 * oc[-1])
    for e in range(len(fo)):
        A = [op(co[e][d], fo[e][d]) for d in range(3)]
        blk = u[5 * of[e]:5 * of[e + 1]].reshape(5, fo[e][2] + 1, fo[e][1] + 1, fo[e][0] + 1)
        r = np.einsum("ck,bj,ai,vkji->vcba", A[2], A[1], A[0], blk)
        out[5 * oc[e]:5 * oc[e + 1]] = r.reshape(-1)
    return out


def _case(seed, isolated):
    rng = np.random.default_rng(seed)
    mesh = wl.box_mesh((2, 2, 2), bc=(0, 0, 1, 1, 0, 0))
    fo = wl.random_orders(8, 2, 7, rng)
    co = np.minimum(fo, rng.integers(1, 7, fo.shape)).astype(np.int32)
    u = wl.random_state(fo, rng)
    dudt = rng.normal(size=u.shape)  # any field: the estimate is linear in it
    return mesh, fo, co, u, dudt


@pytest.mark.parametrize("isolated", [True, False])
@pytest.mark.parametrize("restriction,op", [(oracle.L2, _op_l2), (oracle.SAMPLE, _op_sample)])
def test_estimate_with_independent_restriction(isolated, restriction, op):
    mesh, fo, co, u, dudt = _case(3 + isolated, isolated)
    tn, tt, norms, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=isolated, restriction=restriction)
    uc, rc = _apply(fo, co, u, op), _apply(fo, co, dudt, op)
    exp = oracle.residual(mesh, co, uc, isolated=isolated) - rc
    s = np.max(np.abs(exp))
    assert np.max(np.abs(tn - exp)) < 1e-11 * s
    # traditional form: J w_i w_j w_k (coarse weights) times the new form; J = h^3 / 8
    nc = np.prod(co + 1, axis=1)
    oc = np.concatenate([[0], np.cumsum(nc)])
    J = 0.5 ** 3 / 8.0
    for e in range(8):
        W = np.einsum("k,j,i->kji", *(_lgl_weights(co[e][d]) for d in (2, 1, 0))).reshape(-1)
        blk = slice(5 * oc[e], 5 * oc[e + 1])
        assert np.allclose(tt[blk], J * np.tile(W, 5) * tn[blk], rtol=0, atol=1e-13 * s)
        assert abs(norms[e, 0] - np.max(np.abs(tn[blk]))) == 0.0


def test_l2_and_sampling_differ_below_and_agree_at_the_fine_orders():
    mesh, fo, co, u, dudt = _case(5, True)
    a = oracle.tau(mesh, fo, co, u, dudt, isolated=True, restriction=oracle.L2)[0]
    b = oracle.tau(mesh, fo, co, u, dudt, isolated=True, restriction=oracle.SAMPLE)[0]
    assert np.max(np.abs(a - b)) > 1e-3 * np.max(np.abs(b))
    a = oracle.tau(mesh, fo, fo, u, dudt, isolated=False, restriction=oracle.L2)[0]
    b = oracle.tau(mesh, fo, fo, u, dudt, isolated=False, restriction=oracle.SAMPLE)[0]
    assert np.array_equal(a, b)


def test_l2_restriction_is_the_best_approximation():
    """||g - P g||_L2 <= ||g - I g||_L2 on every element (Gauss quadrature), the L2
    projection P being the best approximation in the coarse space."""
    rng = np.random.default_rng(9)
    fo = wl.random_orders(6, 3, 8, rng)
    co = np.minimum(fo, rng.integers(1, 6, fo.shape)).astype(np.int32)
    g = rng.normal(size=5 * int(np.prod(fo + 1, axis=1).sum()))
    gP = oracle.project(fo, co, g)
    gI = oracle.restrict(fo, co, g)
    x, w = np.polynomial.legendre.leggauss(12)
    nf, nc = np.prod(fo + 1, axis=1), np.prod(co + 1, axis=1)
    of, oc = np.concatenate([[0], np.cumsum(nf)]), np.concatenate([[0], np.cumsum(nc)])
    for e in range(6):
        Bf = [_lagrange(_lgl(fo[e][d]), x) for d in range(3)]
        Bc = [_lagrange(_lgl(co[e][d]), x) for d in range(3)]
        W = np.einsum("k,j,i->kji", w, w, w)

        def at(v, B, o, off):
            blk = v[5 * off[e]:5 * off[e + 1]].reshape(5, o[e][2] + 1, o[e][1] + 1, o[e][0] + 1)
            return np.einsum("zk,yj,xi,vkji->vzyx", B[2], B[1], B[0], blk)

        G = at(g, Bf, fo, of)
        eP = np.sum(W * (G - at(gP, Bc, co, oc)) ** 2)
        eI = np.sum(W * (G - at(gI, Bc, co, oc)) ** 2)
        assert eP <= eI * (1 + 1e-12)


def test_sweep_with_l2_matches_the_estimate_per_combination():
    rng = np.random.default_rng(11)
    mesh = wl.box_mesh((2, 1, 1))
    fo = np.array([[4, 3, 5], [4, 3, 5]], dtype=np.int32)
    u = wl.random_state(fo, rng)
    dudt = rng.normal(size=u.shape)
    ten, tet, offs = oracle.sweep(mesh, fo, u, dudt, restriction=oracle.L2)
    k = 0
    for c3 in range(1, 5):
        for c2 in range(1, 3):
            for c1 in range(1, 4):
                co = np.tile(np.array([c1, c2, c3], dtype=np.int32), (2, 1))
                _, _, norms, _ = oracle.tau(mesh, fo, co, u, dudt, isolated=True, restriction=oracle.L2)
                for e in range(2):
                    assert abs(ten[offs[e] + k] - norms[e, 0]) <= 1e-13 * norms[e, 0]
                    assert abs(tet[offs[e] + k] - norms[e, 1]) <= 1e-13 * norms[e, 1]
                k += 1
