"""Pins of the oracle's 1D nodal tables (DGSEM basis on Gauss-Lobatto nodes, Section 2.1).

Each table is checked against something other than the oracle itself: closed
forms of the low-order Gauss-Lobatto rules, exactness of quadrature and
differentiation on monomials, the summation-by-parts identity, and numpy's
Gauss-Legendre rule for the L2 projection.
"""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle


def test_lgl_closed_forms():
    # Gauss-Lobatto rules with 2, 3 and 4 points (closed forms)
    x, w = oracle.lgl(1)
    assert np.array_equal(x, [-1.0, 1.0]) and np.allclose(w, [1.0, 1.0], atol=1e-15)
    x, w = oracle.lgl(2)
    assert np.array_equal(x, [-1.0, 0.0, 1.0])
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = oracle.lgl(3)
    s = 1.0 / np.sqrt(5.0)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = oracle.lgl(4)
    t = np.sqrt(3.0 / 7.0)
    assert np.allclose(x, [-1, -t, 0, t, 1], atol=1e-15)
    assert np.allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1], atol=1e-15)


@pytest.mark.parametrize("N", range(1, oracle.NMAX + 1))
def test_lgl_quadrature_exactness_and_symmetry(N):
    x, w = oracle.lgl(N)
    assert np.all(np.diff(x) > 0)
    assert np.array_equal(x, -x[::-1])
    assert np.array_equal(w, w[::-1])
    # interior nodes are the roots of L_N' (independent: numpy's Legendre series)
    dL = npleg.legder(np.eye(N + 1)[N])
    if N > 1:
        assert np.max(np.abs(npleg.legval(x[1:-1], dL))) < 1e-11 * N * N
    # N+1 point Gauss-Lobatto integrates degree 2N-1 exactly
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("N", range(1, oracle.NMAX + 1))
def test_dmat_exact_and_sbp(N):
    x, w = oracle.lgl(N)
    D = oracle.dmat(N)
    for k in range(N + 1):
        ref = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(D @ x ** k - ref)) < 1e-12 * max(1, k) * N * N
    # summation by parts: W D + D^T W = diag(-1, 0, ..., 0, 1)
    W = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(W @ D + D.T @ W - B)) < 1e-13 * N * N


@pytest.mark.parametrize("M,N", [(1, 3), (2, 7), (5, 7), (3, 3), (6, 9), (7, 2), (12, 5)])
def test_interp_exact_on_order_N_polynomials(M, N):
    xf, _ = oracle.lgl(N)
    xc, _ = oracle.lgl(M)
    I = oracle.interp(M, N)
    rng = np.random.default_rng(11)
    c = rng.normal(size=N + 1)
    p = np.polyval(c, xf)
    assert np.max(np.abs(I @ p - np.polyval(c, xc))) < 1e-13
    # coinciding nodes give exact unit rows
    for a in range(M + 1):
        hits = np.where(xf == xc[a])[0]
        if len(hits):
            row = np.zeros(N + 1)
            row[hits[0]] = 1.0
            assert np.array_equal(I[a], row)


@pytest.mark.parametrize("N,K", [(1, 2), (2, 5), (3, 3), (4, 7), (6, 9), (1, 9)])
def test_projection_is_l2_projection(N, K):
    P = oracle.proj(N, K)
    S = oracle.interp(K, N)
    assert np.max(np.abs(P @ S - np.eye(N + 1))) < 1e-13
    # orthogonality of the residual g - P g to every degree-N polynomial, checked
    # with numpy's Gauss-Legendre rule (exact for the degrees involved)
    xK, _ = oracle.lgl(K)
    xN, _ = oracle.lgl(N)
    rng = np.random.default_rng(3)
    c = rng.normal(size=K + 1)
    g = np.polyval(c, xK)
    Pg = P @ g
    gq, wq = npleg.leggauss(K + N + 2)
    g_at = np.polyval(c, gq)
    # order-N interpolant of Pg evaluated at the Gauss points
    VN = np.vander(xN, N + 1)
    cp = np.linalg.solve(VN, Pg)
    Pg_at = np.polyval(cp, gq)
    for k in range(N + 1):
        assert abs(np.dot(wq, (g_at - Pg_at) * gq ** k)) < 1e-12
