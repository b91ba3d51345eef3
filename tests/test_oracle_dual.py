"""Pins of the dual time-stepping estimate (Section 2.3, item 2) in the oracle: the
backward-difference weights are exact on polynomials in time of their order (and not
beyond), and on a stored history that satisfies the backward-difference scheme with the
fine residual, the estimate equals the variational estimate (pinned by its own tests)."""
import numpy as np
import pytest

import oracle
import workloads as wl


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_bdf_weights_exact_on_polynomials(k):
    w = oracle.bdf_weights(k)
    s = -np.arange(k + 1, dtype=np.float64)  # abscissae of Q(t_{n+1-j}) in steps
    for m in range(k + 1):
        exact = 1.0 if m == 1 else 0.0  # d/ds s^m at s = 0
        assert abs(np.sum(w * s ** m) - exact) < 1e-12
    assert abs(np.sum(w * s ** (k + 1))) > 1e-3  # order exactly k


@pytest.mark.parametrize("k,isolated", [(1, False), (2, True), (3, False)])
def test_dual_equals_variational_on_a_consistent_history(k, isolated):
    rng = np.random.default_rng(10 + k)
    mesh = wl.box_mesh((3, 2, 2), bc=(0, 0, 1, 1, 0, 0))
    fo = wl.random_orders(12, 2, 6, rng)
    co = np.minimum(fo, rng.integers(1, 6, fo.shape)).astype(np.int32)
    q0 = wl.random_state(fo, rng)
    r0 = oracle.residual(mesh, fo, q0)  # = -dQ/dt of the fine semi-discretisation
    dt = 1e-3
    w = oracle.bdf_weights(k)
    # history Q(t_{n+1-j}): free for j = 1..k-1, the last one closes sum_j w_j Q_j = -dt r0
    hist = [q0] + [q0 + 1e-3 * rng.normal(size=q0.shape) for _ in range(k - 1)]
    rest = -dt * r0 - sum(w[j] * hist[j] for j in range(k))
    hist.append(rest / w[k])
    tn, tt = oracle.tau_dual(mesh, fo, co, hist, dt, isolated=isolated)
    vn, vt, _, _ = oracle.tau(mesh, fo, co, q0, r0, isolated=isolated)
    s = np.max(np.abs(oracle.residual(mesh, co, oracle.restrict(fo, co, q0), isolated=True)))
    assert np.max(np.abs(tn - vn)) < 1e-10 * s
    assert np.max(np.abs(tt - vt)) < 1e-10 * s
