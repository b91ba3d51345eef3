"""Pins of the oracle's Euler fluxes (Roe advective flux, set-up at the start of Section 3; Rusanov option).

Checks use Roe's defining properties (the wave vectors sum to the jump, and
their eigenvalue-weighted sum to the flux jump), consistency, antisymmetry,
rotation invariance and pure upwinding in supersonic flow.
"""
import numpy as np
import pytest

import oracle

G = 1.4


def _state(rng, mach=0.5):
    rho = rng.uniform(0.5, 2.0)
    p = rng.uniform(0.5, 2.0)
    c = np.sqrt(G * p / rho)
    u = rng.normal(size=3)
    u *= mach * c / np.linalg.norm(u)
    E = p / (G - 1) + 0.5 * rho * u @ u
    return np.array([rho, *(rho * u), E])


def _unit(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def _phys(q, n):
    rho, m, E = q[0], q[1:4], q[4]
    u = m / rho
    p = (G - 1) * (E - 0.5 * rho * u @ u)
    un = u @ n
    return np.array([rho * un, *(m * un + p * n), (E + p) * un])


def test_physical_flux_matches_definition():
    rng = np.random.default_rng(0)
    for _ in range(20):
        q, n = _state(rng), _unit(rng)
        assert np.allclose(oracle.flux_n(q, n), _phys(q, n), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", [0, 1])
def test_consistency(kind):
    rng = np.random.default_rng(1)
    for _ in range(20):
        q, n = _state(rng), _unit(rng)
        assert np.allclose(oracle.numflux(q, q, n, G, kind), _phys(q, n), rtol=1e-13, atol=1e-13)


def test_roe_waves_sum_to_jumps():
    rng = np.random.default_rng(2)
    for _ in range(50):
        qL, qR, n = _state(rng), _state(rng), _unit(rng)
        lam, wave = oracle.roe_waves(qL, qR, n, G)
        # property U of Roe's linearisation: dQ = sum_k alpha_k r_k, df = sum_k lam_k alpha_k r_k
        assert np.allclose(wave.sum(axis=0), qR - qL, rtol=1e-12, atol=1e-12)
        assert np.allclose(lam @ wave, _phys(qR, n) - _phys(qL, n), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("kind", [0, 1])
def test_antisymmetry_and_rotation(kind):
    rng = np.random.default_rng(3)
    for _ in range(20):
        qL, qR, n = _state(rng), _state(rng), _unit(rng)
        f = oracle.numflux(qL, qR, n, G, kind)
        g = oracle.numflux(qR, qL, -n, G, kind)
        assert np.allclose(f, -g, rtol=1e-12, atol=1e-12)
        # rotate momentum and normal by a random orthogonal matrix
        Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        rot = lambda q: np.array([q[0], *(Rm @ q[1:4]), q[4]])
        fr = oracle.numflux(rot(qL), rot(qR), Rm @ n, G, kind)
        assert np.allclose(fr, rot(f), rtol=1e-12, atol=1e-12)


def test_roe_supersonic_is_pure_upwind():
    rng = np.random.default_rng(4)
    n = np.array([1.0, 0.0, 0.0])
    for _ in range(10):
        qL, qR = _state(rng), _state(rng)
        for q in (qL, qR):  # make both states supersonic along +n
            rho, p = q[0], (G - 1) * (q[4] - 0.5 * (q[1:4] @ q[1:4]) / q[0])
            c = np.sqrt(G * p / rho)
            u = np.array([3.0 * c, 0.1, -0.2])
            q[1:4] = rho * u
            q[4] = p / (G - 1) + 0.5 * rho * u @ u
        lam, _ = oracle.roe_waves(qL, qR, n, G)
        if np.all(lam > 0):
            assert np.allclose(oracle.numflux(qL, qR, n, G, 0), _phys(qL, n), rtol=1e-12, atol=1e-12)


def test_lf_closed_form():
    qL = np.array([1.0, 0.2, 0.0, 0.0, 2.52])
    qR = np.array([0.8, 0.0, 0.1, 0.0, 2.0])
    n = np.array([1.0, 0.0, 0.0])
    fL, fR = _phys(qL, n), _phys(qR, n)

    def sp(q):
        rho = q[0]
        p = (G - 1) * (q[4] - 0.5 * (q[1:4] @ q[1:4]) / rho)
        return abs(q[1] / rho) + np.sqrt(G * p / rho)

    s = max(sp(qL), sp(qR))
    ref = 0.5 * (fL + fR) - 0.5 * s * (qR - qL)
    assert np.allclose(oracle.numflux(qL, qR, n, G, 1), ref, rtol=1e-14, atol=1e-14)
