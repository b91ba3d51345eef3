"""Pins of the tau-extrapolation oracle (the computed map extended to N_i >= P_i by the
exponential decay of Sections 1 and 2.3, the high value of Section 2.4.2 where a
direction is not in the asymptotic range) and of the selection from extended maps:
closed forms on separable exponential maps, numpy's polyfit for the least-squares
slope, the high-value cases, and the two-stage worked example of Section 2.4.2."""
import json
import math
import os

import numpy as np
import pytest

from oracle import extrapolate as ex
from oracle import select as sel

GOLD = os.path.join(os.path.dirname(__file__), "golden", "select_two_stage_table.json")


def _grid(X):
    """(N1, N2, N3) of the extended layout, N1 fastest."""
    n = np.arange(1, X + 1)
    n3, n2, n1 = np.meshgrid(n, n, n, indexing="ij")
    return n1.reshape(-1), n2.reshape(-1), n3.reshape(-1)


def _separable(P, A, beta):
    return np.array([A * math.exp(-sum(b * n for b, n in zip(beta, N))) for N in sel.combos(P)])


@pytest.mark.parametrize("P,beta", [((5, 4, 7), (1.3, 0.7, 2.1)), ((9, 3, 4), (0.4, 2.5, 1.0))])
def test_separable_exponential_map_is_continued_exactly(P, beta):
    A, X = 3.0, 9
    ext = ex.extrapolate_element(P, _separable(P, A, beta), X)
    n1, n2, n3 = _grid(X)
    exact = A * np.exp(-(beta[0] * n1 + beta[1] * n2 + beta[2] * n3))
    assert np.max(np.abs(ext / exact - 1.0)) < 1e-12


def test_inner_values_are_kept():
    rng = np.random.default_rng(1)
    P = (6, 3, 5)
    vals = rng.uniform(0.1, 2.0, len(sel.combos(P)))
    ext = ex.extrapolate_element(P, vals, 8)
    for idx, N in enumerate(sel.combos(P)):
        k = (N[0] - 1) + 8 * ((N[1] - 1) + 8 * (N[2] - 1))
        assert ext[k] == vals[idx]


def test_slope_is_the_least_squares_fit_of_the_last_three_degrees():
    rng = np.random.default_rng(2)
    P = (7, 2, 2)  # C = (6, 1, 1): one line along x
    vals = np.exp(-0.8 * np.arange(1, 7) + rng.normal(0, 0.2, 6))
    ext = ex.extrapolate_element(P, vals, 9)
    b = np.polyfit(np.arange(4, 7), np.log(vals[3:6]), 1)[0]
    assert b < 0
    for n in range(7, 10):
        assert abs(ext[n - 1] / (vals[5] * math.exp(b * (n - 6))) - 1.0) < 1e-12


def test_two_degrees_are_fitted_one_is_not():
    P = (3, 2, 1)  # C = (2, 1, 1)
    vals = np.array([0.5, 0.1])
    ext = ex.extrapolate_element(P, vals, 4)
    assert abs(ext[2] / (0.1 * 0.2) - 1.0) < 1e-12        # N = (3, 1, 1): ratio 0.2 continued
    assert abs(ext[3] / (0.1 * 0.04) - 1.0) < 1e-12       # N = (4, 1, 1)
    for n2 in range(2, 5):                                # C2 = 1: no fit along y
        assert ext[(n2 - 1) * 4] == math.inf


@pytest.mark.parametrize("line", [[0.3, 0.3, 0.3], [0.1, 0.2, 0.4], [0.4, 0.0, 0.1], [0.4, np.nan, 0.1]])
def test_directions_out_of_the_asymptotic_range_get_the_high_value(line):
    """Flat, growing, touching zero, or not finite (the slope of three points ignores the
    middle one, but a NaN or a zero there still leaves the asymptotic range)."""
    P = (4, 2, 2)  # C = (3, 1, 1)
    ext = ex.extrapolate_element(P, np.array(line, dtype=np.float64), 6)
    assert np.all(np.isinf(ext[3:6]))
    assert np.array_equal(ext[:3], np.array(line), equal_nan=True)


def test_mixed_directions_multiply_the_decays():
    P = (4, 4, 3)
    vals = _separable(P, 1.0, (1.0, 2.0, 0.5))
    ext = ex.extrapolate_element(P, vals, 5)
    k = lambda N: (N[0] - 1) + 5 * ((N[1] - 1) + 5 * (N[2] - 1))
    assert abs(ext[k((5, 5, 2))] / math.exp(-(5.0 + 10.0 + 1.0)) - 1.0) < 1e-12
    assert abs(ext[k((1, 4, 5))] / math.exp(-(1.0 + 8.0 + 2.5)) - 1.0) < 1e-12


def test_selection_from_extended_maps_reaches_beyond_the_reference_degree():
    """On a separable map the selection from the extended map equals the fewest-DOF
    combination of the closed form (numpy over the whole grid), and with a loose
    threshold it equals the selection from the computed map."""
    P, A, beta, X = (4, 5, 3), 1.0, (0.9, 1.4, 2.0), 8
    vals = _separable(P, A, beta)
    ext = ex.extrapolate_element(P, vals, X)
    n1, n2, n3 = _grid(X)
    exact = A * np.exp(-(beta[0] * n1 + beta[1] * n2 + beta[2] * n3))
    for tau_max in (1e-3, 1e-5, 1e-7):
        ndof = (n1 + 1) * (n2 + 1) * (n3 + 1)
        ok = exact < tau_max * (1 - 1e-9)
        keys = np.lexsort((n3, n2, n1, exact, ndof))
        keys = keys[ok[keys]]
        want = (n1[keys[0]], n2[keys[0]], n3[keys[0]])
        got = ex.select_orders_ext([ext], X, tau_max, 1, X)[0]
        assert tuple(got) == want
        assert any(got[d] >= P[d] for d in range(3))
    tau_max = 0.05
    got = ex.select_orders_ext([ext], X, tau_max, 1, X)[0]
    inner = sel.select_orders(np.array([P]), [vals], tau_max, 1, X)[0]
    assert tuple(got) == tuple(inner)


@pytest.mark.parametrize("approach", [1, 2])
def test_table_example_on_extended_maps(approach):
    """The two-stage example of Section 2.4.2 (N_max = 3) written into extended maps with
    N3 = 1 passing and N3 > 1 failing: approach 1 gives (3, 3), approach 2 (2, 2)."""
    with open(GOLD) as f:
        t = json.load(f)
    X = 3
    n1, n2, n3 = _grid(X)
    maps = []
    for st in ("stage1", "stage2"):
        okset = {tuple(c) for c in t["passing"][st]}
        maps.append(np.array([0.25 if (a, b) in okset and c == 1 else 4.0 for a, b, c in zip(n1, n2, n3)]))
    exp = t["approach%d" % approach]["degrees"]
    got = ex.select_orders_ext(maps, X, 1.0, t["nmin"], t["nmax"], approach=approach)[0]
    assert tuple(got) == tuple(exp) + (1,)


def test_extended_map_layout():
    rng = np.random.default_rng(3)
    orders = np.array([[3, 4, 2], [2, 2, 2], [5, 1, 3]], dtype=np.int32)
    offs = sel.combo_offsets(orders)
    m = rng.uniform(0.01, 1.0, int(offs[-1]))
    ext = ex.extrapolate_map(orders, m, 6)
    assert ext.shape == (3, 216)
    for e in range(3):
        assert np.array_equal(ext[e], ex.extrapolate_element(tuple(orders[e]), m[offs[e]:offs[e + 1]], 6))
