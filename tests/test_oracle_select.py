"""Pins of the degree-selection oracle: the two-stage worked example of Section 2.4.2
(tests/golden/select_two_stage_table.json), closed forms of the jump conditions of
Section 3.1 on chains, the graph-distance form of their least fixed point on box
meshes, and the rules for combinations that cannot qualify."""
import json
import os
from collections import deque

import numpy as np
import pytest

from oracle import select as sel
import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden", "select_two_stage_table.json")


def _table():
    with open(GOLD) as f:
        return json.load(f)


def _table_maps(t, tau_max=1.0):
    """The table's element embedded in 3-D: fine orders P = (4, 4, 2), so the sweep's
    combinations are (N1, N2) in 1..3 with N3 = 1; listed combinations get 0.25 tau_max,
    the others 4 tau_max."""
    P = (4, 4, 2)
    maps = []
    for st in ("stage1", "stage2"):
        ok = {tuple(c) for c in t["passing"][st]}
        maps.append(np.array([0.25 * tau_max if (N[0], N[1]) in ok else 4.0 * tau_max
                              for N in sel.combos(P)]))
    return np.array([P], dtype=np.int32), maps


def test_table_fixture_is_consistent():
    t = _table()
    for st in ("stage1", "stage2"):
        assert [(a + 1) * (b + 1) for a, b in t["passing"][st]] == t["ndof_row"][st]
    a1, a2 = t["approach1"], t["approach2"]
    assert (a1["degrees"][0] + 1) * (a1["degrees"][1] + 1) == a1["ndof"]
    assert (a2["degrees"][0] + 1) * (a2["degrees"][1] + 1) == a2["ndof"]


def test_table_per_stage_choice():
    t = _table()
    orders, maps = _table_maps(t)
    for st, m in zip(("stage1", "stage2"), maps):
        got = sel.select_orders(orders, [m], 1.0, t["nmin"], t["nmax"], approach=2)[0]
        assert tuple(got) == tuple(t["per_stage_choice"][st]) + (1,)


@pytest.mark.parametrize("approach", [1, 2])
def test_table_approaches(approach):
    t = _table()
    orders, maps = _table_maps(t)
    exp = t["approach%d" % approach]
    for ms in (maps, maps[::-1]):
        got = sel.select_orders(orders, ms, 1.0, t["nmin"], t["nmax"], approach=approach)[0]
        assert tuple(got) == tuple(exp["degrees"]) + (1,)
        assert (got[0] + 1) * (got[1] + 1) == exp["ndof"]


def test_no_qualifying_combination_gives_nmax():
    P = np.array([[5, 4, 3]], dtype=np.int32)
    m = np.full(len(sel.combos(P[0])), 10.0)
    assert tuple(sel.select_orders(P, [m], 1.0, 1, 7)[0]) == (7, 7, 7)
    # N_i >= P_i never qualifies: with P_3 = 1 the sweep's only c3 is 1 = P_3
    P1 = np.array([[4, 4, 1]], dtype=np.int32)
    m1 = np.zeros(len(sel.combos(P1[0])))
    assert tuple(sel.select_orders(P1, [m1], 1.0, 1, 6)[0]) == (6, 6, 6)
    # NaN never qualifies
    m2 = np.full(len(sel.combos(P[0])), np.nan)
    assert tuple(sel.select_orders(P, [m2], 1.0, 1, 7)[0]) == (7, 7, 7)


def test_degree_range():
    P = np.array([[6, 6, 6]], dtype=np.int32)
    m = np.zeros(len(sel.combos(P[0])))  # everything passes
    assert tuple(sel.select_orders(P, [m], 1.0, 1, 8)[0]) == (1, 1, 1)
    assert tuple(sel.select_orders(P, [m], 1.0, 3, 8)[0]) == (3, 3, 3)
    # threshold is strict
    m[:] = 1.0
    assert tuple(sel.select_orders(P, [m], 1.0, 1, 8)[0]) == (8, 8, 8)


def test_ties_prefer_smaller_value_then_lexicographic():
    P = np.array([[4, 4, 4]], dtype=np.int32)
    cs = sel.combos(P[0])
    m = np.full(len(cs), 5.0)
    # (1, 2, 1), (2, 1, 1), (1, 1, 2) all have 12 degrees of freedom
    for N, v in (((1, 2, 1), 0.5), ((2, 1, 1), 0.5), ((1, 1, 2), 0.7)):
        m[cs.index(N)] = v
    assert tuple(sel.select_orders(P, [m], 1.0, 1, 8)[0]) == (1, 2, 1)
    m[cs.index((2, 1, 1))] = 0.4
    assert tuple(sel.select_orders(P, [m], 1.0, 1, 8)[0]) == (2, 1, 1)


def _chain(n, periodic):
    bc = (0, 0) if periodic else (1, 1)
    return wl.box_mesh((n, 1, 1), bc=bc + (0, 0, 0, 0))


@pytest.mark.parametrize("periodic", [False, True])
def test_jump_chain_closed_forms(periodic):
    n = 11
    mesh = _chain(n, periodic)
    o = np.ones((n, 3), dtype=np.int32)
    o[0, 0] = 8
    o[5, 1] = 6
    dist = [min(k, n - k) if periodic else k for k in range(n)]
    # (b): N_k = max(1, 8 - dist)
    got = sel.apply_jump(mesh, o, 2)
    assert list(got[:, 0]) == [max(1, 8 - d) for d in dist]
    # (a): 8 -> 5 -> 3 -> 2 -> 1 along the chain
    seq = [8, 5, 3, 2, 1]
    got = sel.apply_jump(mesh, o, 1)
    assert list(got[:, 0]) == [seq[d] if d < len(seq) else 1 for d in dist]
    # directions are independent: direction 1 only feels element 5
    assert list(sel.apply_jump(mesh, o, 2)[:, 1]) == [max(1, 6 - abs(k - 5)) for k in range(n)]
    assert np.all(sel.apply_jump(mesh, o, 2)[:, 2] == 1)


def _distances(mesh):
    """All-pairs face-graph distances by breadth-first search from every element."""
    nx, ny, nz = mesh["n"]
    n = (nx, ny, nz)
    E = nx * ny * nz
    D = np.full((E, E), -1, dtype=np.int64)
    for s in range(E):
        D[s, s] = 0
        q = deque([s])
        while q:
            e = q.popleft()
            idx = (e % nx, (e // nx) % ny, e // (nx * ny))
            for d in range(3):
                for side in (-1, 1):
                    j = list(idx)
                    j[d] += side
                    if not 0 <= j[d] < n[d]:
                        if mesh["bc"][2 * d + (side > 0)] != 0:
                            continue
                        j[d] %= n[d]
                    f = j[0] + nx * (j[1] + ny * j[2])
                    if D[s, f] < 0:
                        D[s, f] = D[s, e] + 1
                        q.append(f)
    return D


@pytest.mark.parametrize("kind", [1, 2])
def test_jump_least_fixed_point_is_distance_decay(kind):
    """The least fixed point above N^0 is N_e = max_j f^{dist(e, j)}(N^0_j): f lowers a
    degree, so the strongest bound from j comes along a shortest path."""
    rng = np.random.default_rng(5)
    mesh = wl.box_mesh((5, 4, 3), bc=(0, 0, 1, 1, 2, 2))
    E = 60
    o = rng.integers(1, 9, (E, 3)).astype(np.int32)
    o[rng.random((E, 3)) < 0.7] = 1
    D = _distances(mesh)

    def f_pow(n, k):
        for _ in range(k):
            n = sel.jump_bound(kind, n)
        return n

    exp = np.zeros_like(o)
    for e in range(E):
        for i in range(3):
            exp[e, i] = max(f_pow(int(o[j, i]), int(D[e, j])) for j in range(E) if D[e, j] >= 0)
    got = sel.apply_jump(mesh, o, kind)
    assert np.array_equal(got, exp)
    assert np.array_equal(sel.apply_jump(mesh, got, kind), got)


def test_approach2_choice_qualifies_in_every_stage():
    rng = np.random.default_rng(9)
    o = rng.integers(1, 8, (40, 3)).astype(np.int32)
    offs = sel.combo_offsets(o)
    maps = [rng.random(int(offs[-1])) for _ in range(3)]
    got = sel.select_orders(o, maps, 0.6, 1, 7, approach=2)
    for e in range(len(o)):
        N = tuple(int(v) for v in got[e])
        cs = sel.combos(o[e])
        if N == (7, 7, 7) and N not in cs:
            # fallback: then no combination below P qualifies in all stages
            assert not any(all(m[offs[e] + k] < 0.6 for m in maps) and all(c[d] < o[e, d] for d in range(3))
                           for k, c in enumerate(cs))
            continue
        k = cs.index(N)
        assert all(m[offs[e] + k] < 0.6 for m in maps)
