"""Polynomial-degree selection from truncation-error maps, and the degree-jump
conditions between neighbours.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark are the only users.  The GPU library never loads it and shares no
code with it.  Plain Python loops over elements and combinations.

What it follows (arXiv 2210.03523):
  * Section 2.4.2 (static p-adaptation), approaches 1 and 2 to processing the
    anisotropic truncation-error maps of several estimation stages, with the
    maximum aggregator F_max (the one the paper uses):
      approach 1: select degrees per stage, then N_i = max over stages of N_i^s;
      approach 2: total map ||tau||^e = max over stages of ||tau||^{e,s} for every
                  combination, then select from the total map.
    Selection: among the combinations whose map value is below tau_max, the one of
    fewest degrees of freedom prod_i (N_i + 1).
  * Section 2.4.2, last paragraph: where the map cannot be extended to N_i >= P_i
    (P the order the estimate was computed on), those combinations get a high
    value, i.e. they never qualify.  This module selects from the computed maps, so
    only the combinations of the sweep below P qualify; the extrapolated maps and the
    selection from them are in extrapolate.py.
  * Section 3.2 (dynamic adaptation of the cylinder case): a degree may fall by at most
    one per adaptation stage (applied before the jump conditions; both only raise).
  * Section 3.1, jump conditions (a) N_i^e >= max_j floor(2/3 N_i^j) and
    (b) N_i^e >= max_j (N_i^j - 1) over the face neighbours j of e, in the matching
    direction i; applied after the selection and iterated until no degree changes.

Readings where the paper is silent:
  * ties in the number of degrees of freedom: the smaller map value wins, then the
    smaller (N1, N2, N3) compared lexicographically, N1 first;
  * an element (or, in approach 1, a stage of it) with no qualifying combination
    gets the maximum degree N_max in every direction;
  * a combination qualifies only inside [N_min, N_max] in every direction;
  * the map values are maxima over nodes and variables (the infinity norm of the
    sweep); a NaN never qualifies.

Layout: orders are natural [E][3] integer arrays; a map is a 1-D array holding, for
every element in natural order, its combinations contiguously (c1 fastest, then c2,
then c3, c_d in 1..max(1, P_d - 1)), at the offsets ``combo_offsets(orders)``.
"""
from __future__ import annotations

import numpy as np


def combos(P):
    """Coarse combinations (N1, N2, N3) of an element of fine orders P, in the sweep's order."""
    C = [max(1, int(p) - 1) for p in P]
    return [(c1, c2, c3)
            for c3 in range(1, C[2] + 1)
            for c2 in range(1, C[1] + 1)
            for c1 in range(1, C[0] + 1)]


def combo_offsets(orders) -> np.ndarray:
    o = np.asarray(orders).reshape(-1, 3)
    counts = [len(combos(P)) for P in o]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def select_element(P, stage_values, tau_max: float, nmin: int, nmax: int):
    """Degrees of one element from the map values of its combinations.

    stage_values: one sequence per map, each with the element's values in the order of
    ``combos(P)``.  A combination qualifies when its value is below tau_max in every
    map given (so one map = one stage's selection; all maps = selection from their
    F_max total map)."""
    best_key, best = None, None
    for idx, N in enumerate(combos(P)):
        if any(N[d] < nmin or N[d] > nmax or N[d] >= P[d] for d in range(3)):
            continue  # outside the degree range, or N_i >= P_i (high value)
        vals = [float(v[idx]) for v in stage_values]
        if not all(v < tau_max for v in vals):
            continue
        ndof = (N[0] + 1) * (N[1] + 1) * (N[2] + 1)
        key = (ndof, max(vals), N[0], N[1], N[2])
        if best_key is None or key < best_key:
            best_key, best = key, N
    return best if best is not None else (nmax, nmax, nmax)


def select_orders(orders, maps, tau_max: float, nmin: int, nmax: int, approach: int = 2) -> np.ndarray:
    """Selected degrees [E][3] from one map per estimation stage (natural layout)."""
    o = np.asarray(orders).reshape(-1, 3)
    offs = combo_offsets(o)
    out = np.zeros_like(o, dtype=np.int32)
    for e in range(len(o)):
        P = tuple(int(v) for v in o[e])
        vals = [np.asarray(m)[offs[e]:offs[e + 1]] for m in maps]
        if approach == 2:
            out[e] = select_element(P, vals, tau_max, nmin, nmax)
        elif approach == 1:
            per_stage = [select_element(P, [v], tau_max, nmin, nmax) for v in vals]
            out[e] = [max(s[d] for s in per_stage) for d in range(3)]
        else:
            raise ValueError("approach is 1 or 2")
    return out


def limit_decrease(orders, prev, max_decrease: int, nmax: int) -> np.ndarray:
    """Per-stage decrease limit of dynamic adaptation (Section 3.2: degrees may fall by
    at most one per adaptation stage): N_i >= min(N_max, N_i^prev - max_decrease)."""
    o = np.array(orders, dtype=np.int32).reshape(-1, 3)
    pv = np.asarray(prev, dtype=np.int32).reshape(-1, 3)
    for e in range(len(o)):
        for i in range(3):
            o[e, i] = max(int(o[e, i]), min(nmax, int(pv[e, i]) - max_decrease))
    return o


def face_neighbours(mesh: dict):
    """Face neighbours of every element of the box mesh (natural index e = ix + nx(iy + ny iz)):
    across interior faces, and across the box faces whose boundary is periodic."""
    nx, ny, nz = mesh["n"]
    bc = mesh["bc"]
    n = (nx, ny, nz)
    nb = []
    for e in range(nx * ny * nz):
        idx = [e % nx, (e // nx) % ny, e // (nx * ny)]
        lst = []
        for d in range(3):
            for side in (-1, 1):
                j = list(idx)
                j[d] += side
                if j[d] < 0 or j[d] >= n[d]:
                    if bc[2 * d + (1 if side > 0 else 0)] != 0:
                        continue  # wall or far field: no neighbour
                    j[d] %= n[d]
                lst.append(j[0] + nx * (j[1] + ny * j[2]))
        nb.append(lst)
    return nb


def jump_bound(kind: int, n: int) -> int:
    """Lower bound a neighbour of degree n imposes: (a) floor(2/3 n), (b) n - 1."""
    if kind == 1:
        return (2 * n) // 3
    if kind == 2:
        return n - 1
    raise ValueError("jump condition is 1 (a) or 2 (b)")


def apply_jump(mesh: dict, orders, kind: int) -> np.ndarray:
    """Raise degrees until every element meets the jump condition against all of its
    face neighbours, direction by direction (iterated until nothing changes)."""
    cur = np.array(orders, dtype=np.int32).reshape(-1, 3)
    if kind == 0:
        return cur
    nb = face_neighbours(mesh)
    while True:
        nxt = cur.copy()
        for e in range(len(cur)):
            for j in nb[e]:
                for i in range(3):
                    nxt[e, i] = max(nxt[e, i], jump_bound(kind, int(cur[j, i])))
        if np.array_equal(nxt, cur):
            return cur
        cur = nxt
