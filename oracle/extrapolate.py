"""tau-extrapolation of the isolated truncation-error map to degrees N_i >= P_i.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark are the only users.  The GPU library never loads it and shares no
code with it.  Plain Python loops.

What it follows (arXiv 2210.03523):
  * Section 1 and Section 2.3: the truncation error of smooth solutions decays
    exponentially with the degree, so the map computed below the reference degree P
    can be extended to N_i >= P_i ("tau-extrapolation"; the paper cites the method
    without stating it);
  * Section 2.4.2, last paragraph: approach 2 works on the extrapolated maps; where a
    direction is not in the asymptotic range the extrapolation is not possible and
    the combinations with N_i >= P_i get a high value (they never qualify).

Reading (the steps the paper leaves to the cited work):
  * the computed ("inner") map of an element of fine orders P holds the degrees
    N_i in 1..C_i, C_i = max(1, P_i - 1), in every direction;
  * a combination N of the extended map (N_i in 1..nmax) with N_i <= C_i everywhere
    keeps its computed value;
  * otherwise let D be the directions with N_i > C_i and N' the inner corner
    (N'_i = C_i for i in D, N'_j = N_j elsewhere).  Along each direction i in D the
    map line through N' is fitted over its last L = min(3, C_i) computed degrees by
    least squares, ln tau = alpha + beta_i n; the direction is in the asymptotic
    range when L >= 2, those values are positive and finite and beta_i < 0;
  * if every direction of D is in the asymptotic range the value is
    tau(N') * prod_{i in D} exp(beta_i (N_i - C_i)) (the decay continued from the last
    computed degree, direction by direction); otherwise +inf (the high value).

Layout of an extended map: element by element (natural order here), nmax^3 values,
N1 fastest, then N2, then N3 (N_i in 1..nmax).
"""
from __future__ import annotations

import math

import numpy as np

from .select import combo_offsets, combos


def _inner_index(C, N):
    return (N[0] - 1) + C[0] * ((N[1] - 1) + C[1] * (N[2] - 1))


def _slope(values):
    """Least-squares slope of ln(values) against n = 1, 2, ..., len(values), or None when
    fewer than two values or any of them is not positive and finite."""
    L = len(values)
    if L < 2 or any(not (v > 0.0 and math.isfinite(v)) for v in values):
        return None
    xs = list(range(L))
    ys = [math.log(v) for v in values]
    xm = sum(xs) / L
    ym = sum(ys) / L
    num = sum((x - xm) * (y - ym) for x, y in zip(xs, ys))
    den = sum((x - xm) ** 2 for x in xs)
    return num / den


def extrapolate_element(P, values, nmax: int) -> np.ndarray:
    """Extended map (nmax^3 values, N1 fastest) of one element of fine orders P from its
    computed values in the order of combos(P)."""
    C = [max(1, int(p) - 1) for p in P]
    vals = [float(v) for v in values]
    assert len(vals) == C[0] * C[1] * C[2] == len(combos(P))
    out = np.empty(nmax ** 3)
    for n3 in range(1, nmax + 1):
        for n2 in range(1, nmax + 1):
            for n1 in range(1, nmax + 1):
                N = (n1, n2, n3)
                k = (n1 - 1) + nmax * ((n2 - 1) + nmax * (n3 - 1))
                D = [d for d in range(3) if N[d] > C[d]]
                corner = tuple(C[d] if d in D else N[d] for d in range(3))
                base = vals[_inner_index(C, corner)]
                if not D:
                    out[k] = base
                    continue
                value = base
                for d in D:
                    L = min(3, C[d])
                    line = []
                    for n in range(C[d] - L + 1, C[d] + 1):
                        M = list(corner)
                        M[d] = n
                        line.append(vals[_inner_index(C, M)])
                    beta = _slope(line)
                    if beta is None or not beta < 0.0:
                        value = math.inf
                        break
                    value *= math.exp(beta * (N[d] - C[d]))
                out[k] = value
    return out


def extrapolate_map(orders, te_map, nmax: int) -> np.ndarray:
    """Extended maps of every element (natural order), shape [E, nmax^3]."""
    o = np.asarray(orders).reshape(-1, 3)
    offs = combo_offsets(o)
    m = np.asarray(te_map, dtype=np.float64)
    return np.stack([extrapolate_element(tuple(int(v) for v in o[e]), m[offs[e]:offs[e + 1]], nmax)
                     for e in range(len(o))])


def select_element_ext(stage_values, X: int, tau_max: float, nmin: int, nmax: int):
    """Degrees of one element from extended maps (X^3 values each, N1 fastest): among the
    combinations with nmin <= N_i <= nmax whose value is below tau_max in every map,
    the one of fewest degrees of freedom (ties: smaller value, then lexicographic N1
    first); none: (nmax, nmax, nmax)."""
    best_key, best = None, None
    for n3 in range(1, X + 1):
        for n2 in range(1, X + 1):
            for n1 in range(1, X + 1):
                N = (n1, n2, n3)
                if any(N[d] < nmin or N[d] > nmax for d in range(3)):
                    continue
                k = (n1 - 1) + X * ((n2 - 1) + X * (n3 - 1))
                vals = [float(v[k]) for v in stage_values]
                if not all(v < tau_max for v in vals):
                    continue
                key = ((n1 + 1) * (n2 + 1) * (n3 + 1), max(vals), n1, n2, n3)
                if best_key is None or key < best_key:
                    best_key, best = key, N
    return best if best is not None else (nmax, nmax, nmax)


def select_orders_ext(ext_maps, X: int, tau_max: float, nmin: int, nmax: int, approach: int = 2) -> np.ndarray:
    """Selected degrees [E][3] (natural order) from extended maps [E, X^3], one per stage;
    approaches 1 and 2 as for the inner maps."""
    maps = [np.asarray(m).reshape(-1, X ** 3) for m in ext_maps]
    E = maps[0].shape[0]
    out = np.zeros((E, 3), dtype=np.int32)
    for e in range(E):
        vals = [m[e] for m in maps]
        if approach == 2:
            out[e] = select_element_ext(vals, X, tau_max, nmin, nmax)
        elif approach == 1:
            per = [select_element_ext([v], X, tau_max, nmin, nmax) for v in vals]
            out[e] = [max(s[d] for s in per) for d in range(3)]
        else:
            raise ValueError("approach is 1 or 2")
    return out
