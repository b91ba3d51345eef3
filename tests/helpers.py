"""Small helpers for ragged arrays and error measures used by the tests."""
import numpy as np

import workloads as wl


def elem_view(a, orders, e, nv=5):
    """[nv, n_e] view of element e in a natural ragged array."""
    offs = wl.node_offsets(orders)
    c = int(offs[e + 1] - offs[e])
    return a[nv * int(offs[e]): nv * int(offs[e]) + nv * c].reshape(nv, c)


def split(a, orders, nv=5):
    return [elem_view(a, orders, e, nv) for e in range(len(wl.node_counts(orders)))]


def per_var(a, orders):
    """Stack every element's [5, n_e] block into [5, total_nodes]."""
    return np.concatenate(split(a, orders), axis=1)


def scaled_err(x, ref, scale):
    """max |x - ref| / max(max |ref|, scale)."""
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), scale))


def residual_scale(mesh, orders, u, D_norm=None):
    """Scale of the cancelling terms of the residual: max |f| * max_d |Ja^d| * max ||D|| / J."""
    n = np.asarray(mesh["n"], dtype=float)
    h = (np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / n
    J = h[0] * h[1] * h[2] / 8.0
    Ja = np.array([h[1] * h[2], h[0] * h[2], h[0] * h[1]]) / 4.0
    q = per_var(u, orders)
    g = mesh["gamma"]
    rho = q[0]
    vel = q[1:4] / rho
    p = (g - 1) * (q[4] - 0.5 * rho * np.sum(vel * vel, axis=0))
    fmax = float(np.max(np.abs(q[4] + p) * np.max(np.abs(vel), axis=0) + np.abs(p)
                        + np.max(np.abs(q[1:4]), axis=0) * np.max(np.abs(vel), axis=0)))
    Nmax = int(np.max(orders))
    Dn = D_norm if D_norm is not None else Nmax * (Nmax + 1) / 4.0 * 2
    return fmax * float(np.max(Ja)) * Dn / J


def de_bruijn_pairs(k: int):
    """Cyclic sequence over 1..k in which every ordered pair (a, b) appears once as
    consecutive entries (de Bruijn sequence of order 2)."""
    seq, a = [], [0] * 2 * k

    def db(t, p):
        if t > 2:
            if 2 % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, k):
                a[t] = j
                db(t + 1, t)
    db(1, 1)
    return [s + 1 for s in seq]


def mortar_chain(d: int, rng, kmax: int = 7):
    """Periodic chain of k^2 elements along direction d whose consecutive elements'
    orders in both tangential directions run through every ordered pair of 1..k (the
    second tangential direction shifted along the cycle); small orders along d."""
    seq = de_bruijn_pairs(kmax)
    L = len(seq)
    shape = [1, 1, 1]
    shape[d] = L
    t1, t2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
    orders = np.zeros((L, 3), dtype=np.int32)
    orders[:, d] = rng.integers(1, 3, L)
    orders[:, t1] = seq
    orders[:, t2] = np.roll(seq, 7)
    return wl.box_mesh(tuple(shape), hi=(1.0, 0.7, 1.3)), orders


def tau_scale(mesh, fine_orders, coarse_orders, u, isolated=False, restriction=0):
    """Denominators of the tau tolerances: max |r^Nc(Q^c)| of the coarse residual of the
    restricted state (new form) and of its traditional form, from the oracle's estimate
    with a zero fine time derivative (tau = r^Nc(I u) - I dudt).  The estimate is the
    difference of two terms of this size, so its rounding is measured against it."""
    import oracle
    z = np.zeros_like(u)
    tn, tt, _, _ = oracle.tau(mesh, fine_orders, coarse_orders, u, z, isolated=isolated,
                              restriction=restriction)
    return float(np.max(np.abs(tn))), float(np.max(np.abs(tt)))


def sweep_scale(mesh, orders, u, elems=None, restriction=0, ns=None):
    """As tau_scale for the isolated sweep: the largest entry of the maps of the coarse
    isolated residuals alone (zero fine time derivative), both forms.  ns = (mu, Pr)
    for Navier-Stokes meshes."""
    import oracle
    z = np.zeros_like(u)
    if ns is None:
        ten, tet, _ = oracle.sweep(mesh, orders, u, z, elems=elems, restriction=restriction)
    else:
        ten, tet, _ = oracle.sweep_ns(mesh, orders, u, z, ns[0], ns[1], elems=elems, restriction=restriction)
    return float(np.max(np.abs(ten))), float(np.max(np.abs(tet)))
