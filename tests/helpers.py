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
