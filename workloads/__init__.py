"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the method's arithmetic: it builds mesh
descriptions, order maps and states, and evaluates initial conditions at
node coordinates that the caller supplies.  Every array it returns is in the
natural ragged layout (element ``e`` occupies ``5 * n_e`` values, ordered
``[var][node]``); coordinates come in as ``[e][3][node]`` ragged arrays.

Workload recipes (3D analogues of the paper's advected density pulse, Section
4.1, and its Roe/RK3 set-up; see the design doc for the full recipe):

* ``c1``: 4x4x4 periodic unit cube, N = 3, literal Gaussian pulse
  rho = 1 + 0.5 exp(-|x - 0.5|^2 / (2 * 0.1^2)), u = (1, 0, 0), p = 1.
* ``c2``: 16^3 periodic unit cube, fine N = 7, same pulse plus i.i.d.
  N(0, 1e-3^2) noise on rho at every node (seed 2); coarse map drawn
  ``rng.integers(1, 7, (4096, 3))`` from the same generator, after the noise.
* ``c5``: 64 independent periodic problems, n ~ U{8..20} elements per side,
  orders U{1..7}, pulse centre U([0,1]^3), width U[0.05, 0.2] (seed 5).
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4
PERIODIC, WALL, FARFIELD = 0, 1, 2
ROE, LF = 0, 1


def box_mesh(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(0,) * 6, flux=ROE,
             gamma=GAMMA, qfar=(1.0, 0.0, 0.0, 0.0, 2.5)):
    if np.isscalar(n):
        n = (int(n),) * 3
    return {"n": tuple(int(v) for v in n), "lo": tuple(float(v) for v in lo),
            "hi": tuple(float(v) for v in hi), "bc": tuple(int(v) for v in bc),
            "flux": int(flux), "gamma": float(gamma), "qfar": tuple(float(v) for v in qfar)}


def num_elems(mesh) -> int:
    n = mesh["n"]
    return int(n[0] * n[1] * n[2])


def node_counts(orders) -> np.ndarray:
    o = np.asarray(orders, dtype=np.int64).reshape(-1, 3)
    return np.prod(o + 1, axis=1)


def node_offsets(orders) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(node_counts(orders))]).astype(np.int64)


def uniform_orders(E: int, N) -> np.ndarray:
    if np.isscalar(N):
        N = (N, N, N)
    return np.tile(np.asarray(N, dtype=np.int32), (E, 1))


def random_orders(E: int, lo: int, hi: int, rng) -> np.ndarray:
    """Orders drawn i.i.d. uniform in {lo..hi} per element and direction."""
    return rng.integers(lo, hi + 1, (E, 3)).astype(np.int32)


def conserved(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _ragged_apply(xyz, orders, fn):
    """Evaluate fn(x, y, z) -> [5, npts] per element and scatter into the ragged layout."""
    offs = node_offsets(orders)
    out = np.zeros(5 * int(offs[-1]))
    # all elements at once: coordinates are [e][3][node]; gather x, y, z per node
    counts = node_counts(orders)
    # build index arrays for the [3][node] blocks
    starts = 3 * offs[:-1]
    x = np.empty(int(offs[-1]))
    y = np.empty_like(x)
    z = np.empty_like(x)
    pos = 0
    for e in range(len(counts)):
        c = int(counts[e])
        s = int(starts[e])
        x[pos:pos + c] = xyz[s:s + c]
        y[pos:pos + c] = xyz[s + c:s + 2 * c]
        z[pos:pos + c] = xyz[s + 2 * c:s + 3 * c]
        pos += c
    q = fn(x, y, z)  # [5, ntot]
    pos = 0
    for e in range(len(counts)):
        c = int(counts[e])
        s = 5 * int(offs[e])
        out[s:s + 5 * c] = q[:, pos:pos + c].reshape(-1)
        pos += c
    return out


def pulse_rho(x, y, z, centre=(0.5, 0.5, 0.5), sigma=0.1, amp=0.5, images=False, t=0.0,
              speed=(1.0, 0.0, 0.0)):
    """Gaussian density pulse; ``images=True`` sums the 27 nearest periodic images."""
    cx, cy, cz = (centre[0] + speed[0] * t, centre[1] + speed[1] * t, centre[2] + speed[2] * t)
    shifts = (-1.0, 0.0, 1.0) if images else (0.0,)
    rho = np.ones_like(x)
    for kx in shifts:
        for ky in shifts:
            for kz in shifts:
                r2 = (x - cx - kx) ** 2 + (y - cy - ky) ** 2 + (z - cz - kz) ** 2
                rho = rho + amp * np.exp(-r2 / (2.0 * sigma * sigma))
    return rho


def pulse_state(xyz, orders, centre=(0.5, 0.5, 0.5), sigma=0.1, amp=0.5, images=False,
                gamma=GAMMA):
    """rho = 1 + amp * Gaussian, u = (1, 0, 0), p = 1."""
    def fn(x, y, z):
        rho = pulse_rho(x, y, z, centre, sigma, amp, images)
        one = np.ones_like(x)
        zero = np.zeros_like(x)
        return conserved(rho, one, zero, zero, one, gamma)
    return _ragged_apply(xyz, orders, fn)


def add_rho_noise(u, orders, rng, amp=1e-3):
    """i.i.d. N(0, amp^2) added to rho at every node (rho E unchanged)."""
    offs = node_offsets(orders)
    counts = node_counts(orders)
    out = u.copy()
    noise = rng.normal(0.0, amp, int(offs[-1]))
    pos = 0
    for e in range(len(counts)):
        c = int(counts[e])
        s = 5 * int(offs[e])
        out[s:s + c] += noise[pos:pos + c]
        pos += c
    return out


def random_state(orders, rng, rho=(0.8, 1.2), vel=0.3, p=(0.8, 1.2), gamma=GAMMA):
    """Nodewise i.i.d. admissible states (for parity and invariance tests)."""
    offs = node_offsets(orders)
    n = int(offs[-1])
    r = rng.uniform(rho[0], rho[1], n)
    uu = rng.uniform(-vel, vel, (3, n))
    pp = rng.uniform(p[0], p[1], n)
    q = conserved(r, uu[0], uu[1], uu[2], pp, gamma)
    out = np.zeros(5 * n)
    counts = node_counts(orders)
    pos = 0
    for e in range(len(counts)):
        c = int(counts[e])
        s = 5 * int(offs[e])
        out[s:s + 5 * c] = q[:, pos:pos + c].reshape(-1)
        pos += c
    return out


def uniform_state(orders, q):
    counts = node_counts(orders)
    offs = node_offsets(orders)
    out = np.zeros(5 * int(offs[-1]))
    for e in range(len(counts)):
        c = int(counts[e])
        s = 5 * int(offs[e])
        out[s:s + 5 * c] = np.repeat(np.asarray(q, dtype=np.float64), c)
    return out


# --------------------------------------------------------------------------- configs
def c1():
    mesh = box_mesh(4)
    return mesh, uniform_orders(64, 3)


def c2(seed: int = 2, n: int = 16, N: int = 7, coarse=(1, 6)):
    """Returns (mesh, fine_orders, coarse_orders, rng); the state is drawn by c2_state."""
    mesh = box_mesh(n)
    E = num_elems(mesh)
    return mesh, uniform_orders(E, N), coarse


def c2_state_and_coarse(xyz, mesh, fine_orders, seed: int = 2, coarse=(1, 6)):
    rng = np.random.default_rng(seed)
    u = pulse_state(xyz, fine_orders)
    u = add_rho_noise(u, fine_orders, rng, 1e-3)
    E = num_elems(mesh)
    co = rng.integers(coarse[0], coarse[1] + 1, (E, 3)).astype(np.int32)
    co = np.minimum(co, np.asarray(fine_orders).reshape(-1, 3))
    return u, co
