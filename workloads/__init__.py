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


SINE_MAP = 1


def sine_mapped(mesh, amp: float = 0.05, geo_order=(2, 2, 1)):
    """The box mesh with its points moved by (x, y, z) -> (x + f, y + f, z),
    f = amp sin(2 pi x') sin(2 pi y') (x', y' the box coordinates scaled to [0, 1]),
    each element's geometry the Gauss-Lobatto interpolant of order geo_order."""
    m = dict(mesh)
    m["map"] = (SINE_MAP, float(amp), tuple(int(g) for g in geo_order))
    return m


def column_orders(mesh, lo: int, hi: int, rng, nz_order: int = 1) -> np.ndarray:
    """Orders (Nx, Ny) drawn i.i.d. uniform in {lo..hi} per element column (ix, iy)
    and shared by every layer of the column; Nz = nz_order."""
    nx, ny, nz = mesh["n"]
    col = rng.integers(lo, hi + 1, (nx * ny, 2))
    orders = np.full((nx * ny * nz, 3), nz_order, dtype=np.int32)
    orders[:, :2] = np.tile(col, (nz, 1))
    return orders


def element_orders(mesh, lo: int, hi: int, rng, nz_range=(1, 1)) -> np.ndarray:
    """Orders (Nx, Ny) drawn i.i.d. uniform in {lo..hi} per element, then Nz uniform in
    nz_range per element (a fixed Nz = 1 draws nothing more)."""
    E = num_elems(mesh)
    orders = np.full((E, 3), nz_range[0], dtype=np.int32)
    orders[:, :2] = rng.integers(lo, hi + 1, (E, 2))
    if nz_range[1] > nz_range[0]:
        orders[:, 2] = rng.integers(nz_range[0], nz_range[1] + 1, E)
    return orders


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


def _node_index(orders):
    """Per-node element index and local node index of the natural ragged layout."""
    counts = node_counts(orders)
    offs = node_offsets(orders)
    elem = np.repeat(np.arange(len(counts)), counts)
    local = np.arange(int(offs[-1])) - offs[:-1][elem]
    return counts, offs, elem, local


def _scatter(q, orders):
    """[nv, total_nodes] per-node values -> natural ragged array (nv values per node)."""
    nv = q.shape[0]
    counts, offs, elem, local = _node_index(orders)
    out = np.zeros(nv * int(offs[-1]))
    base = nv * offs[:-1][elem] + local
    for v in range(nv):
        out[base + v * counts[elem]] = q[v]
    return out


def _gather_xyz(xyz, orders):
    counts, offs, elem, local = _node_index(orders)
    ix = 3 * offs[:-1][elem] + local
    c = counts[elem]
    return xyz[ix], xyz[ix + c], xyz[ix + 2 * c]


def _ragged_apply(xyz, orders, fn):
    """Evaluate fn(x, y, z) -> [5, npts] at every node and scatter into the ragged layout."""
    x, y, z = _gather_xyz(np.asarray(xyz), orders)
    return _scatter(fn(x, y, z), orders)


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
    counts, offs, elem, local = _node_index(orders)
    out = u.copy()
    out[5 * offs[:-1][elem] + local] += rng.normal(0.0, amp, int(offs[-1]))
    return out


def random_state(orders, rng, rho=(0.8, 1.2), vel=0.3, p=(0.8, 1.2), gamma=GAMMA):
    """Nodewise i.i.d. admissible states (for parity and invariance tests)."""
    n = int(node_offsets(orders)[-1])
    r = rng.uniform(rho[0], rho[1], n)
    uu = rng.uniform(-vel, vel, (3, n))
    pp = rng.uniform(p[0], p[1], n)
    return _scatter(conserved(r, uu[0], uu[1], uu[2], pp, gamma), orders)


def uniform_state(orders, q):
    n = int(node_offsets(orders)[-1])
    return _scatter(np.repeat(np.asarray(q, dtype=np.float64)[:, None], n, axis=1), orders)


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


def c5(seed: int = 5, nprob: int = 64, nrange=(8, 20), orange=(1, 7)):
    """64 independent periodic unit-cube problems: per problem n ~ U{8..20} elements
    per side, orders U{1..7}, pulse centre U([0,1]^3), width U[0.05, 0.2].
    Returns a list of (mesh, orders, centre, sigma)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nrange[0], nrange[1] + 1, nprob)
    out = []
    for n in ns:
        orders = random_orders(int(n) ** 3, orange[0], orange[1], rng)
        centre = rng.random(3)
        sigma = float(rng.uniform(0.05, 0.2))
        out.append((box_mesh(int(n)), orders, tuple(centre), sigma))
    return out


def c4(n: int = 24, N: int = 5):
    """Slip wall on x = 0, far field (free stream) on x = 1, periodic in y and z."""
    q_inf = conserved(np.array(1.0), np.array(0.3), np.array(0.4), np.array(0.5), np.array(1.0))
    mesh = box_mesh(n, bc=(WALL, FARFIELD, PERIODIC, PERIODIC, PERIODIC, PERIODIC), qfar=tuple(q_inf))
    return mesh, uniform_orders(n ** 3, N)


def c4_state(xyz, orders, seed: int = 4, nmodes: int = 8):
    """rho = 1 + 0.1 * pulse (width 0.1), u = (0.3, 0.4, 0.5) + 1e-2 * (nmodes seeded smooth
    Fourier modes per component), p = 1."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 4, (nmodes, 3))
    ph = rng.random((nmodes, 3)) * 2 * np.pi
    amp = rng.normal(size=(nmodes, 3))

    def fn(x, y, z):
        rho = pulse_rho(x, y, z, amp=0.1, sigma=0.1)
        vel = [np.full_like(x, c) for c in (0.3, 0.4, 0.5)]
        for m in range(nmodes):
            arg = 2 * np.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z)
            for c in range(3):
                vel[c] = vel[c] + 1e-2 * amp[m, c] * np.sin(arg + ph[m, c])
        return conserved(rho, vel[0], vel[1], vel[2], np.ones_like(x))
    return _ragged_apply(xyz, orders, fn)


def ns_mesh(mesh, mu: float, Pr: float = 0.72):
    """A copy of a box mesh description carrying Navier-Stokes parameters."""
    out = dict(mesh)
    out["mu"] = float(mu)
    out["Pr"] = float(Pr)
    return out


def c3(seed: int = 3, n=(32, 32, 2), Re: float = 100.0, Ma: float = 0.2, Pr: float = 0.72,
       curved: bool = True):
    """Navier-Stokes, Re = 100, Ma = 0.2, Pr = 0.72 on [0,1]^2 x [0, 1/16] (32 x 32 x 2 cubes)
    under the sine map of amplitude 0.05 (geometry order (2, 2, 1)), periodic; orders
    (Nx, Ny) drawn U{2..6} per element (the faces between the two layers are
    non-conforming where the layers' orders differ), Nz = 1.  Nondimensional with
    rho = 1, |u| = 1, L = 1: mu = 1/Re, p = 1/(gamma Ma^2).  Returns (mesh, orders, rng)."""
    rng = np.random.default_rng(seed)
    mesh = ns_mesh(box_mesh(n, hi=(1.0, 1.0, n[2] / n[0])), mu=1.0 / Re, Pr=Pr)
    if curved:
        mesh = sine_mapped(mesh)
    orders = element_orders(mesh, 2, 6, rng)
    mesh["p_inf"] = 1.0 / (GAMMA * Ma * Ma)
    return mesh, orders, rng


def c3_state(xyz, orders, mesh, rng, nvort: int = 16, r0: float = 0.05, amp: float = 0.1):
    """Free stream rho = 1, u = (1, 0, 0), p = p_inf plus nvort Gaussian vortices in x-y
    (centres U([0,1]^2), swirl amp * (r/r0) exp((1 - r^2/r0^2)/2), minimum-image distance)."""
    centres = rng.random((nvort, 2))
    p_inf = mesh["p_inf"]

    def fn(x, y, z):
        u = np.ones_like(x)
        v = np.zeros_like(x)
        for cx, cy in centres:
            dx = (x - cx + 0.5) % 1.0 - 0.5
            dy = (y - cy + 0.5) % 1.0 - 0.5
            r2 = dx * dx + dy * dy
            s = amp / r0 * np.exp(0.5 * (1.0 - r2 / (r0 * r0)))
            u = u - s * dy
            v = v + s * dx
        one = np.ones_like(x)
        return conserved(one, u, v, 0.0 * x, p_inf * one)
    return _ragged_apply(xyz, orders, fn)
