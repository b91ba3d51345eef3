"""Plain FP64 CPU oracle for the DGSEM residual and tau-estimation (arXiv 2210.03523).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The GPU library never loads it and
shares no code with it.

The numerical work is done in ``dg_oracle.c`` (plain loops, natural element
order); this module only marshals numpy arrays through ctypes.  Arrays are in
the natural ragged layout: element ``e`` occupies ``5 * n_e`` values starting
at ``5 * noff[e]``, ordered ``[var][node]`` with ``node = i + n1*(j + n2*k)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.environ.get("DG_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

NMAX = 12

# restriction operators of the tau-estimate (Section 2.3)
SAMPLE = 0  # sampling of the fine polynomial at the coarse nodes
L2 = 1      # exact L2 projection onto the coarse tensor-product space


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over elements)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC",
               "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 6), ("flux", ctypes.c_int),
                ("gamma", ctypes.c_double), ("qfar", ctypes.c_double * 5),
                ("map_kind", ctypes.c_int), ("map_amp", ctypes.c_double),
                ("geo_order", ctypes.c_int * 3)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        for name, args in {
            "orc_lgl": [ctypes.c_int, _D, _D],
            "orc_dmat": [ctypes.c_int, _D],
            "orc_interp": [ctypes.c_int, ctypes.c_int, _D],
            "orc_proj": [ctypes.c_int, ctypes.c_int, _D],
            "orc_node_coords": [ctypes.POINTER(_Mesh), _I, _D],
            "orc_metrics": [ctypes.POINTER(_Mesh), _I, _D],
            "orc_sweep_ns": [ctypes.POINTER(_Mesh), _I, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             _I, ctypes.c_int, _D, _D],
            "orc_residual": [ctypes.POINTER(_Mesh), _I, _D, _D, ctypes.c_int, ctypes.c_int],
            "orc_restrict": [ctypes.c_int, _I, _I, _D, _D],
            "orc_project": [ctypes.c_int, _I, _I, _D, _D],
            "orc_bdf_weights": [ctypes.c_int, _D],
            "orc_tau_dual": [ctypes.c_void_p, _I, _I, ctypes.POINTER(_D), ctypes.c_int, ctypes.c_double,
                             ctypes.c_int, _D, _D],
            "orc_tau": [ctypes.POINTER(_Mesh), _I, _I, _D, _D, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D],
            "orc_num_combos": [_I],
            "orc_sweep": [ctypes.POINTER(_Mesh), _I, _D, _D, ctypes.c_int, _I, ctypes.c_int, _D, _D],
            "orc_rk3": [ctypes.POINTER(_Mesh), _I, _D, ctypes.c_double, ctypes.c_int],
            "orc_tau_eta": [ctypes.POINTER(_Mesh), _I, _I, _D, _D, ctypes.c_int, ctypes.c_int, _D, ctypes.c_int,
                            _D],
            "orc_functional": [ctypes.POINTER(_Mesh), _I, _D, _D, _D],
            "orc_gradient": [ctypes.POINTER(_Mesh), _I, _D, ctypes.c_int, _D],
            "orc_residual_ns": [ctypes.POINTER(_Mesh), _I, _D, ctypes.c_double, ctypes.c_double, _D,
                                ctypes.c_int, ctypes.c_int],
            "orc_residual_cstep": [ctypes.POINTER(_Mesh), _I, _D, _D, ctypes.c_double, _D, _D, ctypes.c_int,
                                   ctypes.c_int],
            "orc_residual_jvp": [ctypes.POINTER(_Mesh), _I, _D, _D, _D, ctypes.c_int, ctypes.c_int],
            "orc_residual_vjp": [ctypes.POINTER(_Mesh), _I, _D, _D, _D, ctypes.c_int, ctypes.c_int],
        }.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name in ("orc_flux_n",):
            fn = getattr(lib, name)
            fn.argtypes = [_D, _D, ctypes.c_double, _D]
            fn.restype = None
        lib.orc_numflux.argtypes = [_D, _D, _D, ctypes.c_double, ctypes.c_int, _D]
        lib.orc_numflux.restype = None
        lib.orc_roe_waves.argtypes = [_D, _D, _D, ctypes.c_double, _D, _D]
        lib.orc_roe_waves.restype = None
        lib.orc_viscous_flux.argtypes = [_D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        lib.orc_viscous_flux.restype = None
        lib.orc_flux_jacobian.argtypes = [_D, _D, ctypes.c_double, _D]
        lib.orc_flux_jacobian.restype = None
        lib.orc_numflux_jacobian.argtypes = [_D, _D, _D, ctypes.c_double, ctypes.c_int, _D, _D]
        lib.orc_numflux_jacobian.restype = None
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _mesh(m: dict) -> _Mesh:
    s = _Mesh()
    s.nx, s.ny, s.nz = (int(v) for v in m["n"])
    for d in range(3):
        s.lo[d] = float(m["lo"][d])
        s.hi[d] = float(m["hi"][d])
    for f in range(6):
        s.bc[f] = int(m["bc"][f])
    s.flux = int(m["flux"])
    s.gamma = float(m["gamma"])
    for v in range(5):
        s.qfar[v] = float(m["qfar"][v])
    kind, amp, geo = m.get("map", (0, 0.0, (1, 1, 1)))
    s.map_kind, s.map_amp = int(kind), float(amp)
    for d in range(3):
        s.geo_order[d] = int(geo[d])
    return s


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


# --------------------------------------------------------------------------- tables
def lgl(N: int):
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    _check(_load().orc_lgl(N, _d(x), _d(w)), "lgl")
    return x, w


def dmat(N: int):
    D = np.zeros((N + 1, N + 1))
    _check(_load().orc_dmat(N, _d(D)), "dmat")
    return D


def interp(M: int, N: int):
    out = np.zeros((M + 1, N + 1))
    _check(_load().orc_interp(M, N, _d(out)), "interp")
    return out


def proj(N: int, K: int):
    out = np.zeros((N + 1, K + 1))
    _check(_load().orc_proj(N, K, _d(out)), "proj")
    return out


# --------------------------------------------------------------------------- fluxes
def flux_n(q, n, gamma=1.4):
    q, n = _f64(q), _f64(n)
    f = np.zeros(5)
    _load().orc_flux_n(_d(q), _d(n), gamma, _d(f))
    return f


def numflux(qL, qR, n, gamma=1.4, kind=0):
    qL, qR, n = _f64(qL), _f64(qR), _f64(n)
    f = np.zeros(5)
    _load().orc_numflux(_d(qL), _d(qR), _d(n), gamma, int(kind), _d(f))
    return f


def roe_waves(qL, qR, n, gamma=1.4):
    qL, qR, n = _f64(qL), _f64(qR), _f64(n)
    lam = np.zeros(4)
    wave = np.zeros((4, 5))
    _load().orc_roe_waves(_d(qL), _d(qR), _d(n), gamma, _d(lam), _d(wave))
    return lam, wave


def flux_jacobian(q, n, gamma=1.4):
    """A[i, j] = d (f.n)_i / d q_j (closed form)."""
    q, n = _f64(q), _f64(n)
    A = np.zeros((5, 5))
    _load().orc_flux_jacobian(_d(q), _d(n), gamma, _d(A))
    return A


def numflux_jacobian(qL, qR, n, gamma=1.4, kind=0):
    """(AL, AR): Jacobians of the numerical flux in qL and qR (complex step)."""
    qL, qR, n = _f64(qL), _f64(qR), _f64(n)
    AL, AR = np.zeros((5, 5)), np.zeros((5, 5))
    _load().orc_numflux_jacobian(_d(qL), _d(qR), _d(n), gamma, int(kind), _d(AL), _d(AR))
    return AL, AR


# --------------------------------------------------------------------------- mesh-level
def num_nodes(orders) -> int:
    o = np.asarray(orders).reshape(-1, 3)
    return int(np.prod(o + 1, axis=1).sum())


def node_coords(mesh: dict, orders):
    o = _i32(orders)
    xyz = np.zeros(3 * num_nodes(o))
    m = _mesh(mesh)
    _check(_load().orc_node_coords(ctypes.byref(m), _i(o), _d(xyz)), "node_coords")
    return xyz


def metrics(mesh: dict, orders):
    """Metric terms per node, natural ragged layout [e][10][node]: Ja^1, Ja^2, Ja^3
    (x, y, z components each), then J."""
    o = _i32(orders)
    met = np.zeros(10 * num_nodes(o))
    m = _mesh(mesh)
    _check(_load().orc_metrics(ctypes.byref(m), _i(o), _d(met)), "metrics")
    return met


def residual(mesh: dict, orders, u, form: int = 0, isolated: bool = False):
    """form 0: new form r = M^-1 F^N(u) (= -du/dt); form 1: traditional F^N(u)."""
    o, u = _i32(orders), _f64(u)
    r = np.zeros_like(u)
    m = _mesh(mesh)
    _check(_load().orc_residual(ctypes.byref(m), _i(o), _d(u), _d(r), int(form), int(bool(isolated))),
           "residual")
    return r


def residual_cstep(mesh: dict, orders, u, d, h: float, form: int = 0, isolated: bool = False):
    """Real and imaginary parts of the residual evaluated in complex arithmetic at u + i h d
    (box Euler meshes)."""
    o, u, d = _i32(orders), _f64(u), _f64(d)
    re, im = np.zeros_like(u), np.zeros_like(u)
    m = _mesh(mesh)
    _check(_load().orc_residual_cstep(ctypes.byref(m), _i(o), _d(u), _d(d), float(h), _d(re), _d(im), int(form),
                                      int(bool(isolated))), "residual_cstep")
    return re, im


def residual_jvp(mesh: dict, orders, u, d, form: int = 0, isolated: bool = False):
    """(d r / d u) d by complex step (box Euler meshes)."""
    o, u, d = _i32(orders), _f64(u), _f64(d)
    out = np.zeros_like(u)
    m = _mesh(mesh)
    _check(_load().orc_residual_jvp(ctypes.byref(m), _i(o), _d(u), _d(d), _d(out), int(form), int(bool(isolated))),
           "residual_jvp")
    return out


def residual_vjp(mesh: dict, orders, u, v, form: int = 0, isolated: bool = False):
    """(d r / d u)^T v, the residual's steps transposed by hand (box Euler meshes)."""
    o, u, v = _i32(orders), _f64(u), _f64(v)
    out = np.zeros_like(u)
    m = _mesh(mesh)
    _check(_load().orc_residual_vjp(ctypes.byref(m), _i(o), _d(u), _d(v), _d(out), int(form), int(bool(isolated))),
           "residual_vjp")
    return out


def restrict(fine_orders, coarse_orders, u):
    fo, co, u = _i32(fine_orders), _i32(coarse_orders), _f64(u)
    E = fo.size // 3
    uc = np.zeros(5 * num_nodes(co))
    _check(_load().orc_restrict(E, _i(fo), _i(co), _d(u), _d(uc)), "restrict")
    return uc


def project(from_orders, to_orders, u):
    """Solution transfer onto another order map (interpolation up, L2 projection down)."""
    fo, to, u = _i32(from_orders), _i32(to_orders), _f64(u)
    E = fo.size // 3
    ut = np.zeros(5 * num_nodes(to))
    _check(_load().orc_project(E, _i(fo), _i(to), _d(u), _d(ut)), "project")
    return ut


def bdf_weights(k: int) -> np.ndarray:
    w = np.zeros(k + 1)
    _check(_load().orc_bdf_weights(int(k), _d(w)), "bdf_weights")
    return w


def tau_dual(mesh: dict, fine_orders, coarse_orders, states, dt: float, isolated: bool = False):
    """Dual time-stepping estimate from stored fine states [Q(t_{n+1}), Q(t_n), ...];
    returns (tau_new, tau_trad) in the coarse layout."""
    fo, co = _i32(fine_orders), _i32(coarse_orders)
    st = [_f64(q) for q in states]
    arr = (_D * len(st))(*[_d(q) for q in st])
    nc = num_nodes(co)
    tn, tt = np.zeros(5 * nc), np.zeros(5 * nc)
    m = _mesh(mesh)
    _check(_load().orc_tau_dual(ctypes.byref(m), _i(fo), _i(co), arr, len(st), float(dt), int(bool(isolated)),
                                _d(tn), _d(tt)), "tau_dual")
    return tn, tt


def tau(mesh: dict, fine_orders, coarse_orders, u, dudt, isolated: bool = False, restriction: int = SAMPLE):
    """Returns (tau_new, tau_trad, norms[E,2], varnorms[E,2,5]) in the coarse layout.
    restriction: SAMPLE (the coarse-node sampling) or L2 (the exact L2 projection)."""
    fo, co, u, dudt = _i32(fine_orders), _i32(coarse_orders), _f64(u), _f64(dudt)
    E = fo.size // 3
    nc = num_nodes(co)
    tn = np.zeros(5 * nc)
    tt = np.zeros(5 * nc)
    norms = np.zeros((E, 2))
    vn = np.zeros((E, 2, 5))
    m = _mesh(mesh)
    _check(_load().orc_tau(ctypes.byref(m), _i(fo), _i(co), _d(u), _d(dudt), int(bool(isolated)),
                           int(restriction), _d(tn), _d(tt), _d(norms), _d(vn)), "tau")
    return tn, tt, norms, vn


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops over elements."""
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def num_combos(order3) -> int:
    o = _i32(order3)
    return int(_load().orc_num_combos(_i(o)))


def sweep(mesh: dict, orders, u, dudt, elems=None, restriction: int = SAMPLE):
    """Isolated sweep; returns (te_new, te_trad, combo_offsets) for the listed elements."""
    o, u, dudt = _i32(orders), _f64(u), _f64(dudt)
    E = o.size // 3
    el = _i32(np.arange(E) if elems is None else elems)
    o3 = o.reshape(-1, 3)
    counts = [num_combos(o3[e]) for e in el]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ten = np.zeros(int(offs[-1]))
    tet = np.zeros(int(offs[-1]))
    m = _mesh(mesh)
    _check(_load().orc_sweep(ctypes.byref(m), _i(o), _d(u), _d(dudt), int(restriction), _i(el), len(el),
                             _d(ten), _d(tet)), "sweep")
    return ten, tet, offs


def sweep_ns(mesh: dict, orders, u, dudt, mu: float, Pr: float = 0.72, elems=None, restriction: int = SAMPLE):
    """Isolated sweep of the Navier-Stokes residual; same outputs as sweep()."""
    o, u, dudt = _i32(orders), _f64(u), _f64(dudt)
    E = o.size // 3
    el = _i32(np.arange(E) if elems is None else elems)
    o3 = o.reshape(-1, 3)
    counts = [num_combos(o3[e]) for e in el]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ten = np.zeros(int(offs[-1]))
    tet = np.zeros(int(offs[-1]))
    m = _mesh(mesh)
    _check(_load().orc_sweep_ns(ctypes.byref(m), _i(o), _d(u), _d(dudt), float(mu), float(Pr), int(restriction),
                                _i(el), len(el), _d(ten), _d(tet)), "sweep_ns")
    return ten, tet, offs


def rk3(mesh: dict, orders, u, dt: float, nsteps: int):
    o = _i32(orders)
    out = _f64(u).copy()
    m = _mesh(mesh)
    _check(_load().orc_rk3(ctypes.byref(m), _i(o), _d(out), float(dt), int(nsteps)), "rk3")
    return out


def tau_eta(mesh: dict, fine_orders, coarse_orders, u, dudt, psi, isolated: bool = False,
            restriction: int = SAMPLE, psi_form: int = 1):
    """eta[e] = sum over the coarse nodes and variables of (I psi_t) * tau_trad, I the
    restriction of the estimate and psi_t the traditional-form adjoint: psi itself
    (psi_form 1) or, for the adjoint of the new form (psi_form 0), psi divided by the fine
    mass matrix."""
    fo, co = _i32(fine_orders), _i32(coarse_orders)
    u, dudt, psi = _f64(u), _f64(dudt), _f64(psi)
    E = fo.size // 3
    eta = np.zeros(E)
    m = _mesh(mesh)
    _check(_load().orc_tau_eta(ctypes.byref(m), _i(fo), _i(co), _d(u), _d(dudt), int(bool(isolated)),
                               int(restriction), _d(psi), int(psi_form), _d(eta)), "tau_eta")
    return eta


def functional(mesh: dict, orders, u, grad: bool = True):
    """Pressure force along x on the slip walls and (optionally) its gradient dJ/du."""
    o, u = _i32(orders), _f64(u)
    J = np.zeros(1)
    g = np.zeros_like(u) if grad else None
    m = _mesh(mesh)
    _check(_load().orc_functional(ctypes.byref(m), _i(o), _d(u), _d(J), _d(g) if grad else None), "functional")
    return (float(J[0]), g) if grad else float(J[0])


def gradient(mesh: dict, orders, u, isolated: bool = False):
    """BR1 gradients of the conserved variables, natural layout [e][3][5][node]."""
    o, u = _i32(orders), _f64(u)
    g = np.zeros(3 * u.size)
    m = _mesh(mesh)
    _check(_load().orc_gradient(ctypes.byref(m), _i(o), _d(u), int(bool(isolated)), _d(g)), "gradient")
    return g


def residual_ns(mesh: dict, orders, u, mu: float, Pr: float = 0.72, form: int = 0, isolated: bool = False):
    """Navier-Stokes (BR1) residual, new (0) or traditional (1) form."""
    o, u = _i32(orders), _f64(u)
    r = np.zeros_like(u)
    m = _mesh(mesh)
    _check(_load().orc_residual_ns(ctypes.byref(m), _i(o), _d(u), float(mu), float(Pr), _d(r), int(form),
                                   int(bool(isolated))), "residual_ns")
    return r


def viscous_flux(q, G, d: int, gamma=1.4, mu=0.01, Pr=0.72):
    q, G = _f64(q), _f64(G)
    f = np.zeros(5)
    _load().orc_viscous_flux(_d(q), _d(G), int(d), gamma, mu, Pr, _d(f))
    return f
