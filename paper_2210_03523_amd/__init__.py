"""MI355X (gfx950) DGSEM residual and anisotropic truncation-error estimation.

Thin ctypes binding of ``libdgtau.so`` (C ABI in ``include/dgtau.h``).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments: torch CUDA tensors provide device memory and the current
stream, numpy arrays the host-side order maps.  There is no CPU fallback: if
the library is not built, or no GPU is present, the calls raise.

Layouts: device state arrays use the plan layout (elements grouped into order
buckets, ``[elem][var][node]``); :meth:`Plan.to_plan` and
:meth:`Plan.to_natural` convert from and to the natural ragged layout
(natural element order ``e = ix + nx*(iy + ny*iz)``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdgtau.so")

DG_F64, DG_F32 = 0, 1
FORM_NEW, FORM_TRAD = 0, 1
RESTRICT_SAMPLE, RESTRICT_L2 = 0, 1  # restriction of the tau-estimate: sampling, L2 projection
NMAX = 9


class DGError(RuntimeError):
    pass


class _MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", ctypes.c_int32 * 6), ("flux", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("q_far", ctypes.c_double * 5),
                ("equation", ctypes.c_int32), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("map_kind", ctypes.c_int32), ("map_amp", ctypes.c_double), ("geo_order", ctypes.c_int32 * 3)]


class _AdjointParams(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("form", ctypes.c_int32), ("isolated", ctypes.c_int32), ("precond", ctypes.c_void_p),
                ("precond_sweep", ctypes.c_int32)]


PRECOND_JACOBI, PRECOND_GAUSS_SEIDEL = 0, 1


class _SelectParams(ctypes.Structure):
    _fields_ = [("tau_max", ctypes.c_double), ("nmin", ctypes.c_int32), ("nmax", ctypes.c_int32),
                ("approach", ctypes.c_int32), ("jump", ctypes.c_int32),
                ("prev", ctypes.c_void_p), ("max_decrease", ctypes.c_int32), ("ext_nmax", ctypes.c_int32)]


SELECT_MAX_STAGES = 32


class _AdaptParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("steps_per_stage", ctypes.c_int32), ("nstages", ctypes.c_int32),
                ("steps_after", ctypes.c_int32), ("restriction", ctypes.c_int32), ("form", ctypes.c_int32),
                ("select", _SelectParams)]


class _AdaptReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("ndof_dyn", ctypes.c_double), ("ndof_final", ctypes.c_int64)]

_lib = None
_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)

# exported symbol -> argument types (restype is always dg_status = int32, except dg_last_error)
SIGNATURES = {
    "dg_plan_create": [ctypes.POINTER(_MeshDesc), _I32P, ctypes.POINTER(_P)],
    "dg_plan_create_coarse": [_P, _I32P, ctypes.POINTER(_P)],
    "dg_plan_destroy": [_P],
    "dg_plan_layout": [_P, _I64P, _I64P, _I64P, _I64P, _I32P],
    "dg_node_coords": [_P, _P, _P],
    "dg_plan_metrics": [_P, _P, _P],
    "dg_residual": [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "dg_residual_noalloc": [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "dg_tau_estimate": [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_int32, _P,
                        _P],
    "dg_residual_vjp": [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P],
    "dg_functional": [_P, _P, _P, _P, _P],
    "dg_sweep_layout": [_P, _I64P],
    "dg_tau_sweep": [_P, _P, _P, ctypes.c_int32, _P, _P, _P],
    "dg_select_orders": [_P, ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_SelectParams), _P, _P],
    "dg_project": [_P, _P, _P, _P, _P],
    "dg_map_fmax": [_P, _P, _P, ctypes.c_int32, _P],
    "dg_tau_extrapolate": [_P, _P, ctypes.c_int32, _P, _P],
    "dg_bdf_rate": [_P, ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_double, _P, _P],
    "dg_adjoint_workspace": [_P, ctypes.c_int32, _I64P],
    "dg_adjoint_precond_bytes": [_P, _I64P],
    "dg_adjoint_precond_build": [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P],
    "dg_adjoint_precond_apply": [_P, _P, _P, _P, _P],
    "dg_adjoint_precond_compact_bytes": [_P, _I64P],
    "dg_adjoint_precond_compact": [_P, _P, _P, _P],
    "dg_adjoint_precond_apply_gs": [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P],
    "dg_adjoint_precond_colours": [_P, _P, _I32P],
    "dg_adjoint_solve": [_P, _P, _P, _P, ctypes.POINTER(_AdjointParams), _P, _I32P,
                         ctypes.POINTER(ctypes.c_double), _P],
    "dg_rk3_step": [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P],
    "dg_check": [],
    "dg_check_state": [_P, _P, ctypes.c_int32, _I64P, _P],
    "dg_batch_create": [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)],
    "dg_batch_destroy": [_P],
    "dg_batch_schedule": [_P, _I32P, _I32P, _I32P, _I32P, _I32P],
    "dg_batch_set_schedule": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "dg_batch_residual": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _P],
    "dg_batch_rk3_step": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_double, ctypes.c_int32, _P],
    "dg_batch_to_f64": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _P],
    "dg_adapt_dynamic": [ctypes.POINTER(_P), _P, _P, ctypes.c_int64, ctypes.POINTER(_AdaptParams), _I32P,
                         ctypes.POINTER(_AdaptReport), _P],
    "dg_adapt_static": [ctypes.POINTER(_P), _P, _P, ctypes.c_int64, ctypes.POINTER(_AdaptParams), _I32P,
                        ctypes.POINTER(_AdaptReport), _P],
    "dg_batch_tau_sweep": [_P, ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P), _P],
}


def lib():
    """Load libdgtau.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DGError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.dg_last_error.argtypes = []
        L.dg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise DGError(f"{name} failed ({st}): {lib().dg_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise DGError("no GPU visible: the HIP library needs a gfx950 device")
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise DGError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return DG_F64
    if t.dtype == torch.float32:
        return DG_F32
    raise DGError(f"unsupported dtype {t.dtype}")


def mesh_desc(mesh: dict) -> _MeshDesc:
    m = _MeshDesc()
    m.nx, m.ny, m.nz = (int(v) for v in mesh["n"])
    for d in range(3):
        m.lo[d] = float(mesh["lo"][d])
        m.hi[d] = float(mesh["hi"][d])
    for f in range(6):
        m.bc[f] = int(mesh["bc"][f])
    m.flux = int(mesh["flux"])
    m.gamma = float(mesh["gamma"])
    for v in range(5):
        m.q_far[v] = float(mesh["qfar"][v])
    m.equation = 1 if mesh.get("mu") is not None else 0
    m.mu = float(mesh.get("mu") or 0.0)
    m.Pr = float(mesh.get("Pr", 0.72))
    kind, amp, geo = mesh.get("map", (0, 0.0, (1, 1, 1)))
    m.map_kind, m.map_amp = int(kind), float(amp)
    for d in range(3):
        m.geo_order[d] = int(geo[d])
    return m


class Plan:
    """Device plan of a box mesh with per-element orders (natural order [E][3])."""

    def __init__(self, mesh: dict, orders, _parent: "Plan | None" = None):
        self.mesh = dict(mesh)
        o = np.ascontiguousarray(np.asarray(orders, dtype=np.int32).reshape(-1, 3))
        E = int(np.prod(mesh["n"])) if _parent is None else _parent.n_elems
        if o.shape[0] != E:
            raise DGError(f"{o.shape[0]} order triples given for {E} elements")
        self.orders_natural = o
        h = ctypes.c_void_p()
        if _parent is None:
            md = mesh_desc(mesh)
            _call("dg_plan_create", ctypes.byref(md), o.ctypes.data_as(_I32P), ctypes.byref(h))
        else:
            _call("dg_plan_create_coarse", _parent.handle, o.ctypes.data_as(_I32P), ctypes.byref(h))
        self.handle = h
        self.parent = _parent
        self._layout()

    @classmethod
    def _adopt(cls, mesh: dict, handle) -> "Plan":
        """A Plan object owning a plan handle the library created (adaptation loops)."""
        self = cls.__new__(cls)
        self.mesh = dict(mesh)
        self.handle = handle
        self.parent = None
        self._layout()
        o = np.empty_like(self.orders)
        o[self.perm] = self.orders
        self.orders_natural = o
        return self

    def _layout(self):
        h = self.handle
        ne = ctypes.c_int64()
        nn = ctypes.c_int64()
        _call("dg_plan_layout", h, ctypes.byref(ne), ctypes.byref(nn), None, None, None)
        self.n_elems, self.n_nodes = int(ne.value), int(nn.value)
        self.perm = np.zeros(self.n_elems, dtype=np.int64)
        self.node_offset = np.zeros(self.n_elems + 1, dtype=np.int64)
        self.orders = np.zeros((self.n_elems, 3), dtype=np.int32)
        _call("dg_plan_layout", h, None, None, self.perm.ctypes.data_as(_I64P),
              self.node_offset.ctypes.data_as(_I64P), self.orders.ctypes.data_as(_I32P))
        o = np.empty_like(self.orders)
        o[self.perm] = self.orders
        counts = np.prod(o.astype(np.int64) + 1, axis=1)
        self.natural_offset = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self._idx = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.dg_plan_destroy(h)
            self.handle = None

    # ------------------------------------------------------------------ layout
    def _index(self, nv: int) -> np.ndarray:
        """Gather index: plan position -> natural position (nv values per node)."""
        if nv not in self._idx:
            cnt = np.diff(self.node_offset) * nv
            src = nv * self.natural_offset[self.perm]
            dst = nv * self.node_offset[:-1]
            idx = np.repeat(src - dst, cnt) + np.arange(int(cnt.sum()), dtype=np.int64)
            self._idx[nv] = idx
        return self._idx[nv]

    def to_plan(self, u_nat, dtype=None, nv: int = 5):
        """Natural ragged numpy array -> device tensor in the plan layout."""
        torch = _torch()
        a = np.asarray(u_nat)[self._index(nv)]
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        return t.cuda()

    def to_natural(self, t, nv: int = 5) -> np.ndarray:
        """Device tensor in the plan layout -> natural ragged numpy array."""
        a = t.detach().cpu().numpy()
        out = np.empty_like(a)
        out[self._index(nv)] = a
        return out

    def inv_perm(self) -> np.ndarray:
        """Plan position of every natural element."""
        inv = np.empty_like(self.perm)
        inv[self.perm] = np.arange(self.n_elems)
        return inv

    def elem_to_natural(self, a_plan: np.ndarray) -> np.ndarray:
        """Per-plan-element rows -> natural element order."""
        out = np.empty_like(a_plan)
        out[self.perm] = a_plan
        return out

    def coarse(self, coarse_orders) -> "Plan":
        return Plan(self.mesh, coarse_orders, _parent=self)

    def node_coords(self):
        torch = _torch()
        xyz = torch.empty(3 * self.n_nodes, dtype=torch.float64, device="cuda")
        _call("dg_node_coords", self.handle, _ptr(xyz), _stream())
        return xyz

    def metrics(self):
        """Per-node metric terms, plan layout [E][10][n_p] (Ja^1, Ja^2, Ja^3, J)."""
        torch = _torch()
        met = torch.empty(10 * self.n_nodes, dtype=torch.float64, device="cuda")
        _call("dg_plan_metrics", self.handle, _ptr(met), _stream())
        return met

    def combo_offsets(self) -> np.ndarray:
        off = np.zeros(self.n_elems + 1, dtype=np.int64)
        _call("dg_sweep_layout", self.handle, off.ctypes.data_as(_I64P))
        return off

    def _combo_index(self) -> np.ndarray:
        """Gather index of the sweep layout: plan position -> natural position."""
        if "combo" not in self._idx:
            off = self.combo_offsets()
            cnt = np.diff(off)
            nat_cnt = np.empty_like(cnt)
            nat_cnt[self.perm] = cnt
            nat_off = np.concatenate([[0], np.cumsum(nat_cnt)]).astype(np.int64)
            self._idx["combo"] = np.repeat(nat_off[self.perm] - off[:-1], cnt) + np.arange(int(off[-1]))
        return self._idx["combo"]

    def map_to_plan(self, m_nat):
        """Map in natural element order (combinations of each element contiguous) -> device
        tensor in the sweep layout."""
        torch = _torch()
        return torch.from_numpy(np.ascontiguousarray(np.asarray(m_nat, dtype=np.float64)[self._combo_index()])).cuda()

    def map_to_natural(self, t) -> np.ndarray:
        a = t.detach().cpu().numpy()
        out = np.empty_like(a)
        out[self._combo_index()] = a
        return out

    def ext_to_natural(self, t, nmax: int) -> np.ndarray:
        """Extended map (plan element order) -> numpy [E, nmax^3] in natural element order."""
        a = t.detach().cpu().numpy().reshape(self.n_elems, int(nmax) ** 3)
        out = np.empty_like(a)
        out[self.perm] = a
        return out

    def ext_to_plan(self, m_nat, nmax: int):
        """Extended maps [E, nmax^3] in natural element order -> device tensor, plan order."""
        torch = _torch()
        a = np.asarray(m_nat, dtype=np.float64).reshape(self.n_elems, int(nmax) ** 3)
        return torch.from_numpy(np.ascontiguousarray(a[self.perm]).reshape(-1)).cuda()


# ---------------------------------------------------------------------- entry points
def residual(plan: Plan, u, form: int = FORM_NEW, isolated: bool = False, out=None):
    """r = M^-1 F^N(u) (form 0) or F^N(u) (form 1), plan layout, dtype of u."""
    torch = _torch()
    if u.numel() != 5 * plan.n_nodes:
        raise DGError("state size does not match the plan")
    r = torch.empty_like(u) if out is None else out
    _call("dg_residual", plan.handle, _ptr(u), _ptr(r), _dtype_code(u), int(form), int(bool(isolated)),
          _stream())
    return r


def residual_noalloc(plan: Plan, u, out, form: int = FORM_NEW, isolated: bool = False):
    """As residual(), with the library's static scratch instead of the plan's buffers
    (dg_residual_noalloc); out is required (nothing is allocated)."""
    if u.numel() != 5 * plan.n_nodes or out.numel() != u.numel() or out.dtype != u.dtype:
        raise DGError("state or output size does not match the plan")
    _call("dg_residual_noalloc", plan.handle, _ptr(u), _ptr(out), _dtype_code(u), int(form),
          int(bool(isolated)), _stream())
    return out


def tau_estimate(fine: Plan, coarse: Plan, u, dudt=None, isolated: bool = False, psi=None,
                 restriction: int = RESTRICT_SAMPLE, psi_form: int = FORM_TRAD, varnorms: bool = False):
    """Returns (tau_new, tau_trad, norms[E,2]) in the coarse plan layout (float64), plus
    eta[E] (sum of (I psi_t) * tau_trad per coarse element, psi_t the traditional-form
    adjoint) when an adjoint weight psi is given; psi_form is the form of the residual psi
    is the adjoint of (FORM_NEW: psi is divided by the fine mass matrix first).
    restriction: RESTRICT_SAMPLE (coarse-node sampling) or RESTRICT_L2 (L2 projection).
    varnorms=True appends the per-variable maxima [E,2,5] to the returned tuple."""
    torch = _torch()
    if coarse.parent is not fine:
        raise DGError("coarse plan was not built from this fine plan")
    for t in (u, dudt, psi):
        if t is not None and t.dtype != torch.float64:
            raise DGError("the tau-estimate runs in float64")
    tn = torch.empty(5 * coarse.n_nodes, dtype=torch.float64, device="cuda")
    tt = torch.empty_like(tn)
    norms = torch.empty((coarse.n_elems, 2), dtype=torch.float64, device="cuda")
    eta = torch.empty(coarse.n_elems, dtype=torch.float64, device="cuda") if psi is not None else None
    vn = torch.empty((coarse.n_elems, 2, 5), dtype=torch.float64, device="cuda") if varnorms else None
    _call("dg_tau_estimate", fine.handle, coarse.handle, _ptr(u), _ptr(dudt), int(bool(isolated)),
          int(restriction), _ptr(tn), _ptr(tt), _ptr(norms), _ptr(vn), _ptr(psi), int(psi_form), _ptr(eta),
          _stream())
    out = (tn, tt, norms) if psi is None else (tn, tt, norms, eta)
    return out + (vn,) if varnorms else out


def residual_vjp(plan: Plan, u, v, form: int = FORM_NEW, isolated: bool = False):
    """(d r / d u)^T v for the residual of `residual` (float64)."""
    torch = _torch()
    if u.dtype != torch.float64 or v.dtype != torch.float64:
        raise DGError("the adjoint runs in float64")
    out = torch.empty_like(u)
    _call("dg_residual_vjp", plan.handle, _ptr(u), _ptr(v), _ptr(out), int(form), int(bool(isolated)), _stream())
    return out


def functional(plan: Plan, u, grad: bool = True):
    """x-pressure force on the slip walls, J (device scalar) and dJ/du (plan layout)."""
    torch = _torch()
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(u) if grad else None
    _call("dg_functional", plan.handle, _ptr(u), _ptr(J), _ptr(g), _stream())
    return (J, g) if grad else J


class ResidualFn:
    """torch.autograd.Function: forward = dg_residual, backward = dg_residual_vjp."""

    @staticmethod
    def apply(plan: Plan, u, form: int = FORM_NEW, isolated: bool = False):
        return _residual_fn().apply(plan, u, form, isolated)


_RES_FN = None


def _residual_fn():
    global _RES_FN
    if _RES_FN is None:
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, plan, u, form, isolated):
                ctx.plan, ctx.form, ctx.isolated = plan, form, isolated
                ctx.save_for_backward(u)
                return residual(plan, u.detach().contiguous(), form=form, isolated=isolated)

            @staticmethod
            def backward(ctx, grad):
                (u,) = ctx.saved_tensors
                gu = residual_vjp(ctx.plan, u.detach().contiguous(), grad.contiguous(), ctx.form, ctx.isolated)
                return None, gu, None, None

        _RES_FN = _Fn
    return _RES_FN


def tau_sweep(plan: Plan, u, dudt=None, restriction: int = RESTRICT_SAMPLE):
    """Isolated TE map: (te_new, te_trad) per (plan element, combo), c1 fastest."""
    torch = _torch()
    off = plan.combo_offsets()
    ten = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    tet = torch.empty_like(ten)
    _call("dg_tau_sweep", plan.handle, _ptr(u), _ptr(dudt), int(restriction), _ptr(ten), _ptr(tet), _stream())
    return ten, tet


def select_orders(plan: Plan, maps, tau_max: float, nmin: int = 1, nmax: int = NMAX, approach: int = 2,
                  jump: int = 0, prev=None, max_decrease: int = 1, ext_nmax: int = 0):
    """Degrees [E][3] (device int32, natural element order) selected from truncation-error
    maps of the plan's sweep layout (or extended maps of tau_extrapolate, ext_nmax > 0),
    one map per estimation stage (approach 1: select per stage then the maximum;
    approach 2: select from the maximum of the maps), no degree more than max_decrease
    below prev (device int32 [E][3], optional), with the jump condition jump = 1
    (floor(2/3 N_j)), 2 (N_j - 1) or 0 (none) enforced."""
    torch = _torch()
    maps = list(maps)
    n = plan.n_elems * ext_nmax ** 3 if ext_nmax else int(plan.combo_offsets()[-1])
    for m in maps:
        if m.dtype != torch.float64 or m.numel() != n:
            raise DGError("maps must be float64 tensors in the layout of the plan")
    out = torch.empty((plan.n_elems, 3), dtype=torch.int32, device="cuda")
    if prev is not None and (prev.dtype != torch.int32 or prev.numel() != 3 * plan.n_elems):
        raise DGError("prev must be an int32 [E][3] device tensor")
    prm = _SelectParams(float(tau_max), int(nmin), int(nmax), int(approach), int(jump),
                        None if prev is None else _ptr(prev).value, int(max_decrease), int(ext_nmax))
    arr = (_P * max(1, len(maps)))(*[_ptr(m).value for m in maps])
    _call("dg_select_orders", plan.handle, arr, len(maps), ctypes.byref(prm), _ptr(out), _stream())
    return out


def adjoint_precond(plan: Plan, u, form: int = FORM_TRAD, isolated: bool = False):
    """Element-block Jacobi preconditioner of (dr/du)^T at u (dg_adjoint_precond_build):
    device memory (a uint8 tensor) to pass to adjoint_solve(precond=...)."""
    torch = _torch()
    if u.dtype != torch.float64 or u.numel() != 5 * plan.n_nodes:
        raise DGError("u must be a float64 state of the plan")
    nb = ctypes.c_int64()
    _call("dg_adjoint_precond_bytes", plan.handle, ctypes.byref(nb))
    pc = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    work = torch.empty(2 * u.numel(), dtype=torch.float64, device="cuda")
    _call("dg_adjoint_precond_build", plan.handle, _ptr(u), int(form), int(bool(isolated)), _ptr(pc), _ptr(work),
          _stream())
    return pc


def adjoint_precond_compact(plan: Plan, pc):
    """The compact (FP16 blocks, per-column scales) form of a preconditioner of
    adjoint_precond (dg_adjoint_precond_compact): new device memory; pc is left as it is."""
    torch = _torch()
    nb = ctypes.c_int64()
    _call("dg_adjoint_precond_compact_bytes", plan.handle, ctypes.byref(nb))
    pc16 = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    _call("dg_adjoint_precond_compact", plan.handle, _ptr(pc), _ptr(pc16), _stream())
    return pc16


def adjoint_precond_apply_gs(plan: Plan, pc, u, x, form: int = FORM_TRAD, isolated: bool = False):
    """z = (D + L)^-1 x, the colour-ordered block Gauss-Seidel sweep (dg_adjoint_precond_apply_gs)."""
    torch = _torch()
    z = torch.empty_like(x)
    work = torch.empty_like(x)
    _call("dg_adjoint_precond_apply_gs", plan.handle, _ptr(pc), _ptr(u), int(form), int(bool(isolated)), _ptr(x),
          _ptr(z), _ptr(work), _stream())
    return z


def adjoint_precond_colours(plan: Plan, pc):
    """The preconditioner's colour of every element (natural order, numpy int32)."""
    import numpy as np
    c = np.empty(plan.n_elems, dtype=np.int32)
    _call("dg_adjoint_precond_colours", plan.handle, _ptr(pc), c.ctypes.data_as(_I32P))
    return c


def adjoint_precond_apply(plan: Plan, pc, x):
    """z = M^-1 x with a preconditioner of adjoint_precond."""
    z = _torch().empty_like(x)
    _call("dg_adjoint_precond_apply", plan.handle, _ptr(pc), _ptr(x), _ptr(z), _stream())
    return z


def adjoint_solve(plan: Plan, u, g, psi=None, restart: int = 30, max_iter: int = 2000, rtol: float = 1e-10,
                  form: int = FORM_TRAD, isolated: bool = False, precond=None, sweep: int = PRECOND_JACOBI):
    """Solve (dr/du)^T psi = g by restarted GMRES on the residual VJP; returns
    (psi, iterations, relative residual).  psi (optional) is the initial guess; precond
    (optional) a preconditioner of adjoint_precond for the same state, form and flag,
    applied as block Jacobi or as the colour-ordered block Gauss-Seidel sweep."""
    torch = _torch()
    n = 5 * plan.n_nodes
    for t in (u, g):
        if t.dtype != torch.float64 or t.numel() != n:
            raise DGError("u and g must be float64 states of the plan")
    x = torch.zeros(n, dtype=torch.float64, device="cuda") if psi is None else psi.clone()
    nw = ctypes.c_int64()
    _call("dg_adjoint_workspace", plan.handle, int(restart), ctypes.byref(nw))
    work = torch.empty(int(nw.value), dtype=torch.float64, device="cuda")
    prm = _AdjointParams(int(restart), int(max_iter), float(rtol), int(form), int(bool(isolated)),
                         _ptr(precond).value if precond is not None else None, int(sweep))
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    _call("dg_adjoint_solve", plan.handle, _ptr(u), _ptr(g), _ptr(x), ctypes.byref(prm), _ptr(work),
          ctypes.byref(it), ctypes.byref(rr), _stream())
    return x, int(it.value), float(rr.value)


def bdf_rate(plan: Plan, states, dt: float):
    """dudt = -(delta_p/delta t) Q from stored states [Q(t_{n+1}), Q(t_n), ...] (2..4 of
    them, float64 plan layout): the fine term of the dual time-stepping estimate."""
    torch = _torch()
    states = list(states)
    for q in states:
        if q.dtype != torch.float64 or q.numel() != 5 * plan.n_nodes:
            raise DGError("states must be float64 states of the plan")
    out = torch.empty(5 * plan.n_nodes, dtype=torch.float64, device="cuda")
    arr = (_P * max(1, len(states)))(*[_ptr(q).value for q in states])
    _call("dg_bdf_rate", plan.handle, arr, len(states), float(dt), _ptr(out), _stream())
    return out


def map_fmax(plan: Plan, acc, m, ext_nmax: int = 0):
    """acc <- max(acc, m) in place (F_max total map of static adaptation; NaN sticky);
    maps in the sweep layout, or extended maps of tau_extrapolate with ext_nmax > 0."""
    torch = _torch()
    n = plan.n_elems * ext_nmax ** 3 if ext_nmax else int(plan.combo_offsets()[-1])
    for t in (acc, m):
        if t.dtype != torch.float64 or t.numel() != n:
            raise DGError("maps must be float64 tensors in the layout of the plan")
    _call("dg_map_fmax", plan.handle, _ptr(acc), _ptr(m), int(ext_nmax), _stream())
    return acc


def tau_extrapolate(plan: Plan, m, nmax: int = NMAX):
    """Extended truncation-error map [E * nmax^3] (plan element order, N1 fastest, N_i in
    1..nmax) from a sweep-layout map: computed values below the reference degree, the
    extrapolated decay (or +inf, the high value) at and above it."""
    torch = _torch()
    if m.dtype != torch.float64 or m.numel() != int(plan.combo_offsets()[-1]):
        raise DGError("the map must be a float64 tensor in the sweep layout of the plan")
    out = torch.empty(plan.n_elems * int(nmax) ** 3, dtype=torch.float64, device="cuda")
    _call("dg_tau_extrapolate", plan.handle, _ptr(m), int(nmax), _ptr(out), _stream())
    return out


def project(src: Plan, dst: Plan, u):
    """Solution u (plan layout of src, float64) transferred onto the order map of dst:
    interpolation where an order rises, exact L2 projection where it falls."""
    torch = _torch()
    if u.dtype != torch.float64 or u.numel() != 5 * src.n_nodes:
        raise DGError("u must be a float64 state of the source plan")
    ut = torch.empty(5 * dst.n_nodes, dtype=torch.float64, device="cuda")
    _call("dg_project", src.handle, dst.handle, _ptr(u), _ptr(ut), _stream())
    return ut


def check_state(plan: Plan, u) -> int:
    """Number of non-physical nodes of u (rho <= 0, p <= 0 or not finite); raises DGError
    (status -5) when there are any."""
    n = ctypes.c_int64()
    _call("dg_check_state", plan.handle, _ptr(u), _dtype_code(u), ctypes.byref(n), _stream())
    return int(n.value)


def rk3_step(plan: Plan, u, g, dt: float, nsteps: int = 1):
    """Advance u in place by nsteps Williamson RK3 steps (g is scratch of the same shape)."""
    if u.dtype != g.dtype or u.numel() != g.numel() or u.numel() != 5 * plan.n_nodes:
        raise DGError("u and g must match the plan and each other")
    _call("dg_rk3_step", plan.handle, _ptr(u), _ptr(g), float(dt), int(nsteps), _dtype_code(u), _stream())
    return u


def check():
    _call("dg_check")


# ---------------------------------------------------------------------- batches
class Batch:
    """Independent problems advanced by shared persistent launches (dtype fixed)."""

    def __init__(self, plans, dtype=None):
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        self.plans = list(plans)
        self.dtype = dtype
        arr = (_P * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        code = DG_F64 if dtype == torch.float64 else DG_F32
        _call("dg_batch_create", arr, len(self.plans), code, ctypes.byref(h))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.dg_batch_destroy(h)
            self.handle = None

    def schedule(self):
        """(tile capacity in nodes, element grid, face grid) chosen by the autotuner."""
        return self.schedule_info()[:3]

    def schedule_info(self):
        """(tile capacity, element grid, face grid, element-kernel shape, from_cache)."""
        v = [ctypes.c_int32() for _ in range(5)]
        _call("dg_batch_schedule", self.handle, *[ctypes.byref(x) for x in v])
        return tuple(x.value for x in v[:4]) + (bool(v[4].value),)

    def set_schedule(self, tile_cap: int, elem_grid: int, face_grid: int, shape: int):
        """Replace the autotuner's schedule (synchronous; drops the captured RK3 graphs)."""
        _call("dg_batch_set_schedule", self.handle, int(tile_cap), int(elem_grid), int(face_grid), int(shape))

    def _ptrs(self, ts):
        if len(ts) != len(self.plans):
            raise DGError("one tensor per problem expected")
        for t, p in zip(ts, self.plans):
            if t.dtype != self.dtype or t.numel() != 5 * p.n_nodes:
                raise DGError("tensor does not match its plan or the batch dtype")
        return (_P * len(ts))(*[t.data_ptr() for t in ts])


def batch_residual(batch: Batch, us, rs=None):
    rs = [_torch().empty_like(u) for u in us] if rs is None else rs
    _call("dg_batch_residual", batch.handle, batch._ptrs(us), batch._ptrs(rs), _stream())
    return rs


def batch_rk3_step(batch: Batch, us, gs, dt: float, nsteps: int = 1):
    _call("dg_batch_rk3_step", batch.handle, batch._ptrs(us), batch._ptrs(gs), float(dt), int(nsteps), _stream())
    return us


def batch_to_f64(batch: Batch, us, u64=None):
    """Every problem's state in float64 (promoted exactly from a float32 batch)."""
    torch = _torch()
    u64 = [torch.empty(u.numel(), dtype=torch.float64, device="cuda") for u in us] if u64 is None else u64
    for t, p in zip(u64, batch.plans):
        if t.dtype != torch.float64 or t.numel() != 5 * p.n_nodes:
            raise DGError("u64 tensors must be float64 and match their plans")
    arr = (_P * len(u64))(*[t.data_ptr() for t in u64])
    _call("dg_batch_to_f64", batch.handle, batch._ptrs(us), arr, _stream())
    return u64


def batch_tau_sweep(batch: Batch, u64, restriction: int = RESTRICT_SAMPLE):
    """FP64 isolated truncation-error maps of every problem: [(te_new, te_trad)] per
    problem in its sweep layout."""
    torch = _torch()
    if len(u64) != len(batch.plans):
        raise DGError("one state per problem expected")
    maps = []
    for t, p in zip(u64, batch.plans):
        if t.dtype != torch.float64 or t.numel() != 5 * p.n_nodes:
            raise DGError("u64 tensors must be float64 and match their plans")
        n = int(p.combo_offsets()[-1])
        maps.append((torch.empty(n, dtype=torch.float64, device="cuda"),
                     torch.empty(n, dtype=torch.float64, device="cuda")))
    n = len(u64)
    ua = (_P * n)(*[t.data_ptr() for t in u64])
    na = (_P * n)(*[m[0].data_ptr() for m in maps])
    ta = (_P * n)(*[m[1].data_ptr() for m in maps])
    _call("dg_batch_tau_sweep", batch.handle, ua, int(restriction), na, ta, _stream())
    return maps


def _adapt(name, plan: Plan, u, dt, steps_per_stage, nstages, tau_max, nmin, nmax, jump, approach,
           max_decrease, steps_after, restriction, form):
    torch = _torch()
    E = plan.n_elems
    cap = max(5 * E * (nmax + 1) ** 3, 5 * plan.n_nodes)
    if u.dtype != torch.float64 or u.numel() != 5 * plan.n_nodes:
        raise DGError("u must be a float64 state of the plan")
    ub = torch.empty(cap, dtype=torch.float64, device="cuda")
    ub[:u.numel()].copy_(u)
    work = torch.empty_like(ub)
    prm = _AdaptParams(float(dt), int(steps_per_stage), int(nstages), int(steps_after), int(restriction), int(form),
                       _SelectParams(float(tau_max), int(nmin), int(nmax), int(approach), int(jump), None,
                                     int(max_decrease), 0))
    rep = _AdaptReport()
    h = ctypes.c_void_p(plan.handle.value)
    orders = np.zeros((nstages if name == "dg_adapt_dynamic" else 1, E, 3), dtype=np.int32)
    _call(name, ctypes.byref(h), _ptr(ub), _ptr(work), int(cap), ctypes.byref(prm), orders.ctypes.data_as(_I32P),
          ctypes.byref(rep), _stream())
    new = plan if h.value == plan.handle.value else Plan._adopt(plan.mesh, h)
    return new, ub[:5 * new.n_nodes].clone(), orders, {"steps": int(rep.steps), "ndof_dyn": float(rep.ndof_dyn),
                                                        "ndof_final": int(rep.ndof_final)}


def adapt_dynamic(plan: Plan, u, dt: float, steps_per_stage: int, nstages: int, tau_max: float, nmin: int = 1,
                  nmax: int = 8, jump: int = 2, max_decrease: int = 1, restriction: int = RESTRICT_SAMPLE,
                  form: int = FORM_NEW):
    """Dynamic p-adaptation loop: (final plan, final state, degrees selected per stage
    [nstages][E][3] natural, report with NDOF_dyn)."""
    return _adapt("dg_adapt_dynamic", plan, u, dt, steps_per_stage, nstages, tau_max, nmin, nmax, jump, 1,
                  max_decrease, 0, restriction, form)


def adapt_static(plan: Plan, u, dt: float, steps_per_stage: int, nstages: int, steps_after: int, tau_max: float,
                 nmin: int = 1, nmax: int = 8, jump: int = 2, approach: int = 2,
                 restriction: int = RESTRICT_SAMPLE, form: int = FORM_NEW):
    """Static p-adaptation loop: (final plan, final state, adapted degrees [1][E][3]
    natural, report)."""
    return _adapt("dg_adapt_static", plan, u, dt, steps_per_stage, nstages, tau_max, nmin, nmax, jump, approach,
                  0, steps_after, restriction, form)
