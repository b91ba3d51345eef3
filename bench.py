"""Benchmark of the hot path on one MI355X.

Workload (16^3 periodic unit cube, affine hexahedra, fine order N = 7 in every
direction = 2,097,152 nodes; Gaussian density pulse plus seeded N(0, 1e-3^2)
noise on rho; coarse orders drawn per element and direction from {1..6}; FP64).
One step is one pass of the whole estimation path on that state:

  1. fine residual r = M^-1 F^N(u)                         (dg_residual)
  2. coupled tau-estimate on the drawn coarse map, both forms (dg_tau_estimate)
  3. isolated anisotropic sweep, all 216 coarse combinations
     per element, both forms                               (dg_tau_sweep)

`value` is the step throughput in fine GDOF/s (fine nodes / step time).  The
line also carries the per-stage rates (residual GDOF/s, tau-estimates/s), the
FP32 residual rate and its speed-up over FP64 with both errors against the
oracle, the roofline of the dominant kernel (the sweep, FP64 vector ALU) and the
oracle's CPU rate on a bounded sample.  Outside the timed step: degree selection
(from the map and from its extrapolation to N_max = 9), plan rebuild and projection, the L2-restriction estimate and sweep, the dual
time-stepping rate, and the secondary legs (64-problem FP32 batch, curved
Navier-Stokes mesh with its sweep and coupled estimate, adjoint VJP / functional /
GMRES solve).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0


def sweep_flops_per_element(n: int) -> float:
    """Algorithmic FP64 flops of the isolated sweep of one element with n = N+1 nodes
    per direction (shared-prefix sum factorisation of the restriction of Q and of the
    time derivative, then the coarse volume residual, flux and tau per coarse node)."""
    ms = np.arange(2, n)              # coarse node counts m = c+1, c = 1..N-1
    S1, S2 = ms.sum(), (ms ** 2).sum()
    interp = 2 * 10 * (n ** 3 * S1 + n ** 2 * S1 ** 2 + n * S1 ** 3)
    deriv = 10 * 3 * S2 * S1 ** 2     # sum_c M_c (m1 + m2 + m3) * 5 vars * 2 flops
    other = 50 * S1 ** 3              # flux, difference, scaling and max per coarse node
    return float(interp + deriv + other)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-c5", action="store_true", help="skip the batched 64-problem leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the curved Navier-Stokes (32x32x2) and adjoint (24^3) legs")
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 256 MiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--only", choices=["c3", "c4", "c5"], default=None,
                    help="run one secondary leg alone and print its JSON (for kernel traces)")
    ap.add_argument("--no-precond", action="store_true",
                    help="adjoint leg: only the unpreconditioned solve (for per-dispatch counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import torch
    import paper_2210_03523_amd as dg

    torch.cuda.set_device(0)
    if args.only:
        stream = torch.cuda.current_stream()
        leg = {"c3": lambda: c3_leg(dg, torch, stream, check=not args.no_cpu),
               "c4": lambda: c4_leg(dg, torch, stream, check=not args.no_cpu, precond=not args.no_precond),
               "c5": lambda: c5_leg(dg, torch, stream, steps=5, warmup=1, check=not args.no_cpu)}[args.only]
        print(json.dumps({"leg": args.only, "result": leg()}))
        return
    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    mesh = wl.box_mesh(args.n)
    E = wl.num_elems(mesh)
    fo = wl.uniform_orders(E, 7)
    plan = dg.Plan(mesh, fo)
    xyz = plan.to_natural(plan.node_coords(), nv=3)
    u_nat, co = wl.c2_state_and_coarse(xyz, mesh, fo)
    cplan = plan.coarse(co)
    u = plan.to_plan(u_nat)
    r = torch.empty_like(u)
    n_fine = plan.n_nodes
    n_est = int(plan.combo_offsets()[-1])
    stream = torch.cuda.current_stream()

    def step(ev=None):
        dg.residual(plan, u, out=r)
        if ev:
            ev[0].record(stream)
        tn, tt, norms = dg.tau_estimate(plan, cplan, u, r)
        if ev:
            ev[1].record(stream)
        te = dg.tau_sweep(plan, u, r)
        if ev:
            ev[2].record(stream)
        return te

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][3].record(stream)
        step(evs[k][:3])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_res = np.array([e[3].elapsed_time(e[0]) for e in evs])
    t_tau = np.array([e[0].elapsed_time(e[1]) for e in evs])
    t_swp = np.array([e[1].elapsed_time(e[2]) for e in evs])
    ms_step = wall * 1e3 / args.steps

    # FP32 residual rate on the same mesh
    u32 = u.float()
    r32 = torch.empty_like(u32)
    for _ in range(3):
        dg.residual(plan, u32, out=r32)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    a.record(stream)
    for _ in range(reps):
        dg.residual(plan, u32, out=r32)
    b.record(stream)
    torch.cuda.synchronize()
    t_res32 = a.elapsed_time(b) / reps
    a.record(stream)
    for _ in range(reps):
        dg.residual(plan, u, out=r)
    b.record(stream)
    torch.cuda.synchronize()
    t_res64 = a.elapsed_time(b) / reps

    # degree selection from the sweep's map: three estimation stages (the map of this
    # step thrice), approach 2 with jump condition (b); tau_max the median map value
    ten_s, _ = step()
    tau_sel = float(torch.median(ten_s))
    t_select = _timed(torch, stream, lambda: dg.select_orders(plan, [ten_s] * 3, tau_max=tau_sel, nmin=1, nmax=8,
                                                              approach=2, jump=2), 10)
    sel_orders = dg.select_orders(plan, [ten_s] * 3, tau_max=tau_sel, nmin=1, nmax=8, approach=2, jump=2)
    sel_ndof = int(torch.prod(sel_orders.long() + 1, dim=1).sum())
    # tau-extrapolation of the map to N_max = 9 and the selection from the extended maps
    t_extrap = _timed(torch, stream, lambda: dg.tau_extrapolate(plan, ten_s, 9), 10)
    ext_s = dg.tau_extrapolate(plan, ten_s, 9)
    t_select_ext = _timed(torch, stream, lambda: dg.select_orders(plan, [ext_s] * 3, tau_max=tau_sel, nmin=1,
                                                                  nmax=9, approach=2, jump=2, ext_nmax=9), 10)
    # adaptation onto the selected map: plan rebuild (host tables, sort, faces, uploads)
    # and the projection of the solution onto it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    new_plan = dg.Plan(mesh, sel_orders.cpu().numpy())
    torch.cuda.synchronize()
    t_replan = (time.perf_counter() - t0) * 1e3
    t_project = _timed(torch, stream, lambda: dg.project(plan, new_plan, u), 10)
    proj_bytes = 40.0 * (n_fine + new_plan.n_nodes)

    # estimator variants on the same state: the L2-projection restriction (coupled
    # estimate and sweep) and the dual time-stepping rate over three stored states
    L2 = dg.RESTRICT_L2
    t_tau_l2 = _timed(torch, stream, lambda: dg.tau_estimate(plan, cplan, u, r, restriction=L2), 10)
    t_sweep_l2 = _timed(torch, stream, lambda: dg.tau_sweep(plan, u, r, restriction=L2), 5)
    hist = [u, u * (1.0 + 1e-6), u * (1.0 + 2e-6)]
    t_bdf = _timed(torch, stream, lambda: dg.bdf_rate(plan, hist, 1e-3), 10)
    del hist

    flops_sweep = sweep_flops_per_element(8) * E
    t_sweep_ms = float(np.mean(t_swp))
    achieved = flops_sweep / (t_sweep_ms * 1e-3) / 1e12
    traffic = _traffic("k_sweep_iso_c2_traffic.txt")

    out = {
        "metric": "GDOF/s residual + tau-estimates/s, batched FP32 vs plain FP64 at stated err",
        "value": n_fine / (ms_step * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler-16^3-N7-tau-sweep", "elements": E, "fine_order": 7,
                   "fine_nodes": n_fine, "coarse_nodes": cplan.n_nodes, "coarse_orders": "U{1..6}^3 seed 2",
                   "sweep_combos": n_est, "step": "residual + coupled tau (both forms) + isolated sweep"},
        "stages": {
            "residual_fp64_ms": float(np.mean(t_res)),
            "residual_fp64_gdof_s": n_fine / (t_res64 * 1e-3) / 1e9,
            "coupled_tau_ms": float(np.mean(t_tau)),
            "coupled_tau_fine_gdof_s": n_fine / (np.mean(t_tau) * 1e-3) / 1e9,
            "sweep_ms": t_sweep_ms,
            "tau_estimates_per_s": n_est / (t_sweep_ms * 1e-3),
            "residual_fp32_gdof_s": n_fine / (t_res32 * 1e-3) / 1e9,
            "fp32_over_fp64_residual_speedup": t_res64 / t_res32,
            "select_degrees_ms": t_select,
            "select_note": "3 stages of the sweep map, approach 2, jump (b), tau_max = median map value",
            "selected_nodes": sel_ndof,
            "adapt_replan_ms": t_replan,
            "adapt_project_ms": t_project,
            "adapt_project_hbm_frac": proj_bytes / (t_project * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "extrapolate_to_nmax9_ms": t_extrap,
            "select_degrees_extended_ms": t_select_ext,
            "coupled_tau_l2_restriction_ms": t_tau_l2,
            "sweep_l2_restriction_ms": t_sweep_l2,
            "dual_bdf2_rate_ms": t_bdf,
            "dual_bdf2_rate_hbm_frac": 160.0 * n_fine / (t_bdf * 1e-3) / 1e9 / PEAK_HBM_GBS,
        },
        "roofline": {"bound": "alu", "kernel": "k_sweep", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops_sweep},
        # HBM fractions of the bandwidth-bound stages: algorithmic bytes (state in, result
        # out; 80 B per fine node FP64, 40 B FP32; coupled tau adds 80 B per coarse node)
        "roofline_stages": {
            "unit": "fraction of 8 TB/s",
            "residual_fp64": 80.0 * n_fine / (t_res64 * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "residual_fp32": 40.0 * n_fine / (t_res32 * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "coupled_tau": (80.0 * n_fine + 80.0 * cplan.n_nodes) / (np.mean(t_tau) * 1e-3) / 1e9 / PEAK_HBM_GBS,
        },
    }
    if not args.no_c5:
        out["batched"] = c5_leg(dg, torch, stream, steps=5, warmup=1, check=not args.no_cpu)
    if not args.no_extra:
        out["navier_stokes_curved"] = c3_leg(dg, torch, stream, check=not args.no_cpu)
        out["adjoint"] = c4_leg(dg, torch, stream, check=not args.no_cpu, precond=not args.no_precond)
    if not args.no_cpu:
        base, ref = cpu_baseline(mesh, fo, co, u_nat, n_fine, n_est, E)
        out["cpu_baseline"] = base
        # errors against the oracle: max |x - x_oracle| / max(max |x_oracle|, s), s = scale of
        # the cancelling terms of the residual
        s = _scale(mesh, u_nat, 7)
        dg.residual(plan, u, out=r)
        dg.residual(plan, u32, out=r32)
        tn, _, _ = dg.tau_estimate(plan, cplan, u, r)
        ten, _ = dg.tau_sweep(plan, u, r)
        off = plan.combo_offsets()
        ten_h = ten.cpu().numpy()
        got = np.concatenate([ten_h[off[p]:off[p + 1]] for p in plan.inv_perm()[ref["sweep_elems"]]])
        out["errors"] = {
            "measure": "max|x - oracle| / max(max|oracle|, s), s = max|f| |Ja| ||D|| / J",
            "residual_fp64": _err(plan.to_natural(r), ref["dudt"], s),
            "residual_fp32": _err(plan.to_natural(r32).astype(np.float64), ref["dudt"], s),
            "coupled_tau_new_fp64": _err(cplan.to_natural(tn), ref["tau_new"], s),
            "sweep_te_new_fp64": _err(got, ref["te_new"], s),
        }
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


def _timed(torch, stream, fn, reps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def c3_leg(dg, torch, stream, check=True, dt=1e-5, nsteps=10):
    """Navier-Stokes (BR1) on the sine-mapped 32 x 32 x 2 mesh, orders (Nx, Ny) U{2..6},
    Nz = 1, 16 vortices: FP32 RK3 steps (graph replays), FP64 and FP32 residual rates, the
    isolated FP64 sweep; errors of the FP32 steps and of the sweep against the oracle."""
    mesh, orders, rng = wl.c3()
    plan = dg.Plan(mesh, orders)
    xyz = plan.to_natural(plan.node_coords(), nv=3)
    u_nat = wl.c3_state(xyz, orders, mesh, rng)
    n = plan.n_nodes
    u64 = plan.to_plan(u_nat)
    u32 = plan.to_plan(u_nat, dtype=torch.float32)
    r64, r32 = torch.empty_like(u64), torch.empty_like(u32)
    t64 = _timed(torch, stream, lambda: dg.residual(plan, u64, out=r64), 20)
    t32 = _timed(torch, stream, lambda: dg.residual(plan, u32, out=r32), 20)
    dudt = dg.residual(plan, u64)
    n_est = int(plan.combo_offsets()[-1])
    tsw = _timed(torch, stream, lambda: dg.tau_sweep(plan, u64, dudt), 10)
    # coupled estimate on a coarse map at or above the geometry order (2, 2, 1)
    co = orders.copy()
    co[:, :2] = np.maximum(2, np.minimum(orders[:, :2], np.random.default_rng(33).integers(1, 6, (len(orders), 2))))
    cplan = plan.coarse(co)
    tcp = _timed(torch, stream, lambda: dg.tau_estimate(plan, cplan, u64, dudt), 10)
    us = u32.clone()
    g = torch.empty_like(us)
    dg.rk3_step(plan, us, g, dt, 1)          # capture
    us.copy_(u32)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    dg.rk3_step(plan, us, g, dt, nsteps)
    b.record(stream)
    torch.cuda.synchronize()
    trk = a.elapsed_time(b) / nsteps
    res = {"workload": "NS Re=100 Ma=0.2 Pr=0.72, 32x32x2 sine-mapped hexes (geometry order 2,2,1), "
                       "(Nx,Ny) U{2..6} per element, Nz=1, 16 vortices, seed 3",
           "nodes": n, "sweep_combos": n_est,
           "residual_fp64_ms": t64, "residual_fp64_gdof_s": n / (t64 * 1e-3) / 1e9,
           "residual_fp32_ms": t32, "residual_fp32_gdof_s": n / (t32 * 1e-3) / 1e9,
           "rk3_fp32_ms_per_step": trk, "rk3_fp32_gdof_steps_s": n / (trk * 1e-3) / 1e9,
           "sweep_fp64_ms": tsw, "tau_estimates_per_s": n_est / (tsw * 1e-3),
           "coupled_tau_fp64_ms": tcp, "coupled_tau_coarse_nodes": cplan.n_nodes}
    if check:
        import oracle
        A, B = (0.0, -5.0 / 9.0, -153.0 / 128.0), (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
        ref = u_nat.copy()
        for _ in range(nsteps):
            G = np.zeros_like(ref)
            for k in range(3):
                r = oracle.residual_ns(mesh, orders, ref, mesh["mu"], mesh["Pr"])
                G = -dt * r if k == 0 else A[k] * G - dt * r
                ref = ref + B[k] * G
        d_ref = oracle.residual_ns(mesh, orders, u_nat, mesh["mu"], mesh["Pr"])
        ten_r, _, _ = oracle.sweep_ns(mesh, orders, u_nat, d_ref, mesh["mu"], mesh["Pr"])
        ten, _ = dg.tau_sweep(plan, u64, plan.to_plan(d_ref))
        off = plan.combo_offsets()
        got = np.concatenate([ten.cpu().numpy()[off[p]:off[p + 1]] for p in plan.inv_perm()])
        s = _scale(mesh, u_nat, int(np.max(orders)), orders)
        res["err_vs_oracle"] = {
            "rk3_fp32": float(np.max(np.abs(plan.to_natural(us).astype(np.float64) - ref)) / np.max(np.abs(ref))),
            "residual_fp64": _err(plan.to_natural(dudt), d_ref, s),
            "sweep_te_new_fp64": _err(got, ten_r, s),
            "measure": "rk3: max|u - u_oracle| / max|u_oracle| after 10 steps; others as in errors"}
    return res


def c4_leg(dg, torch, stream, check=True, precond=True):
    """Adjoint workload (24^3, N = 5, slip wall at x = 0, far field at x = 1): the residual
    VJP and the wall functional; the VJP is checked against the oracle's hand-transposed
    VJP over the whole field."""
    mesh, orders = wl.c4()
    plan = dg.Plan(mesh, orders)
    xyz = plan.to_natural(plan.node_coords(), nv=3)
    u_nat = wl.c4_state(xyz, orders)
    n = plan.n_nodes
    u = plan.to_plan(u_nat)
    rng = np.random.default_rng(44)
    v_nat = rng.normal(size=u_nat.shape)
    v = plan.to_plan(v_nat)
    out = torch.empty_like(u)
    tv = _timed(torch, stream, lambda: dg.residual_vjp(plan, u, v), 10)
    tf = _timed(torch, stream, lambda: dg.functional(plan, u), 10)
    # adjoint of the wall force: (dr/du)^T psi = dJ/du by GMRES(30) on the VJP, without a
    # preconditioner (it stalls) and with the element-block Jacobi one (built from probing
    # VJPs, FP32 inverse blocks)
    _, dJ = dg.functional(plan, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters0, relres0 = dg.adjoint_solve(plan, u, dJ, restart=30, max_iter=300, rtol=1e-8, form=dg.FORM_TRAD)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) * 1e3
    if not precond:
        return {"workload": "Euler 24^3 N=5, slip wall x=0, far field x=1, seed 4", "nodes": n, "vjp_ms": tv,
                "functional_ms": tf, "adjoint_solve": {"unpreconditioned": {"iterations": iters0, "relres": relres0,
                                                                            "ms": t_plain}}}
    t0 = time.perf_counter()
    pc32 = dg.adjoint_precond(plan, u, form=dg.FORM_TRAD)
    torch.cuda.synchronize()
    t_pc = (time.perf_counter() - t0) * 1e3
    pc32_gb = pc32.numel() / 1e9
    # the compact form (FP16 blocks over per-column scales) is the one the solve uses
    t0 = time.perf_counter()
    pc = dg.adjoint_precond_compact(plan, pc32)
    torch.cuda.synchronize()
    t_compact = (time.perf_counter() - t0) * 1e3
    del pc32
    torch.cuda.empty_cache()
    pc_gb = pc.numel() / 1e9
    # block Jacobi, then the colour-ordered block Gauss-Seidel sweep (the reported solve)
    t0 = time.perf_counter()
    _, iters_j, relres_j = dg.adjoint_solve(plan, u, dJ, restart=30, max_iter=4000, rtol=1e-8, form=dg.FORM_TRAD,
                                            precond=pc)
    torch.cuda.synchronize()
    t_adj_j = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    psi, iters, relres = dg.adjoint_solve(plan, u, dJ, restart=30, max_iter=4000, rtol=1e-8, form=dg.FORM_TRAD,
                                          precond=pc, sweep=dg.PRECOND_GAUSS_SEIDEL)
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - t0) * 1e3
    del pc
    torch.cuda.empty_cache()
    true_rel = float((dg.residual_vjp(plan, u, psi, form=dg.FORM_TRAD) - dJ).norm() / dJ.norm())
    res = {"workload": "Euler 24^3 N=5, slip wall x=0, far field x=1, seed 4", "nodes": n,
           "vjp_ms": tv, "vjp_gdof_s": n / (tv * 1e-3) / 1e9,
           "vjp_hbm_frac": 120.0 * n / (tv * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "functional_ms": tf,
           "adjoint_solve": {"method": "GMRES(30) on the residual VJP, right-preconditioned by the colour-ordered "
                                       "block Gauss-Seidel sweep of the element blocks (inverse blocks from probing "
                                       "VJPs, inverted in FP32, stored as FP16 over per-column scales), rtol 1e-8",
                             "block_jacobi": {"iterations": iters_j, "relres": relres_j, "ms": t_adj_j,
                                              "ms_per_iteration": t_adj_j / max(iters_j, 1)},
                             "precond_build_ms": t_pc, "precond_fp32_gb": pc32_gb,
                             "precond_compact_ms": t_compact, "precond_gb": pc_gb,
                             "ms": t_adj, "iterations": iters, "ms_per_iteration": t_adj / max(iters, 1),
                             "gmres_relres": relres, "true_relres": true_rel,
                             "unpreconditioned": {"iterations": iters0, "relres": relres0, "ms": t_plain}}}
    if check:
        import oracle
        jtv = plan.to_natural(dg.residual_vjp(plan, u, v))
        ref = oracle.residual_vjp(mesh, orders, u_nat, v_nat)
        res["err_vs_oracle"] = {"vjp": float(np.max(np.abs(jtv - ref)) / np.max(np.abs(ref))),
                                "measure": "max|J^T v - oracle J^T v| / max|oracle J^T v| over the whole field"}
    return res


def c5_leg(dg, torch, stream, steps=5, warmup=1, check=True, dt=1e-4):
    """64 independent periodic problems (n ~ U{8..20} elements per side, orders U{1..7},
    seeded pulses): RK3 steps of the FP32 batch (one graph per step, one persistent face and
    one persistent element launch per stage) against plain FP64 per-problem RK3 steps."""
    probs = wl.c5()
    plans, u0 = [], []
    for mesh, orders, centre, sigma in probs:
        p = dg.Plan(mesh, orders)
        xyz = p.to_natural(p.node_coords(), nv=3)
        plans.append(p)
        u0.append(wl.pulse_state(xyz, orders, centre=centre, sigma=sigma))
    nodes = sum(p.n_nodes for p in plans)
    batch = dg.Batch(plans, dtype=torch.float32)
    u32 = [p.to_plan(u, dtype=torch.float32) for p, u in zip(plans, u0)]
    g32 = [torch.empty_like(u) for u in u32]
    u64 = [p.to_plan(u) for p, u in zip(plans, u0)]
    g64 = [torch.empty_like(u) for u in u64]

    def timed(fn):
        fn(warmup)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn(steps)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    t32 = timed(lambda k: dg.batch_rk3_step(batch, u32, g32, dt, k))
    t64 = timed(lambda k: [dg.rk3_step(p, u, g, dt, k) for p, u, g in zip(plans, u64, g64)])
    # FP64 estimate of the FP32-stepped batch: exact promotion, then every problem's
    # FP64 fine residual and isolated sweep
    w64 = dg.batch_to_f64(batch, u32)
    maps = dg.batch_tau_sweep(batch, w64)
    combos = sum(int(p.combo_offsets()[-1]) for p in plans)
    t_prom = timed(lambda k: [dg.batch_to_f64(batch, u32, w64) for _ in range(k)])
    t_tau = timed(lambda k: [dg.batch_tau_sweep(batch, w64) for _ in range(k)])
    res = {"workload": "64 periodic Euler problems, n ~ U{8..20}^3 elements, orders U{1..7}^3, seed 5",
           "problems": len(plans), "nodes": nodes, "dt": dt,
           "schedule": dict(zip(("tile_cap", "elem_grid", "face_grid", "elem_shape", "from_cache"),
                                batch.schedule_info())),
           "fp32_batched_ms_per_rk3_step": t32, "fp64_plain_ms_per_rk3_step": t64,
           "fp32_batched_gdof_steps_s": nodes / (t32 * 1e-3) / 1e9,
           "fp64_plain_gdof_steps_s": nodes / (t64 * 1e-3) / 1e9,
           "speedup_fp32_batched_over_fp64_plain": t64 / t32,
           "fp64_tau": {"what": "promotion of the FP32 batch state to FP64, then the FP64 fine residuals "
                                "of all problems (one batched pass) and their isolated sweeps (both "
                                "forms, one launch per fine node count)",
                        "promote_ms": t_prom, "sweep_ms": t_tau, "tau_estimates": combos,
                        "tau_estimates_per_s": combos / ((t_prom + t_tau) * 1e-3)}}
    if check:
        import oracle
        order = np.argsort([p.n_nodes for p in plans])[:2]
        e32, e64 = 0.0, 0.0
        for i in order:
            mesh, orders, _, _ = probs[i]
            ref = oracle.rk3(mesh, orders, u0[i], dt, warmup + steps)
            scale = np.max(np.abs(ref))
            e32 = max(e32, float(np.max(np.abs(plans[i].to_natural(u32[i]).astype(np.float64) - ref)) / scale))
            e64 = max(e64, float(np.max(np.abs(plans[i].to_natural(u64[i]) - ref)) / scale))
        et = 0.0
        for i in order:
            mesh, orders, _, _ = probs[i]
            un = plans[i].to_natural(w64[i])
            ref, _, _ = oracle.sweep(mesh, orders, un, oracle.residual(mesh, orders, un))
            zs, _, _ = oracle.sweep(mesh, orders, un, np.zeros_like(un))
            off = plans[i].combo_offsets()
            a = maps[i][0].cpu().numpy()
            got = np.concatenate([a[off[q]:off[q + 1]] for q in np.argsort(plans[i].perm)])
            et = max(et, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), np.max(np.abs(zs)))))
        res["err_vs_oracle"] = {"measure": f"max|u - u_oracle| / max|u_oracle| after {warmup + steps} steps, "
                                           "two smallest problems; tau: max|te - te_oracle| / max(max|te_oracle|, "
                                           "max|r^Nc(Q^c)|) of the promoted state, same problems",
                                "fp32_batched": e32, "fp64_plain": e64, "fp64_tau_sweep": et}
    return res


def _traffic(name):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or None when
    the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    src = os.path.join(ROOT, kv["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["source_sha256_16"]:
        return None
    return float(kv["bytes_per_launch"])


def _scale(mesh, u_nat, N, orders=None):
    """Scale of the cancelling terms of the residual, max |f| * |Ja| * ||D|| / J, with
    ||D|| = N(N+1)/2 (the error measure of the parity tests); N the largest order,
    orders (natural [E][3]) for a mixed-order state."""
    if orders is None:
        q = u_nat.reshape(-1, 5, (N + 1) ** 3).transpose(1, 0, 2).reshape(5, -1)
    else:
        offs = wl.node_offsets(orders)
        q = np.concatenate([u_nat[5 * offs[e]:5 * offs[e + 1]].reshape(5, -1) for e in range(len(orders))], axis=1)
    g = mesh["gamma"]
    vel = q[1:4] / q[0]
    p = (g - 1) * (q[4] - 0.5 * q[0] * np.sum(vel * vel, axis=0))
    fmax = float(np.max(np.abs(q[4] + p) * np.max(np.abs(vel), axis=0) + np.abs(p)
                        + np.max(np.abs(q[1:4]), axis=0) * np.max(np.abs(vel), axis=0)))
    h = (np.asarray(mesh["hi"]) - np.asarray(mesh["lo"])) / np.asarray(mesh["n"])
    J = h.prod() / 8
    return fmax * (h[1] * h[2] / 4) * N * (N + 1) / 2 / J


def _err(x, ref, s):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), s))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, fo, co, u_nat, n_fine, n_est, E, runs=5):
    """The oracle as it stands on the host cores, median of `runs` timings after one
    warm-up, on all the process's cores and on one core: the full fine residual and the
    full coupled tau-estimate, and the isolated sweep on an evenly spaced sample of the
    elements (256 on all cores, 32 on one core), scaled to one step.  Returns the rate
    and the oracle outputs of the all-core run (the sweep on its sample)."""
    import oracle
    cores = len(os.sched_getaffinity(0))

    def leg(threads, nsample):
        oracle.set_threads(threads)
        sample = np.linspace(0, E - 1, nsample).astype(np.int64)
        t = {"res": [], "tau": [], "swp": []}
        out = None
        for r in range(runs + 1):
            t0 = time.perf_counter()
            dudt = oracle.residual(mesh, fo, u_nat)
            t1 = time.perf_counter()
            tn, tt, norms, _ = oracle.tau(mesh, fo, co, u_nat, dudt)
            t2 = time.perf_counter()
            ten, tet, _ = oracle.sweep(mesh, fo, u_nat, dudt, elems=sample)
            t3 = time.perf_counter()
            if r == 0:  # warm-up
                out = {"dudt": dudt, "tau_new": tn, "sweep_elems": sample, "te_new": ten, "te_trad": tet}
                continue
            t["res"].append(t1 - t0)
            t["tau"].append(t2 - t1)
            t["swp"].append((t3 - t2) * E / nsample)
        med = {k: float(np.median(v)) for k, v in t.items()}
        step = med["res"] + med["tau"] + med["swp"]
        return {"value": n_fine / step / 1e9, "threads": threads, "ms_per_step": step * 1e3,
                "residual_gdof_s": n_fine / med["res"] / 1e9, "coupled_tau_s": med["tau"],
                "tau_estimates_per_s": n_est / med["swp"], "sweep_sample_elements": nsample}, out

    allc, out = leg(cores, 256)
    one, _ = leg(1, 32)
    oracle.set_threads(cores)
    base = {"value": allc["value"], "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": f"median of {runs} runs after one warm-up: the full fine residual and coupled tau on "
                      f"the whole mesh, the isolated sweep on {allc['sweep_sample_elements']} of {E} evenly "
                      f"spaced elements scaled to all elements; the one-core leg samples "
                      f"{one['sweep_sample_elements']} elements",
            "cpu_model": _cpu_model(), "statistic": "median", "runs": runs,
            "residual_gdof_s": allc["residual_gdof_s"], "tau_estimates_per_s": allc["tau_estimates_per_s"],
            "all_cores": allc, "one_core": one}
    return base, out


if __name__ == "__main__":
    main()
