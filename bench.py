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
oracle's CPU rate on a bounded sample.
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
    ap.add_argument("--n", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import torch
    import paper_2210_03523_amd as dg

    torch.cuda.set_device(0)
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

    flops_sweep = sweep_flops_per_element(8) * E
    t_sweep_ms = float(np.mean(t_swp))
    achieved = flops_sweep / (t_sweep_ms * 1e-3) / 1e12
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "sweep_c2_traffic.json")
    if os.path.exists(tpath):
        traffic = json.load(open(tpath)).get("bytes_per_launch")

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
        },
        "roofline": {"bound": "alu", "kernel": "k_sweep", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops_sweep},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, fo, co, u_nat, n_fine, n_est, E)
        # errors of the GPU results against the oracle on the sampled elements
        out["stages"].update(out["cpu_baseline"].pop("errors"))
        out["stages"]["err_residual_fp32"] = _err32(plan, r32, out["cpu_baseline"].pop("_ref"))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


def _err32(plan, r32, ref):
    got = plan.to_natural(r32).astype(np.float64)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def cpu_baseline(mesh, fo, co, u_nat, n_fine, n_est, E):
    """The oracle as it stands on the host cores: the full fine residual, the full
    coupled tau-estimate and the sweep on a sample of 8 elements, scaled to a step."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    dudt = oracle.residual(mesh, fo, u_nat)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.tau(mesh, fo, co, u_nat, dudt)
    t_tau = time.perf_counter() - t0
    sample = np.arange(0, E, E // 8)[:8]
    t0 = time.perf_counter()
    oracle.sweep(mesh, fo, u_nat, dudt, elems=sample)
    t_swp = (time.perf_counter() - t0) * E / len(sample)
    t_step = t_res + t_tau + t_swp
    return {"value": n_fine / t_step / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": f"full fine residual ({t_res:.2f} s) and coupled tau ({t_tau:.2f} s) on the whole "
                      f"mesh; isolated sweep on {len(sample)} of {E} elements, scaled by {E // len(sample)}",
            "residual_gdof_s": n_fine / t_res / 1e9,
            "tau_estimates_per_s": n_est / t_swp,
            "errors": {},
            "_ref": dudt}


if __name__ == "__main__":
    main()
