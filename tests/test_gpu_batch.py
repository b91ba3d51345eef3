"""GPU parity of the batched form: many independent problems of uneven size and
random anisotropic orders in shared persistent launches, against the FP64 oracle
problem by problem (FP64 within 1e-12, FP32 within 1e-5 of the cancelling-term scale)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import residual_scale, sweep_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2210_03523_amd as dg  # noqa: E402


def _problems(nprob=7, seed=31):
    probs = wl.c5(seed=seed, nprob=nprob, nrange=(1, 4), orange=(1, 7))
    out = []
    for mesh, orders, centre, sigma in probs:
        u = wl.pulse_state(oracle.node_coords(mesh, orders), orders, centre=centre, sigma=max(sigma, 0.15))
        out.append((mesh, orders, u))
    return out


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_batch_residual(dtype, tol):
    probs = _problems()
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=dtype)
    cap, eg, fg = batch.schedule()
    assert cap in (256, 512) and eg > 0 and fg > 0
    us = [p.to_plan(u, dtype=dtype) for p, (_, _, u) in zip(plans, probs)]
    rs = dg.batch_residual(batch, us)
    for p, (m, o, u), r in zip(plans, probs, rs):
        ref = oracle.residual(m, o, u)
        s = residual_scale(m, o, u)
        e = np.max(np.abs(p.to_natural(r).astype(np.float64) - ref)) / max(np.max(np.abs(ref)), s)
        assert e < tol
        # same answer as the single-problem path
        r1 = dg.residual(p, us[plans.index(p)])
        if dtype == torch.float64:
            assert torch.allclose(r1, r, rtol=0, atol=1e-13 * s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_every_schedule_gives_the_same_residual(dtype):
    """Forced schedules -- both tile capacities and all three element-kernel shapes, grids
    from one workgroup (one persistent workgroup runs every tile and face, through the
    element pass's software pipeline from its first tile to its last) to one per work
    item -- give the tuned schedule's residuals and RK3 states bit for bit."""
    probs = _problems(nprob=6, seed=41)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=dtype)
    us = [p.to_plan(u, dtype=dtype) for p, (_, _, u) in zip(plans, probs)]
    ref = [r.clone() for r in dg.batch_residual(batch, us)]
    ref_rk = [u.clone() for u in us]
    dg.batch_rk3_step(batch, ref_rk, [torch.zeros_like(u) for u in us], 1e-3)
    max_npe = max(int(np.prod(np.asarray(o) + 1, axis=1).max()) for _, o, _ in probs)
    nt_big = sum(p.n_nodes for p in plans)  # above any tile or face count
    for cap, shape in ((256, 0), (512, 1), (512, 2)):
        if cap < max_npe:
            with pytest.raises(dg.DGError, match="tile capacity"):
                batch.set_schedule(cap, 8, 8, shape)
            continue
        for eg, fg in ((1, 1), (3, 7), (64, 1000), (nt_big, nt_big)):
            batch.set_schedule(cap, eg, fg, shape)
            assert batch.schedule_info()[:4] == (cap, eg, fg, shape)
            got = dg.batch_residual(batch, us)
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (cap, shape, eg, fg)
            uu = [u.clone() for u in us]
            dg.batch_rk3_step(batch, uu, [torch.zeros_like(u) for u in us], 1e-3)
            for a, b in zip(uu, ref_rk):
                assert torch.equal(a, b), (cap, shape, eg, fg)
    with pytest.raises(dg.DGError, match="shape"):
        batch.set_schedule(512, 8, 8, 3)
    with pytest.raises(dg.DGError, match="256 goes with shape 0"):
        batch.set_schedule(256, 8, 8, 2)
    with pytest.raises(dg.DGError, match="positive"):
        batch.set_schedule(512, 0, 8, 2)


def test_schedule_cache():
    """A second batch of the same composition (new plans of the same meshes and orders)
    takes the autotuner's cached schedule and gives the same residuals bit for bit; a
    batch of the other precision is tuned afresh."""
    probs = _problems(nprob=5, seed=33)
    pa = [dg.Plan(m, o) for m, o, _ in probs]
    a = dg.Batch(pa, dtype=torch.float32)
    assert a.schedule_info()[4] is False
    pb = [dg.Plan(m, o) for m, o, _ in probs]
    b = dg.Batch(pb, dtype=torch.float32)
    ia, ib = a.schedule_info(), b.schedule_info()
    assert ib[4] is True and ia[:4] == ib[:4]
    ua = [p.to_plan(u, dtype=torch.float32) for p, (_, _, u) in zip(pa, probs)]
    ub = [p.to_plan(u, dtype=torch.float32) for p, (_, _, u) in zip(pb, probs)]
    for ra, rb in zip(dg.batch_residual(a, ua), dg.batch_residual(b, ub)):
        assert torch.equal(ra, rb)
    c = dg.Batch(pb, dtype=torch.float64)
    assert c.schedule_info()[4] is False


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_batch_rk3_graph(dtype, tol):
    probs = _problems(nprob=5, seed=32)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=dtype)
    us = [p.to_plan(u, dtype=dtype) for p, (_, _, u) in zip(plans, probs)]
    gs = [torch.empty_like(u) for u in us]
    refs = [u.copy() for _, _, u in probs]
    dt = 1e-3
    for chunk in (1, 3):  # replays of the captured step, with syncs in between
        dg.batch_rk3_step(batch, us, gs, dt, chunk)
        torch.cuda.synchronize()
        for i, (m, o, _) in enumerate(probs):
            refs[i] = oracle.rk3(m, o, refs[i], dt, chunk)
            got = plans[i].to_natural(us[i]).astype(np.float64)
            assert np.max(np.abs(got - refs[i])) / np.max(np.abs(refs[i])) < tol


def _sweep_nat(plan, t):
    off = plan.combo_offsets()
    a = t.cpu().numpy()
    return np.concatenate([a[off[p]:off[p + 1]] for p in np.argsort(plan.perm)])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batch_tau_sweep(dtype):
    """The FP64 estimate of a batch: states (FP32 ones promoted exactly), each problem's
    FP64 fine residual and isolated sweep, against the oracle's sweep of the same
    (promoted) state, every problem, both forms."""
    probs = _problems(nprob=5, seed=35)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=dtype)
    us = [p.to_plan(u, dtype=dtype) for p, (_, _, u) in zip(plans, probs)]
    gs = [torch.empty_like(u) for u in us]
    dg.batch_rk3_step(batch, us, gs, 1e-3, 2)
    u64 = dg.batch_to_f64(batch, us)
    for a, b in zip(u64, us):
        assert torch.equal(a, b.double())
    maps = dg.batch_tau_sweep(batch, u64)
    for p, (m, o, _), x, (ten, tet) in zip(plans, probs, u64, maps):
        un = p.to_natural(x)
        ten_r, tet_r, _ = oracle.sweep(m, o, un, oracle.residual(m, o, un))
        sn, st = sweep_scale(m, o, un)
        assert np.max(np.abs(_sweep_nat(p, ten) - ten_r)) < 1e-12 * max(np.max(np.abs(ten_r)), sn)
        assert np.max(np.abs(_sweep_nat(p, tet) - tet_r)) < 1e-12 * max(np.max(np.abs(tet_r)), st)


def test_batch_tau_sweep_matches_each_plan():
    """The merged work lists of the batched sweep (one launch per fine node count over
    every problem) give each problem exactly its own plan's sweep: the same kernels, the
    same per-node arithmetic, only the launch composition differs."""
    probs = _problems(nprob=6, seed=36)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=torch.float64)
    u64 = [p.to_plan(u) for p, (_, _, u) in zip(plans, probs)]
    maps = dg.batch_tau_sweep(batch, u64)
    for p, x, (ten, tet) in zip(plans, u64, maps):
        a, b = dg.tau_sweep(p, x, None)
        assert torch.equal(ten, a) and torch.equal(tet, b)


def test_batch_rejects_a_repeated_plan():
    probs = _problems(nprob=2, seed=33)
    p = dg.Plan(probs[0][0], probs[0][1])
    with pytest.raises(dg.DGError, match="appears twice"):
        dg.Batch([p, p], dtype=torch.float32)


def test_eager_ring_and_graph_cache_reuse():
    """Ten eager residual calls issued back to back (more than the four descriptor
    slots) into distinct outputs, and RK3 steps on ten distinct state sets (more than
    the eight cached graphs, so the least recently used ones are evicted and captured
    again): every result equals the same call made alone with a synchronisation around
    it, bit for bit (the batched kernels are deterministic)."""
    probs = _problems(nprob=3, seed=34)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=torch.float64)
    us = [p.to_plan(u) for p, (_, _, u) in zip(plans, probs)]
    ins = [[u * (1.0 + 0.01 * k) for u in us] for k in range(10)]
    torch.cuda.synchronize()
    outs = [dg.batch_residual(batch, x) for x in ins]
    torch.cuda.synchronize()
    for x, rs in zip(ins, outs):
        alone = dg.batch_residual(batch, x)
        torch.cuda.synchronize()
        for a, b in zip(rs, alone):
            assert torch.equal(a, b)
    dt = 1e-3
    sets = [([u.clone() for u in us], [torch.empty_like(u) for u in us]) for _ in range(10)]
    for _ in range(2):
        for ub, gb in sets:
            dg.batch_rk3_step(batch, ub, gb, dt, 1)
    torch.cuda.synchronize()
    ref = [u.clone() for u in us]
    gref = [torch.empty_like(u) for u in us]
    for _ in range(2):
        dg.batch_rk3_step(batch, ref, gref, dt, 1)
        torch.cuda.synchronize()
    for ub, _ in sets:
        for a, b in zip(ub, ref):
            assert torch.equal(a, b)
    for p, (m, o, u), r in zip(plans, probs, ref):
        want = oracle.rk3(m, o, u, dt, 2)
        assert np.max(np.abs(p.to_natural(r) - want)) < 1e-12 * np.max(np.abs(want))


def test_batch_rejects_mismatched_tensors():
    probs = _problems(nprob=2, seed=33)
    plans = [dg.Plan(m, o) for m, o, _ in probs]
    batch = dg.Batch(plans, dtype=torch.float32)
    us = [p.to_plan(u, dtype=torch.float64) for p, (_, _, u) in zip(plans, probs)]
    with pytest.raises(dg.DGError):
        dg.batch_residual(batch, us)


@pytest.mark.slow
def test_c5_workload():
    """The 64-problem batched workload at full size (26.3M nodes, orders U{1..7}^3): six
    FP32 batched RK3 steps and six FP64 per-problem steps at dt = 1e-4, checked against
    the oracle on the two smallest problems and, on every problem, FP32 against FP64;
    then the FP64 estimate (promotion, fine residual, isolated sweep) of the FP32 state
    against the oracle on eight problems spread across sizes."""
    probs = wl.c5()
    plans, u0 = [], []
    for mesh, orders, centre, sigma in probs:
        p = dg.Plan(mesh, orders)
        plans.append(p)
        u0.append(wl.pulse_state(p.to_natural(p.node_coords(), nv=3), orders, centre=centre, sigma=sigma))
    batch = dg.Batch(plans, dtype=torch.float32)
    u32 = [p.to_plan(u, dtype=torch.float32) for p, u in zip(plans, u0)]
    g32 = [torch.empty_like(u) for u in u32]
    u64 = [p.to_plan(u) for p, u in zip(plans, u0)]
    g64 = [torch.empty_like(u) for u in u64]
    dt, n = 1e-4, 6
    dg.batch_rk3_step(batch, u32, g32, dt, n)
    for p, u, g in zip(plans, u64, g64):
        dg.rk3_step(p, u, g, dt, n)
    for i in np.argsort([p.n_nodes for p in plans])[:2]:
        mesh, orders, _, _ = probs[i]
        ref = oracle.rk3(mesh, orders, u0[i], dt, n)
        s = np.max(np.abs(ref))
        assert np.max(np.abs(plans[i].to_natural(u64[i]) - ref)) < 1e-12 * s
        assert np.max(np.abs(plans[i].to_natural(u32[i]).astype(np.float64) - ref)) < 1e-5 * s
    for a, b in zip(u32, u64):
        assert float((a.double() - b).abs().max()) < 1e-5 * float(b.abs().max())
    # FP64 estimate of the FP32-stepped batch on eight problems spread across sizes
    w = dg.batch_to_f64(batch, u32)
    maps = dg.batch_tau_sweep(batch, w)
    sizes = np.argsort([p.n_nodes for p in plans])
    for i in sizes[np.linspace(0, len(plans) - 1, 8).astype(int)]:
        mesh, orders, _, _ = probs[i]
        un = plans[i].to_natural(w[i])
        ten_r, tet_r, _ = oracle.sweep(mesh, orders, un, oracle.residual(mesh, orders, un))
        sn, st = sweep_scale(mesh, orders, un)
        assert np.max(np.abs(_sweep_nat(plans[i], maps[i][0]) - ten_r)) < 1e-12 * max(np.max(np.abs(ten_r)), sn)
        assert np.max(np.abs(_sweep_nat(plans[i], maps[i][1]) - tet_r)) < 1e-12 * max(np.max(np.abs(tet_r)), st)
