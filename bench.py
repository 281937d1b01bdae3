"""Benchmark of the batched SF on one MI355X.

One step = one batched forward (sf_project, L* iterations, checkpoints saved)
plus the adjoint (sf_project_backward) over the whole batch: every step of the
hot path.  The checkpoint interval k is chosen from the device memory: every
iterate is kept when the history fits in a quarter of the free HBM (the
adjoint then recomputes nothing), else the smallest k that fits; a workload
that specifies k uses it.  The rate at k = 10 is reported beside it.  Default workload: 64 independent problems of 32 robots and 20
obstacles (12 m arena, 11 Bernstein coefficients per axis, 100 time steps),
run for L* iterations, the smallest multiple of 10 at which every problem's
FP64-oracle residual is <= 1e-3, capped at 2000 (determined offline by
oracle/lstar.py; at the cap the fraction of outputs at or below 1e-3 is
reported beside the rate, which counts every problem of the batch).

Prints one JSON line.  Extra fields: the forward-only rate, the plain
per-problem path's forward rate (one problem per launch group, per-stage
kernels) and the batched/plain ratio, the batched-but-unfused forward rate (the
same per-stage kernels, each launch over the whole batch) so that the gain can
be attributed to batching and to fusion, the plan setup time (host FP64
factors and workspace tables), the residual check on the GPU outputs, the
candidate-selection pipeline around the SF on the 32-candidate context, the
3D (spheroid) forward on 64 problems of 32 robots, the other workloads at
their own L* (configs: single-problem latency, the 32-candidate batch, the
uneven batch through graph replays, the large batch with its checkpoint
interval of 10, each with batched forward and forward + adjoint rates, the
plain per-problem forward rate on a sample and the roofline), the roofline of
the dominant kernel (against the published FP32 vector peak and the scalar
FP32 peak) and the FP64 oracle timed on one host core and on all available
cores (one process per problem), with the host CPU model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SF problems/s (fwd, fwd+bwd) at 32 robots, residual≤1e-3; batched vs plain"
RHO = 0.5
# L* per workload at rho = 0.5 (oracle/lstar.py on every problem of c1-c4 and a
# sample of c5; the runs are recorded in the design doc)
LSTAR = {1: 100, 2: 560, 3: 2000, 4: 2000, 5: 2000}
CKPT_SPECIFIED = {5: 10}     # workloads whose description fixes the checkpoint interval
CKPT_REFERENCE = 10


def choose_checkpoint_interval(L, coef_total, free_bytes, budget_frac=0.25):
    """Smallest k whose checkpoint area (ceil(L/k) iterates of 2 coefficient
    arrays, FP32) fits in budget_frac of the free device memory."""
    per_iterate = 2 * coef_total * 4
    budget = budget_frac * free_bytes
    k = 1
    while k < max(L, 1) and -(-L // k) * per_iterate > budget:
        k += 1
    return k
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz; FMA = 2 flops.  Packed FP32
# is disabled in this build, so scalar FP32 FMA is the attainable ceiling.
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12          # 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3


def algorithmic_flops(problems, T, nc, L, kind):
    """Data-independent algorithmic flop count of one launch (FMA = 2):
    distance tests of every unordered robot pair and robot-obstacle pair per
    step (6 flops), box residuals (4 per coordinate), the coefficient<->time maps
    (2 n_d n T nc FMAs each), the mode products on coefficients (2 n_d n nc^2
    FMAs each) and ~10 flops per coefficient of elementwise work.  Work on active
    constraints (data dependent, a small fraction) is not counted."""
    tot = 0.0
    for p in problems:
        n, M = p.n, p.M
        Sc = 2 * n * nc
        tests = 6.0 * (n * (n - 1) / 2 + n * M) * T + 4.0 * 2 * n * T
        maps = 2.0 * 2 * n * T * nc
        modes = 2.0 * Sc * nc
        if kind == "fwd":
            per_it = tests + 2 * maps + 2 * modes + 10.0 * Sc
            tot += per_it * L + tests + maps          # + residual of the returned iterate
        else:
            per_it = tests + 3 * maps + 2 * modes + 10.0 * Sc
            tot += per_it * L
    return tot


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known
    size), or None when there is none or the library sources have changed since
    the counters were taken."""
    from paper_2510_09204_amd.build import source_digest
    path = os.path.join(ROOT, "profiles", f"sf_fused_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith(("source-digest", "traffic-bytes")):
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source-digest") != source_digest():
        return None
    v = vals.get(f"traffic-bytes {kernel}")
    return int(v) if v else None


def _oracle_times(problem, budget_s):
    """Seconds per forward iteration and per forward+adjoint iteration of the
    FP64 oracle on one problem, on one thread: forward iterations for about
    half the budget, then an adjoint (forward + reverse sweep) sized to about a
    quarter of it.  Returns (t_fwd, n_fwd, t_fwd_bwd, n_fwd_bwd)."""
    from threadpoolctl import threadpool_limits

    from oracle import SFAdjoint, SFOracle
    with threadpool_limits(limits=1):
        orc = SFOracle.for_problem(problem, RHO)
        t0 = time.perf_counter()
        n_f = 0
        xib, lam = orc.flat(problem.xi), np.zeros(problem.xi.size)
        xi = orc.flat(problem.xi)
        while time.perf_counter() - t0 < budget_s / 2:
            xib, lam, _, _ = orc.step(xi, xib, lam)
            n_f += 1
        t_f = (time.perf_counter() - t0) / n_f
        n_b = max(5, int(0.25 * budget_s / (3 * t_f)))
        g = np.ones(problem.xi.shape)
        t1 = time.perf_counter()
        SFAdjoint(orc).gradient(problem.xi, problem.xi, None, n_b, g, np.zeros_like(g))
        t_fb = (time.perf_counter() - t1) / n_b
    return t_f, n_f, t_fb, n_b


def _pool_worker(job):
    problem, budget_s = job
    return _oracle_times(problem, budget_s)


def cpu_pool_rates(problems, L, budget_s=8.0):
    """The same oracle timing on every available host core at once (at most
    16), one process per core, each on its own problem of the workload;
    aggregate problems/s at L iterations.  Run before the GPU is touched (the
    workers are forked)."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(problems[w % len(problems)], budget_s) for w in range(workers)]
    # close + join (not terminate) so that no pool thread outlives the call:
    # a lingering handler thread competes for the interpreter lock with the
    # host side of the later GPU timings
    pool = mp.get_context("fork").Pool(workers)
    try:
        times = pool.map(_pool_worker, jobs)
    finally:
        pool.close()
        pool.join()
    return dict(value=sum(1.0 / (t[2] * L) for t in times), unit="problems/s",
                cores=workers, fwd_value=sum(1.0 / (t[0] * L) for t in times),
                sample=f"{workers} problems, one per process, each timed as the one-core "
                       f"sample with a {budget_s:g} s budget")


def cpu_baseline(problem, L, budget_s=20.0, pool=None):
    """The FP64 oracle on one problem of the workload, on one host core,
    scaled to problems/s at L iterations; `pool` (the all-cores rate) is
    attached when given."""
    t_f, n_f, t_fb, n_b = _oracle_times(problem, budget_s)
    out = dict(value=1.0 / (t_fb * L), unit="problems/s", cores=1, kind="oracle",
               sample=f"1 problem ({problem.n} robots, {problem.M} obstacles): {n_f} forward "
                      f"iterations ({t_f * 1e3:.1f} ms each) and a {n_b}-iteration forward+"
                      f"adjoint ({t_fb * 1e3:.1f} ms per iteration), scaled to {L} iterations",
               fwd_value=1.0 / (t_f * L))
    if pool is not None:
        out["all_cores"] = pool
    return out


def candidate_pipeline_timing(dev, steps=5):
    """The planning pipeline around the SF on the 32-candidate, 16-robot
    context (raw ranking, SF refinement of the best 10 for that workload's
    L*, choice by feasibility and smoothness), plans built once; ms per
    pipeline from HIP events on the stream."""
    import torch

    from paper_2510_09204_amd import select_candidates
    from workloads import WORKLOADS, make_batch, pack
    probs = make_batch(WORKLOADS[2])
    p0, pk = probs[0], pack(probs)
    xi = torch.from_numpy(pk.xi).to(dev)
    bnd = torch.from_numpy(pk.boundary[:p0.n * 4].copy()).to(dev)
    obs = torch.from_numpy(pk.obstacles[:p0.M * 3].copy()).to(dev)
    k, L = 10, LSTAR[2]
    args = (xi, p0.n, p0.M, float(pk.robot_a[0]), pk.box[0], bnd, obs, p0.n_coef,
            p0.n_steps, RHO, k, L, 1e-3, 5.0)
    out = select_candidates(*args)
    plans = out["plans"]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = select_candidates(*args, plans=plans)
    e1.record(stream)
    torch.cuda.synchronize()
    res = out["residual_refined"].cpu().numpy()
    best = int(out["best"].cpu()[0])
    return dict(workload=f"{WORKLOADS[2].name}: 32 candidates -> top {k} -> SF {L} iterations -> "
                         "best by feasibility and smoothness",
                ms=round(e0.elapsed_time(e1) / steps, 4),
                threads=[int(pl.threads) for pl in plans],
                chosen=int(out["topk"].cpu()[best]),
                chosen_residual=float(np.hypot(res[best, 0], res[best, 1])),
                chosen_cost=float(out["cost"].cpu()[best]))


def roofline_of(kernel, flops, ms):
    """Roofline object of one kernel launch: algorithmic flops over its
    measured duration against the published FP32 vector peak, and against the
    scalar (unpacked) FP32 peak that this build's instruction mix can reach."""
    ach = flops / (ms / 1e3) / 1e12
    return dict(bound="alu", kernel=kernel, achieved=round(ach, 3),
                peak=PEAK_FP32_PACKED_TFLOPS, unit="TFLOP/s",
                frac=round(ach / PEAK_FP32_PACKED_TFLOPS, 4),
                frac_vs_unpacked_fp32_peak=round(ach / PEAK_ALU_TFLOPS, 4))


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def config_rates(cfg_id, dev, steps=3, graph=False, plain_sample=2):
    """One workload at its L*: the batched fused forward (through SF_GRAPH
    replays on a side stream when `graph`), the batched forward + adjoint
    (checkpoint interval as in the headline step), the plain per-problem
    forward on the first `plain_sample` problems (a host loop of one-problem
    launch groups, so its rate is per problem), the roofline of the dominant
    kernel and the fraction of outputs at residual <= 1e-3.  Times from HIP
    events on the launch stream; problems/s = batch / time."""
    import torch

    from paper_2510_09204_amd import SFPlan, to_device
    from workloads import WORKLOADS, make_batch, pack
    cfg = WORKLOADS[cfg_id]
    L = LSTAR[cfg_id]
    probs = make_batch(cfg)
    pk = pack(probs)
    B = len(probs)
    ckpt = CKPT_SPECIFIED.get(cfg_id) or choose_checkpoint_interval(
        L, int(pk.xi.size), torch.cuda.mem_get_info(dev)[0])
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, pk.n_coef, pk.n_steps, RHO,
                  checkpoint_every=ckpt, max_iters=L, device=dev)
    t = to_device(pk, dev)
    args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"])
    stream = torch.cuda.Stream(dev) if graph else torch.cuda.current_stream(dev)
    outs = (torch.empty_like(t["xi"]), torch.empty_like(t["xi"]),
            torch.empty((B, 4), dtype=torch.float32, device=dev))
    g_out = torch.ones_like(t["xi"])
    with torch.cuda.stream(stream):
        plan.project(*args, L, graph=graph, out=outs)           # tunes; captures the graph
        plan.project(*args, L, save=True)
        plan.backward(g_out, None, None)
        torch.cuda.synchronize()
        e = _events(2)
        e[0].record(stream)
        for _ in range(steps):
            plan.project(*args, L, graph=graph, out=outs)
        e[1].record(stream)
        torch.cuda.synchronize()
        fwd_ms = e[0].elapsed_time(e[1]) / steps
        res = outs[2].cpu().numpy()
        ev = [_events(3) for _ in range(steps)]
        for q in range(steps):
            ev[q][0].record(stream)
            plan.project(*args, L, save=True)
            ev[q][1].record(stream)
            plan.backward(g_out, None, None)
            ev[q][2].record(stream)
        torch.cuda.synchronize()
    f_ms = float(np.mean([x[0].elapsed_time(x[1]) for x in ev]))
    b_ms = float(np.mean([x[1].elapsed_time(x[2]) for x in ev]))
    sub = probs[:max(1, min(plain_sample, B))]
    spk = pack(sub)
    splan = SFPlan(spk.n_robots, spk.n_obs, spk.robot_a, spk.box, spk.n_coef, spk.n_steps, RHO,
                   device=dev)
    st = to_device(spk, dev)
    sargs = (st["xi"], st["xi0"], st["lam0"], st["boundary"], st["obstacles"])
    splan.project(*sargs, 1, plain=True)
    e = _events(2)
    cur = torch.cuda.current_stream(dev)
    e[0].record(cur)
    splan.project(*sargs, L, plain=True)
    e[1].record(cur)
    torch.cuda.synchronize()
    plain_ms = e[0].elapsed_time(e[1])
    plain_rate = len(sub) / (plain_ms / 1e3)
    nc, T = pk.n_coef, pk.n_steps
    f_fwd = algorithmic_flops(probs, T, nc, L, "fwd")
    f_bwd = algorithmic_flops(probs, T, nc, L, "bwd")
    dom = ("sf_bwd_fused", f_bwd, b_ms) if b_ms >= f_ms else ("sf_fwd_fused", f_fwd, f_ms)
    r = np.hypot(res[:, 0], res[:, 1])
    fwd_rate = B / (fwd_ms / 1e3)
    out = dict(workload=f"{cfg.name}: {cfg.description}", batch=B,
               robots=[int(pk.n_robots.min()), int(pk.n_robots.max())],
               obstacles=[int(pk.n_obs.min()), int(pk.n_obs.max())], n_coef=nc, n_steps=T,
               iters=L, checkpoint_every=ckpt, graph=graph, threads_fwd=plan.threads,
               fwd_ms=round(fwd_ms, 4), fwd_problems_per_s=round(fwd_rate, 2),
               fwd_bwd_ms=round(f_ms + b_ms, 4),
               fwd_bwd_problems_per_s=round(B / ((f_ms + b_ms) / 1e3), 2),
               plain_fwd_problems_per_s=round(plain_rate, 3),
               plain_sample=f"first {len(sub)} problem(s), {L} iterations, one launch group each",
               batched_over_plain_fwd=round(fwd_rate / plain_rate, 2),
               batched_fwd_bwd_over_plain_fwd=round(B / ((f_ms + b_ms) / 1e3) / plain_rate, 2),
               frac_residual_le_tol=float(np.mean(r <= 1e-3)),
               residual_median=float(np.median(r)), status_nonzero=int(np.sum(res[:, 3] != 0)),
               roofline=dict(roofline_of(dom[0], dom[1], dom[2]),
                             kernels={"sf_fwd_fused": dict(ms=round(f_ms, 4), tflops=round(
                                 f_fwd / f_ms / 1e9, 3)),
                                      "sf_bwd_fused": dict(ms=round(b_ms, 4), tflops=round(
                                          f_bwd / b_ms / 1e9, 3))}))
    if B == 1:
        out["latency_ms"] = dict(fwd=round(fwd_ms, 4), fwd_bwd=round(f_ms + b_ms, 4),
                                 plain_fwd=round(plain_ms, 4))
    if graph and B > 1:
        # the costliest problem alone (same thread count, same graph path):
        # with no more problems than compute units every block has a CU of
        # its own, so the batch takes about as long as its largest problem
        cost = [T * (0.5 * p.n * (p.n - 1) + p.n * p.M + p.n) + 4.0 * p.n * nc * nc
                for p in probs]
        big = probs[int(np.argmax(cost))]
        bpk = pack([big])
        bplan = SFPlan(bpk.n_robots, bpk.n_obs, bpk.robot_a, bpk.box, bpk.n_coef, bpk.n_steps,
                       RHO, threads=plan.threads, device=dev)
        bt = to_device(bpk, dev)
        bargs = (bt["xi"], bt["xi0"], bt["lam0"], bt["boundary"], bt["obstacles"])
        bouts = (torch.empty_like(bt["xi"]), torch.empty_like(bt["xi"]),
                 torch.empty((1, 4), dtype=torch.float32, device=dev))
        with torch.cuda.stream(stream):
            bplan.project(*bargs, L, graph=True, out=bouts)
            torch.cuda.synchronize()
            e = _events(2)
            e[0].record(stream)
            for _ in range(steps):
                bplan.project(*bargs, L, graph=True, out=bouts)
            e[1].record(stream)
            torch.cuda.synchronize()
        big_ms = e[0].elapsed_time(e[1]) / steps
        out["largest_alone"] = dict(robots=int(big.n), obstacles=int(big.M),
                                    fwd_ms=round(big_ms, 4),
                                    batch_over_largest=round(fwd_ms / big_ms, 3))
        bplan.close()
    plan.close()
    splan.close()
    return out


def uneven_scaling(dev, L=500, sizes=(48, 256, 1024)):
    """Uneven batches of the c4 recipe (robots U{8..64}) at growing batch
    size, one fused forward launch each (1024 threads, L iterations): with no
    more problems than compute units the batch takes about as long as its
    largest problem; beyond, the time grows with the work."""
    import torch

    from paper_2510_09204_amd import SFPlan, to_device
    from workloads import WORKLOADS, make_batch, pack
    rows = []
    for B in sizes:
        probs = make_batch(WORKLOADS[4], batch=B)
        pk = pack(probs)
        plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, pk.n_coef, pk.n_steps, RHO,
                      threads=1024, device=dev)
        t = to_device(pk, dev)
        args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
        plan.project(*args)
        torch.cuda.synchronize()
        e = _events(2)
        e[0].record(torch.cuda.current_stream(dev))
        plan.project(*args)
        e[1].record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1])
        rows.append(dict(batch=B, ms=round(ms, 3), problems_per_s=round(B / (ms / 1e3), 1),
                         robots_max=int(pk.n_robots.max())))
        plan.close()
    for r in rows:
        r["time_over_smallest_batch"] = round(r["ms"] / rows[0]["ms"], 3)
    return dict(workload="c4 recipe, robots U{8..64}, obstacles U{0..30}", iters=L, threads=1024,
                runs=rows)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def algorithmic_flops3d(problems, T, nc, L, kind="fwd"):
    """algorithmic_flops for the 3D (spheroid) SF: a distance test costs 8
    flops per unordered robot pair and robot-obstacle pair per step, box
    residuals 4 per coordinate, the maps and mode products run over three
    axes; the adjoint counts the tests, three maps and two mode products per
    iteration (its recompute excluded)."""
    tot = 0.0
    for p in problems:
        n, M = p.n, p.M
        Sc = 3 * n * nc
        tests = 8.0 * (n * (n - 1) / 2 + n * M) * T + 4.0 * 3 * n * T
        maps = 2.0 * 3 * n * T * nc
        modes = 2.0 * Sc * nc
        if kind == "fwd":
            tot += (tests + 2 * maps + 2 * modes + 10.0 * Sc) * L + tests + maps
        else:
            tot += (tests + 3 * maps + 2 * modes + 10.0 * Sc) * L
    return tot


def spheroid_3d_timing(dev, steps=5):
    """The 3D (spheroid) forward on 64 problems of 32 robots and 20 obstacles
    (sf_setup with n_dim = 3), for the workload's iteration count and 10x
    that; ms per launch from HIP events on the stream."""
    import torch

    from paper_2510_09204_amd import SFPlan
    from workloads.gen3d import WORKLOADS_3D, make_batch3d, pack3d
    cfg = WORKLOADS_3D[32]
    probs = make_batch3d(cfg)
    pk = pack3d(probs)
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_ab, pk.box, pk.n_coef, pk.n_steps, RHO,
                  n_dim=3, device=dev)
    t = {k: torch.from_numpy(getattr(pk, k)).to(dev) for k in ("xi", "xi0", "lam0",
                                                                "boundary", "obstacles")}
    stream = torch.cuda.current_stream(dev)
    out = {"candidate_lists": plan.set_candidate_lists(True)}

    def fwd_ms(args):
        plan.project(*args)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            res = plan.project(*args)[2]
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, res

    for L in (cfg.iters, 10 * cfg.iters):
        args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
        if L == cfg.iters:
            # every pair and obstacle visited at every step (same bits)
            plan.set_candidate_lists(False)
            full_ms = fwd_ms(args)[0]
            plan.set_candidate_lists(True)
            out[f"L{L}_full_sweep_ms"] = round(full_ms, 4)
        ms, res = fwd_ms(args)
        r = np.hypot(res[:, 0].cpu().numpy(), res[:, 1].cpu().numpy())
        out[f"L{L}"] = dict(ms=round(ms, 4), problems_per_s=round(len(probs) / (ms / 1e3), 2),
                            us_per_iter=round(ms * 1e3 / L, 3),
                            residual_median=float(np.median(r)),
                            frac_residual_le_tol=float(np.mean(r <= 1e-3)),
                            status_nonzero=int(np.sum(res[:, 3].cpu().numpy() != 0)),
                            roofline=roofline_of(
                                "fwd3_kernel", algorithmic_flops3d(probs, pk.n_steps, pk.n_coef, L),
                                ms))
    # the plain per-problem forward (each stage its own launch, the state in
    # the workspace) on the first two problems, one launch group each
    L = cfg.iters
    sub = probs[:2]
    spk = pack3d(sub)
    splan = SFPlan(spk.n_robots, spk.n_obs, spk.robot_ab, spk.box, spk.n_coef, spk.n_steps, RHO,
                   n_dim=3, device=dev)
    st = {k: torch.from_numpy(getattr(spk, k)).to(dev) for k in ("xi", "xi0", "lam0",
                                                                  "boundary", "obstacles")}
    sargs = (st["xi"], st["xi0"], st["lam0"], st["boundary"], st["obstacles"])
    splan.project(*sargs, 1, plain=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    splan.project(*sargs, L, plain=True)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    splan.close()
    plain_rate = len(sub) / (plain_ms / 1e3)
    out["plain"] = dict(sample=f"first {len(sub)} problems, {L} iterations, one launch group each",
                        ms=round(plain_ms, 4), fwd_problems_per_s=round(plain_rate, 2),
                        batched_over_plain_fwd=round(out[f"L{L}"]["problems_per_s"] / plain_rate,
                                                     2))
    # forward + adjoint at the workload's iteration count, every iterate kept
    planb = SFPlan(pk.n_robots, pk.n_obs, pk.robot_ab, pk.box, pk.n_coef, pk.n_steps, RHO,
                   n_dim=3, max_iters=L, checkpoint_every=1, device=dev)
    args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
    g_out = torch.ones_like(t["xi"])

    def fwd_bwd_ms():
        planb.project(*args, save=True)
        planb.backward(g_out, None, None)
        torch.cuda.synchronize()
        ev = [_events(3) for _ in range(steps)]
        for q in range(steps):
            ev[q][0].record(stream)
            planb.project(*args, save=True)
            ev[q][1].record(stream)
            planb.backward(g_out, None, None)
            ev[q][2].record(stream)
        torch.cuda.synchronize()
        return (float(np.mean([x[0].elapsed_time(x[1]) for x in ev])),
                float(np.mean([x[1].elapsed_time(x[2]) for x in ev])))

    planb.set_candidate_lists(False)
    full_f, full_b = fwd_bwd_ms()
    planb.set_candidate_lists(True)
    f_ms, b_ms = fwd_bwd_ms()
    out[f"L{L}_fwd_bwd"] = dict(
        candidate_lists=planb.set_candidate_lists(True), full_sweep_fwd_ms=round(full_f, 4),
        full_sweep_bwd_ms=round(full_b, 4), fwd_ms=round(f_ms, 4), bwd_ms=round(b_ms, 4),
        problems_per_s=round(len(probs) / ((f_ms + b_ms) / 1e3), 2),
        roofline=roofline_of("bwd3_kernel",
                             algorithmic_flops3d(probs, pk.n_steps, pk.n_coef, L, "bwd"), b_ms))
    planb.close()
    return dict(workload=f"{cfg.name}: {cfg.description}", batch=len(probs),
                robots=int(pk.n_robots.max()), obstacles=int(pk.n_obs.max()),
                n_coef=pk.n_coef, n_steps=pk.n_steps, threads=plan.threads, **out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--ckpt", type=int, default=0, help="checkpoint interval (0 = from memory)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (c1, c2, c4, c5)")
    ap.add_argument("--no-ref", action="store_true",
                    help="skip the rate at the reference checkpoint interval")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-pool-budget", type=float, default=8.0,
                    help="seconds per process of the all-cores oracle timing (0 = skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--spheroid-3d-only", action="store_true",
                    help="only time the 3D (spheroid) forward and print its JSON object")
    ap.add_argument("--configs-only", type=str, default=None, metavar="IDS",
                    help="only time the listed workloads (e.g. 1,2,4,5) at their L* and print "
                         "one JSON object per workload")
    a = ap.parse_args(argv)
    if a.configs_only:
        import torch
        from paper_2510_09204_amd import load_library
        load_library()
        for c in (int(x) for x in a.configs_only.split(",")):
            t0 = time.perf_counter()
            out = config_rates(c, torch.device("cuda:0"), steps=2 if c == 5 else 3,
                               graph=(c == 4), plain_sample=1 if c == 5 else 2)
            out["wall_s"] = round(time.perf_counter() - t0, 2)
            print(json.dumps({f"c{c}": out}), flush=True)
        return 0
    if a.spheroid_3d_only:
        import torch
        from paper_2510_09204_amd import load_library
        load_library()
        print(json.dumps(spheroid_3d_timing(torch.device("cuda:0"), steps=a.steps)), flush=True)
        return 0
    if a.copy_probe:
        import torch
        # the last kernel of the run is the calibration copy: an elementwise
        # shader kernel that reads MIB MiB and writes MIB MiB
        src = torch.ones(a.copy_probe * (1 << 18), dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_probe_bytes=src.numel() * 4)))
        return 0
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for {a.gpus}); "
              "the problems of a batch are independent, so a multi-GPU run would shard "
              "them across GPUs without communication.", file=sys.stderr)
        return 2

    from workloads import WORKLOADS, make_batch, pack

    cfg = WORKLOADS[a.config]
    L = a.iters if a.iters is not None else LSTAR[a.config]
    probs = make_batch(cfg)
    pool = None
    if not a.no_cpu and a.cpu_pool_budget > 0:
        pool = cpu_pool_rates(probs, L, a.cpu_pool_budget)

    import torch

    from paper_2510_09204_amd import SFPlan, load_library, to_device

    load_library()
    dev = torch.device("cuda:0")
    pk = pack(probs)
    B = len(probs)
    torch.cuda.synchronize()
    if a.ckpt:
        ckpt = a.ckpt
    elif a.config in CKPT_SPECIFIED:
        ckpt = CKPT_SPECIFIED[a.config]
    else:
        ckpt = choose_checkpoint_interval(L, int(pk.xi.size), torch.cuda.mem_get_info(dev)[0])
    t_setup = time.perf_counter()
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, pk.n_coef, pk.n_steps, RHO,
                  checkpoint_every=ckpt, max_iters=L, threads=a.threads, device=dev)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    t = to_device(pk, dev)
    args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"])
    g_out = torch.ones_like(t["xi"])
    g_res = torch.zeros((B, 4), dtype=torch.float32, device=dev)
    g_res[:, 0] = 1.0
    g_res[:, 1] = 1.0
    stream = torch.cuda.current_stream(dev)

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        xo, lo, res = plan.project(*args, L, save=True)
        if evs is not None:
            evs[1].record(stream)
        g = plan.backward(g_out, None, g_res)
        if evs is not None:
            evs[2].record(stream)
        return xo, lo, res, g

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    kev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        out = step(kev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in kev]))
    bwd_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in kev]))
    ms_per_step = wall * 1e3 / a.steps
    res = out[2].cpu().numpy()
    resid = np.hypot(res[:, 0], res[:, 1])

    # forward only
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.project(*args, L)
    e0.record(stream)
    for _ in range(a.steps):
        plan.project(*args, L)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_only_ms = e0.elapsed_time(e1) / a.steps

    # the selection pipeline is launch-bound (small kernels from the host);
    # timed after the plain runs (hundreds of thousands of launches) it read
    # 12 ms against 3.9 ms alone in a fresh process, so it goes first
    pipeline = None if a.no_plain else candidate_pipeline_timing(dev)

    unfused = None
    if not a.no_plain:
        e0.record(stream)
        xu, lu, ru = plan.project(*args, L, unfused=True)
        e1.record(stream)
        torch.cuda.synchronize()
        unfused_ms = e0.elapsed_time(e1)
        unfused = dict(ms=unfused_ms, problems_per_s=B / (unfused_ms / 1e3),
                       max_abs_diff_vs_batched=float((xu - out[0]).abs().max().item()))

    # the same step with checkpoints every CKPT_REFERENCE iterates (recompute in the adjoint)
    ref_rate = None
    if ckpt != CKPT_REFERENCE and not a.no_ref:
        plan_k = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, pk.n_coef, pk.n_steps, RHO,
                        checkpoint_every=CKPT_REFERENCE, max_iters=L, threads=a.threads,
                        device=dev)
        plan_k.project(*args, L, save=True)
        plan_k.backward(g_out, None, g_res)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            plan_k.project(*args, L, save=True)
            plan_k.backward(g_out, None, g_res)
        torch.cuda.synchronize()
        ref_rate = B / ((time.perf_counter() - t0) / a.steps)
        plan_k.close()

    plain = None
    if not a.no_plain:
        e0.record(stream)
        xp, lp, rp = plan.project(*args, L, plain=True)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        plain = dict(ms=plain_ms, problems_per_s=B / (plain_ms / 1e3),
                     max_abs_diff_vs_batched=float((xp - out[0]).abs().max().item()))

    nc, T = pk.n_coef, pk.n_steps
    f_fwd = algorithmic_flops(probs, T, nc, L, "fwd")
    f_bwd = algorithmic_flops(probs, T, nc, L, "bwd")
    dom = ("sf_bwd_fused", f_bwd, bwd_ms) if bwd_ms >= fwd_ms else ("sf_fwd_fused", f_fwd, fwd_ms)
    roofline = roofline_of(*dom)
    roofline["traffic"] = measured_traffic(f"c{a.config}", dom[0])
    roofline["kernels"] = {"sf_fwd_fused": dict(ms=round(fwd_ms, 4),
                                                tflops=round(f_fwd / fwd_ms / 1e9, 3)),
                           "sf_bwd_fused": dict(ms=round(bwd_ms, 4),
                                                tflops=round(f_bwd / bwd_ms / 1e9, 3))}
    sph3d = None if a.no_plain else spheroid_3d_timing(dev)
    others = None
    if not a.no_configs:
        # the other workloads at their own L*: c1 latency, c2 candidates, c4 uneven
        # through graph replays, c5 with its specified checkpoint interval
        others = {f"c{c}": config_rates(c, dev, steps=2 if c == 5 else 3, graph=(c == 4),
                                        plain_sample=1 if c == 5 else 2)
                  for c in (1, 2, 4, 5) if c != a.config}
        others["uneven_scaling"] = uneven_scaling(dev)
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(probs[0], L, a.cpu_budget, pool)
        cpu["cpu_model"] = cpu_model()

    value = B / (ms_per_step / 1e3)
    line = dict(metric=METRIC, value=round(value, 2), unit="problems/s", n_gpus=1,
                steps=a.steps, warmup=a.warmup, ms_per_step=round(ms_per_step, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(workload=f"{cfg.name}: {cfg.description}", global_batch=B,
                            robots=int(pk.n_robots.max()), obstacles=int(pk.n_obs.max()),
                            n_coef=nc, n_steps=T, iters=L, rho=RHO, checkpoint_every=ckpt,
                            threads_fwd=plan.threads, residual_tol=1e-3,
                            iters_rule="L* = smallest multiple of 10 at which every FP64-oracle "
                                       "problem has residual <= 1e-3, capped at 2000; "
                                       "value counts every problem of the batch",
                            frac_residual_le_tol=float(np.mean(resid <= 1e-3))),
                fwd_problems_per_s=round(B / (fwd_only_ms / 1e3), 2),
                fwd_bwd_problems_per_s_ckpt10=None if ref_rate is None else round(ref_rate, 2),
                fwd_ms=round(fwd_only_ms, 4),
                plain_fwd_problems_per_s=None if plain is None else round(plain["problems_per_s"], 2),
                batched_over_plain_fwd=None if plain is None else
                round((B / (fwd_only_ms / 1e3)) / plain["problems_per_s"], 2),
                plain_max_abs_diff=None if plain is None else plain["max_abs_diff_vs_batched"],
                unfused_fwd_problems_per_s=None if unfused is None else
                round(unfused["problems_per_s"], 2),
                batched_over_unfused_fwd=None if unfused is None else
                round((B / (fwd_only_ms / 1e3)) / unfused["problems_per_s"], 2),
                unfused_max_abs_diff=None if unfused is None else
                unfused["max_abs_diff_vs_batched"],
                setup_ms=round(setup_ms, 2),
                residual_max=float(resid.max()), residual_median=float(np.median(resid)),
                frac_residual_le_tol=float(np.mean(resid <= 1e-3)),
                status_nonzero=int(np.sum(res[:, 3] != 0)),
                feasible_problems_per_s=round(float(np.sum(resid <= 1e-3)) /
                                              (ms_per_step / 1e3), 2),
                batched_fwd_bwd_over_plain_fwd=None if plain is None else
                round(value / plain["problems_per_s"], 2),
                candidate_pipeline=pipeline, spheroid_3d=sph3d, configs=others,
                roofline=roofline, cpu_baseline=cpu)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
