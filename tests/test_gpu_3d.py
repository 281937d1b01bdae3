"""The 3D (spheroid) SF forward (sf_setup with n_dim = 3, sf_project through
the C ABI) against the FP64 oracle with dim=3 on the same float32 inputs."""
import numpy as np
import pytest

from oracle import SFOracle
from sf_testlib import check_against, finish_parity, rel_err, report
from workloads import WORKLOADS, make_batch, pack, unpack_coefs
from workloads.gen3d import WORKLOADS_3D, make_batch3d, pack3d, scaled3d, unpack3d

pytestmark = pytest.mark.gpu
RHO = 0.5


def _inputs3d(pk, probs):
    xi = unpack3d(pk.xi.astype(np.float64), probs)
    xi0 = unpack3d(pk.xi0.astype(np.float64), probs)
    lam0 = unpack3d(pk.lam0.astype(np.float64), probs)
    out, r, o = [], 0, 0
    for b, p in enumerate(probs):
        out.append(dict(
            n=p.n, M=p.M, n_coef=p.n_coef, n_steps=p.n_steps,
            a=float(pk.robot_ab[b, 0]), b=float(pk.robot_ab[b, 1]),
            box=pk.box[b].astype(np.float64),
            obstacles=pk.obstacles[o * 5:(o + p.M) * 5].astype(np.float64).reshape(p.M, 5),
            boundary=pk.boundary[r * 6:(r + p.n) * 6].astype(np.float64).reshape(p.n, 2, 3),
            xi=xi[b], xi0=xi0[b], lam0=lam0[b]))
        r += p.n
        o += p.M
    return out


def _oracle(inp, objective="projection"):
    return SFOracle(inp["n"], inp["M"], inp["n_coef"], inp["n_steps"], RHO, inp["a"],
                    inp["box"], inp["obstacles"], inp["boundary"], dim=3, robot_b=inp["b"],
                    objective=objective)


def _plan(pk, threads=0, objective=0, max_iters=0, ckpt=1):
    from paper_2510_09204_amd import SFPlan
    return SFPlan(pk.n_robots, pk.n_obs, pk.robot_ab, pk.box, pk.n_coef, pk.n_steps, RHO,
                  threads=threads, n_dim=3, objective=objective, max_iters=max_iters,
                  checkpoint_every=ckpt)


def _run(probs, L, threads=0, objective=0):
    import torch
    pk = pack3d(probs)
    plan = _plan(pk, threads, objective)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    xi = None if objective else t["xi"]
    xo, lo, res = plan.project(xi, t["xi0"], t["lam0"], t["boundary"],
                               t["obstacles"] if pk.obstacles.size else None, L)
    torch.cuda.synchronize()
    return pk, xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy(), plan, t


def _compare(probs, L, objective="projection", final=True, **kw):
    pk, xo, lo, res = _run(probs, L, objective=0 if objective == "projection" else 1, **kw)[:4]
    gx, gl = unpack3d(xo, probs), unpack3d(lo, probs)
    errs = []
    for b, inp in enumerate(_inputs3d(pk, probs)):
        xi = inp["xi"] if objective == "projection" else np.zeros_like(inp["xi"])
        ref = _oracle(inp, objective).solve(xi, inp["xi0"], inp["lam0"], L)
        errs.append(check_against(ref, gx[b], gl[b], res[b]))
    report(f"3d {objective} n={probs[0].n} L={L}", errs)
    if final:
        finish_parity(errs)
    return pk, xo, lo, res, errs


@pytest.mark.parametrize("cfg_id,batch,L", [(16, 3, 60), (48, 6, 40), (32, 2, 40)])
def test_3d_matches_oracle(gpu, cfg_id, batch, L):
    _compare(make_batch3d(WORKLOADS_3D[cfg_id], batch=batch), L)


def test_3d_chunked_horizon_matches_oracle(gpu):
    """64 robots, 15 coefficients, 120 steps: the horizon runs in two LDS time
    chunks."""
    cfg = scaled3d(WORKLOADS_3D[32], n_robots=(64, 64), n_obs=(30, 30), side=16.0,
                   height=8.0, n_coef=15, n_steps=120)
    _compare(make_batch3d(cfg, batch=1), 12)


def test_3d_large_ragged_problem_matches_oracle(gpu):
    """98 robots (a ragged last group of the four-robots-per-thread stage),
    13 coefficients (a partial MFMA K step), 77 steps in three LDS time
    chunks of 26 (partial step tiles), 294 position rows (a partial row
    tile)."""
    cfg = scaled3d(WORKLOADS_3D[32], n_robots=(98, 98), n_obs=(7, 7), side=14.0, height=7.0,
                   n_coef=13, n_steps=77)
    _compare(make_batch3d(cfg, batch=1), 6)


def test_3d_single_robot_without_obstacles_and_zero_iterations(gpu):
    cfg = scaled3d(WORKLOADS_3D[16], n_robots=(1, 1), n_obs=(0, 0), side=2.0, height=1.0)
    probs = make_batch3d(cfg, batch=2)
    errs = _compare(probs, 25, final=False)[4]
    pk, xo, lo, res = _run(probs, 0)[:4]
    np.testing.assert_array_equal(xo, pk.xi0)
    np.testing.assert_array_equal(lo, pk.lam0)
    assert np.all(res[:, 2] == 0.0)
    finish_parity(errs)


def test_3d_accel_objective_matches_oracle(gpu):
    _compare(make_batch3d(WORKLOADS_3D[16], batch=2), 40, objective="accel")


def test_3d_threads_and_graph_give_the_same_bits(gpu):
    """Each output entry, and the residual norms, are summed in a fixed order
    whatever the block size; graph replays (eager work between them) repeat
    the eager bits."""
    import torch
    probs = make_batch3d(WORKLOADS_3D[48], batch=5)
    base = _run(probs, 30, threads=512)
    for th in (256, 1024):
        got = _run(probs, 30, threads=th)
        np.testing.assert_array_equal(got[1], base[1])
        np.testing.assert_array_equal(got[2], base[2])
        np.testing.assert_array_equal(got[3][:, [0, 1, 3]], base[3][:, [0, 1, 3]])
    plan, t = base[4], base[5]
    outs = (torch.empty_like(t["xi"]), torch.empty_like(t["xi"]),
            torch.empty((len(probs), 4), device=t["xi"].device))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        with torch.cuda.stream(side):
            outs[0].fill_(float("nan"))
            plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], 30,
                         graph=True, out=outs)
        side.synchronize()
        _ = (t["xi"] * 2.0).sum().item()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(outs[0].cpu().numpy(), base[1])
        np.testing.assert_array_equal(outs[2].cpu().numpy(), base[3])


def test_3d_flat_problem_matches_the_planar_gpu_path(gpu):
    """A 3D problem with every z value 0 is the planar problem: its x, y
    coefficients match the planar fused kernel's within float32 rounding."""
    import torch
    from sf_testlib import gpu_forward
    probs = make_batch(WORKLOADS[3], batch=2)
    pk2 = pack(probs)
    x2 = unpack_coefs(gpu_forward(probs, RHO, 50)["xi"], probs)
    from paper_2510_09204_amd import SFPlan
    B = len(probs)
    ab = np.stack([pk2.robot_a, np.full(B, 0.5, np.float32)], axis=1)
    box = np.concatenate([pk2.box, np.array([[[-1.0], [1.0]]] * B, np.float32)], axis=2)
    xi3 = np.concatenate([np.concatenate([p.xi.astype(np.float32), np.zeros((1, p.n, p.n_coef),
                                          np.float32)]).ravel() for p in probs])
    bnd3 = np.concatenate([np.concatenate([p.boundary.astype(np.float32),
                                           np.zeros((p.n, 2, 1), np.float32)], axis=2).ravel()
                           for p in probs])
    obs3 = np.concatenate([np.column_stack([p.obstacles[:, :2], np.zeros(p.M), p.obstacles[:, 2],
                                            np.full(p.M, 0.6)]).astype(np.float32).ravel()
                           for p in probs])
    plan = SFPlan(pk2.n_robots, pk2.n_obs, ab, box, pk2.n_coef, pk2.n_steps, RHO, n_dim=3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xo, _, res = plan.project(dev(xi3), dev(xi3), dev(np.zeros_like(xi3)), dev(bnd3), dev(obs3),
                              50)
    torch.cuda.synchronize()
    x3 = unpack3d(xo.cpu().numpy(), [type("P", (), dict(n=p.n, n_coef=p.n_coef))
                                     for p in probs])
    for b in range(B):
        assert rel_err(x3[b][:2], x2[b]) <= 2e-5, b
        assert np.max(np.abs(x3[b][2])) <= 1e-6


def test_3d_unsupported_calls_fail_loudly(gpu):
    import torch
    from paper_2510_09204_amd import SFError
    probs = make_batch3d(WORKLOADS_3D[16], batch=1)
    pk = pack3d(probs)
    plan = _plan(pk)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], 5)
    # saving needs max_iters >= L; the plain path does not save
    with pytest.raises(SFError):
        plan.project(*args, save=True)
    with pytest.raises(SFError) as e:
        plan.backward(t["xi0"], None, None)
    assert e.value.code == -4
    # the candidate-list switch is for 3D plans; planar fused kernels always use lists
    from sf_testlib import make_plan
    plan2, _ = make_plan(make_batch(WORKLOADS[1], batch=1), RHO, 0, 1, 0)
    with pytest.raises(SFError) as e:
        plan2.set_candidate_lists(False)
    assert e.value.code == -1


@pytest.mark.parametrize("cfg_id,batch,L", [(16, 3, 50), (48, 5, 40)])
def test_3d_moving_obstacles_match_oracle(gpu, cfg_id, batch, L):
    """Obstacle centres c + d tau (sf_set_obstacle_motion with [sum M][3]);
    resetting the motion restores the static result bit for bit."""
    import torch
    probs = make_batch3d(WORKLOADS_3D[cfg_id], batch=batch)
    pk = pack3d(probs)
    disp = np.random.default_rng(cfg_id).uniform(-2.0, 2.0, (int(pk.n_obs.sum()), 3))
    disp = disp.astype(np.float32)
    static = _run(probs, L)
    plan, t = static[4], static[5]
    plan.set_obstacle_motion(torch.from_numpy(disp).cuda())
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
    torch.cuda.synchronize()
    xo, lo, res = xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy()
    assert not np.array_equal(xo, static[1])
    gx, gl = unpack3d(xo, probs), unpack3d(lo, probs)
    o, errs = 0, []
    for b, inp in enumerate(_inputs3d(pk, probs)):
        d = disp[o:o + inp["M"]].astype(np.float64)
        o += inp["M"]
        ref = SFOracle(inp["n"], inp["M"], inp["n_coef"], inp["n_steps"], RHO, inp["a"],
                       inp["box"], inp["obstacles"], inp["boundary"], dim=3,
                       robot_b=inp["b"], obstacle_displacement=d).solve(
                           inp["xi"], inp["xi0"], inp["lam0"], L)
        errs.append(check_against(ref, gx[b], gl[b], res[b]))
    report("3d moving", errs)
    plan.set_obstacle_motion(None)
    back, _, _ = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back.cpu().numpy(), static[1])
    finish_parity(errs)


# ---------------------------------------------------------------- 3D adjoint
def _run_grad(probs, L, ckpt, seed, g_res=None, fp_weight=0.0, threads=0):
    import torch
    pk = pack3d(probs)
    plan = _plan(pk, threads=threads, max_iters=L, ckpt=ckpt)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"],
                               t["obstacles"] if pk.obstacles.size else None, L, save=True)
    rng = np.random.default_rng(seed)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    dev = lambda gs: torch.from_numpy(np.concatenate([g.ravel() for g in gs])
                                      .astype(np.float32)).cuda()
    gr = None if g_res is None else torch.from_numpy(g_res.astype(np.float32)).cuda()
    g = plan.backward(dev(g_xi), dev(g_lam), gr, fp_weight)
    torch.cuda.synchronize()
    return pk, [unpack3d(x.cpu().numpy(), probs) for x in g], g_xi, g_lam, res.cpu().numpy()


def _check_grad(probs, pk, grads, L, g_xi, g_lam, g_res=None, fp_weight=0.0, idx=None):
    from oracle import SFAdjoint
    from sf_testlib import GRAD_REL_TOL
    inps = _inputs3d(pk, probs)
    for b in (range(len(probs)) if idx is None else idx):
        inp = inps[b]
        gr1 = 0.0 if g_res is None else float(np.float32(g_res[b, 0]))
        gr2 = 0.0 if g_res is None else float(np.float32(g_res[b, 1]))
        ref = SFAdjoint(_oracle(inp)).gradient(
            inp["xi"], inp["xi0"], inp["lam0"], L,
            g_xi[b].astype(np.float32).astype(np.float64),
            g_lam[b].astype(np.float32).astype(np.float64), gr1, gr2, fp_weight)
        errs = {name: rel_err(gv, rv) for name, gv, rv in
                (("xi", grads[0][b], ref.g_xi), ("xi0", grads[1][b], ref.g_xi0),
                 ("lam0", grads[2][b], ref.g_lam0))}
        print(f"[grad3d] L={L} problem {b} (n={inp['n']}, M={inp['M']}): "
              + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for name, e in errs.items():
            assert e <= GRAD_REL_TOL, (b, name, e)


@pytest.mark.parametrize("cfg_id,batch,L,ckpt", [(16, 2, 30, 1), (32, 2, 25, 5),
                                                  (48, 4, 20, 3)])
def test_3d_adjoint_matches_oracle(gpu, cfg_id, batch, L, ckpt):
    """The 3D reverse sweep (sf_project_backward, n_dim = 3) against the FP64
    oracle's on the three 3D workloads, with checkpoint recompute."""
    probs = make_batch3d(WORKLOADS_3D[cfg_id], batch=batch)
    pk, grads, g_xi, g_lam, _ = _run_grad(probs, L, ckpt, seed=cfg_id)
    _check_grad(probs, pk, grads, L, g_xi, g_lam)


def test_3d_adjoint_with_residual_and_fixed_point_terms(gpu):
    cfg = scaled3d(WORKLOADS_3D[16], n_robots=(6, 6), n_obs=(4, 4), side=2.5, height=1.4)
    probs = make_batch3d(cfg, batch=2)
    g_res = np.array([[0.7, 0.4, 0.0, 0.0], [1.3, 0.6, 0.0, 0.0]])
    pk, grads, g_xi, g_lam, res = _run_grad(probs, 12, 4, seed=3, g_res=g_res, fp_weight=0.25)
    # both residual terms are exercised (pair/obstacle and box, nonzero norms)
    assert res[:, 0].max() > 1e-2 and res[:, 1].max() > 1e-2, res
    _check_grad(probs, pk, grads, 12, g_xi, g_lam, g_res, 0.25)


def test_3d_adjoint_time_chunked_horizon(gpu):
    """64 robots, 15 coefficients, 120 steps: the recompute runs the forward's
    LDS time chunks and the VJP its own shorter chunks."""
    cfg = scaled3d(WORKLOADS_3D[32], n_robots=(64, 64), n_obs=(30, 30), side=16.0,
                   height=8.0, n_coef=15, n_steps=120)
    probs = make_batch3d(cfg, batch=1)
    pk, grads, g_xi, g_lam, _ = _run_grad(probs, 8, 3, seed=5)
    _check_grad(probs, pk, grads, 8, g_xi, g_lam)


def test_3d_adjoint_checkpoint_interval_and_threads_give_the_same_bits(gpu):
    probs = make_batch3d(WORKLOADS_3D[48], batch=4)
    g_res = np.tile([[0.5, 0.5, 0.0, 0.0]], (4, 1))
    ref = _run_grad(probs, 24, 1, seed=9, g_res=g_res, fp_weight=0.1, threads=1024)[1]
    for ckpt, th in ((5, 1024), (24, 1024), (5, 256)):
        got = _run_grad(probs, 24, ckpt, seed=9, g_res=g_res, fp_weight=0.1, threads=th)[1]
        for q in range(3):
            for b in range(4):
                np.testing.assert_array_equal(got[q][b], ref[q][b])


def test_3d_autograd_function(gpu):
    """SFProject on a 3D plan: the loss sum ||xi_bar^L - straight||^2 + ||r_1||^2
    through the library's forward and adjoint against the oracle's gradient."""
    import torch
    from oracle import SFAdjoint
    from paper_2510_09204_amd import SFProject
    from sf_testlib import GRAD_REL_TOL
    cfg = scaled3d(WORKLOADS_3D[16], n_robots=(5, 5), n_obs=(3, 3), side=3.0, height=1.6)
    probs = make_batch3d(cfg, batch=2)
    pk = pack3d(probs)
    L = 15
    plan = _plan(pk, max_iters=L, ckpt=4)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    straight = torch.from_numpy(np.concatenate([p.straight.ravel() for p in probs])
                                .astype(np.float32)).cuda()
    xi = t["xi"].clone().requires_grad_(True)
    xi0 = t["xi0"].clone().requires_grad_(True)
    xo, lo, res = SFProject.apply(xi, xi0, t["lam0"], t["boundary"], t["obstacles"], plan, L)
    loss = ((xo - straight) ** 2).sum() + (res[:, 0] ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g_out = unpack3d(2.0 * (xo.detach().cpu().numpy() - straight.cpu().numpy()), probs)
    r = res.detach().cpu().numpy()
    for b, inp in enumerate(_inputs3d(pk, probs)):
        ref = SFAdjoint(_oracle(inp)).gradient(inp["xi"], inp["xi0"], inp["lam0"], L, g_out[b],
                                               np.zeros_like(g_out[b]), 2.0 * float(r[b, 0]))
        got_xi = unpack3d(xi.grad.cpu().numpy(), probs)[b]
        got_xi0 = unpack3d(xi0.grad.cpu().numpy(), probs)[b]
        assert rel_err(got_xi, ref.g_xi) <= GRAD_REL_TOL, b
        assert rel_err(got_xi0, ref.g_xi0) <= GRAD_REL_TOL, b


# ------------------------------------------------------- 3D candidate lists
def _bits(probs, L, lists, disp=None, grad=None, threads=0):
    """Forward (and with grad = (ckpt, g_res, fp_weight) the adjoint) with the
    candidate lists switched on or off; returns the outputs as numpy arrays."""
    import torch
    pk = pack3d(probs)
    plan = _plan(pk, threads=threads, max_iters=L if grad else 0, ckpt=grad[0] if grad else 1)
    assert plan.set_candidate_lists(lists) == lists
    if disp is not None:
        plan.set_obstacle_motion(torch.from_numpy(disp).cuda())
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"],
                               t["obstacles"] if pk.obstacles.size else None, L,
                               save=grad is not None)
    out = [xo, lo, res]
    if grad is not None:
        rng = np.random.default_rng(11)
        g_xi = torch.from_numpy(rng.standard_normal(pk.xi.size).astype(np.float32)).cuda()
        g_lam = torch.from_numpy(rng.standard_normal(pk.xi.size).astype(np.float32)).cuda()
        gr = torch.from_numpy(np.tile(np.array([grad[1], grad[1], 0, 0], np.float32),
                                      (len(probs), 1))).cuda()
        out += list(plan.backward(g_xi, g_lam, gr, grad[2]))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def _same_bits(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("case", ["32r", "uneven", "chunked64", "ragged98", "single"])
def test_3d_candidate_lists_give_the_same_bits(gpu, case):
    """The lists only skip rows that add exact zeros: forward outputs and
    residuals with and without them are identical, on LDS-resident and
    time-chunked horizons (chunks of a multiple of the 16-step window, a
    ragged last window), ragged robot groups and a lone robot."""
    cfg, batch, L = {
        "32r": (WORKLOADS_3D[32], 2, 60),
        "uneven": (WORKLOADS_3D[48], 6, 40),
        "chunked64": (scaled3d(WORKLOADS_3D[32], n_robots=(64, 64), n_obs=(30, 30), side=16.0,
                               height=8.0, n_coef=15, n_steps=120), 1, 12),
        "ragged98": (scaled3d(WORKLOADS_3D[32], n_robots=(98, 98), n_obs=(7, 7), side=14.0,
                              height=7.0, n_coef=13, n_steps=77), 1, 6),
        "single": (scaled3d(WORKLOADS_3D[16], n_robots=(1, 1), n_obs=(0, 0), side=2.0,
                            height=1.0), 2, 25),
    }[case]
    probs = make_batch3d(cfg, batch=batch)
    on = _bits(probs, L, True)
    off = _bits(probs, L, False)
    print(f"[lists3d] {case}: residual max {on[2][:, 0].max():.3e}, "
          f"status {on[2][:, 3].max()}", flush=True)
    _same_bits(on, off)


def test_3d_candidate_lists_with_moving_obstacles_give_the_same_bits(gpu):
    probs = make_batch3d(WORKLOADS_3D[16], batch=3)
    pk = pack3d(probs)
    disp = np.random.default_rng(16).uniform(-2.0, 2.0, (int(pk.n_obs.sum()), 3))
    disp = disp.astype(np.float32)
    _same_bits(_bits(probs, 50, True, disp=disp), _bits(probs, 50, False, disp=disp))


@pytest.mark.parametrize("case", ["uneven", "tight"])
def test_3d_adjoint_candidate_lists_give_the_same_bits(gpu, case):
    """The adjoint's recompute, residual-cotangent pass and VJP with and
    without the lists: identical gradients (checkpoint segments jump back and
    forth over iterates, so the lists are rebuilt on demand)."""
    if case == "uneven":
        probs = make_batch3d(WORKLOADS_3D[48], batch=4)
        grad = (5, 0.5, 0.1)
    else:
        cfg = scaled3d(WORKLOADS_3D[16], n_robots=(6, 6), n_obs=(4, 4), side=2.5, height=1.4)
        probs = make_batch3d(cfg, batch=2)
        grad = (4, 0.9, 0.25)
    on = _bits(probs, 24, True, grad=grad)
    off = _bits(probs, 24, False, grad=grad)
    _same_bits(on, off)


def test_3d_candidate_lists_through_skin_changes_give_the_same_bits(gpu):
    """Long runs on the 32-robot workload, long enough for the list skin to
    halve once lists last sixteen passes (and to double again where they stop
    lasting): forward over 400 iterations, adjoint over 150 with every
    iterate kept and with checkpoints every 4; outputs and gradients stay
    those of the full sweep bit for bit."""
    probs = make_batch3d(WORKLOADS_3D[32], batch=2)
    _same_bits(_bits(probs, 400, True), _bits(probs, 400, False))
    for ckpt in (1, 4):
        grad = (ckpt, 0.3, 0.05)
        _same_bits(_bits(probs, 150, True, grad=grad), _bits(probs, 150, False, grad=grad))


# ------------------------------------------------------------ 3D early exit
def _oracle_early_exit3(inp, L, tol, every, rel_margin=1e-3):
    """The 3D oracle under the rule of sf_set_early_exit: at every iteration l
    that is a multiple of `every`, if the residual of xi_bar^l is <= tol,
    iteration l is completed and the run stops.  Returns (iterations run,
    xi_bar, lambda, near) with `near` set when a tested residual lies within
    rel_margin of tol (FP32 may then decide otherwise)."""
    orc = _oracle(inp)
    xi = orc.flat(inp["xi"])
    xib, lam = orc.flat(inp["xi0"]).copy(), orc.flat(inp["lam0"]).copy()
    near = False
    for l in range(L):
        stop = False
        if l % every == 0:
            res = orc.residual_of(xib)
            near = near or abs(res - tol) <= rel_margin * tol
            stop = res <= tol
        xib, lam, _, _ = orc.step(xi, xib, lam)
        if stop:
            return l + 1, orc.shaped(xib), orc.shaped(lam), near
    return L, orc.shaped(xib), orc.shaped(lam), near


def _early3(probs, L, tol, every, save=False, ckpt=1):
    import torch
    pk = pack3d(probs)
    plan = _plan(pk, max_iters=L if save else 0, ckpt=ckpt)
    plan.set_early_exit(tol, every)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L,
                               save=save)
    its = plan.iterations()
    torch.cuda.synchronize()
    return plan, pk, xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy(), its.cpu().numpy()


def test_3d_early_exit_matches_oracle_rule(gpu):
    """Per-problem early exit on 3D plans: the iteration counts, outputs and
    residual rows against the oracle run under the same rule."""
    from sf_testlib import REL_TOL, lam_err
    probs = make_batch3d(WORKLOADS_3D[16], batch=4)
    L, tol, every = 200, 2e-2, 10
    _, pk, xo, lo, res, its = _early3(probs, L, tol, every)
    gx, gl = unpack3d(xo, probs), unpack3d(lo, probs)
    stopped, checked = 0, 0
    for b, inp in enumerate(_inputs3d(pk, probs)):
        n_ref, xb_ref, lam_ref, near = _oracle_early_exit3(inp, L, tol, every)
        print(f"[early3d] problem {b}: GPU {its[b]} iterations, oracle {n_ref}"
              f"{' (near tol)' if near else ''}", flush=True)
        if near:
            continue
        checked += 1
        assert its[b] == n_ref, (b, its[b], n_ref)
        stopped += n_ref < L
        assert rel_err(gx[b], xb_ref) <= REL_TOL, b
        assert lam_err(gl[b], lam_ref) <= REL_TOL, b
        r1, r2 = _oracle(inp).residual_terms(_oracle(inp).flat(gx[b]))[:2]
        assert abs(res[b, 0] - np.linalg.norm(r1)) <= 1e-5 + 1e-5 * np.linalg.norm(r1)
        assert abs(res[b, 1] - np.linalg.norm(r2)) <= 1e-5 + 1e-5 * np.linalg.norm(r2)
        assert res[b, 3] == 0.0
    assert checked >= 2 and stopped >= 1, (checked, stopped)
    # a tolerance every iterate meets: each problem runs exactly one iteration
    assert (_early3(probs, 40, 1e9, 7)[5] == 1).all()


def test_3d_adjoint_follows_each_problems_own_chain(gpu):
    import torch
    from oracle import SFAdjoint
    from sf_testlib import GRAD_REL_TOL
    cfg = scaled3d(WORKLOADS_3D[16], n_robots=(5, 5), n_obs=(3, 3), side=3.0, height=1.6)
    probs = make_batch3d(cfg, batch=4)
    L, tol, every = 60, 3e-2, 4
    plan, pk, xo, lo, res, its = _early3(probs, L, tol, every, save=True, ckpt=3)
    rng = np.random.default_rng(17)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    dev = lambda gs: torch.from_numpy(np.concatenate([g.ravel() for g in gs])
                                      .astype(np.float32)).cuda()
    grads = plan.backward(dev(g_xi), dev(g_lam), None, 0.05)
    torch.cuda.synchronize()
    grads = [unpack3d(g.cpu().numpy(), probs) for g in grads]
    print(f"[early3d] iterations {its.tolist()}", flush=True)
    assert len(set(its.tolist())) >= 2, its   # problems stopped at different iterations
    for b, inp in enumerate(_inputs3d(pk, probs)):
        n_ref, _, _, near = _oracle_early_exit3(inp, L, tol, every)
        assert near or its[b] == n_ref, (b, its[b], n_ref)
        ref = SFAdjoint(_oracle(inp)).gradient(
            inp["xi"], inp["xi0"], inp["lam0"], int(its[b]),
            g_xi[b].astype(np.float32).astype(np.float64),
            g_lam[b].astype(np.float32).astype(np.float64), 0.0, 0.0, 0.05)
        for name, gv, rv in (("xi", grads[0][b], ref.g_xi), ("xi0", grads[1][b], ref.g_xi0),
                             ("lam0", grads[2][b], ref.g_lam0)):
            assert rel_err(gv, rv) <= GRAD_REL_TOL, (b, name)


# --------------------------------------------------------- 3D plain path
@pytest.mark.parametrize("case", ["uneven", "chunked64", "moving"])
def test_3d_plain_and_unfused_paths_match_fused_bitwise(gpu, case):
    """SF_PLAIN (one problem per launch group) and SF_UNFUSED (each stage
    launch over the batch) run the forward's stages as separate launches with
    the state in the workspace: the same coefficients and multipliers bit for
    bit, and the residual norms (the final pass sums in the same fixed order);
    ||z' - z|| is summed over a different block size, so it matches to
    rounding."""
    import torch
    if case == "chunked64":
        cfg = scaled3d(WORKLOADS_3D[32], n_robots=(64, 64), n_obs=(30, 30), side=16.0,
                       height=8.0, n_coef=15, n_steps=120)
        probs, L = make_batch3d(cfg, batch=1), 10
    else:
        probs, L = make_batch3d(WORKLOADS_3D[48], batch=5), 25
    pk = pack3d(probs)
    plan = _plan(pk)
    if case == "moving":
        disp = np.random.default_rng(48).uniform(-2.0, 2.0, (int(pk.n_obs.sum()), 3))
        plan.set_obstacle_motion(torch.from_numpy(disp.astype(np.float32)).cuda())
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    args = (t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L)
    runs = {}
    for name, kw in (("fused", {}), ("plain", dict(plain=True)), ("unfused", dict(unfused=True))):
        xo, lo, res = plan.project(*args, **kw)
        torch.cuda.synchronize()
        runs[name] = (xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy())
    for name in ("plain", "unfused"):
        np.testing.assert_array_equal(runs[name][0], runs["fused"][0])
        np.testing.assert_array_equal(runs[name][1], runs["fused"][1])
        np.testing.assert_array_equal(runs[name][2][:, [0, 1, 3]], runs["fused"][2][:, [0, 1, 3]])
        np.testing.assert_allclose(runs[name][2][:, 2], runs["fused"][2][:, 2], rtol=1e-5,
                                   atol=1e-7)


# ------------------------------------------- 3D at the benchmark's configuration
def test_3d_bench_configuration_sampled(gpu):
    """The 3D benchmark's launch as timed: all 64 problems of 32 spheroid
    robots and 20 obstacles, 1024 threads, candidate lists, L = 100 with every
    iterate saved, then the adjoint; two sampled problems' forward outputs and
    gradients against the oracle."""
    import torch
    from oracle import SFAdjoint
    from sf_testlib import GRAD_REL_TOL
    probs = make_batch3d(WORKLOADS_3D[32])
    assert len(probs) == 64
    L, picks = 100, (0, 37)
    pk = pack3d(probs)
    plan = _plan(pk, max_iters=L, ckpt=1)
    assert plan.set_candidate_lists(True)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L,
                               save=True)
    rng = np.random.default_rng(32)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    dev = lambda gs: torch.from_numpy(np.concatenate([g.ravel() for g in gs])
                                      .astype(np.float32)).cuda()
    g = plan.backward(dev(g_xi), dev(g_lam), None)
    torch.cuda.synchronize()
    print(f"[3d bench] GPU done, oracle on problems {picks}", flush=True)
    res = res.cpu().numpy()
    assert np.all(res[:, 3] == 0.0)
    gx, gl = unpack3d(xo.cpu().numpy(), probs), unpack3d(lo.cpu().numpy(), probs)
    grads = [unpack3d(x.cpu().numpy(), probs) for x in g]
    inps = _inputs3d(pk, probs)
    errs, misses = [], []
    for b in picks:
        inp = inps[b]
        ref = _oracle(inp).solve(inp["xi"], inp["xi0"], inp["lam0"], L)
        errs.append(check_against(ref, gx[b], gl[b], res[b]))
        gref = SFAdjoint(_oracle(inp)).gradient(
            inp["xi"], inp["xi0"], inp["lam0"], L,
            g_xi[b].astype(np.float32).astype(np.float64),
            g_lam[b].astype(np.float32).astype(np.float64), 0.0, 0.0, 0.0)
        ge = {name: rel_err(gv, rv) for name, gv, rv in
              (("xi", grads[0][b], gref.g_xi), ("xi0", grads[1][b], gref.g_xi0),
               ("lam0", grads[2][b], gref.g_lam0))}
        print(f"[3d bench] problem {b}: residual {np.hypot(res[b, 0], res[b, 1]):.3e}, "
              + ", ".join(f"g_{k} {v:.2e}" for k, v in ge.items()), flush=True)
        misses += [f"problem {b} g_{k} {v:.2e}" for k, v in ge.items() if v > GRAD_REL_TOL]
    report("3d bench L=100", errs)
    assert not misses, misses
    finish_parity(errs)   # the residual bar on unconverged outputs: reported, expected
