"""Per-problem early exit (sf_set_early_exit / sf_project_iterations) against
the FP64 oracle run under the same rule, forward and adjoint."""
import numpy as np
import pytest

from sf_testlib import (GRAD_REL_TOL, REL_TOL, lam_err, make_plan, oracle_early_exit, oracle_grad,
                        oracle_inputs, oracle_residual_terms, rel_err)
from workloads import WORKLOADS, make_batch, make_problem, scaled, unpack_coefs

pytestmark = pytest.mark.gpu
RHO = 0.5


def _forward(probs, L, tol, every, save=False, ckpt=1):
    import torch
    from paper_2510_09204_amd import to_device
    plan, pk = make_plan(probs, RHO, L=L if save else 0, ckpt=ckpt)
    plan.set_early_exit(tol, every)
    t = to_device(pk)
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L,
                               save=save)
    its = plan.iterations()
    torch.cuda.synchronize()
    return plan, pk, xo, lo, res.cpu().numpy(), its.cpu().numpy()


def test_early_exit_matches_oracle_rule(gpu):
    probs = make_batch(WORKLOADS[2], batch=6)
    L, tol, every = 300, 1e-3, 10
    _, pk, xo, lo, res, its = _forward(probs, L, tol, every)
    inps = oracle_inputs(pk, probs)
    gx = unpack_coefs(xo.cpu().numpy(), probs)
    gl = unpack_coefs(lo.cpu().numpy(), probs)
    stopped = 0
    for b, inp in enumerate(inps):
        n_ref, xb_ref, lam_ref, near = oracle_early_exit(inp, RHO, L, tol, every)
        if near:
            continue
        assert its[b] == n_ref, (b, its[b], n_ref)
        stopped += n_ref < L
        assert rel_err(gx[b], xb_ref) <= REL_TOL, b
        assert lam_err(gl[b], lam_ref) <= REL_TOL, b
        o1, o2 = oracle_residual_terms(inp, RHO, gx[b])
        assert abs(res[b, 0] - o1) <= 1e-5 + 1e-5 * o1 and abs(res[b, 1] - o2) <= 1e-5 + 1e-5 * o2
        assert res[b, 3] == 0.0
    assert stopped >= 1, "no problem stopped early: the case does not test the exit"


def test_iterations_without_early_exit_and_switching_off(gpu):
    probs = make_batch(WORKLOADS[2], batch=3)
    _, _, _, _, _, its = _forward(probs, 40, 1e-3, 0)
    assert (its == 40).all()
    # a tolerance every iterate meets: each problem runs exactly one iteration
    _, _, _, _, _, its = _forward(probs, 40, 1e9, 7)
    assert (its == 1).all()


def test_early_exit_rejected_with_plain_path(gpu):
    import torch
    from paper_2510_09204_amd import SFError, to_device
    probs = make_batch(WORKLOADS[2], batch=2)
    plan, pk = make_plan(probs, RHO)
    plan.set_early_exit(1e-3, 5)
    t = to_device(pk)
    with pytest.raises(SFError):
        plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], 10, plain=True)
    with pytest.raises(SFError):
        plan.set_early_exit(-1.0, 5)
    torch.cuda.synchronize()


def test_adjoint_follows_each_problems_own_chain(gpu):
    import torch
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0)
    probs = [make_problem(cfg, i) for i in range(4)]
    L, tol, every = 60, 2e-2, 4
    plan, pk, xo, lo, res, its = _forward(probs, L, tol, every, save=True, ckpt=3)
    rng = np.random.default_rng(7)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    gx = torch.from_numpy(np.concatenate([g.ravel() for g in g_xi]).astype(np.float32)).cuda()
    gl = torch.from_numpy(np.concatenate([g.ravel() for g in g_lam]).astype(np.float32)).cuda()
    grads = plan.backward(gx, gl, None, 0.05)
    torch.cuda.synchronize()
    grads = [unpack_coefs(g.cpu().numpy(), probs) for g in grads]
    inps = oracle_inputs(pk, probs)
    assert len(set(its.tolist())) >= 2, its   # problems stopped at different iterations
    for b, inp in enumerate(inps):
        n_ref, _, _, near = oracle_early_exit(inp, RHO, L, tol, every)
        assert near or its[b] == n_ref, (b, its[b], n_ref)
        ref = oracle_grad(inp, RHO, int(its[b]), g_xi[b].astype(np.float32).astype(np.float64),
                          g_lam[b].astype(np.float32).astype(np.float64), 0.0, 0.0, 0.05)
        for name, gv, rv in (("xi", grads[0][b], ref.g_xi), ("xi0", grads[1][b], ref.g_xi0),
                             ("lam0", grads[2][b], ref.g_lam0)):
            assert rel_err(gv, rv) <= GRAD_REL_TOL, (b, name)
