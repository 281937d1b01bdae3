"""The acceleration objective (SF_OBJECTIVE_ACCEL: the smoothness cost of the
trajectory optimiser in place of the distance to the sample) through the C
ABI, against the FP64 oracle with the same objective."""
import numpy as np
import pytest

from oracle import SFOracle
from oracle.adjoint import SFAdjoint
from sf_testlib import GRAD_REL_TOL, check_against, finish_parity, oracle_inputs, rel_err, report
from workloads import WORKLOADS, make_batch, make_problem, pack, scaled, unpack_coefs

pytestmark = pytest.mark.gpu
RHO = 0.5


def _plan(problems, L=0, ckpt=1):
    from paper_2510_09204_amd import SF_OBJECTIVE_ACCEL, SFPlan
    pk = pack(problems)
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, pk.n_coef, pk.n_steps, RHO,
                  checkpoint_every=ckpt, max_iters=L, objective=SF_OBJECTIVE_ACCEL)
    return plan, pk


def _oracle(inp):
    return SFOracle(inp["n"], inp["M"], inp["n_coef"], inp["n_steps"], RHO, inp["a"],
                    inp["box"], inp["obstacles"], inp["boundary"], objective="accel")


def _run(problems, L, plain=False):
    import torch
    from paper_2510_09204_amd import to_device
    plan, pk = _plan(problems)
    t = to_device(pk)
    xo, lo, res = plan.project(None, t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L,
                               plain=plain)
    torch.cuda.synchronize()
    return pk, xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy()


@pytest.mark.parametrize("cfg_id,batch,L", [(1, None, 100), (3, 3, 60), (4, 4, 40)])
def test_accel_objective_matches_oracle(gpu, cfg_id, batch, L):
    probs = make_batch(WORKLOADS[cfg_id], batch=batch)
    pk, xo, lo, res = _run(probs, L)
    inps = oracle_inputs(pk, probs)
    gx, gl = unpack_coefs(xo, probs), unpack_coefs(lo, probs)
    errs = []
    for b, inp in enumerate(inps):
        ref = _oracle(inp).solve(np.zeros_like(inp["xi"]), inp["xi0"], inp["lam0"], L)
        errs.append(check_against(ref, gx[b], gl[b], res[b]))
    report(f"accel c{cfg_id}", errs)
    finish_parity(errs)


def test_accel_objective_plain_path_matches_fused_bitwise(gpu):
    probs = make_batch(WORKLOADS[3], batch=3)
    _, xf, lf, _ = _run(probs, 30)
    _, xp, lp, _ = _run(probs, 30, plain=True)
    np.testing.assert_array_equal(xp, xf)
    np.testing.assert_array_equal(lp, lf)


def test_accel_objective_adjoint_matches_oracle(gpu):
    import torch
    from paper_2510_09204_amd import to_device
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0)
    probs = [make_problem(cfg, i) for i in range(2)]
    L = 20
    plan, pk = _plan(probs, L=L)
    t = to_device(pk)
    plan.project(None, t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L, save=True)
    rng = np.random.default_rng(9)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    gx = torch.from_numpy(np.concatenate([g.ravel() for g in g_xi]).astype(np.float32)).cuda()
    gl = torch.from_numpy(np.concatenate([g.ravel() for g in g_lam]).astype(np.float32)).cuda()
    g = plan.backward(gx, gl, None)
    torch.cuda.synchronize()
    out = [unpack_coefs(x.cpu().numpy(), probs) for x in g]
    inps = oracle_inputs(pk, probs)
    for b, inp in enumerate(inps):
        assert np.all(out[0][b] == 0.0)
        ref = SFAdjoint(_oracle(inp)).gradient(
            np.zeros_like(inp["xi"]), inp["xi0"], inp["lam0"], L,
            g_xi[b].astype(np.float32).astype(np.float64),
            g_lam[b].astype(np.float32).astype(np.float64))
        assert rel_err(out[1][b], ref.g_xi0) <= GRAD_REL_TOL, b
        assert rel_err(out[2][b], ref.g_lam0) <= GRAD_REL_TOL, b
