"""Moving obstacles (sf_set_obstacle_motion: centre c + d tau) through the C
ABI against the FP64 oracle with the same motion."""
import numpy as np
import pytest

from oracle import SFOracle
from oracle.adjoint import SFAdjoint
from sf_testlib import (GRAD_REL_TOL, check_against, finish_parity, make_plan, oracle_inputs,
                        rel_err, report)
from workloads import WORKLOADS, make_batch, make_problem, pack, scaled, unpack_coefs

pytestmark = pytest.mark.gpu
RHO = 0.5


def _disp(pk, seed, scale=3.0):
    n_obs = int(pk.n_obs.sum())
    return np.random.default_rng(seed).uniform(-scale, scale, (n_obs, 2)).astype(np.float32)


def _oracle(inp, disp):
    return SFOracle(inp["n"], inp["M"], inp["n_coef"], inp["n_steps"], RHO, inp["a"],
                    inp["box"], inp["obstacles"], inp["boundary"],
                    obstacle_displacement=disp.astype(np.float64))


def _forward(probs, disp, L, plain=False, save=False, ckpt=1):
    import torch
    from paper_2510_09204_amd import to_device
    plan, pk = make_plan(probs, RHO, L=L if save else 0, ckpt=ckpt)
    t = to_device(pk)
    plan.set_obstacle_motion(None if disp is None else torch.from_numpy(disp).cuda())
    xo, lo, res = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L,
                               plain=plain, save=save)
    torch.cuda.synchronize()
    return plan, pk, t, xo.cpu().numpy(), lo.cpu().numpy(), res.cpu().numpy()


def _split(disp, probs):
    out, o = [], 0
    for p in probs:
        out.append(disp[o:o + p.M])
        o += p.M
    return out


@pytest.mark.parametrize("cfg_id,batch,L", [(3, 3, 60), (4, 4, 40), (5, 1, 12)])
def test_moving_obstacles_match_oracle(gpu, cfg_id, batch, L):
    """c5's 120-step horizon runs in LDS time chunks: the obstacle boxes of
    each chunk's windows start at the chunk's global step."""
    probs = make_batch(WORKLOADS[cfg_id], batch=batch)
    pk = pack(probs)
    disp = _disp(pk, cfg_id)
    _, pk, _, xo, lo, res = _forward(probs, disp, L)
    inps = oracle_inputs(pk, probs)
    gx, gl = unpack_coefs(xo, probs), unpack_coefs(lo, probs)
    errs = []
    for b, (inp, d) in enumerate(zip(inps, _split(disp, probs))):
        ref = _oracle(inp, d).solve(inp["xi"], inp["xi0"], inp["lam0"], L)
        errs.append(check_against(ref, gx[b], gl[b], res[b]))
    report(f"moving c{cfg_id}", errs)
    finish_parity(errs)


def test_moving_obstacles_plain_path_matches_fused_bitwise(gpu):
    probs = make_batch(WORKLOADS[4], batch=5)
    disp = _disp(pack(probs), 7)
    xf, lf = _forward(probs, disp, 30)[3:5]
    xp, lp = _forward(probs, disp, 30, plain=True)[3:5]
    np.testing.assert_array_equal(xp, xf)
    np.testing.assert_array_equal(lp, lf)


def test_motion_reset_restores_static_obstacles(gpu):
    import torch
    probs = make_batch(WORKLOADS[3], batch=3)
    static = _forward(probs, None, 40)
    plan, pk, t = static[0], static[1], static[2]
    plan.set_obstacle_motion(torch.from_numpy(_disp(pk, 3)).cuda())
    moved, _, _ = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], 40)
    plan.set_obstacle_motion(None)
    back, _, _ = plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], 40)
    torch.cuda.synchronize()
    assert not np.array_equal(moved.cpu().numpy(), static[3])
    np.testing.assert_array_equal(back.cpu().numpy(), static[3])


def test_moving_obstacles_adjoint_matches_oracle(gpu):
    import torch
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0)
    probs = [make_problem(cfg, i) for i in range(2)]
    pk = pack(probs)
    L = 20
    disp = _disp(pk, 11, scale=1.0)
    plan, pk, t, _, _, _ = _forward(probs, disp, L, save=True)
    rng = np.random.default_rng(12)
    g_xi = [rng.standard_normal(p.xi.shape) for p in probs]
    g_lam = [rng.standard_normal(p.xi.shape) for p in probs]
    gx = torch.from_numpy(np.concatenate([g.ravel() for g in g_xi]).astype(np.float32)).cuda()
    gl = torch.from_numpy(np.concatenate([g.ravel() for g in g_lam]).astype(np.float32)).cuda()
    g = plan.backward(gx, gl, None)
    torch.cuda.synchronize()
    out = [unpack_coefs(x.cpu().numpy(), probs) for x in g]
    for b, (inp, d) in enumerate(zip(oracle_inputs(pk, probs), _split(disp, probs))):
        ref = SFAdjoint(_oracle(inp, d)).gradient(
            inp["xi"], inp["xi0"], inp["lam0"], L,
            g_xi[b].astype(np.float32).astype(np.float64),
            g_lam[b].astype(np.float32).astype(np.float64))
        for q, rv in enumerate((ref.g_xi, ref.g_xi0, ref.g_lam0)):
            assert rel_err(out[q][b], rv) <= GRAD_REL_TOL, (b, q)
