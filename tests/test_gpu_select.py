"""Candidate selection around the SF on the GPU (sf_smoothness, sf_rank_residual,
sf_select_best, sf_gather_blocks through the C ABI) against the FP64 oracle of
oracle/select.py."""
import dataclasses

import numpy as np
import pytest

from oracle.select import rank_residual as o_rank
from oracle.select import select_best as o_best
from oracle.select import select_candidates as o_select
from oracle.select import smoothness_cost
from sf_testlib import make_plan, rel_err
from workloads import WORKLOADS, make_batch, pack, unpack_coefs

pytestmark = pytest.mark.gpu
RHO = 0.5
T_FINAL = 5.0


def _f32(problems):
    """Copies of the problems holding exactly the float32 values the GPU sees."""
    out = []
    for p in problems:
        out.append(dataclasses.replace(
            p, xi=p.xi.astype(np.float32).astype(np.float64),
            boundary=p.boundary.astype(np.float32).astype(np.float64),
            obstacles=p.obstacles.astype(np.float32).astype(np.float64),
            box=p.box.astype(np.float32).astype(np.float64),
            a=float(np.float32(p.a))))
    return out


@pytest.mark.parametrize("cfg_id", [2, 4, 5])
def test_smoothness_matches_oracle(gpu, cfg_id):
    import torch
    probs = make_batch(WORKLOADS[cfg_id], batch=6)
    plan, pk = make_plan(probs, RHO)
    xi = torch.from_numpy(pk.xi).cuda()
    cost = plan.smoothness(xi, T_FINAL).cpu().numpy()
    xs = unpack_coefs(pk.xi.astype(np.float64), probs)
    for b, p in enumerate(probs):
        ref = smoothness_cost(xs[b], p.n_steps, T_FINAL)
        assert cost[b] == pytest.approx(ref, rel=1e-5), (b, cost[b], ref)


def test_rank_and_best_are_exact_on_crafted_rows(gpu):
    import torch
    from paper_2510_09204_amd import rank_residual, select_best
    rng = np.random.default_rng(11)
    n = 3000                                   # several rows per thread
    rows = np.zeros((n, 4), dtype=np.float32)
    rows[:, 0] = rng.choice(np.float32([1e-4, 5e-4, 9e-4, 2e-3, 0.3]), n)
    rows[:, 1] = rng.choice(np.float32([0.0, 1e-4]), n)
    rows[rng.integers(0, n, 50), 3] = 1.0      # flagged rows rank last
    rows[7, 0] = np.nan
    cost = rng.choice(np.float32([0.5, 0.25, 0.125]), n).astype(np.float32)
    cost[3] = np.inf
    t_rows = torch.from_numpy(rows).cuda()
    t_cost = torch.from_numpy(cost).cuda()
    for k in (1, 10, 256, n):
        got = rank_residual(t_rows, k).cpu().numpy()
        np.testing.assert_array_equal(got, o_rank(rows, k))
    for tol in (0.0, 1e-4, 1e-3, 1.0):
        assert int(select_best(t_rows, t_cost, tol).cpu()[0]) == o_best(rows, cost, tol)


def test_gather_blocks_exact_and_invalid_index_gives_nan(gpu):
    import torch
    from paper_2510_09204_amd import gather_blocks
    src = torch.arange(7 * 300, dtype=torch.float32, device="cuda")
    idx = torch.tensor([6, 0, 3, 3, 7, -1], dtype=torch.int32, device="cuda")
    out = gather_blocks(src, idx, 300).reshape(6, 300).cpu().numpy()
    ref = src.reshape(7, 300).cpu().numpy()
    for q, j in enumerate([6, 0, 3, 3]):
        np.testing.assert_array_equal(out[q], ref[j])
    assert np.isnan(out[4]).all() and np.isnan(out[5]).all()


def test_candidate_pipeline_matches_oracle(gpu):
    """32 candidates of one 16-robot context: raw ranking, SF refinement of the
    best 10 for 200 iterations, choice by feasibility and smoothness.  The
    top-k sets agree unless two raw keys are within float32 rounding of the
    oracle's; the refined trajectories agree to the SF tolerance; the choice
    agrees unless the oracle itself sees a near-tie."""
    import torch
    from paper_2510_09204_amd import select_candidates
    probs = _f32(make_batch(WORKLOADS[2]))
    k, L, tol = 10, 200, 1e-3
    p0 = probs[0]
    pk = pack(probs)
    xi = torch.from_numpy(pk.xi).cuda()
    bnd = torch.from_numpy(pk.boundary[:p0.n * 4].copy()).cuda()
    obs = torch.from_numpy(pk.obstacles[:p0.M * 3].copy()).cuda()
    out = select_candidates(xi, p0.n, p0.M, float(pk.robot_a[0]), pk.box[0], bnd, obs,
                            p0.n_coef, p0.n_steps, RHO, k, L, tol, T_FINAL)
    torch.cuda.synchronize()
    ref = o_select(probs, k, L, tol, T_FINAL, RHO)
    raw = out["residual_raw"].cpu().numpy()
    np.testing.assert_allclose(raw[:, :2], ref["residual_raw"][:, :2], rtol=1e-4, atol=1e-6)
    top = out["topk"].cpu().numpy()
    # the GPU ranking is exactly the oracle ranking of the GPU's own rows
    np.testing.assert_array_equal(top, o_rank(raw, k))
    print(f"top-k GPU {list(top)} oracle {list(ref['topk'])}; chosen GPU "
          f"{int(top[int(out['best'].cpu()[0])])} oracle {int(ref['topk'][ref['best']])}")
    if set(top) != set(ref["topk"]):
        keys = np.hypot(ref["residual_raw"][:, 0], ref["residual_raw"][:, 1])
        edge = np.sort(keys)[k - 1:k + 1]
        assert abs(edge[1] - edge[0]) <= 1e-4 * edge[1], (top, ref["topk"])
        return
    xo = out["xi_refined"].cpu().numpy().reshape(k, 2, p0.n, p0.n_coef)
    order = {int(b): q for q, b in enumerate(ref["topk"])}
    for q, b in enumerate(top):
        e = rel_err(xo[q], ref["xi_refined"][order[int(b)]])
        assert e <= 1e-4, (q, b, e)
    cost = out["cost"].cpu().numpy()
    for q, b in enumerate(top):
        assert cost[q] == pytest.approx(ref["cost"][order[int(b)]], rel=1e-3)
    best = int(out["best"].cpu()[0])
    rows = out["residual_refined"].cpu().numpy()
    assert best == o_best(rows, cost, tol)              # exact on the GPU's own values
    if int(top[best]) != int(ref["topk"][ref["best"]]):
        rc = ref["cost"]
        srt = np.sort(rc)
        assert abs(srt[1] - srt[0]) <= 1e-3 * srt[1], (top[best], ref["topk"][ref["best"]])
