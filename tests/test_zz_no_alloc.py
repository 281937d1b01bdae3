"""sf_project_backward_static (the adjoint for callers that cannot allocate:
its recompute area is the library's static device array) against
sf_project_backward on the same saved forwards, through the C ABI.  Both run
the same kernel with the same summation order, so the gradients must agree bit
for bit.  Two static calls run back to back, the second on a smaller batch
(the array keeps the first call's contents); a recompute area larger than the
array is rejected before anything is launched."""
import numpy as np
import pytest

from sf_testlib import make_plan
from workloads import WORKLOADS, make_batch, make_problem, scaled

pytestmark = pytest.mark.gpu
RHO = 0.5


def _forward(problems, L, ckpt):
    import torch
    from paper_2510_09204_amd import to_device
    plan, pk = make_plan(problems, RHO, L=L, ckpt=ckpt)
    t = to_device(pk)
    plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L, save=True)
    rng = np.random.default_rng(len(problems) * 1000 + L)
    cot = [torch.from_numpy(rng.standard_normal(plan.coef_size).astype(np.float32)).cuda()
           for _ in range(2)]
    g_res = torch.from_numpy(np.tile(np.float32([[0.6, 0.3, 0.0, 0.0]]),
                                     (plan.B, 1))).cuda()
    torch.cuda.synchronize()
    return plan, cot, g_res


def _outputs(plan):
    import torch
    return [torch.full((plan.coef_size,), float("nan"), dtype=torch.float32, device="cuda")
            for _ in range(3)]


def test_static_area_backward_matches_workspace_backward(gpu):
    import torch
    big = make_batch(WORKLOADS[3], batch=4)                 # 32 robots, 20 obstacles
    small_cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0)
    small = [make_problem(small_cfg, i) for i in range(2)]
    runs = [(big, 40, 10, 0.1), (small, 20, 5, 0.0)]
    fwd = [_forward(p, L, k) for p, L, k, _ in runs]
    # two static calls in a row, the second on the smaller batch
    got = []
    for (plan, cot, g_res), (_, L, k, fw) in zip(fwd, runs):
        outs = _outputs(plan)
        print(f"[static] B={plan.B} n={plan.n_robots[0]} L={L} ckpt={k}", flush=True)
        plan.backward(cot[0], cot[1], g_res, fw, out=outs, static_area=True)
        got.append(outs)
    torch.cuda.synchronize()
    for (plan, cot, g_res), (_, L, k, fw), g in zip(fwd, runs, got):
        ref = plan.backward(cot[0], cot[1], g_res, fw)
        torch.cuda.synchronize()
        for name, a, b in zip(("g_xi", "g_xi0", "g_lam0"), g, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.isfinite(b).all(), name
            print(f"[static] B={plan.B} {name}: max |diff| {np.abs(a - b).max():.3e}",
                  flush=True)
            np.testing.assert_array_equal(a, b)


def test_static_area_rejects_a_recompute_area_beyond_its_size(gpu):
    import torch
    from paper_2510_09204_amd import SFError
    probs = make_batch(WORKLOADS[3], batch=4)
    # 4 problems x 704 floats x 2 (xi_bar, lambda) x 2000 iterates x 4 B = 45 MB > 32 MiB
    plan, cot, g_res = _forward(probs, 1, 2000)
    with pytest.raises(SFError) as err:
        plan.backward(cot[0], cot[1], g_res, 0.0, static_area=True)
    assert err.value.code == -2
    g = plan.backward(cot[0], cot[1], g_res, 0.0)       # the workspace path still runs
    torch.cuda.synchronize()
    assert all(np.isfinite(x.cpu().numpy()).all() for x in g)


def test_static_area_backward_matches_workspace_backward_3d(gpu):
    """The same on a 3D (spheroid) plan: the 3D adjoint's segment recompute
    goes to the static array."""
    import torch
    from paper_2510_09204_amd import SFPlan, to_device
    from workloads.gen3d import WORKLOADS_3D, make_batch3d, pack3d
    probs = make_batch3d(WORKLOADS_3D[48], batch=3)
    pk = pack3d(probs)
    L = 20
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_ab, pk.box, pk.n_coef, pk.n_steps, RHO,
                  n_dim=3, max_iters=L, checkpoint_every=5)
    t = {k: torch.from_numpy(getattr(pk, k)).cuda() for k in ("xi", "xi0", "lam0",
                                                               "boundary", "obstacles")}
    plan.project(t["xi"], t["xi0"], t["lam0"], t["boundary"], t["obstacles"], L, save=True)
    rng = np.random.default_rng(48)
    cot = [torch.from_numpy(rng.standard_normal(plan.coef_size).astype(np.float32)).cuda()
           for _ in range(2)]
    g_res = torch.from_numpy(np.tile(np.float32([[0.5, 0.5, 0.0, 0.0]]), (plan.B, 1))).cuda()
    outs = _outputs(plan)
    print(f"[static] 3D B={plan.B} L={L} ckpt=5", flush=True)
    plan.backward(cot[0], cot[1], g_res, 0.1, out=outs, static_area=True)
    ref = plan.backward(cot[0], cot[1], g_res, 0.1)
    torch.cuda.synchronize()
    for name, a, b in zip(("g_xi", "g_xi0", "g_lam0"), outs, ref):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(b).all(), name
        np.testing.assert_array_equal(a, b)
