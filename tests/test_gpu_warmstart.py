"""The learned warm start trained through sf_project_backward (eq. NN_loss):
the fixed-point terms reach the network through the adjoint's fixed-point
weight, and a short training run lowers the objective."""
import numpy as np
import pytest

from workloads import WORKLOADS, make_batch, pack, scaled

pytestmark = pytest.mark.gpu
RHO = 0.5


def _batch(B=16, L=20):
    import torch
    from paper_2510_09204_amd import SFPlan
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0, n_steps=50)
    probs = make_batch(cfg, batch=B)
    pk = pack(probs)
    n, M, nc = probs[0].n, probs[0].M, probs[0].n_coef
    dev = torch.device("cuda")
    xi = torch.from_numpy(pk.xi).to(dev).reshape(B, 2, n, nc)
    bnd = torch.from_numpy(pk.boundary).to(dev).reshape(B, n, 2, 2)
    obs = torch.from_numpy(pk.obstacles).to(dev).reshape(B, M, 3)
    plan = SFPlan(pk.n_robots, pk.n_obs, pk.robot_a, pk.box, nc, pk.n_steps, RHO,
                  checkpoint_every=1, max_iters=L, device=dev)
    return plan, xi, bnd, obs


def _objective(net, plan, xi, bnd, obs, L):
    """||xi_bar^L - xi||^2 + sum_l ||z^{l+1} - z^l||^2, evaluated one iteration
    per call (the state (xi_bar, lambda) is the whole iterate)."""
    import torch
    with torch.no_grad():
        x, lam = net(xi, bnd, obs)
        x, lam = x.reshape(-1).contiguous(), lam.reshape(-1).contiguous()
        fp = 0.0
        for _ in range(L):
            x, lam, res = plan.project(xi.reshape(-1).contiguous(), x, lam, bnd.reshape(-1),
                                       obs.reshape(-1), 1)
            fp += float((res[:, 2].double() ** 2).sum())
        return float(((x - xi.reshape(-1)) ** 2).sum()) + fp


def test_warm_start_training_lowers_the_objective(gpu):
    import torch
    from paper_2510_09204_amd.warmstart import WarmStartNet, warm_start_loss
    torch.manual_seed(0)
    L = 20
    plan, xi, bnd, obs = _batch(L=L)
    net = WarmStartNet(xi.shape[-1]).cuda()
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    j0 = _objective(net, plan, xi, bnd, obs, L)
    for step in range(80):
        opt.zero_grad()
        loss, _, _, res = warm_start_loss(net, plan, xi, bnd, obs, L, fp_weight=1.0)
        loss.backward()
        if step == 0:
            gnorm = sum(float(p.grad.norm()) for p in net.parameters() if p.grad is not None)
            assert np.isfinite(gnorm) and gnorm > 0.0
        opt.step()
    j1 = _objective(net, plan, xi, bnd, obs, L)
    print(f"objective {j0:.4g} -> {j1:.4g}")
    assert np.isfinite(j1) and j1 < 0.8 * j0, (j0, j1)


def test_untrained_net_is_the_default_warm_start(gpu):
    """The output layer starts at zero: xi_bar^0 = xi and lambda^0 = 0."""
    import torch
    from paper_2510_09204_amd.warmstart import WarmStartNet
    plan, xi, bnd, obs = _batch(B=4)
    net = WarmStartNet(xi.shape[-1]).cuda()
    x0, l0 = net(xi, bnd, obs)
    assert torch.equal(x0, xi) and torch.count_nonzero(l0) == 0
