"""Pins of the 3D (spheroid) oracle (dim=3) against what the mathematics fixes.

The 3D steps are pinned without restating them: a problem flat in z reduces to
the planar oracle (pinned on its own); with spheres (b = a) the iteration is
equivariant under rotations; with spheroids it is equivariant under scaling z
together with b and b_o (the map that turns a spheroid into a sphere); the e
step's composition has a closed form on the spheroid surface; a well-separated
feasible input is a fixed point.
"""
import numpy as np
import pytest

from oracle import sf as O
from workloads import WORKLOADS, make_problem
from workloads.gen3d import WORKLOADS_3D, make_problem3d, scaled3d

RHO = 0.5


def _solve3(p, L, **over):
    kw = dict(a=p.a, b=p.b, box=p.box, obstacles=p.obstacles, boundary=p.boundary, xi=p.xi)
    kw.update(over)
    orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, kw["a"], kw["box"], kw["obstacles"],
                     kw["boundary"], dim=3, robot_b=kw["b"])
    return orc.solve(kw["xi"], n_iters=L, keep_history=True)


def _tight3d(idx=0, **kw):
    cfg = scaled3d(WORKLOADS_3D[16], n_robots=(5, 5), n_obs=(3, 3), side=3.0, height=1.6,
                   n_coef=7, n_steps=30, sigma=0.4, **kw)
    return make_problem3d(cfg, idx)


def test_z_flat_problem_reduces_to_the_planar_oracle():
    p = make_problem(WORKLOADS[1], 0)
    L = 40
    ref = O.SFOracle.for_problem(p, RHO).solve(p.xi, n_iters=L, keep_history=True)
    n, M, nc = p.n, p.M, p.n_coef
    xi3 = np.concatenate([p.xi, np.zeros((1, n, nc))])
    bnd3 = np.concatenate([p.boundary, np.zeros((n, 2, 1))], axis=2)
    obs3 = np.column_stack([p.obstacles[:, :2], np.zeros(M), p.obstacles[:, 2],
                            np.full(M, 0.7)])
    box3 = np.column_stack([p.box, [-1.0, 1.0]])
    orc = O.SFOracle(n, M, nc, p.n_steps, RHO, p.a, box3, obs3, bnd3, dim=3, robot_b=0.45)
    got = orc.solve(xi3, n_iters=L)
    np.testing.assert_allclose(got.xi_bar[:2], ref.xi_bar, rtol=0, atol=1e-11)
    np.testing.assert_allclose(got.lam[:2], ref.lam, rtol=0, atol=1e-11)
    # z stays at zero up to rounding (cos(beta) at beta = pi/2 is ~6e-17)
    assert np.max(np.abs(got.xi_bar[2])) < 1e-12 and np.max(np.abs(got.lam[2])) < 1e-12
    assert got.residual == pytest.approx(ref.residual, rel=1e-10, abs=1e-13)
    assert ref.history[0, 0] > 0.0             # constraints were active


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("seed", [0, 2])
def test_spheres_are_rotation_equivariant(seed):
    """b = a and b_o = a_o; the box is far away (inactive): rotating the
    sample, the boundary and the obstacle centres rotates the solution."""
    p = _tight3d(seed)
    Q = _rotation(seed + 10)
    obs = p.obstacles.copy()
    obs[:, 4] = obs[:, 3]
    box = np.array([[-50.0] * 3, [50.0] * 3])
    L = 40
    base = _solve3(p, L, b=p.a, obstacles=obs, box=box)
    assert base.history[0, 0] > 1e-3
    rot = lambda c: np.einsum("xy,yic->xic", Q, c)
    obs_r = obs.copy()
    obs_r[:, :3] = obs[:, :3] @ Q.T
    got = _solve3(p, L, b=p.a, obstacles=obs_r, box=box, xi=rot(p.xi),
                  boundary=p.boundary @ Q.T)
    np.testing.assert_allclose(got.xi_bar, rot(base.xi_bar), rtol=0, atol=1e-9)
    np.testing.assert_allclose(got.lam, rot(base.lam), rtol=0, atol=1e-9)
    assert got.residual == pytest.approx(base.residual, rel=1e-8)


@pytest.mark.parametrize("kappa", [0.6, 1.7])
def test_spheroids_are_equivariant_under_z_scaling(kappa):
    """Scaling z by kappa together with b, b_o and the box maps the problem to
    one with the same constraint geometry: the solution's z scales, x and y
    stay."""
    p = _tight3d(3)
    L = 40
    base = _solve3(p, L)
    assert base.history[0, 0] > 1e-3
    S = np.diag([1.0, 1.0, kappa])
    obs = p.obstacles.copy()
    obs[:, 2] *= kappa
    obs[:, 4] *= kappa
    got = _solve3(p, L, b=p.b * kappa, obstacles=obs, box=p.box @ S,
                  xi=np.einsum("xy,yic->xic", S, p.xi), boundary=p.boundary @ S)
    np.testing.assert_allclose(got.xi_bar[:2], base.xi_bar[:2], rtol=0, atol=1e-9)
    np.testing.assert_allclose(got.xi_bar[2], kappa * base.xi_bar[2], rtol=0, atol=1e-9)
    np.testing.assert_allclose(got.lam[2], kappa * base.lam[2], rtol=0, atol=1e-9)


def test_e_step_lands_on_the_spheroid_or_keeps_delta():
    """After the alpha, beta and d steps, e = Delta outside the spheroid
    ((dx^2 + dy^2)/a^2 + dz^2/b^2 >= 1) and the radial point Delta/s on its
    surface inside; at Delta = 0 (the tie) e = (0, 0, b)."""
    rng = np.random.default_rng(5)
    a, b = 0.4, 0.7
    D = rng.uniform(-1.0, 1.0, (4000, 3))
    ex, ey, ez = O.e_block_3d(D[:, 0], D[:, 1], D[:, 2], a, b)
    E = np.stack([ex, ey, ez], axis=1)
    s = np.sqrt((D[:, 0] ** 2 + D[:, 1] ** 2) / a ** 2 + D[:, 2] ** 2 / b ** 2)
    out = s >= 1.0
    assert out.any() and (~out).any()
    np.testing.assert_allclose(E[out], D[out], atol=1e-12)
    np.testing.assert_allclose(E[~out], D[~out] / s[~out, None], atol=1e-12)
    on = (E[~out, 0] ** 2 + E[~out, 1] ** 2) / a ** 2 + E[~out, 2] ** 2 / b ** 2
    np.testing.assert_allclose(on, 1.0, atol=1e-12)
    assert O.e_block_3d(np.zeros(1), np.zeros(1), np.zeros(1), a, b) == (0.0, 0.0, b)


def test_sphere_e_step_is_the_nearest_feasible_point_by_brute_force():
    """b = a: e is the point of {|e| >= a} nearest to Delta (grid search)."""
    a = 0.5
    th = np.linspace(0, np.pi, 181)
    ph = np.linspace(-np.pi, np.pi, 361)
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    rng = np.random.default_rng(8)
    for _ in range(10):
        d = rng.uniform(-0.4, 0.4, 3)
        e = np.array(O.e_block_3d(d[:1], d[1:2], d[2:], a, a)).ravel()
        cand = np.concatenate([a * dirs, d[None] if np.linalg.norm(d) >= a else np.zeros((0, 3))])
        best = np.min(np.linalg.norm(cand - d, axis=1))
        assert np.linalg.norm(e - d) <= best + 1e-9
        assert np.linalg.norm(e) == pytest.approx(a, rel=1e-12) or np.linalg.norm(d) >= a


def test_separated_feasible_lines_are_a_fixed_point():
    starts = np.array([[-2.0, -2.0, -1.0], [2.0, 2.0, 1.0]])
    goals = np.array([[2.0, -2.0, -1.0], [-2.0, 2.0, 1.0]])
    from workloads import straight_coefficients
    xi = straight_coefficients(starts, goals, 8)
    obs = np.array([[0.0, 0.0, 0.0, 0.5, 0.4]])
    box = np.array([[-3.0] * 3, [3.0] * 3])
    orc = O.SFOracle(2, 1, 8, 30, RHO, 0.4, box, obs, np.stack([starts, goals], 1), dim=3,
                     robot_b=0.6)
    res = orc.solve(xi, n_iters=15)
    np.testing.assert_allclose(res.xi_bar, xi, atol=1e-12)
    # e = d u reproduces Delta up to rounding of the angles
    assert res.residual < 1e-13 and np.max(np.abs(res.lam)) < 1e-13


def test_3d_residual_decreases_on_a_generated_problem():
    p = _tight3d(7)
    res = _solve3(p, 200)
    h = np.hypot(res.history[:, 0], res.history[:, 1])
    assert h[0] > 1e-2 and res.residual < 0.05 * h[0]


def test_moving_obstacles_are_galilean_equivariant():
    """Obstacles moving by d over the horizon (centre c + d tau) against the
    same problem seen from a frame moving with them: there the obstacles are
    static and every robot's sample and boundary are shifted by -d tau, i.e.
    by -d c/(n_coef - 1) on coefficient c (linear precision of the Bernstein
    basis).  Pair differences are unchanged and the box is far away, so the
    iterates differ by exactly that shift."""
    p = _tight3d(2)
    box = np.array([[-50.0] * 3, [50.0] * 3])
    d = np.array([0.7, -0.4, 0.3])
    L = 40
    disp = np.tile(d, (p.M, 1))
    mov = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, box, p.obstacles, p.boundary,
                     dim=3, robot_b=p.b, obstacle_displacement=disp).solve(
                         p.xi, n_iters=L, keep_history=True)
    assert mov.history[0, 0] > 1e-3
    shift = d[:, None, None] * (np.arange(p.n_coef) / (p.n_coef - 1))[None, None, :]
    bnd = p.boundary - np.stack([np.zeros(3), d])[None]
    sta = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, box, p.obstacles, bnd,
                     dim=3, robot_b=p.b).solve(p.xi - shift, n_iters=L)
    np.testing.assert_allclose(mov.xi_bar - shift, sta.xi_bar, rtol=0, atol=1e-9)
    np.testing.assert_allclose(mov.lam, sta.lam, rtol=0, atol=1e-9)
    assert mov.residual == pytest.approx(sta.residual, rel=1e-8, abs=1e-12)


def test_pins_catch_swapped_spheroid_axes(monkeypatch):
    """A planted mistake in the beta step (a and b swapped) breaks the
    z-scaling equivariance that the pin above checks."""
    p = _tight3d(3)
    L = 20
    kappa = 1.7

    def wrong_beta(dx, dy, dz, alpha, a, b):
        rho_xy = dx * np.cos(alpha) + dy * np.sin(alpha)
        return np.arctan2(rho_xy / b, dz / a)

    monkeypatch.setattr(O, "beta_step", wrong_beta)
    base = _solve3(p, L)
    S = np.diag([1.0, 1.0, kappa])
    obs = p.obstacles.copy()
    obs[:, 2] *= kappa
    obs[:, 4] *= kappa
    got = _solve3(p, L, b=p.b * kappa, obstacles=obs, box=p.box @ S,
                  xi=np.einsum("xy,yic->xic", S, p.xi), boundary=p.boundary @ S)
    dev = max(np.max(np.abs(got.xi_bar[:2] - base.xi_bar[:2])),
              np.max(np.abs(got.xi_bar[2] - kappa * base.xi_bar[2])))
    assert dev > 1e-6


# ---------------------------------------------------------------- 3D adjoint
def _kink_margin3(orc, its):
    """Smallest distance of any pair/obstacle scaled length from 1 (the d
    step's clip) and of any box coordinate from its bound."""
    o = orc.ops
    R, Pr = o.n_pair_rows + o.n_obs_rows, o.n_pair_rows
    m = np.inf
    for xib, _ in its:
        q = o.F @ xib
        x, y, z = q[:R], q[R:2 * R], q[2 * R:]
        s = np.sqrt((x[:Pr] ** 2 + y[:Pr] ** 2) / orc.a ** 2 + z[:Pr] ** 2 / orc.robot_b ** 2)
        m = min(m, np.min(np.abs(s - 1.0))) if Pr else m
        if o.M:
            ox, oy, oz = (x[Pr:] - orc.obs_cen[0], y[Pr:] - orc.obs_cen[1],
                          z[Pr:] - orc.obs_cen[2])
            so = np.sqrt((ox ** 2 + oy ** 2) / orc.obs_ao[0] ** 2 + oz ** 2 / orc.obs_ao[1] ** 2)
            m = min(m, np.min(np.abs(so - 1.0)))
        m = min(m, np.min(np.abs(o.G @ xib - orc.h)))
    return m


@pytest.fixture(scope="module")
def fd3_case():
    p = _tight3d(4)
    orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles, p.boundary,
                     dim=3, robot_b=p.b)
    return p, orc, np.random.default_rng(21)


def _fd_check(p, orc, rng, L, wr1, wr2, fp_weight, adjoint_cls=None, tol=1e-6):
    from oracle.adjoint import SFAdjoint, loss_value
    adjoint_cls = adjoint_cls or SFAdjoint
    lam0 = 0.05 * rng.standard_normal(p.xi.shape)
    its = orc.solve(p.xi, p.xi, lam0, L, keep_iterates=True).iterates
    assert _kink_margin3(orc, its) > 1e-4
    w_xi = rng.standard_normal(p.xi.shape)
    w_lam = rng.standard_normal(p.xi.shape)
    g = adjoint_cls(orc).gradient(p.xi, p.xi, lam0, L, w_xi, w_lam, wr1, wr2, fp_weight)
    h = 1e-6
    worst = 0.0
    for which, gv in ((0, g.g_xi), (1, g.g_xi0), (2, g.g_lam0)):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in p.xi.shape)
            args = [p.xi.copy(), p.xi.copy(), lam0.copy()]
            args[which][idx] += h
            fp = loss_value(orc, *args, L, w_xi, w_lam, wr1, wr2, fp_weight)
            args[which][idx] -= 2 * h
            fm = loss_value(orc, *args, L, w_xi, w_lam, wr1, wr2, fp_weight)
            fd = (fp - fm) / (2 * h)
            worst = max(worst, abs(fd - gv[idx]) / max(1.0, abs(fd)))
    return worst


@pytest.mark.parametrize("fp_weight,wr1,wr2", [(0.0, 0.0, 0.0), (0.3, 0.8, 0.5)])
def test_3d_oracle_adjoint_matches_central_finite_differences(fd3_case, fp_weight, wr1, wr2):
    """The reverse sweep through the alpha, beta and d steps (reading Q1) against
    central differences (h = 1e-6) of the loss it differentiates."""
    p, orc, rng = fd3_case
    hist = orc.solve(p.xi, n_iters=15, keep_history=True).history
    assert hist[0, 0] > 1e-3                    # spheroid constraints were active
    assert _fd_check(p, orc, rng, 15, wr1, wr2, fp_weight) <= 1e-6


def test_3d_oracle_adjoint_dot_product_identity(fd3_case):
    """<J v, w> = <v, J^T w> for the Jacobian of xi_bar^L w.r.t. lambda^0."""
    from oracle.adjoint import SFAdjoint
    p, orc, rng = fd3_case
    L = 12
    v = rng.standard_normal(p.xi.shape)
    w = rng.standard_normal(p.xi.shape)
    g = SFAdjoint(orc).gradient(p.xi, p.xi, None, L, w, np.zeros_like(w))
    h = 1e-6
    jv = (orc.solve(p.xi, p.xi, h * v, L).xi_bar - orc.solve(p.xi, p.xi, -h * v, L).xi_bar) / (2 * h)
    assert abs(np.sum(jv * w) - np.sum(v * g.g_lam0)) < 1e-6 * max(1.0, abs(np.sum(jv * w)))


def test_3d_adjoint_pins_catch_swapped_spheroid_axes(fd3_case, monkeypatch):
    """A planted mistake in the reverse sweep (the spheroid sizes a and b
    swapped in the reverse alpha/beta/d chain) fails the finite-difference
    pin."""
    import oracle.adjoint as A
    p, orc, _ = fd3_case
    real = A._e3_vjp

    def wrong(dx, dy, dz, a, b, g_ex, g_ey, g_ez):
        return real(dx, dy, dz, b, a, g_ex, g_ey, g_ez)

    monkeypatch.setattr(A, "_e3_vjp", wrong)
    assert _fd_check(p, orc, np.random.default_rng(21), 15, 0.0, 0.0, 0.0) > 1e-4
