"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, a closed form, brute force, an optimality condition or an invariance.
The paper prints no worked SF instance, so no test compares with printed values
of a solve.
"""
import numpy as np
import pytest
import scipy.optimize as so
from scipy.interpolate import BPoly

from oracle import sf as O
from oracle.adjoint import SFAdjoint, loss_value
from workloads import WORKLOADS, make_problem, scaled, straight_coefficients

RHO = 0.5


def _line_problem(starts, goals, n_coef=7, T=25, obstacles=None, half=5.0, a=0.4):
    starts, goals = np.asarray(starts, float), np.asarray(goals, float)
    xi = straight_coefficients(starts, goals, n_coef)
    obs = np.zeros((0, 3)) if obstacles is None else np.asarray(obstacles, float)
    box = np.array([[-half, -half], [half, half]])
    bnd = np.stack([starts, goals], axis=1)
    return xi, obs, box, bnd


def _scipy_W(n_coef, T):
    tau = np.arange(T) / (T - 1)
    cols = []
    for c in range(n_coef):
        coef = np.zeros((n_coef, 1))
        coef[c, 0] = 1.0
        cols.append(BPoly(coef, [0.0, 1.0])(tau))
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------- P1: basis W
@pytest.mark.parametrize("n_coef,T", [(11, 50), (11, 100), (15, 120), (2, 2), (5, 7)])
def test_bernstein_matches_library_bpoly(n_coef, T):
    W = O.bernstein_W(n_coef, T)
    np.testing.assert_allclose(W, _scipy_W(n_coef, T), rtol=0, atol=1e-13)
    np.testing.assert_allclose(W.sum(axis=1), 1.0, atol=1e-13)      # partition of unity
    assert np.allclose(W[0], np.eye(n_coef)[0]) and np.allclose(W[-1], np.eye(n_coef)[-1])


def test_linear_precision_of_straight_lines():
    s, g = np.array([[0.3, -1.2]]), np.array([[2.0, 0.7]])
    xi = straight_coefficients(s, g, 11)
    W = _scipy_W(11, 40)
    tau = np.arange(40) / 39
    for ax in range(2):
        np.testing.assert_allclose(W @ xi[ax, 0], s[0, ax] + tau * (g[0, ax] - s[0, ax]),
                                   atol=1e-13)


# ---------------------------------------------------------------- P2: operators
def test_F_rows_are_pair_differences_and_robot_positions():
    n, M, nc, T = 5, 3, 6, 9
    ops = O.build_operators(n, M, nc, T)
    rng = np.random.default_rng(1)
    xi_axis = rng.standard_normal(n * nc)
    X = _scipy_W(nc, T) @ xi_axis.reshape(n, nc).T          # [T][n]
    rows = ops.F_axis @ xi_axis
    P = n * (n - 1) // 2
    assert ops.n_pair_rows == P * T and ops.n_obs_rows == n * M * T   # dimension table
    assert ops.G_axis.shape == (2 * n * T, n * nc) and ops.A_axis.shape == (2 * n, n * nc)
    expect_pairs = [X[:, i] - X[:, j] for i in range(n) for j in range(i + 1, n)]
    np.testing.assert_allclose(rows[:P * T], np.concatenate(expect_pairs), atol=1e-13)
    expect_obs = [X[:, i] for i in range(n) for _ in range(M)]
    np.testing.assert_allclose(rows[P * T:], np.concatenate(expect_obs), atol=1e-13)


def test_FtF_is_complete_graph_laplacian_kron_WtW():
    n, M, nc, T = 5, 3, 6, 9
    ops = O.build_operators(n, M, nc, T)
    W = _scipy_W(nc, T)
    expect = np.kron((n + M) * np.eye(n) - np.ones((n, n)), W.T @ W)
    np.testing.assert_allclose((ops.F_axis.T @ ops.F_axis).toarray(), expect, atol=1e-12)
    np.testing.assert_allclose((ops.G_axis.T @ ops.G_axis).toarray(),
                               np.kron(2 * np.eye(n), W.T @ W), atol=1e-12)


# ---------------------------------------------------------------- P3: alpha/d step
@pytest.mark.parametrize("dx,dy", [(0.1, 0.05), (-0.2, 0.1), (0.3, -0.4), (1.5, 0.7),
                                   (-0.01, -0.02), (0.0, 0.35)])
def test_alpha_d_step_is_brute_force_minimiser(dx, dy):
    a = 0.4
    alphas = np.linspace(-np.pi, np.pi, 62832 + 1)
    ds = np.linspace(1.0, 5.0, 4001)
    # minimise over d for each alpha in closed form would reuse the oracle's
    # algebra; use a dense grid over both instead
    best = (np.inf, None)
    for chunk in np.array_split(alphas, 16):
        A, D = np.meshgrid(chunk, ds, indexing="ij")
        f = (dx - a * D * np.cos(A)) ** 2 + (dy - a * D * np.sin(A)) ** 2
        k = np.unravel_index(np.argmin(f), f.shape)
        if f[k] < best[0]:
            best = (f[k], (A[k], D[k]))
    al, d = best[1]
    e_brute = a * d * np.array([np.cos(al), np.sin(al)])
    al_o = O.alpha_step(np.array([dx]), np.array([dy]))
    d_o = O.d_step(np.array([dx]), np.array([dy]), al_o, a)
    e_o = a * d_o * np.array([np.cos(al_o), np.sin(al_o)]).ravel()
    np.testing.assert_allclose(e_o, e_brute, atol=2e-3)


# ---------------------------------------------------------------- P4: s step
def test_s_step_is_brute_force_minimiser_over_nonnegative_slack():
    rng = np.random.default_rng(2)
    Gx = rng.uniform(-2, 2, 50)
    h = rng.uniform(-1, 1, 50)
    grid = np.linspace(0, 5, 50001)
    brute = np.array([grid[np.argmin((g - hh + grid) ** 2)] for g, hh in zip(Gx, h)])
    np.testing.assert_allclose(O.s_step(Gx, h), brute, atol=1e-4)


# ---------------------------------------------------------------- P5: xi_bar step
def _aug_lagrangian(orc, xib, xi, e, s, lam):
    """The augmented Lagrangian (eq. aug_lag) as a scalar."""
    F, G = orc.ops.F, orc.ops.G
    return (0.5 * np.sum((xib - xi) ** 2) + 0.5 * orc.rho * np.sum((F @ xib - e) ** 2)
            + 0.5 * orc.rho * np.sum((G @ xib - orc.h + s) ** 2) - lam @ xib)


def test_xi_step_minimises_augmented_lagrangian_on_the_equality_set():
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=3.0, n_steps=20)
    p = make_problem(cfg, 3)
    orc = O.SFOracle.for_problem(p, RHO)
    xi = orc.flat(p.xi)
    rng = np.random.default_rng(3)
    xib = xi + 0.2 * rng.standard_normal(xi.size)
    lam = 0.3 * rng.standard_normal(xi.size)
    xib1, lam1, _, _ = orc.step(xi, xib, lam)
    _, _, e, s, _ = orc.residual_terms(xib)
    np.testing.assert_allclose(orc.ops.A @ xib1, orc.b, atol=1e-11)
    # directional derivatives of L along the null space of A vanish, and L is
    # not decreased by any feasible step
    Z = np.linalg.svd(orc.ops.A)[2][orc.ops.A.shape[0]:].T
    h = 1e-5
    f0 = _aug_lagrangian(orc, xib1, xi, e, s, lam1)
    for q in range(12):
        d = Z @ rng.standard_normal(Z.shape[1])
        d /= np.linalg.norm(d)
        fp = _aug_lagrangian(orc, xib1 + h * d, xi, e, s, lam1)
        fm = _aug_lagrangian(orc, xib1 - h * d, xi, e, s, lam1)
        assert abs(fp - fm) / (2 * h) < 1e-6 * max(1.0, abs(f0))
        assert fp >= f0 - 1e-9 and fm >= f0 - 1e-9


# ---------------------------------------------------------------- P6: fixed point
def test_feasible_well_separated_input_is_a_fixed_point():
    starts = [[-3.0, -2.0], [-3.0, 0.0], [-3.0, 2.0]]
    goals = [[3.0, -2.0], [3.0, 0.0], [3.0, 2.0]]
    xi, obs, box, bnd = _line_problem(starts, goals, obstacles=[[0.0, 4.0, 0.5]])
    orc = O.SFOracle(3, 1, xi.shape[2], 25, RHO, 0.4, box, obs, bnd)
    res = orc.solve(xi, n_iters=3)
    np.testing.assert_allclose(res.xi_bar, xi, atol=1e-12)
    np.testing.assert_allclose(res.lam, 0.0, atol=1e-12)
    assert res.residual < 1e-12


# ---------------------------------------------------------------- P7: special case
def test_single_robot_converges_monotonically_to_affine_projection():
    rng = np.random.default_rng(4)
    xi = straight_coefficients(np.array([[-1.0, 0.5]]), np.array([[1.0, -0.5]]), 9)
    xi = xi + 0.3 * rng.standard_normal(xi.shape)
    bnd = np.array([[[-1.0, 0.5], [1.0, -0.5]]])
    box = np.array([[-10.0, -10.0], [10.0, 10.0]])
    orc = O.SFOracle(1, 0, 9, 30, RHO, 0.4, box, np.zeros((0, 3)), bnd)
    A, b = orc.ops.A, orc.b
    x = orc.flat(xi)
    proj = x - A.T @ np.linalg.solve(A @ A.T, A @ x - b)
    res = orc.solve(xi, n_iters=400, keep_iterates=True)
    errs = [np.linalg.norm(it[0] - proj) for it in res.iterates[1:]]
    assert errs[-1] < 1e-10
    assert all(e2 <= e1 + 1e-15 for e1, e2 in zip(errs[:-1], errs[1:]))


# ---------------------------------------------------------------- P8: equivariances
def _solve(p, L=60, **over):
    kw = dict(n=p.n, M=p.M, n_coef=p.n_coef, n_steps=p.n_steps, rho=RHO, a=p.a, box=p.box,
              obstacles=p.obstacles, boundary=p.boundary)
    kw.update(over)
    xi = kw.pop("xi", p.xi)
    orc = O.SFOracle(**kw)
    return orc.solve(xi, n_iters=L)


@pytest.fixture(scope="module")
def small_problem():
    cfg = scaled(WORKLOADS[3], n_robots=(5, 5), n_obs=(3, 3), arena=3.5, n_steps=30)
    return make_problem(cfg, 1)


def test_robot_permutation_equivariance(small_problem):
    p = small_problem
    perm = np.array([3, 0, 4, 1, 2])
    base = _solve(p)
    out = _solve(p, xi=p.xi[:, perm], boundary=p.boundary[perm])
    np.testing.assert_allclose(out.xi_bar, base.xi_bar[:, perm], atol=1e-9)
    np.testing.assert_allclose(out.lam, base.lam[:, perm], atol=1e-9)


def test_obstacle_permutation_invariance(small_problem):
    p = small_problem
    base = _solve(p)
    out = _solve(p, obstacles=p.obstacles[::-1].copy())
    np.testing.assert_allclose(out.xi_bar, base.xi_bar, atol=1e-9)


def test_rotation_by_90_degrees_equivariance(small_problem):
    p = small_problem
    rot = lambda v: np.stack([-v[..., 1], v[..., 0]], axis=-1)     # (x, y) -> (-y, x)
    xi_r = np.stack([-p.xi[1], p.xi[0]])
    obs_r = p.obstacles.copy()
    obs_r[:, :2] = rot(p.obstacles[:, :2])
    base = _solve(p)
    out = _solve(p, xi=xi_r, obstacles=obs_r, boundary=rot(p.boundary))
    np.testing.assert_allclose(out.xi_bar, np.stack([-base.xi_bar[1], base.xi_bar[0]]),
                               atol=1e-9)
    assert abs(out.residual - base.residual) < 1e-9


def test_translation_equivariance(small_problem):
    p = small_problem
    t = np.array([0.7, -1.3])
    obs_t = p.obstacles.copy()
    obs_t[:, :2] += t
    base = _solve(p)
    out = _solve(p, xi=p.xi + t[:, None, None], obstacles=obs_t, boundary=p.boundary + t,
                 box=p.box + t)
    np.testing.assert_allclose(out.xi_bar, base.xi_bar + t[:, None, None], atol=1e-9)
    np.testing.assert_allclose(out.lam, base.lam, atol=1e-9)


# ---------------------------------------------------------------- P9: converged iterate
def test_converged_iterate_is_feasible_and_stationary():
    """Two robots swapping sides past one obstacle, run to convergence.  Then
    (a) every original constraint (inter-robot, obstacle, workspace, boundary)
    holds, evaluated from library Bernstein positions; (b) with r_1 = r_2 = 0 the
    xi_bar step's optimality leaves xi_bar - xi - lambda in the range of A^T.
    (The limit is generally not a KKT point of the projection itself: once every
    constraint holds strictly, r_1 = 0 freezes lambda at what it accumulated.)"""
    nc, T, a = 6, 16, 0.5
    starts, goals = [[-1.5, 0.05], [1.5, -0.05]], [[1.5, 0.05], [-1.5, -0.05]]
    xi, obs, box, bnd = _line_problem(starts, goals, n_coef=nc, T=T,
                                      obstacles=[[0.0, 1.2, 0.5]], half=3.0, a=a)
    orc = O.SFOracle(2, 1, nc, T, RHO, a, box, obs, bnd)
    res = orc.solve(xi, n_iters=3000)
    assert res.residual < 1e-9
    W = _scipy_W(nc, T)
    pos = np.einsum("kc,aic->aik", W, res.xi_bar)      # [2][n][T]
    d = np.hypot(*(pos[:, 0] - pos[:, 1]))
    assert d.min() >= a - 1e-9
    for i in range(2):
        assert np.hypot(*(pos[:, i] - obs[0, :2, None])).min() >= obs[0, 2] - 1e-9
    assert pos.min() >= box[0, 0] - 1e-9 and pos.max() <= box[1, 0] + 1e-9
    np.testing.assert_allclose(pos[:, :, 0], np.array(starts).T, atol=1e-10)
    np.testing.assert_allclose(pos[:, :, -1], np.array(goals).T, atol=1e-10)
    v = orc.flat(res.xi_bar) - orc.flat(xi) - orc.flat(res.lam)
    A = orc.ops.A
    nu = np.linalg.lstsq(A.T, v, rcond=None)[0]
    assert np.linalg.norm(A.T @ nu - v) < 1e-8 * max(1.0, np.linalg.norm(v))


# ---------------------------------------------------------------- P12: residual units
def test_head_on_residual_has_hand_computable_magnitude():
    """Two robots head-on along y = 0: each step's r_1 row has length
    max(0, a - |x_i - x_j|) (metres), so ||r_1||^2 is a sum of those squares."""
    T, nc, a = 41, 7, 0.5
    xi, obs, box, bnd = _line_problem([[-1.0, 0.0], [1.0, 0.0]], [[1.0, 0.0], [-1.0, 0.0]],
                                      n_coef=nc, T=T, a=a)
    orc = O.SFOracle(2, 0, nc, T, RHO, a, box, obs, bnd)
    r1, r2, _, _, _ = orc.residual_terms(orc.flat(xi))
    tau = np.arange(T) / (T - 1)
    gap = np.abs((-1 + 2 * tau) - (1 - 2 * tau))
    expect = np.sqrt(np.sum(np.maximum(0.0, a - gap) ** 2))
    assert abs(np.linalg.norm(r1) - expect) < 1e-12
    assert np.linalg.norm(r2) == 0.0


# ---------------------------------------------------------------- P10: adjoint
@pytest.fixture(scope="module")
def fd_case():
    cfg = scaled(WORKLOADS[3], n_robots=(4, 4), n_obs=(3, 3), arena=4.0, n_steps=30)
    p = make_problem(cfg, 0)
    orc = O.SFOracle.for_problem(p, RHO)
    rng = np.random.default_rng(5)
    return p, orc, rng


def _kink_margin(orc, its):
    """Smallest distance of any pair/obstacle/box quantity from its kink."""
    m = np.inf
    for xib, _ in its:
        q = orc.ops.F @ xib
        R = orc.ops.n_pair_rows + orc.ops.n_obs_rows
        Pr = orc.ops.n_pair_rows
        x, y = q[:R], q[R:]
        d = np.hypot(x[:Pr], y[:Pr])
        m = min(m, np.min(np.abs(d - orc.a)))
        if orc.ops.M:
            do = np.hypot(x[Pr:] - orc.obs_cen[0], y[Pr:] - orc.obs_cen[1])
            m = min(m, np.min(np.abs(do - orc.obs_ao)))
        m = min(m, np.min(np.abs(orc.ops.G @ xib - orc.h)))
    return m


@pytest.mark.parametrize("fp_weight,wr1,wr2", [(0.0, 0.0, 0.0), (0.3, 0.8, 0.5)])
def test_oracle_adjoint_matches_central_finite_differences(fd_case, fp_weight, wr1, wr2):
    p, orc, rng = fd_case
    L = 20
    lam0 = 0.05 * rng.standard_normal(p.xi.shape)
    its = orc.solve(p.xi, p.xi, lam0, L, keep_iterates=True).iterates
    assert _kink_margin(orc, its) > 1e-4
    w_xi = rng.standard_normal(p.xi.shape)
    w_lam = rng.standard_normal(p.xi.shape)
    g = SFAdjoint(orc).gradient(p.xi, p.xi, lam0, L, w_xi, w_lam, wr1, wr2, fp_weight)
    h = 1e-6
    for which, gv in ((0, g.g_xi), (1, g.g_xi0), (2, g.g_lam0)):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in p.xi.shape)
            args = [p.xi.copy(), p.xi.copy(), lam0.copy()]
            args[which][idx] += h
            fp = loss_value(orc, *args, L, w_xi, w_lam, wr1, wr2, fp_weight)
            args[which][idx] -= 2 * h
            fm = loss_value(orc, *args, L, w_xi, w_lam, wr1, wr2, fp_weight)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gv[idx]) <= 1e-6 * max(1.0, abs(fd)), (which, idx, fd, gv[idx])


def test_oracle_adjoint_dot_product_identity(fd_case):
    """<J v, w> = <v, J^T w> for the Jacobian of xi_bar^L w.r.t. lambda^0, with J v
    from a central difference along v (a linear-algebra identity)."""
    p, orc, rng = fd_case
    L = 15
    v = rng.standard_normal(p.xi.shape)
    w = rng.standard_normal(p.xi.shape)
    g = SFAdjoint(orc).gradient(p.xi, p.xi, None, L, w, np.zeros_like(w))
    h = 1e-6
    plus = orc.solve(p.xi, p.xi, h * v, L).xi_bar
    minus = orc.solve(p.xi, p.xi, -h * v, L).xi_bar
    jv = (plus - minus) / (2 * h)
    assert abs(np.sum(jv * w) - np.sum(v * g.g_lam0)) < 1e-6 * max(1.0, abs(np.sum(jv * w)))


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_the_printed_slack_sign(monkeypatch):
    """The s step as printed (max(0, -G xi - h)) is not the slack minimiser."""
    rng = np.random.default_rng(6)
    Gx, h = rng.uniform(-2, 2, 20), rng.uniform(-1, 1, 20)
    printed = np.maximum(0.0, -Gx - h)
    grid = np.linspace(0, 5, 50001)
    brute = np.array([grid[np.argmin((g - hh + grid) ** 2)] for g, hh in zip(Gx, h)])
    assert np.max(np.abs(printed - brute)) > 1e-2


def test_pins_catch_a_kkt_without_workspace_terms():
    """Dropping rho G^T G / rho G^T (h - s) (the printed M and eta) breaks the
    optimality pin of the xi_bar step whenever a box bound is active."""
    starts, goals = [[-1.0, 0.0]], [[1.0, 0.0]]
    xi, obs, box, bnd = _line_problem(starts, goals, n_coef=7, T=25, half=0.5)
    xi = xi.copy()
    xi[1, 0, 3] += 2.0                                   # push outside the box
    orc = O.SFOracle(1, 0, 7, 25, RHO, 0.4, box, obs, bnd, include_G=False)
    x = orc.flat(xi)
    xib1, lam1, _, _ = orc.step(x, x, np.zeros_like(x))
    _, _, e, s, _ = orc.residual_terms(x)
    Z = np.linalg.svd(orc.ops.A)[2][orc.ops.A.shape[0]:].T
    grads = []
    for q in range(Z.shape[1]):
        d = Z[:, q]
        hstep = 1e-5
        grads.append((_aug_lagrangian(orc, xib1 + hstep * d, x, e, s, lam1)
                      - _aug_lagrangian(orc, xib1 - hstep * d, x, e, s, lam1)) / (2 * hstep))
    assert max(abs(g) for g in grads) > 1e-3


# ------------------------------------- acceleration objective (trajectory optimiser)
def test_accel_objective_reaches_the_straight_line_without_constraints():
    """With the smoothness cost, one robot, no obstacles and an inactive box,
    the xi_bar steps are proximal steps on 1/2 ||Wdd xi_bar||^2 subject to the
    boundary rows; its unique minimiser is the zero-acceleration trajectory,
    the straight line between the endpoints."""
    nc, T = 7, 40
    starts, goals = np.array([[-1.0, 0.5]]), np.array([[1.5, -0.5]])
    rng = np.random.default_rng(2)
    xi0 = straight_coefficients(starts, goals, nc) + 0.3 * rng.standard_normal((2, 1, nc))
    box = np.array([[-50.0, -50.0], [50.0, 50.0]])
    bnd = np.stack([starts, goals], axis=1)
    orc = O.SFOracle(1, 0, nc, T, RHO, 0.4, box, np.zeros((0, 3)), bnd, objective="accel")
    r = orc.solve(np.zeros_like(xi0), xi0, None, 3000)
    np.testing.assert_allclose(r.xi_bar, straight_coefficients(starts, goals, nc), atol=1e-8)


def test_accel_objective_ignores_the_sample():
    """The sample xi enters only the projection's cost: with the acceleration
    objective two different samples give the same iterates."""
    cfg = scaled(WORKLOADS[3], n_robots=(3, 3), n_obs=(2, 2), arena=4.0, n_steps=25)
    p = make_problem(cfg, 1)
    orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles, p.boundary,
                     objective="accel")
    a = orc.solve(p.xi, p.xi, None, 30).xi_bar
    b = orc.solve(np.zeros_like(p.xi), p.xi, None, 30).xi_bar
    np.testing.assert_array_equal(a, b)


def test_accel_xi_step_minimises_its_lagrangian_on_the_equality_set():
    """One xi_bar step with the acceleration objective minimises
    1/2 xi'^T Q xi' + rho/2 ||F xi' - e||^2 + rho/2 ||G xi' - h + s||^2
    - lambda'^T xi' ... on {A xi' = b}: the gradient there lies in range(A^T)."""
    cfg = scaled(WORKLOADS[3], n_robots=(3, 3), n_obs=(2, 2), arena=4.0, n_steps=25)
    p = make_problem(cfg, 2)
    orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles, p.boundary,
                     objective="accel")
    xib = orc.flat(p.xi)
    lam = 0.1 * np.random.default_rng(4).standard_normal(xib.size)
    xn, lam_n, _, _ = orc.step(np.zeros_like(xib), xib, lam)
    r1, r2, e, s, _ = orc.residual_terms(xib)
    Q = O.objective_block(orc.ops, "accel")
    F, G = orc.ops.F, orc.ops.G
    grad = Q @ xn + RHO * (F.T @ (F @ xn - e)) + RHO * (G.T @ (G @ xn - orc.h + s)) - lam_n
    A = orc.ops.A
    nu, *_ = np.linalg.lstsq(A.T, grad, rcond=None)
    assert np.linalg.norm(grad - A.T @ nu) <= 1e-9 * max(1.0, np.linalg.norm(grad))
    np.testing.assert_allclose(A @ xn, orc.b, atol=1e-10)


def test_accel_objective_adjoint_matches_central_finite_differences(fd_case):
    p, _, rng = fd_case
    orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles, p.boundary,
                     objective="accel")
    L = 12
    lam0 = 0.05 * rng.standard_normal(p.xi.shape)
    its = orc.solve(p.xi, p.xi, lam0, L, keep_iterates=True).iterates
    assert _kink_margin(orc, its) > 1e-4
    w_xi = rng.standard_normal(p.xi.shape)
    w_lam = rng.standard_normal(p.xi.shape)
    g = SFAdjoint(orc).gradient(p.xi, p.xi, lam0, L, w_xi, w_lam)
    assert np.all(g.g_xi == 0.0)
    h = 1e-6
    for which, gv in ((1, g.g_xi0), (2, g.g_lam0)):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in p.xi.shape)
            args = [p.xi.copy(), p.xi.copy(), lam0.copy()]
            args[which][idx] += h
            fp = loss_value(orc, *args, L, w_xi, w_lam)
            args[which][idx] -= 2 * h
            fm = loss_value(orc, *args, L, w_xi, w_lam)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gv[idx]) <= 1e-6 * max(1.0, abs(fd)), (which, idx, fd, gv[idx])


# ------------------------------------------------------------- moving obstacles
def test_moving_obstacle_residual_is_the_closed_form_overlap():
    """A robot parked at the origin and an obstacle crossing it along x from
    -1 to +1 over the horizon: at sample k the obstacle row's residual has
    length max(0, a_o - |c(tau_k)|), |c(tau_k)| = |2 tau_k - 1| (metres)."""
    T, nc, ao = 41, 7, 0.3
    xi = np.zeros((2, 1, nc))
    box = np.array([[-5.0, -5.0], [5.0, 5.0]])
    bnd = np.zeros((1, 2, 2))
    obs = np.array([[-1.0, 0.0, ao]])
    orc = O.SFOracle(1, 1, nc, T, RHO, 0.4, box, obs, bnd,
                     obstacle_displacement=np.array([[2.0, 0.0]]))
    r1, r2, _, _, _ = orc.residual_terms(orc.flat(xi))
    tau = np.arange(T) / (T - 1)
    expect = np.sqrt(np.sum(np.maximum(0.0, ao - np.abs(2 * tau - 1)) ** 2))
    assert abs(np.linalg.norm(r1) - expect) < 1e-12
    assert np.linalg.norm(r2) == 0.0


def test_zero_displacement_is_the_static_oracle():
    cfg = scaled(WORKLOADS[3], n_robots=(3, 3), n_obs=(2, 2), arena=4.0, n_steps=25)
    p = make_problem(cfg, 3)
    a = O.SFOracle.for_problem(p, RHO).solve(p.xi, n_iters=15).xi_bar
    b = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles, p.boundary,
                   obstacle_displacement=np.zeros((p.M, 2))).solve(p.xi, n_iters=15).xi_bar
    np.testing.assert_array_equal(a, b)


def test_moving_obstacle_adjoint_matches_central_finite_differences(fd_case):
    p, _, rng = fd_case
    L = 12
    # first displacement (fixed seeds) whose iterates keep every pair,
    # obstacle and box quantity away from its kink (else reseed)
    for seed in range(20):
        disp = np.random.default_rng(100 + seed).uniform(-1.0, 1.0, (p.M, 2))
        orc = O.SFOracle(p.n, p.M, p.n_coef, p.n_steps, RHO, p.a, p.box, p.obstacles,
                         p.boundary, obstacle_displacement=disp)
        its = orc.solve(p.xi, p.xi, None, L, keep_iterates=True).iterates
        if _kink_margin(orc, its) > 1e-4:
            break
    else:
        pytest.fail("no kink-free displacement among the seeds")
    w_xi = rng.standard_normal(p.xi.shape)
    w_lam = rng.standard_normal(p.xi.shape)
    g = SFAdjoint(orc).gradient(p.xi, p.xi, None, L, w_xi, w_lam)
    h = 1e-6
    for which, gv in ((0, g.g_xi), (1, g.g_xi0)):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in p.xi.shape)
            args = [p.xi.copy(), p.xi.copy(), None]
            args[which][idx] += h
            fp = loss_value(orc, *args, L, w_xi, w_lam)
            args[which][idx] -= 2 * h
            fm = loss_value(orc, *args, L, w_xi, w_lam)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gv[idx]) <= 1e-6 * max(1.0, abs(fd)), (which, idx, fd, gv[idx])
