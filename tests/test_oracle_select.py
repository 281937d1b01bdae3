"""Pins of the candidate-selection oracle (oracle/select.py) against facts that
do not come from it: a library routine for the basis derivative, closed forms
of the smoothness cost, and brute-force orderings."""
import numpy as np
import pytest
from scipy.interpolate import BPoly

from oracle.select import (accel_basis, rank_residual, residual_key, select_best,
                           smoothness_cost)
from workloads import straight_coefficients


@pytest.mark.parametrize("nc,T", [(11, 100), (15, 120), (3, 7), (4, 50)])
def test_accel_basis_matches_scipy_bernstein_derivative(nc, T):
    tau = np.arange(T) / (T - 1)
    D = accel_basis(nc, T)
    for c in range(nc):
        coef = np.zeros((nc, 1))
        coef[c, 0] = 1.0
        ref = BPoly(coef, [0.0, 1.0]).derivative(2)(tau)
        np.testing.assert_allclose(D[:, c], ref, rtol=1e-9, atol=1e-9 * max(1.0, np.abs(ref).max()))


def test_accel_basis_of_low_degrees_is_zero():
    # degree 1 (two coefficients): straight lines only
    assert np.all(accel_basis(2, 20) == 0.0)


def test_straight_lines_have_zero_smoothness_cost():
    rng = np.random.default_rng(3)
    starts, goals = rng.uniform(-3, 3, (5, 2)), rng.uniform(-3, 3, (5, 2))
    xi = straight_coefficients(starts, goals, 11)
    assert smoothness_cost(xi, 100, 5.0) < 1e-20


@pytest.mark.parametrize("t_final", [1.0, 5.0])
def test_quadratic_trajectory_has_constant_acceleration(t_final):
    """x(tau) = tau^2 has Bernstein coefficients c_j = j (j - 1) / (N (N - 1))
    (degree elevation of tau^2); its time acceleration is 2 / t_final^2 at
    every step, so for one robot with y = 0 the cost is T (2 / t_final^2)^2."""
    nc, T = 11, 100
    N = nc - 1
    j = np.arange(nc)
    xi = np.zeros((2, 1, nc))
    xi[0, 0] = j * (j - 1) / (N * (N - 1))
    expect = T * (2.0 / t_final ** 2) ** 2
    assert smoothness_cost(xi, T, t_final) == pytest.approx(expect, rel=1e-10)


def test_cost_is_an_average_over_robots():
    nc, T = 11, 60
    rng = np.random.default_rng(5)
    one = rng.standard_normal((2, 1, nc))
    both = np.concatenate([one, one], axis=1)
    assert smoothness_cost(both, T, 5.0) == pytest.approx(smoothness_cost(one, T, 5.0), rel=1e-12)


def test_residual_key_is_float32_and_flags_rank_last():
    row = np.array([0.3, 0.4, 0.0, 0.0], dtype=np.float32)
    k = residual_key(row)
    assert k.dtype == np.float32
    r1, r2 = np.float32(0.3), np.float32(0.4)
    assert k == np.float32(np.float32(r1 * r1) + np.float32(r2 * r2))
    assert residual_key(np.array([0.0, 0.0, 0.0, 1.0])) == np.inf
    assert residual_key(np.array([np.nan, 0.0, 0.0, 0.0])) == np.inf


def test_rank_matches_brute_force_with_ties_and_flags():
    rng = np.random.default_rng(7)
    rows = np.zeros((40, 4), dtype=np.float32)
    rows[:, 0] = rng.choice([0.1, 0.2, 0.3], 40)          # many exact ties
    rows[:, 1] = rng.choice([0.0, 0.05], 40)
    rows[5, 3] = 1.0                                       # flagged
    rows[9, 0] = np.inf
    keys = [(float(np.float32(np.float32(r[0] * r[0]) + np.float32(r[1] * r[1])))
             if r[3] == 0 and np.isfinite(r[0]) else np.inf, b) for b, r in enumerate(rows)]
    brute = [b for _, b in sorted(keys)]
    for k in (1, 10, 40):
        assert list(rank_residual(rows, k)) == brute[:k]


def test_select_best_rules():
    tol = 1e-3
    rows = np.array([[2e-3, 0, 0, 0],      # infeasible, least residual among infeasible
                     [5e-4, 0, 0, 0],      # feasible, cost 3
                     [1e-4, 0, 0, 0],      # feasible, cost 2 (tie with 3)
                     [2e-4, 0, 0, 0],      # feasible, cost 2, larger key than 2
                     [0.0, 0, 0, 1.0]],    # flagged
                    dtype=np.float32)
    cost = np.array([0.1, 3.0, 2.0, 2.0, 0.0])
    assert select_best(rows, cost, tol) == 2
    cost_nan = cost.copy()
    cost_nan[2] = np.nan                   # non-finite cost counts as +inf
    assert select_best(rows, cost_nan, tol) == 3
    infeasible = rows.copy()
    infeasible[1:4, 0] = [3e-3, 4e-3, 5e-3]
    assert select_best(infeasible, cost, tol) == 0
