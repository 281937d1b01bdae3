"""FP64 oracle of the candidate selection around the SF.

TEST INFRASTRUCTURE ONLY (imported by the tests, never by the product path);
shares no code with the HIP implementation.

The planning pipeline of the paper ("Validation and Benchmarking": the
three-stage figure and "Qualitative Validation"): sampled candidate
trajectories of one context are sorted by constraint residual (eq.
primal_residual), the best k (the paper uses about 256 samples and k = 10)
are refined by the SF, and the feasible refined trajectory with the least
smoothness cost is returned.  The smoothness cost is the squared acceleration
norm summed over the time steps and averaged over the robots ("Smoothness
Cost", "Implementation Details").

Readings fixed here (each is a named choice):
  S1  "feasible" means primal residual <= tol (the benchmark's 1e-3 m); when
      no refined candidate is feasible the one of least residual is returned.
  S2  ranking key: ||r_1||^2 + ||r_2||^2 (monotone in the residual of R4),
      taken in float32 with each operation rounded, so that a ranking of
      float32 residual rows is reproduced exactly; ties go to the lower index;
      a row with its status word set ranks last.
  S3  accelerations are time derivatives: t = tau * t_final, so p'' =
      (1/t_final^2) d^2 p / d tau^2 (t_final = 5 s for the benchmark contexts).
"""
from __future__ import annotations

import numpy as np

from .basis import accel_basis
from .sf import SFOracle


def smoothness_cost(xi: np.ndarray, n_steps: int, t_final: float) -> float:
    """(1/n) sum_i sum_k |p_i''(t_k)|^2 for xi [2][n][n_coef] (S3)."""
    xi = np.asarray(xi, dtype=np.float64)
    n, nc = xi.shape[1], xi.shape[2]
    D = accel_basis(nc, n_steps) / t_final ** 2
    acc = np.einsum("kc,aic->aik", D, xi)
    return float(np.sum(acc ** 2) / n)


def residual_key(row) -> np.float32:
    """S2: float32 key of a residual row (||r_1||, ||r_2||, ., status)."""
    r1, r2 = np.float32(row[0]), np.float32(row[1])
    with np.errstate(over="ignore", invalid="ignore"):
        k = np.float32(np.float32(r1 * r1) + np.float32(r2 * r2))
    if row[3] != 0 or not np.isfinite(k):
        return np.float32(np.inf)
    return k


def rank_residual(rows, k: int) -> np.ndarray:
    """Indices of the k smallest keys, increasing, ties by index (S2)."""
    keys = [residual_key(r) for r in np.asarray(rows, dtype=np.float32)]
    order = sorted(range(len(keys)), key=lambda b: (keys[b], b))
    return np.array(order[:k], dtype=np.int64)


def select_best(rows, cost, tol: float) -> int:
    """S1: feasible (key <= tol^2 in float32) of least cost, ties by key then
    index; else least key, ties by index.  Non-finite costs count as +inf."""
    rows = np.asarray(rows, dtype=np.float32)
    tol2 = np.float32(np.float32(tol) * np.float32(tol))
    best, best_t = None, None
    for b, row in enumerate(rows):
        key = residual_key(row)
        c = np.float32(cost[b])
        c = c if np.isfinite(c) else np.float32(np.inf)
        feas = key <= tol2
        t = (0, c, key, b) if feas else (1, key, key, b)
        if best_t is None or t < best_t:
            best, best_t = b, t
    return int(best)


def residual_row(orc: SFOracle, xib) -> np.ndarray:
    """(||r_1||, ||r_2||, 0, 0) of xi_bar, FP64."""
    r1, r2, _, _, _ = orc.residual_terms(orc.flat(xib))
    return np.array([np.linalg.norm(r1), np.linalg.norm(r2), 0.0, 0.0])


def select_candidates(problems, k: int, n_iters: int, tol: float, t_final: float,
                      rho: float) -> dict:
    """The pipeline on candidates of one context (problems share everything
    but xi): raw residual rows, the top-k, the k refined solutions (xi_bar^0 =
    xi, lambda^0 = 0), their residual rows and smoothness costs, and the chosen
    index into the top-k list."""
    orc = SFOracle.for_problem(problems[0], rho)
    raw = np.stack([residual_row(orc, p.xi) for p in problems])
    top = rank_residual(raw, k)
    refined, rows, costs = [], [], []
    for b in top:
        r = orc.solve(problems[b].xi, n_iters=n_iters)
        refined.append(r.xi_bar)
        rows.append([r.res_r1, r.res_r2, 0.0, 0.0])
        costs.append(smoothness_cost(r.xi_bar, problems[0].n_steps, t_final))
    rows = np.array(rows)
    best = select_best(rows, costs, tol)
    return dict(residual_raw=raw, topk=top, xi_refined=refined, residual_refined=rows,
                cost=np.array(costs), best=best)


__all__ = ["accel_basis", "smoothness_cost", "residual_key", "rank_residual", "select_best",
           "residual_row", "select_candidates"]
