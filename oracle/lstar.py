"""Iteration count L* at which every problem of a workload reaches residual <= tol.

TEST INFRASTRUCTURE (uses only the FP64 oracle and the seeded generator).  The
benchmark runs every problem for exactly L* iterations; L* is the smallest
multiple of 10, at least the workload's own iteration count, at which the
oracle's residual sqrt(||r_1||^2 + ||r_2||^2) of the current iterate is <= tol
for all problems at once (the residual is not monotone, so a problem that
dipped below tol earlier may be above it at L*).  Capped at `cap`; when capped
the fraction of problems at or below tol is reported instead.

  python -m oracle.lstar --config 3 --rho 0.5 [--problems 64] [--cap 2000] [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from multiprocessing import Pool

import numpy as np


def _history(args):
    cfg_id, b, rho, cap = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle.sf import SFOracle
    from workloads import WORKLOADS, make_batch
    cfg = WORKLOADS[cfg_id]
    p = make_batch(cfg, batch=b + 1)[b]
    orc = SFOracle.for_problem(p, rho)
    res = orc.solve(p.xi, n_iters=cap, keep_history=True)
    h = np.hypot(res.history[:, 0], res.history[:, 1])      # residual of iterate l
    return b, np.append(h, res.residual)                    # ... and of iterate cap


def lstar(cfg_id: int, rho: float, problems: int, cap: int = 2000, tol: float = 1e-3,
          jobs: int = 8):
    from workloads import WORKLOADS
    cfg = WORKLOADS[cfg_id]
    with Pool(jobs) as pool:
        hist = dict(pool.imap_unordered(_history, [(cfg_id, b, rho, cap)
                                                   for b in range(problems)]))
    H = np.stack([hist[b] for b in range(problems)])        # [B][cap+1]
    first = [int(np.argmax(h <= tol)) if np.any(h <= tol) else -1 for h in H]
    L = None
    for cand in range(max(10, int(np.ceil(cfg.iters / 10)) * 10), cap + 1, 10):
        if np.all(H[:, cand] <= tol):
            L = cand
            break
    out = dict(config=cfg_id, rho=rho, problems=problems, cap=cap, tol=tol,
               lstar=L if L is not None else cap,
               capped=L is None,
               frac_at_lstar=float(np.mean(H[:, L if L is not None else cap] <= tol)),
               first_reach=first,
               residual_at_config_iters=[float(x) for x in H[:, cfg.iters]])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--rho", type=float, default=0.5)
    ap.add_argument("--problems", type=int, default=None)
    ap.add_argument("--cap", type=int, default=2000)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-3)
    a = ap.parse_args(argv)
    from workloads import WORKLOADS
    n = a.problems or WORKLOADS[a.config].batch
    print(json.dumps(lstar(a.config, a.rho, n, a.cap, a.tol, a.jobs)))


if __name__ == "__main__":
    sys.exit(main())
