"""Second derivative of the Bernstein basis for the oracle (test
infrastructure only; shares no code with the HIP path)."""
from __future__ import annotations

from math import comb

import numpy as np


def accel_basis(n_coef: int, n_steps: int) -> np.ndarray:
    """Second tau-derivative of the Bernstein basis at tau_k = k/(T-1),
    [T][n_coef], by differentiating each basis polynomial's power-series
    coefficients (C(N,c) tau^c (1-tau)^(N-c) expanded with the binomial
    theorem) twice -- a route independent of the degree-elevation identity
    used by the library."""
    N = n_coef - 1
    tau = np.arange(n_steps, dtype=np.float64) / (n_steps - 1)
    out = np.zeros((n_steps, n_coef))
    for c in range(n_coef):
        # C(N,c) tau^c (1-tau)^(N-c) = sum_q C(N,c) C(N-c,q) (-1)^q tau^(c+q)
        for q in range(N - c + 1):
            p = c + q
            if p < 2:
                continue
            coef = comb(N, c) * comb(N - c, q) * (-1.0) ** q
            out[:, c] += coef * p * (p - 1) * tau ** (p - 2)
    return out
