"""FP64 CPU oracle of the safety-filter (SF) fixed-point iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the HIP
path: it builds the paper's matrices explicitly (F, G, A, the KKT matrix) and
takes the alternating-minimisation steps one by one, in the order and notation
of the Appendix ("Derivation of Fixed-Point Iteration Form"), in float64.

Readings of the paper that this oracle fixes (each is a named choice):
  R1  the KKT matrix carries rho*G^T G and eta carries rho*G^T(h - s): both
      follow from the augmented Lagrangian (eq. aug_lag); the printed M/eta
      omit them.
  R2  s-step: s = max(0, h - G xi_bar), the minimiser over s >= 0 (the printed
      sign is flipped).
  R3  r_1 = F xi_bar^l - e^{l+1} (the printed r_1 drops the bar).
  R4  reported residual = sqrt(||r_1||^2 + ||r_2||^2), in metres.
  R5  fixed-point residual = ||z^{l+1} - z^l||^2 with z = (xi_bar, lambda).
  R6  F_r = D (x) W, D the pair incidence matrix (rows (i, j), i < j).
  R7  G = [W_bar; -W_bar], h = [p_max; -p_min] per axis (two-sided box).
  R10 2D: beta = pi/2, so sin(beta) = 1 and only a, a_o enter.
  R11 xi_bar^{l+1} = first block of K^{-1} [eta; b].
  R12 atan2(0, 0) = 0; ||Delta|| = a is inactive (d = 1 exactly, e = Delta).
  R13 Jacobi order: alpha, d, s from xi_bar^l; lambda before xi_bar.
  R15 without an initialisation network xi_bar^0 = xi, lambda^0 = 0.
  R16 tau_k = k/(T-1): both ends of the horizon are sampled.
  R17 boundary rows are positions at k = 0 and k = K only.
  D1  moving obstacles: centre c_m + d_m tau_k at time sample k (d_m the
      displacement over the horizon); F and K are unchanged, only e moves.
  O1  objective="accel" (the trajectory optimiser of the problem formulation,
      used for the paper's dataset): the identity block of the KKT matrix
      becomes Wdd^T Wdd per robot and axis (Wdd the second tau-derivative of
      the basis) and the sample drops out of eta; everything else is the SF.
  Q1  3D (dim=3, spheroids (a, a, b) and (a_o, a_o, b_o), eqs.
      inter_robot_polar, workspace_polar, f_e): the alpha, beta and d steps
      are all taken at xi_bar^l (Jacobi order as R13).  The paper prints a
      closed form for the alpha step only (after eq. d_step) and refers the
      rest to prior work.  alpha = atan2(dy, dx), the printed form and the
      exact minimiser over alpha.  beta is this oracle's reading of eq.
      beta_step: beta = atan2(rho_xy / a, dz / b) with rho_xy = dx cos(alpha) +
      dy sin(alpha), the polar angle of Delta in the spheroid's scaled
      coordinates, so that u(alpha, beta) points along Delta.  For a != b this
      is not the Euclidean argmin over beta with d held at its previous value;
      for spheres (a = b) it is.  d is the exact least-squares minimiser over
      d >= 1 of ||Delta - d u(alpha, beta)||^2 with alpha, beta fixed.  At
      Delta = 0: alpha = beta = 0, so u = (0, 0, b) and e = (0, 0, b) (the tie
      convention of R12 in 3D).
"""
from __future__ import annotations

from dataclasses import dataclass
from math import comb
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import accel_basis

N_DIM = 2          # the planar SF; dim=3 selects the spheroid variant (Q1)


# --------------------------------------------------------------------------
# Polynomial parametrisation (eq. poly): positions p = W xi per axis.
# --------------------------------------------------------------------------
def bernstein_W(n_coef: int, n_steps: int) -> np.ndarray:
    """W[k, c] = C(n_coef-1, c) tau_k^c (1 - tau_k)^(n_coef-1-c), tau_k = k/(T-1)."""
    deg = n_coef - 1
    tau = np.arange(n_steps, dtype=np.float64) / (n_steps - 1)
    W = np.empty((n_steps, n_coef))
    for c in range(n_coef):
        W[:, c] = comb(deg, c) * tau ** c * (1.0 - tau) ** (deg - c)
    return W


# --------------------------------------------------------------------------
# Operators of the reformulated problem (eqs. reform_*, f_e; matrix F_r, F_o).
# Rows/columns are per axis; the full operators are block diagonal over axes
# because the coefficient vector is stacked axis-major.
# --------------------------------------------------------------------------
def pair_list(n: int):
    """Unordered robot pairs (i, j), i < j, in the row order of
    F_r = [F_{r,1}; ...; F_{r,n-1}]: block i holds the pairs (i, j), j > i."""
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def pair_incidence(n: int) -> np.ndarray:
    """D with rows [F_{r,i}] = [F_i, -I]: +1 in column i, -1 in column j."""
    pairs = pair_list(n)
    D = np.zeros((len(pairs), n))
    for row, (i, j) in enumerate(pairs):
        D[row, i] = 1.0
        D[row, j] = -1.0
    return D


@dataclass
class Operators:
    n: int
    M: int
    n_coef: int
    n_steps: int
    W: np.ndarray            # [T, n_coef]
    F_axis: sp.csr_matrix     # [(P + n*M)*T, n*n_coef], P = n(n-1)/2
    G_axis: sp.csr_matrix     # [2*n*T, n*n_coef]
    A_axis: np.ndarray        # [2n, n*n_coef]
    F: sp.csr_matrix          # block-diag over axes
    G: sp.csr_matrix
    A: np.ndarray
    n_pair_rows: int          # P*T rows per axis
    n_obs_rows: int           # n*M*T rows per axis
    dim: int = N_DIM          # workspace dimension n_d (2 or 3)


def build_operators(n: int, M: int, n_coef: int, n_steps: int, dim: int = N_DIM) -> Operators:
    W = bernstein_W(n_coef, n_steps)
    Ws = sp.csr_matrix(W)
    D = sp.csr_matrix(pair_incidence(n))
    F_r = sp.kron(D, Ws, format="csr")                                   # R6
    # Block-diagonal stacks are written as Kronecker products with identities
    # (I (x) X has X on its diagonal blocks): the same matrices as stacking
    # the blocks one by one, built without per-block copies.
    if M > 0:
        P = sp.kron(np.ones((M, 1)), Ws, format="csr")                    # 1_M (x) W
        F_o = sp.kron(sp.identity(n, format="csr"), P, format="csr")      # I_n (x) P
    else:
        F_o = sp.csr_matrix((0, n * n_coef))
    F_axis = sp.vstack([F_r, F_o], format="csr")
    Wbar = sp.kron(sp.identity(n, format="csr"), Ws, format="csr")       # eq. poly
    G_axis = sp.vstack([Wbar, -Wbar], format="csr")                      # R7
    A1 = np.stack([W[0], W[-1]])                                         # R17
    A_axis = np.kron(np.eye(n), A1)
    F = sp.kron(sp.identity(dim, format="csr"), F_axis, format="csr")
    G = sp.kron(sp.identity(dim, format="csr"), G_axis, format="csr")
    A = sla.block_diag(*([A_axis] * dim))
    return Operators(n, M, n_coef, n_steps, W, F_axis, G_axis, A_axis, F, G, A,
                     F_r.shape[0], F_o.shape[0], dim)


def objective_block(ops: Operators, objective: str) -> np.ndarray:
    """Quadratic term of the xi_bar step's objective: I for the projection
    (eq. proj_cost, 1/2 ||xi_bar - xi||^2); for the acceleration objective
    (the smoothness cost of the trajectory optimiser, 1/2 sum ||Wdd xi_bar||^2
    per robot and axis, Wdd the second tau-derivative of the basis) the block
    diagonal of Wdd^T Wdd."""
    Sz = ops.F.shape[1]
    if objective == "projection":
        return np.eye(Sz)
    if objective == "accel":
        D = accel_basis(ops.n_coef, ops.n_steps)
        return np.kron(np.eye(ops.dim * ops.n), D.T @ D)
    raise ValueError(objective)


def kkt_matrix(ops: Operators, rho: float, include_G: bool = True,
               objective: str = "projection") -> np.ndarray:
    """K = [[Q + rho (F^T F + G^T G), A^T], [A, 0]] with Q = I for the
    projection (R1, R11)."""
    Sz = ops.F.shape[1]
    FtF = (ops.F.T @ ops.F).toarray()
    Q = objective_block(ops, objective) + rho * FtF
    if include_G:
        Q += rho * (ops.G.T @ ops.G).toarray()
    nA = ops.A.shape[0]
    K = np.zeros((Sz + nA, Sz + nA))
    K[:Sz, :Sz] = Q
    K[:Sz, Sz:] = ops.A.T
    K[Sz:, :Sz] = ops.A
    return K


# --------------------------------------------------------------------------
# Problem data as the paper's vectors.
# --------------------------------------------------------------------------
def h_vector(ops: Operators, box: np.ndarray) -> np.ndarray:
    """h = [p_max 1; -p_min 1] per axis (eq. workspace_con, R7)."""
    nT = ops.n * ops.n_steps
    parts = []
    for ax in range(ops.dim):
        parts.append(np.concatenate([np.full(nT, box[1, ax]), np.full(nT, -box[0, ax])]))
    return np.concatenate(parts)


def b_vector(boundary: np.ndarray) -> np.ndarray:
    """b = (b_{i,0}, b_{i,K}) per robot, axis-major (eq. boundary_con)."""
    n, dim = boundary.shape[0], boundary.shape[2]
    return np.concatenate([boundary[:, :, ax].reshape(n * 2) for ax in range(dim)])


def obstacle_rows(ops: Operators, obstacles: np.ndarray, displacement=None):
    """Obstacle centres per axis stacked over (robot, obstacle, time) as F_o's
    rows, and the sizes: a_o in 2D (obstacles [M][3] = x, y, a_o); the pair
    (a_o, b_o) in 3D (obstacles [M][5] = x, y, z, a_o, b_o).  With a
    displacement d ([M][dim]) obstacle m's centre at time sample k is
    c_m + d_m tau_k (moving obstacles; tau_k = k/(T-1))."""
    n, M, T, dim = ops.n, ops.M, ops.n_steps, ops.dim
    if M == 0:
        z = np.zeros(0)
        return [z] * dim, (z if dim == 2 else (z, z))
    tau = np.arange(T, dtype=np.float64) / (T - 1)
    d = np.zeros((M, dim)) if displacement is None else np.asarray(displacement, np.float64)
    cen = [np.tile((obstacles[:, ax][:, None] + d[:, ax][:, None] * tau[None, :]).reshape(-1), n)
           for ax in range(dim)]
    size = [np.tile(np.repeat(obstacles[:, q], T), n) for q in range(dim, 2 * dim - 1)]
    return cen, (size[0] if dim == 2 else tuple(size))


# --------------------------------------------------------------------------
# Closed-form steps (eqs. alpha_step, d_step, s_step; 2D with beta = pi/2).
# --------------------------------------------------------------------------
def alpha_step(dx: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """alpha = atan2(dy, dx); atan2(0, 0) = 0 (R12)."""
    return np.arctan2(dy, dx)


def d_step(dx, dy, alpha, size):
    """argmin over 1 <= d <= inf of ||Delta - size*d*(cos a, sin a)||^2:
    the unconstrained minimiser (dx cos a + dy sin a)/size clipped below at 1."""
    return np.maximum(1.0, (dx * np.cos(alpha) + dy * np.sin(alpha)) / size)


def s_step(Gxi: np.ndarray, h: np.ndarray) -> np.ndarray:
    """s = max(0, h - G xi_bar) (R2)."""
    return np.maximum(0.0, h - Gxi)


def split_axes(v: np.ndarray, rows_per_axis: int, dim: int = N_DIM):
    return [v[ax * rows_per_axis:(ax + 1) * rows_per_axis] for ax in range(dim)]


def e_vector(ops: Operators, Fxi: np.ndarray, a: float, obs_cen, obs_ao):
    """e(alpha, beta, d) of eq. f_e, from the alpha and d steps at xi_bar^l.
    Returns e (stacked like F's rows) and the intermediates (alpha, d)."""
    R = ops.n_pair_rows + ops.n_obs_rows
    comp = split_axes(Fxi, R)
    Pr = ops.n_pair_rows
    # robot pairs: F_r xi_bar = p_i - p_j
    dx, dy = comp[0][:Pr], comp[1][:Pr]
    alpha = alpha_step(dx, dy)
    d = d_step(dx, dy, alpha, a)
    # robot-obstacle rows: F_o xi_bar = p_i, Delta = p_i - p_o
    ox = comp[0][Pr:] - obs_cen[0]
    oy = comp[1][Pr:] - obs_cen[1]
    alpha_o = alpha_step(ox, oy)
    d_o = d_step(ox, oy, alpha_o, obs_ao) if ops.M > 0 else np.zeros(0)
    ex = np.concatenate([a * d * np.cos(alpha), obs_cen[0] + obs_ao * d_o * np.cos(alpha_o)])
    ey = np.concatenate([a * d * np.sin(alpha), obs_cen[1] + obs_ao * d_o * np.sin(alpha_o)])
    return np.concatenate([ex, ey]), (alpha, d, alpha_o, d_o)


# --------------------------------------------------------------------------
# 3D closed-form steps (eqs. inter_robot_polar, workspace_polar, alpha_step,
# beta_step, d_step; reading Q1).  Delta = (dx, dy, dz), spheroid sizes (a, b).
# --------------------------------------------------------------------------
def beta_step(dx, dy, dz, alpha, a, b):
    """beta = atan2(rho_xy / a, dz / b), rho_xy = dx cos(alpha) + dy sin(alpha)."""
    rho_xy = dx * np.cos(alpha) + dy * np.sin(alpha)
    return np.arctan2(rho_xy / a, dz / b)


def spheroid_direction(alpha, beta, a, b):
    """u(alpha, beta) = (a cos(alpha) sin(beta), a sin(alpha) sin(beta), b cos(beta))."""
    return (a * np.cos(alpha) * np.sin(beta), a * np.sin(alpha) * np.sin(beta),
            b * np.cos(beta))


def d_step_3d(dx, dy, dz, alpha, beta, a, b):
    """argmin over 1 <= d <= inf of ||Delta - d u(alpha, beta)||^2: the least-squares
    d = <Delta, u> / <u, u>, clipped below at 1."""
    ux, uy, uz = spheroid_direction(alpha, beta, a, b)
    return np.maximum(1.0, (dx * ux + dy * uy + dz * uz) / (ux * ux + uy * uy + uz * uz))


def e_block_3d(dx, dy, dz, a, b):
    """e - centre = d u(alpha, beta) after the alpha, beta and d steps at Delta."""
    alpha = alpha_step(dx, dy)
    beta = beta_step(dx, dy, dz, alpha, a, b)
    d = d_step_3d(dx, dy, dz, alpha, beta, a, b)
    ux, uy, uz = spheroid_direction(alpha, beta, a, b)
    return d * ux, d * uy, d * uz


def e_vector_3d(ops: Operators, Fxi: np.ndarray, a: float, b: float, obs_cen, obs_ab):
    """e(alpha, beta, d) of eq. f_e in 3D (x, y, z blocks of F's rows)."""
    R = ops.n_pair_rows + ops.n_obs_rows
    comp = split_axes(Fxi, R, 3)
    Pr = ops.n_pair_rows
    ep = e_block_3d(comp[0][:Pr], comp[1][:Pr], comp[2][:Pr], a, b)
    if ops.M > 0:
        off = [comp[ax][Pr:] - obs_cen[ax] for ax in range(3)]
        eo = e_block_3d(off[0], off[1], off[2], obs_ab[0], obs_ab[1])
        eo = [obs_cen[ax] + eo[ax] for ax in range(3)]
    else:
        eo = [np.zeros(0)] * 3
    return np.concatenate([np.concatenate([ep[ax], eo[ax]]) for ax in range(3)]), None


# --------------------------------------------------------------------------
# The SF solver.
# --------------------------------------------------------------------------
@dataclass
class SFResult:
    xi_bar: np.ndarray            # [N_DIM][n][n_coef]
    lam: np.ndarray
    res_r1: float                 # ||r_1(xi_bar^L)||
    res_r2: float                 # ||r_2(xi_bar^L)||
    res_dz: float                 # ||z^L - z^{L-1}||
    history: Optional[np.ndarray] = None   # [L][3]: ||r1||, ||r2||, ||dz|| per iteration
    iterates: Optional[List[tuple]] = None  # (xi_bar^l, lambda^l) l = 0..L

    @property
    def residual(self) -> float:
        """R4: sqrt(||r_1||^2 + ||r_2||^2) of the returned xi_bar^L."""
        return float(np.hypot(self.res_r1, self.res_r2))


class SFOracle:
    """Literal SF for one problem (one context + one target xi).  dim=3 is the
    spheroid variant: robot_b is b, obstacles are [M][5] = x, y, z, a_o, b_o,
    box [2][3], boundary [n][2][3]."""

    def __init__(self, n: int, M: int, n_coef: int, n_steps: int, rho: float,
                 a: float, box: np.ndarray, obstacles: np.ndarray,
                 boundary: np.ndarray, include_G: bool = True,
                 objective: str = "projection", obstacle_displacement=None,
                 dim: int = N_DIM, robot_b: Optional[float] = None):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim = dim
        self.ops = build_operators(n, M, n_coef, n_steps, dim)
        self.rho = float(rho)
        self.a = float(a)
        self.robot_b = float(a if robot_b is None else robot_b)
        self.box = np.asarray(box, dtype=np.float64)
        self.obstacles = np.asarray(obstacles, dtype=np.float64).reshape(M, 2 * dim - 1)
        self.include_G = include_G
        self.h = h_vector(self.ops, self.box)
        self.b = b_vector(np.asarray(boundary, dtype=np.float64))
        self.obs_cen, self.obs_ao = obstacle_rows(self.ops, self.obstacles,
                                                  obstacle_displacement)
        self.objective = objective
        self.K = kkt_matrix(self.ops, self.rho, include_G, objective)
        self.K_lu = sla.lu_factor(self.K)            # pre-stored factorisation
        self.Sz = self.ops.F.shape[1]

    @classmethod
    def for_problem(cls, prob, rho: float, **kw) -> "SFOracle":
        dim = getattr(prob, "dim", N_DIM)
        if dim == 3:
            kw = dict(kw, dim=3, robot_b=prob.b)
        return cls(prob.n, prob.M, prob.n_coef, prob.n_steps, rho, prob.a,
                   prob.box, prob.obstacles, prob.boundary, **kw)

    # vector <-> [N_DIM][n][n_coef]
    def flat(self, x: np.ndarray) -> np.ndarray:
        return np.asarray(x, dtype=np.float64).reshape(-1)

    def shaped(self, v: np.ndarray) -> np.ndarray:
        return v.reshape(self.dim, self.ops.n, self.ops.n_coef).copy()

    def residual_terms(self, xib: np.ndarray):
        """r_1, r_2, e, s at xi_bar (steps alpha..s of one iteration)."""
        Fxi = self.ops.F @ xib
        if self.dim == 3:
            e, geo = e_vector_3d(self.ops, Fxi, self.a, self.robot_b, self.obs_cen, self.obs_ao)
        else:
            e, geo = e_vector(self.ops, Fxi, self.a, self.obs_cen, self.obs_ao)
        Gxi = self.ops.G @ xib
        s = s_step(Gxi, self.h)
        r1 = Fxi - e                                                     # R3
        r2 = Gxi - self.h + s
        return r1, r2, e, s, geo

    def step(self, xi: np.ndarray, xib: np.ndarray, lam: np.ndarray):
        """One application of the fixed-point operator T (eq. fixed_point):
        alpha, d, s from xi_bar^l; lambda^{l+1}; xi_bar^{l+1} = first block
        of K^{-1} eta.  Returns (xi_bar^{l+1}, lambda^{l+1}, ||r1||, ||r2||)."""
        rho, F, G = self.rho, self.ops.F, self.ops.G
        r1, r2, e, s, _ = self.residual_terms(xib)
        lam_new = lam - rho * (F.T @ r1) - rho * (G.T @ r2)             # lambda_step
        eta_top = rho * (F.T @ e) + lam_new
        if self.objective == "projection":
            eta_top = eta_top + xi                                       # the sample
        if self.include_G:
            eta_top = eta_top + rho * (G.T @ (self.h - s))               # R1
        sol = sla.lu_solve(self.K_lu, np.concatenate([eta_top, self.b]))
        return sol[:self.Sz], lam_new, float(np.linalg.norm(r1)), float(np.linalg.norm(r2))

    def solve(self, xi, xi0=None, lam0=None, n_iters: int = 100,
              keep_history: bool = False, keep_iterates: bool = False) -> SFResult:
        xi = self.flat(xi)
        xib = xi.copy() if xi0 is None else self.flat(xi0).copy()       # R15
        lam = np.zeros_like(xi) if lam0 is None else self.flat(lam0).copy()
        hist = np.zeros((n_iters, 3)) if keep_history else None
        its = [(xib.copy(), lam.copy())] if keep_iterates else None
        dz = 0.0
        for l in range(n_iters):
            xib_new, lam_new, n1, n2 = self.step(xi, xib, lam)
            dz = float(np.sqrt(np.sum((xib_new - xib) ** 2) + np.sum((lam_new - lam) ** 2)))
            if keep_history:
                hist[l] = (n1, n2, dz)
            xib, lam = xib_new, lam_new
            if keep_iterates:
                its.append((xib.copy(), lam.copy()))
        r1, r2, _, _, _ = self.residual_terms(xib)                       # R22
        return SFResult(self.shaped(xib), self.shaped(lam), float(np.linalg.norm(r1)),
                        float(np.linalg.norm(r2)), dz, hist, its)

    def residual_of(self, xib) -> float:
        r1, r2, _, _, _ = self.residual_terms(self.flat(xib))
        return float(np.hypot(np.linalg.norm(r1), np.linalg.norm(r2)))


def solve_problem(prob, rho: float, n_iters: int, xi0=None, lam0=None, **kw) -> SFResult:
    """Run the oracle on one generated problem (xi_bar^0 = xi, lambda^0 = 0 by default)."""
    orc = SFOracle.for_problem(prob, rho)
    return orc.solve(prob.xi, xi0, lam0, n_iters, **kw)
