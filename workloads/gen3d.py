"""Seeded synthetic workloads of the 3D (spheroid) SF.

The 3D variant of the projection problem: robots are axis-aligned spheroids
(a/2, a/2, b/2) and obstacles spheroids inflated by the robot, (a_o, a_o, b_o)
(problem formulation; Appendix eqs. inter_robot_polar, workspace_polar).  As
in the planar generator, straight start-to-goal lines plus seeded Gaussian
noise on every coefficient stand in for the flow sampler.  The paper's 3D rows
(16 and 32 robots) give robot counts only; the arena, heights and sizes below
are proposed values in the spirit of the planar workloads.

Conventions: arena [-side/2, side/2]^2 x [-height/2, height/2]; box bounds
shrunk by the robot's half-extent per axis; a = 2 r_robot, b = 2 h_robot (the
minimum centre distances in the horizontal plane and along z); a_o = r_o +
r_robot, b_o = h_o + h_robot.  Holds no arithmetic of the SF itself.

Random streams: PCG64 seeded with SeedSequence([cfg_id, problem_idx]) for the
context and SeedSequence([cfg_id, problem_idx, 0, 1]) for the noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .gen import straight_coefficients

DIM = 3


@dataclass(frozen=True)
class SFConfig3D:
    cfg_id: int
    name: str
    n_robots: Tuple[int, int]
    n_obs: Tuple[int, int]
    side: float                      # arena side in x and y [m]
    height: float                    # arena extent in z [m]
    r_robot: float                   # horizontal semi-axis
    h_robot: float                   # vertical semi-axis
    r_obs: Tuple[float, float]       # obstacle horizontal semi-axis range
    h_obs: Tuple[float, float]       # obstacle vertical semi-axis range
    n_coef: int
    n_steps: int
    batch: int
    iters: int
    sigma: float
    description: str = ""


WORKLOADS_3D = {
    16: SFConfig3D(16, "3d_16r", (16, 16), (10, 10), 8.0, 4.0, 0.2, 0.3, (0.2, 0.5),
                   (0.3, 0.8), 11, 100, batch=64, iters=100, sigma=0.3,
                   description="64 problems of 16 spheroid robots, 10 spheroid "
                               "obstacles, 8x8x4 m arena"),
    32: SFConfig3D(32, "3d_32r", (32, 32), (20, 20), 12.0, 6.0, 0.2, 0.3, (0.2, 0.5),
                   (0.3, 0.8), 11, 100, batch=64, iters=100, sigma=0.3,
                   description="64 problems of 32 spheroid robots, 20 spheroid "
                               "obstacles, 12x12x6 m arena"),
    48: SFConfig3D(48, "3d_uneven", (4, 40), (0, 12), 10.0, 5.0, 0.2, 0.3, (0.2, 0.5),
                   (0.3, 0.8), 11, 100, batch=24, iters=100, sigma=0.3,
                   description="24 problems, robots U{4..40}, obstacles U{0..12}"),
}


@dataclass
class Problem3D:
    """One 3D SF instance (float64; coefficient stacking axis-major)."""
    n: int
    M: int
    n_coef: int
    n_steps: int
    a: float                      # horizontal minimum centre distance
    b: float                      # vertical minimum centre distance
    box: np.ndarray               # [2][3]
    obstacles: np.ndarray         # [M][5]: x, y, z, a_o, b_o
    boundary: np.ndarray          # [n][2][3]
    xi: np.ndarray                # [3][n][n_coef]
    straight: np.ndarray
    seed: Tuple[int, ...] = field(default_factory=tuple)
    dim: int = DIM

    @property
    def xi0(self) -> np.ndarray:
        return self.xi.copy()

    @property
    def lam0(self) -> np.ndarray:
        return np.zeros_like(self.xi)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _scaled_dist(p, q, sx, sz):
    d = p - q
    return np.sqrt((d[..., 0] ** 2 + d[..., 1] ** 2) / sx ** 2 + d[..., 2] ** 2 / sz ** 2)


def make_problem3d(cfg: SFConfig3D, idx: int) -> Problem3D:
    ctx = _rng(cfg.cfg_id, idx)
    n = int(ctx.integers(cfg.n_robots[0], cfg.n_robots[1] + 1))
    M = int(ctx.integers(cfg.n_obs[0], cfg.n_obs[1] + 1))
    hi = np.array([cfg.side / 2 - cfg.r_robot, cfg.side / 2 - cfg.r_robot,
                   cfg.height / 2 - cfg.h_robot])
    a, b = 2 * cfg.r_robot, 2 * cfg.h_robot

    def points(count):
        pts = np.zeros((count, 3))
        for i in range(count):
            for _ in range(100000):
                p = ctx.uniform(-hi, hi)
                if i == 0 or np.min(_scaled_dist(pts[:i], p, a, b)) >= 1.5:
                    pts[i] = p
                    break
            else:
                raise RuntimeError("could not place robots")
        return pts

    start, goal = points(n), points(n)
    ends = np.concatenate([start, goal])
    obs = np.zeros((M, 5))
    for m in range(M):
        ao = ctx.uniform(*cfg.r_obs) + cfg.r_robot
        bo = ctx.uniform(*cfg.h_obs) + cfg.h_robot
        for t in range(100000):
            c = ctx.uniform([-cfg.side / 2, -cfg.side / 2, -cfg.height / 2],
                            [cfg.side / 2, cfg.side / 2, cfg.height / 2])
            if np.min(_scaled_dist(ends, c, ao, bo)) <= 1.1:
                continue
            if t < 2000 and m > 0:
                # disjoint bounding spheres, 0.1 m apart
                rad = np.maximum(obs[:m, 3], obs[:m, 4])
                if np.any(np.linalg.norm(obs[:m, :3] - c, axis=1) < rad + max(ao, bo) + 0.1):
                    continue
            obs[m] = (c[0], c[1], c[2], ao, bo)
            break
        else:
            raise RuntimeError("could not place an obstacle")
    straight = straight_coefficients(start, goal, cfg.n_coef)
    xi = straight + cfg.sigma * _rng(cfg.cfg_id, idx, 0, 1).standard_normal(straight.shape)
    return Problem3D(n=n, M=M, n_coef=cfg.n_coef, n_steps=cfg.n_steps, a=a, b=b,
                     box=np.stack([-hi, hi]), obstacles=obs,
                     boundary=np.stack([start, goal], axis=1), xi=xi, straight=straight,
                     seed=(cfg.cfg_id, idx))


def make_batch3d(cfg: SFConfig3D, batch: Optional[int] = None, first: int = 0) -> List[Problem3D]:
    B = cfg.batch if batch is None else batch
    return [make_problem3d(cfg, first + q) for q in range(B)]


def scaled3d(cfg: SFConfig3D, **kw) -> SFConfig3D:
    return replace(cfg, **kw)


@dataclass
class PackedBatch3D:
    """Flat arrays in the C-ABI layout of the 3D SF (n_dim = 3)."""
    n_robots: np.ndarray        # int32 [B]
    n_obs: np.ndarray           # int32 [B]
    robot_ab: np.ndarray        # float32 [B][2] = a, b
    box: np.ndarray             # float32 [B][2][3]
    xi: np.ndarray              # float32 [sum 3 n nc]
    xi0: np.ndarray
    lam0: np.ndarray
    boundary: np.ndarray        # float32 [sum n][2][3]
    obstacles: np.ndarray       # float32 [sum M][5]
    n_coef: int
    n_steps: int


def pack3d(problems: Sequence[Problem3D], dtype=np.float32) -> PackedBatch3D:
    nc, T = problems[0].n_coef, problems[0].n_steps
    if any(p.n_coef != nc or p.n_steps != T for p in problems):
        raise ValueError("all problems of a batch share n_coef and n_steps")
    obs = [p.obstacles.reshape(-1) for p in problems]
    return PackedBatch3D(
        n_robots=np.array([p.n for p in problems], dtype=np.int32),
        n_obs=np.array([p.M for p in problems], dtype=np.int32),
        robot_ab=np.array([[p.a, p.b] for p in problems], dtype=dtype),
        box=np.stack([p.box for p in problems]).astype(dtype),
        xi=np.concatenate([p.xi.ravel() for p in problems]).astype(dtype),
        xi0=np.concatenate([p.xi0.ravel() for p in problems]).astype(dtype),
        lam0=np.concatenate([p.lam0.ravel() for p in problems]).astype(dtype),
        boundary=np.concatenate([p.boundary.ravel() for p in problems]).astype(dtype),
        obstacles=np.concatenate(obs).astype(dtype) if sum(o.size for o in obs)
        else np.zeros(0, dtype),
        n_coef=nc, n_steps=T)


def unpack3d(flat: np.ndarray, problems: Sequence[Problem3D]) -> List[np.ndarray]:
    out, o = [], 0
    for p in problems:
        size = DIM * p.n * p.n_coef
        out.append(np.asarray(flat[o:o + size]).reshape(DIM, p.n, p.n_coef))
        o += size
    return out
