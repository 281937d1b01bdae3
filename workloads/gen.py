"""Seeded synthetic safety-filter (SF) workloads.

This module produces the inputs of the SF projection problem (Sec. "Fast
Inference-Time Refinement", eqs. proj_cost..proj_robot): a sampled joint
trajectory xi, the boundary positions b, the box bounds, the robot size a and
the obstacle centres and inflated sizes a_o.  It stands in for the paper's
flow-matching sampler and its datasets, neither of which exists here: the flow
output is replaced by straight start-to-goal lines plus seeded Gaussian noise on
every coefficient.

It holds no arithmetic of the SF method itself.  Both the FP64 oracle and the
GPU path read the arrays it returns; neither is imported here.

Conventions (shared by every configuration):
  * arena square, centred at the origin (Sec. "Data Collection");
  * box bounds p_min/p_max = -/+ (side/2 - r_robot), so the robot body stays in
    the arena;
  * a = 2 r_robot (minimum centre distance, the spheroid matrix M_r of the
    problem statement), a_o = r_obs + r_robot (obstacle inflated by the robot);
  * straight-line Bernstein coefficients c_j = s + j/(n_coef-1) (g - s);
  * xi = straight + sigma * N(0, 1) on every coefficient; warm start
    xi_bar^0 = xi, lambda^0 = 0.

Random streams: numpy PCG64 seeded with SeedSequence([cfg_id, problem_idx])
for the context (starts, goals, obstacles) and SeedSequence([cfg_id,
problem_idx, cand_idx, 1]) for the noise, so candidates of one context share it.
Draw order inside the context stream: robot count, obstacle count (uneven
configurations only), starts, goals, then per obstacle radius and centre.
Obstacles are placed with disjoint inflated discs (0.1 m apart) where the arena
allows it: overlapping discs form walls with slits that a local projection
cannot resolve, which would make convergence a property of the generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

N_DIM = 2


@dataclass(frozen=True)
class SFConfig:
    cfg_id: int
    name: str
    n_robots: Tuple[int, int]          # inclusive range; equal ends = fixed
    n_obs: Tuple[int, int]
    arena: Optional[float]             # side [m]; None -> 2*sqrt(n_robots)
    r_robot: float
    r_obs: Tuple[float, float]
    n_coef: int
    n_steps: int
    batch: int
    iters: int
    sigma: float
    candidates: bool = False           # True: the whole batch shares one context
    layout: str = "random"             # "random" | "antipodal"
    circle_radius: float = 1.5
    checkpoint_every: int = 1
    description: str = ""


# The five workloads.  Values marked "proposed" are not fixed by the workload
# statement and were chosen to match its neighbours.
WORKLOADS = {
    1: SFConfig(1, "c1_single_4r", (4, 4), (3, 3), 4.0, 0.15, (0.2, 0.4), 11, 50,
                batch=1, iters=100, sigma=0.3, layout="antipodal", circle_radius=1.5,
                description="plain SF, one problem: 4 robots swapping antipodal "
                            "positions on a 1.5 m circle, 3 obstacles, 4x4 m arena"),
    2: SFConfig(2, "c2_candidates_16r", (16, 16), (10, 10), 8.0, 0.2, (0.2, 0.5), 11, 100,
                batch=32, iters=200, sigma=0.4, candidates=True,
                description="32 noisy candidates of one 16-robot, 10-obstacle "
                            "context, 8x8 m arena"),
    3: SFConfig(3, "c3_batch64_32r", (32, 32), (20, 20), 12.0, 0.2, (0.2, 0.5), 11, 100,
                batch=64, iters=100, sigma=0.3,
                description="64 independent 32-robot, 20-obstacle problems, "
                            "12x12 m arena (r_robot, r_obs, sigma proposed)"),
    4: SFConfig(4, "c4_uneven48", (8, 64), (0, 30), None, 0.2, (0.2, 0.5), 11, 100,
                batch=48, iters=150, sigma=0.3,
                description="48 problems, robots U{8..64}, obstacles U{0..30}, "
                            "arena side 2*sqrt(robots)"),
    5: SFConfig(5, "c5_large_64r", (64, 64), (50, 50), 16.0, 0.2, (0.2, 0.6), 15, 120,
                batch=128, iters=200, sigma=0.3, checkpoint_every=10,
                description="128 problems of 64 robots, 50 obstacles, 16x16 m "
                            "arena, 15 coefficients, 120 steps"),
}


@dataclass
class Problem:
    """One SF instance.  Arrays are float64; layouts follow the coefficient
    stacking of the compact form (axis-major, then robot, then coefficient)."""
    n: int
    M: int
    n_coef: int
    n_steps: int
    r_robot: float
    a: float                      # minimum centre distance
    box: np.ndarray               # [2][N_DIM]: p_min, p_max
    obstacles: np.ndarray         # [M][3]: centre x, centre y, a_o (inflated)
    boundary: np.ndarray          # [n][2][N_DIM]: b_{i,0}, b_{i,K}
    xi: np.ndarray                # [N_DIM][n][n_coef] flow-sample stand-in
    straight: np.ndarray          # [N_DIM][n][n_coef] noise-free straight lines
    seed: Tuple[int, ...] = field(default_factory=tuple)

    @property
    def xi0(self) -> np.ndarray:
        return self.xi.copy()

    @property
    def lam0(self) -> np.ndarray:
        return np.zeros_like(self.xi)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _points_with_separation(rng, count, lo, hi, min_sep, max_tries=100000):
    pts = np.zeros((count, N_DIM))
    for i in range(count):
        for _ in range(max_tries):
            p = rng.uniform(lo, hi, size=N_DIM)
            if i == 0 or np.min(np.linalg.norm(pts[:i] - p, axis=1)) >= min_sep:
                pts[i] = p
                break
        else:
            raise RuntimeError("could not place points with the requested separation")
    return pts


def _place_obstacles(rng, M, side, r_robot, r_obs, keep_clear, margin=0.05,
                     gap=0.1, disjoint_tries=2000, max_tries=100000):
    """Per obstacle: radius, then centre.  A centre is redrawn while its
    inflated disc (plus margin) holds a start or goal, or while it comes
    closer than `gap` to an already placed inflated disc.  After
    `disjoint_tries` draws the second rule is dropped for that obstacle (dense
    small arenas cannot hold every obstacle disjointly)."""
    obs = np.zeros((M, 3))
    half = side / 2.0
    for m in range(M):
        radius = rng.uniform(r_obs[0], r_obs[1])
        a_o = radius + r_robot
        for t in range(max_tries):
            c = rng.uniform(-half, half, size=N_DIM)
            if np.min(np.linalg.norm(keep_clear - c, axis=1)) <= a_o + margin:
                continue
            if t < disjoint_tries and m > 0:
                dist = np.linalg.norm(obs[:m, :2] - c, axis=1)
                if np.any(dist < obs[:m, 2] + a_o + gap):
                    continue
            obs[m] = (c[0], c[1], a_o)
            break
        else:
            raise RuntimeError("could not place an obstacle clear of starts/goals")
    return obs


def straight_coefficients(start: np.ndarray, goal: np.ndarray, n_coef: int) -> np.ndarray:
    """[N_DIM][n][n_coef] coefficients of straight start->goal lines in the
    Bernstein basis (its control points are evenly spaced on the line)."""
    frac = np.arange(n_coef) / (n_coef - 1)
    out = start.T[:, :, None] + frac[None, None, :] * (goal - start).T[:, :, None]
    return np.ascontiguousarray(out)


def make_problem(cfg: SFConfig, problem_idx: int, cand_idx: int = 0) -> Problem:
    ctx = _rng(cfg.cfg_id, problem_idx)
    n = int(ctx.integers(cfg.n_robots[0], cfg.n_robots[1] + 1)) \
        if cfg.n_robots[0] != cfg.n_robots[1] else cfg.n_robots[0]
    M = int(ctx.integers(cfg.n_obs[0], cfg.n_obs[1] + 1)) \
        if cfg.n_obs[0] != cfg.n_obs[1] else cfg.n_obs[0]
    side = cfg.arena if cfg.arena is not None else 2.0 * np.sqrt(n)
    half_box = side / 2.0 - cfg.r_robot
    if cfg.layout == "antipodal":
        ang = 2.0 * np.pi * np.arange(n) / n
        start = cfg.circle_radius * np.stack([np.cos(ang), np.sin(ang)], axis=1)
        goal = -start
    else:
        min_sep = max(0.5, 2.0 * cfg.r_robot + 0.1)
        start = _points_with_separation(ctx, n, -half_box, half_box, min_sep)
        goal = _points_with_separation(ctx, n, -half_box, half_box, min_sep)
    obstacles = _place_obstacles(ctx, M, side, cfg.r_robot, cfg.r_obs,
                                 np.concatenate([start, goal], axis=0))
    straight = straight_coefficients(start, goal, cfg.n_coef)
    noise_rng = _rng(cfg.cfg_id, problem_idx, cand_idx, 1)
    xi = straight + cfg.sigma * noise_rng.standard_normal(straight.shape)
    box = np.array([[-half_box] * N_DIM, [half_box] * N_DIM])
    boundary = np.stack([start, goal], axis=1)
    return Problem(n=n, M=M, n_coef=cfg.n_coef, n_steps=cfg.n_steps,
                   r_robot=cfg.r_robot, a=2.0 * cfg.r_robot, box=box,
                   obstacles=obstacles, boundary=boundary, xi=xi,
                   straight=straight, seed=(cfg.cfg_id, problem_idx, cand_idx))


def make_batch(cfg: SFConfig, batch: Optional[int] = None, first: int = 0) -> List[Problem]:
    B = cfg.batch if batch is None else batch
    if cfg.candidates:
        return [make_problem(cfg, first, c) for c in range(B)]
    return [make_problem(cfg, first + b, 0) for b in range(B)]


def scaled(cfg: SFConfig, **kw) -> SFConfig:
    """A copy of cfg with some fields replaced (e.g. the 4-robot copy of a
    workload used for finite-difference checks)."""
    return replace(cfg, **kw)


@dataclass
class PackedBatch:
    """Flat arrays in the C-ABI layout (see include/sf.h)."""
    n_robots: np.ndarray        # int32 [B]
    n_obs: np.ndarray           # int32 [B]
    robot_a: np.ndarray         # float32 [B]
    box: np.ndarray             # float32 [B][2][N_DIM]
    xi: np.ndarray              # float32 [sum_b N_DIM*n_b*n_coef]
    xi0: np.ndarray
    lam0: np.ndarray
    boundary: np.ndarray        # float32 [sum n][2][N_DIM]
    obstacles: np.ndarray       # float32 [sum M][3]
    coef_offsets: np.ndarray    # int64 [B+1] start of each problem's coefficient block
    n_coef: int
    n_steps: int


def pack(problems: Sequence[Problem], dtype=np.float32,
         xi0: Optional[Sequence[np.ndarray]] = None,
         lam0: Optional[Sequence[np.ndarray]] = None) -> PackedBatch:
    n_coef = problems[0].n_coef
    n_steps = problems[0].n_steps
    offs = [0]
    for p in problems:
        if p.n_coef != n_coef or p.n_steps != n_steps:
            raise ValueError("all problems of a batch share n_coef and n_steps")
        offs.append(offs[-1] + N_DIM * p.n * n_coef)
    xi0 = [p.xi0 for p in problems] if xi0 is None else xi0
    lam0 = [p.lam0 for p in problems] if lam0 is None else lam0
    obstacles = [p.obstacles.reshape(-1, 3) for p in problems]
    return PackedBatch(
        n_robots=np.array([p.n for p in problems], dtype=np.int32),
        n_obs=np.array([p.M for p in problems], dtype=np.int32),
        robot_a=np.array([p.a for p in problems], dtype=dtype),
        box=np.stack([p.box for p in problems]).astype(dtype),
        xi=np.concatenate([p.xi.ravel() for p in problems]).astype(dtype),
        xi0=np.concatenate([np.asarray(x).ravel() for x in xi0]).astype(dtype),
        lam0=np.concatenate([np.asarray(x).ravel() for x in lam0]).astype(dtype),
        boundary=np.concatenate([p.boundary.reshape(-1) for p in problems]).astype(dtype),
        obstacles=(np.concatenate(obstacles).ravel() if sum(o.size for o in obstacles)
                   else np.zeros(0)).astype(dtype),
        coef_offsets=np.array(offs, dtype=np.int64),
        n_coef=n_coef, n_steps=n_steps)


def unpack_coefs(flat: np.ndarray, problems: Sequence[Problem]) -> List[np.ndarray]:
    """Split a flat [sum N_DIM*n*n_coef] array into per-problem [N_DIM][n][n_coef]."""
    out, o = [], 0
    for p in problems:
        size = N_DIM * p.n * p.n_coef
        out.append(np.asarray(flat[o:o + size]).reshape(N_DIM, p.n, p.n_coef))
        o += size
    return out
