"""Seeded synthetic workloads for the batched safety filter.

This module only draws inputs.  It holds none of the filter's arithmetic and is
shared by the FP64 oracle tests, the GPU parity tests and the benchmark.

The paper's data (expert trajectories and trained generative priors, Sec. V-A)
is not available, so generative samples are stood in for by straight-line
Bernstein fits between start and goal plus i.i.d. Gaussian noise on every
coefficient.  Start/goal positions follow Sec. V-A: origin-centred workspaces,
zero boundary velocity and acceleration.

Coefficient arrays use the layout [sample, robot, axis, coeff] (C order).
Boundary values are [robot, axis, 6] = (p0, v0, a0, pH, vH, aH).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np


@dataclass(frozen=True)
class SwarmConfig:
    """Problem shape and constraint parameters of one swarm size."""
    n_robots: int
    dims: int
    degree: int
    horizon: int
    t_final: float
    safety_a: float          # centre-to-centre separation (x, y semi-axis)
    safety_b: float          # centre-to-centre separation (z semi-axis)
    vmax: float
    amax: float
    rho_coll: float = 1.0
    rho_vel: float = 1.0
    rho_acc: float = 1.0
    ws_a: float = 0.0        # workspace spheroid semi-axes (x, y and z); 0 switches it off
    ws_b: float = 0.0
    rho_ws: float = 1.0
    ws_x: float = 0.0        # workspace centre
    ws_y: float = 0.0
    ws_z: float = 0.0

    @property
    def m(self) -> int:
        return self.degree + 1


@dataclass
class Problem:
    """One start/goal instance with its batch of sampled trajectories."""
    cfg: SwarmConfig
    xi_bar: np.ndarray       # [S, n, D, m] float64
    bvals: np.ndarray        # [n, D, 6] float64
    starts: np.ndarray       # [n, D]
    goals: np.ndarray        # [n, D]


@dataclass
class Workload:
    name: str
    problems: List[Problem]
    iters: int
    precision: str
    ckpt_every: int = 0
    notes: str = ""

    @property
    def n_samples(self) -> int:
        return sum(p.xi_bar.shape[0] for p in self.problems)


def _rngs(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]


def straight_line_coeffs(starts: np.ndarray, goals: np.ndarray, degree: int) -> np.ndarray:
    """Bernstein coefficients of the constant-velocity line from start to goal.

    A Bernstein polynomial with equally spaced control points on a segment is
    that segment traversed at constant speed, so c_k = s + (k/N)(g - s).
    Returns [n, D, m]."""
    k = np.arange(degree + 1, dtype=np.float64) / degree
    return starts[:, :, None] + k[None, None, :] * (goals - starts)[:, :, None]


def boundary_values(starts: np.ndarray, goals: np.ndarray) -> np.ndarray:
    n, d = starts.shape
    b = np.zeros((n, d, 6), dtype=np.float64)
    b[:, :, 0] = starts
    b[:, :, 3] = goals
    return b


def sample_coeffs(rng, starts, goals, degree, n_samples, sigma) -> np.ndarray:
    base = straight_line_coeffs(starts, goals, degree)
    noise = rng.normal(0.0, sigma, size=(n_samples,) + base.shape)
    return base[None] + noise


def box_starts(rng, n, lo, hi, min_sep, max_tries=100000) -> np.ndarray:
    """Uniform positions in an axis-aligned box, rejecting any closer than min_sep."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place robots with the requested separation")
        p = lo + (hi - lo) * rng.random(lo.shape[0])
        if all(np.linalg.norm(p - q) >= min_sep for q in pts):
            pts.append(p)
    return np.stack(pts)


def circle_problem(cfg: SwarmConfig, n_samples: int, sigma: float, radius: float, seed: int) -> Problem:
    """Robots evenly spaced on a circle, goals antipodal (the swarm-crossing case)."""
    _, _, r_noise = _rngs(seed)
    th = 2.0 * np.pi * np.arange(cfg.n_robots) / cfg.n_robots
    starts = np.zeros((cfg.n_robots, cfg.dims))
    starts[:, 0] = radius * np.cos(th)
    starts[:, 1] = radius * np.sin(th)
    goals = -starts
    xi = sample_coeffs(r_noise, starts, goals, cfg.degree, n_samples, sigma)
    return Problem(cfg, xi, boundary_values(starts, goals), starts, goals)


def box_problem(cfg: SwarmConfig, n_samples: int, sigma: float, seed: int,
                box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), min_sep: float = 0.5,
                rngs=None) -> Problem:
    """Starts uniform in a box with a minimum separation; goals a permutation of the starts."""
    r_start, r_perm, r_noise = rngs if rngs is not None else _rngs(seed)
    lo = np.asarray(box[0])[: cfg.dims]
    hi = np.asarray(box[1])[: cfg.dims]
    starts = box_starts(r_start, cfg.n_robots, lo, hi, min_sep)
    goals = starts[r_perm.permutation(cfg.n_robots)]
    xi = sample_coeffs(r_noise, starts, goals, cfg.degree, n_samples, sigma)
    return Problem(cfg, xi, boundary_values(starts, goals), starts, goals)


# --- the five workloads -----------------------------------------------------

ROBOT_RADIUS = 0.15
SEP = 2 * ROBOT_RADIUS            # centre-to-centre safety distance


def cfg_tiny2d() -> SwarmConfig:
    return SwarmConfig(n_robots=4, dims=2, degree=10, horizon=100, t_final=5.0,
                       safety_a=SEP, safety_b=SEP, vmax=1.5, amax=2.0)


def cfg_swarm(n: int, degree: int = 10, horizon: int = 100) -> SwarmConfig:
    return SwarmConfig(n_robots=n, dims=3, degree=degree, horizon=horizon, t_final=10.0,
                       safety_a=SEP, safety_b=SEP, vmax=1.5, amax=2.0)


def tiny2d(n_samples: int = 8) -> Workload:
    """4 robots in 2D on a circle of radius 2 m, antipodal goals, 8 samples, sigma 0.3, 200 iterations, FP64."""
    p = circle_problem(cfg_tiny2d(), n_samples, 0.3, 2.0, seed=1)
    return Workload("tiny2d_n4_fp64", [p], iters=200, precision="fp64")


def swarm16(n_samples: int = 1024, iters: int = 300) -> Workload:
    """16 robots in 3D, 6x6x2 m box, 1024 samples, sigma 0.4, degree 10, H 100, T 10 s, 300 iterations."""
    p = box_problem(cfg_swarm(16), n_samples, 0.4, seed=2)
    return Workload("swarm16_3d", [p], iters=iters, precision="fp32")


def swarm16ws(n_samples: int = 1024, iters: int = 300) -> Workload:
    """The 16-robot instance with the workspace constraint on: an origin-centred spheroid of
    semi-axes 4.8, 4.8, 2.2 m, just large enough to hold the 6x6x2 m box of starts and goals,
    so that the sampled trajectories that bulge out near its corners are pulled back in."""
    cfg = replace(cfg_swarm(16), ws_a=4.8, ws_b=2.2)
    p = box_problem(cfg, n_samples, 0.4, seed=2)
    return Workload("swarm16ws_3d", [p], iters=iters, precision="fp32")


def swarm16sph(n_samples: int = 1024, iters: int = 300) -> Workload:
    """The 16-robot instance with spheroidal robots: centre-to-centre semi-axes 0.3 m in x and y
    and 0.6 m in z (a taller keep-out, as for the downwash below a quadrotor)."""
    cfg = replace(cfg_swarm(16), safety_b=2 * SEP)
    p = box_problem(cfg, n_samples, 0.4, seed=2)
    return Workload("swarm16sph_3d", [p], iters=iters, precision="fp32")


def eqqp16(n_samples: int = 1 << 20) -> Workload:
    """Decoder outputs for the equality-only QP layer: the 16-robot instance's straight-line
    coefficients plus N(0, 0.4) noise on every coefficient (so the end coefficients miss the
    boundary values).  Only 8 samples are drawn here; the benchmark draws the full batch of
    n_samples on the device from a seeded generator, in the same form."""
    p = box_problem(cfg_swarm(16), 8, 0.4, seed=2)
    return Workload("eqqp16_3d", [p], iters=0, precision="fp32", notes=f"n_samples={n_samples}")


def swarm32(n_samples: int = 4096, iters: int = 300) -> Workload:
    """32 robots in 3D, degree 12, H 120, 4096 samples, 300 iterations."""
    p = box_problem(cfg_swarm(32, degree=12, horizon=120), n_samples, 0.4, seed=4)
    return Workload("swarm32_3d_deg12", [p], iters=iters, precision="bf16")


def diff16(n_samples: int = 512, iters: int = 100) -> Workload:
    """16 robots in 3D, 512 samples, 100 unrolled iterations, checkpoints every 10."""
    p = box_problem(cfg_swarm(16), n_samples, 0.4, seed=5)
    return Workload("diff16_3d", [p], iters=iters, precision="fp32", ckpt_every=10)


def ragged(n_problems: int = 3000, sizes=(8, 16, 32), max_samples: int = 256,
           iters: int = 300, seed: int = 3) -> Workload:
    """Uneven batch: equal numbers of problems per swarm size (seeded interleave),
    1..max_samples samples per problem drawn log-uniformly."""
    r_start, r_perm, r_noise = _rngs(seed)
    per = n_problems // len(sizes)
    order = np.repeat(np.arange(len(sizes)), per)
    order = np.concatenate([order, np.arange(n_problems - order.size) % len(sizes)])
    order = r_perm.permutation(order)
    counts = np.minimum(max_samples,
                        np.floor(np.exp(r_noise.random(n_problems) * np.log(max_samples + 1)))).astype(int)
    counts = np.maximum(counts, 1)
    cfgs = {n: cfg_swarm(n) for n in sizes}
    probs = []
    for k in range(n_problems):
        n = sizes[order[k]]
        probs.append(box_problem(cfgs[n], int(counts[k]), 0.4, seed=0,
                                 rngs=(r_start, r_perm, r_noise)))
    return Workload("ragged_3000", probs, iters=iters, precision="fp32")


def small3d(n_robots: int = 5, n_samples: int = 6, degree: int = 10, horizon: int = 40,
            sigma: float = 0.4, seed: int = 11, box=((-1.2, -1.2, -0.5), (1.2, 1.2, 0.5)),
            t_final: float = 6.0) -> Problem:
    """A small 3D instance for parity tests: several time tiles and a ragged tail."""
    cfg = SwarmConfig(n_robots=n_robots, dims=3, degree=degree, horizon=horizon, t_final=t_final,
                      safety_a=SEP, safety_b=SEP, vmax=1.5, amax=2.0)
    return box_problem(cfg, n_samples, sigma, seed=seed, box=box, min_sep=0.5)


WORKLOADS = {
    "tiny2d": tiny2d,
    "swarm16": swarm16,
    "swarm16ws": swarm16ws,
    "swarm16sph": swarm16sph,
    "eqqp16": eqqp16,
    "ragged": ragged,
    "swarm32": swarm32,
    "diff16": diff16,
}
