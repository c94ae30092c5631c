"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module draws random numbers and nothing else: MLP weights (Xavier-uniform),
reference positions, initial latents and per-step sample index lists. It holds none
of the method's arithmetic (no field evaluation, no transfer, no projection), so the
oracle and the library can both consume what it produces without sharing code.

Conventions (the readings the project fixes where the paper is silent):
  * Every stream is a NumPy ``Generator(PCG64(seed))``. Field weights use ``seed``,
    positions ``seed + 1``, the latent ``seed + 2``; sample plans use
    ``PCG64((plan_seed, step))`` per step.
  * Each MLP has 6 affine maps (5 hidden ELU layers, output linear), widths
    ``3 + r -> w -> w -> w -> w -> w -> d`` (supplementary "Network architecture").
  * Weights are drawn in float64 from U(-a, a), a = sqrt(6 / (fan_in + fan_out)), each
    ``W`` of shape (out, in), drawn row-major, then rounded once to float32. Those
    float32 values ARE the model everywhere. Biases are zero unless ``bias_scale`` is
    given (tests use nonzero biases so a dropped bias cannot hide).
  * Positions are float32 structure-of-arrays, shape (3, n).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

FIELD_NAMES = ("g", "h", "l")
FIELD_OUT = {"g": 3, "h": 6, "l": 9}
N_AFFINE = 6

Layer = Tuple[np.ndarray, np.ndarray]  # (W (out, in) float32, b (out,) float32)


def xavier_mlp(rng: np.random.Generator, in_dim: int, width: int, out_dim: int,
               bias_scale: float = 0.0, n_hidden: int = 5) -> List[Layer]:
    """Draw one MLP's parameters, layer 1 to layer n_hidden + 1."""
    dims = [in_dim] + [width] * n_hidden + [out_dim]
    layers: List[Layer] = []
    for k in range(n_hidden + 1):
        fan_in, fan_out = dims[k], dims[k + 1]
        a = math.sqrt(6.0 / (fan_in + fan_out))
        W = rng.uniform(-a, a, size=(fan_out, fan_in)).astype(np.float32)
        if bias_scale > 0.0:
            b = rng.uniform(-bias_scale, bias_scale, size=(fan_out,)).astype(np.float32)
        else:
            b = np.zeros((fan_out,), np.float32)
        layers.append((W, b))
    return layers


def make_fields(seed: int, r: int, width: int, bias_scale: float = 0.0,
                n_mu: int = 0) -> Dict[str, List[Layer]]:
    """Weights for the three fields g (3 out), h (6 out), l (9 out); draw order g, h, l.
    With n_mu > 0 the stress field h takes n_mu problem parameters after the latent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {name: xavier_mlp(rng, 3 + r + (n_mu if name == "h" else 0), width, FIELD_OUT[name], bias_scale)
            for name in FIELD_NAMES}


def box_points(seed: int, n: int, lo: Sequence[float], hi: Sequence[float]) -> np.ndarray:
    """n reference positions uniform in the box [lo, hi], float32 SoA (3, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    X = rng.uniform(0.0, 1.0, size=(3, n)) * (hi - lo)[:, None] + lo[:, None]
    return X.astype(np.float32)


def falling_cube_points(seed: int = 0, n: int = 50_000) -> np.ndarray:
    """The fitting workload's cube: n reference positions uniform in the cube of side 0.2
    centred at (0.5, 0.5, 0.4), float64 (n, 3) (one U(-0.1, 0.1) draw of shape (n, 3))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-0.1, 0.1, size=(n, 3)) + np.array([0.5, 0.5, 0.4])


def latent(seed: int, r: int, std: float) -> np.ndarray:
    """z0 ~ N(0, std^2), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, std, size=(r,))


def sample_plan(plan_seed: int, n_particles: int, n_integration: int, steps: int) -> np.ndarray:
    """Per-step index lists, int32 (steps, n_integration).

    Row n is a uniform draw without replacement from range(n_particles). When
    n_integration == n_particles every row is the identity (all particles integrate).
    """
    if n_integration == n_particles:
        return np.tile(np.arange(n_particles, dtype=np.int32), (steps, 1))
    out = np.empty((steps, n_integration), np.int32)
    for s in range(steps):
        rng = np.random.Generator(np.random.PCG64((plan_seed, s)))
        out[s] = rng.choice(n_particles, size=n_integration, replace=False).astype(np.int32)
    return out


@dataclasses.dataclass
class Knife:
    """A moving blade imposed as a grid velocity boundary.

    Nodes i with |n . x_i - offset| <= half_thickness and x_i[2] >= edge_z0 - edge_speed * t
    take the blade velocity (t = the time the updated grid velocity belongs to).
    """
    enabled: bool = False
    normal: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    offset: float = 0.5
    half_thickness: float = 0.0
    edge_z0: float = 0.0
    edge_speed: float = 0.0
    velocity: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Workload:
    """Everything one reduced simulation needs, as plain arrays and numbers."""
    name: str
    r: int
    width: int
    fields: Dict[str, List[Layer]]
    X: np.ndarray                      # (3, P) float32
    z0: np.ndarray                     # (r,) float64
    z_prev: np.ndarray                 # (r,) float64
    plan: np.ndarray                   # (plan_steps, N) int32; first n_sample entries are S
    n_sample: int
    grid_n: int
    dx: float
    dt: float
    gravity: Tuple[float, float, float]
    wall_nodes: int
    rho: float
    body_volume: float
    out_scale: Dict[str, np.ndarray]   # per-channel de-normalisation scale
    out_shift: Dict[str, np.ndarray]
    gn_iters: int
    steps: int
    knife: Knife = dataclasses.field(default_factory=Knife)
    gn_damping: float = 0.0            # Marquardt damping of the Gauss-Newton solves
    # "plan": N = S = the step's plan row. "closure": S = plan[0][:n_sample], fixed, and N
    # is the closure of S's stencils each step, with room for closure_cap particles.
    integration: str = "plan"
    closure_cap: int = 0
    # problem parameters of the stress field h(X, z, mu) (empty: h(X, z))
    mu: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))

    @property
    def n_particles(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_integration(self) -> int:
        return int(self.plan.shape[1])


def default_scales(r: int = 0) -> Tuple[Dict[str, np.ndarray], Dict[str, np.ndarray]]:
    scale = {"g": np.full(3, 1e-2), "h": np.ones(6), "l": np.ones(9)}
    shift = {k: np.zeros(FIELD_OUT[k]) for k in FIELD_NAMES}
    return scale, shift


def small_cube(seed: int = 0, r: int = 6, width: int = 64, n: int = 1024, steps: int = 10,
               bias_scale: float = 0.0) -> Workload:
    """1,024 points uniform in [0.4, 0.6]^3, 32^3 grid, dx = 1/32, dt = 1e-4, sticky walls,
    gravity -9.8 z, 2 Gauss-Newton iterations, all particles integrate and sample."""
    fields = make_fields(seed, r, width, bias_scale)
    X = box_points(seed + 1, n, (0.4, 0.4, 0.4), (0.6, 0.6, 0.6))
    z0 = latent(seed + 2, r, 0.1)
    scale, shift = default_scales()
    return Workload(
        name=f"cube{n}_w{width}_r{r}", r=r, width=width, fields=fields, X=X, z0=z0,
        z_prev=z0.copy(), plan=sample_plan(0, n, n, 1), n_sample=n, grid_n=32,
        dx=1.0 / 32, dt=1e-4, gravity=(0.0, 0.0, -9.8), wall_nodes=3, rho=1.0,
        body_volume=0.2 ** 3, out_scale=scale, out_shift=shift, gn_iters=2, steps=steps)


def cake_slab(seed: int = 0, r: int = 6, width: int = 128, n: int = 200_000,
              n_integration: int = 8192, steps: int = 100, plan_steps: int | None = None,
              grid_n: int = 128, bias_scale: float = 0.0) -> Workload:
    """Cake-scale single instance: n points uniform in [0.35,0.65]x[0.35,0.65]x[0.05,0.20],
    n_integration resampled uniformly per step (all of them are sample particles),
    128^3 grid, dt = 5e-5, and a knife moving down at 0.5 m/s through x = 0.5."""
    fields = make_fields(seed, r, width, bias_scale)
    X = box_points(seed + 1, n, (0.35, 0.35, 0.05), (0.65, 0.65, 0.20))
    z0 = latent(seed + 2, r, 0.1)
    scale, shift = default_scales()
    dx = 1.0 / grid_n
    plan = sample_plan(seed + 3, n, n_integration, plan_steps or steps)
    knife = Knife(enabled=True, normal=(1.0, 0.0, 0.0), offset=0.5, half_thickness=dx,
                  edge_z0=0.20, edge_speed=0.5, velocity=(0.0, 0.0, -0.5))
    return Workload(
        name=f"slab{n}_s{n_integration}_w{width}_r{r}", r=r, width=width, fields=fields, X=X,
        z0=z0, z_prev=z0.copy(), plan=plan, n_sample=n_integration, grid_n=grid_n, dx=dx,
        dt=5e-5, gravity=(0.0, 0.0, -9.8), wall_nodes=3, rho=1.0,
        body_volume=0.3 * 0.3 * 0.15, out_scale=scale, out_shift=shift, gn_iters=2,
        steps=steps, knife=knife)


def clustered_samples(seed: int, X: np.ndarray, n: int, center: Sequence[float],
                      sigma: float) -> np.ndarray:
    """n distinct particle indices drawn without replacement with weights
    exp(-|X_p - center|^2 / (2 sigma^2)): a sample set clustered around `center`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d2 = ((np.asarray(X, np.float64).T - np.asarray(center, np.float64)[None, :]) ** 2).sum(1)
    p = np.exp(-d2 / (2.0 * sigma * sigma))
    return rng.choice(X.shape[1], size=n, replace=False, p=p / p.sum()).astype(np.int32)


def cake_closure(seed: int = 0, r: int = 6, width: int = 128, n: int = 200_000,
                 n_sample: int = 700, sigma: float = 0.02, closure_cap: int = 32_768,
                 steps: int = 100, grid_n: int = 128, bias_scale: float = 0.0) -> Workload:
    """The cake slab with the paper's own integration set: n_sample sample particles
    clustered around the middle of the slab (fixed over time) and N the closure of their
    stencils, recomputed every step."""
    w = cake_slab(seed=seed, r=r, width=width, n=n, n_integration=1, steps=steps, plan_steps=1,
                  grid_n=grid_n, bias_scale=bias_scale)
    S = clustered_samples(seed + 5, w.X, n_sample, (0.5, 0.5, 0.125), sigma)
    w.plan = S[None, :]
    w.n_sample = n_sample
    w.integration = "closure"
    w.closure_cap = closure_cap
    w.name = f"slab{n}_closure{n_sample}_w{width}_r{r}"
    return w


def served_mix(n_requests: int = 256, seed: int = 4, rate_hz: float = 200.0,
               p_lo: float = 5e3, p_hi: float = 2e5, sample_frac: float = 0.04,
               r_choices: Sequence[int] = (6, 12, 24), grids: Sequence[int] = (64, 128)):
    """Request stream for the served batch: Poisson arrivals, log-uniform particle counts,
    4% sample points, r uniform over r_choices, grid size uniform over grids. Returns
    a list of dicts (arrival time in s, n_particles, n_integration, r, grid_n, weight seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    P = np.round(np.exp(rng.uniform(math.log(p_lo), math.log(p_hi), size=n_requests))).astype(int)
    rs = rng.choice(np.asarray(r_choices), size=n_requests)
    gs = rng.choice(np.asarray(grids), size=n_requests)
    out = []
    for i in range(n_requests):
        nP = int(P[i])
        out.append(dict(arrival_s=float(t[i]), n_particles=nP,
                        n_integration=max(1, int(round(sample_frac * nP))), r=int(rs[i]),
                        grid_n=int(gs[i]), weight_seed=1000 + i))
    return out


def served_instance(req: dict, width: int = 128, steps: int = 1000, plan_steps: int = 16) -> Workload:
    """Materialise one served request as a Workload (slab geometry, dt = 5e-5, no knife)."""
    w = cake_slab(seed=req["weight_seed"], r=req["r"], width=width, n=req["n_particles"],
                  n_integration=req["n_integration"], steps=steps, plan_steps=plan_steps,
                  grid_n=req["grid_n"])
    w.knife = Knife()
    w.name = f"req{req['weight_seed']}_P{req['n_particles']}_r{req['r']}_g{req['grid_n']}"
    return w
