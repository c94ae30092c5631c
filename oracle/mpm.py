"""MLS-MPM transfers on a uniform grid, FP64 (paper Sec. 3.2-3.3).

Readings:
  * Nodes sit at x_i = i * dx, i = 0 .. n-1 per axis. The quadratic B-spline stencil of a
    point starts at base = floor(x / dx - 0.5) and covers base .. base + 2 per axis.
  * P2G (Sec. 3.3 step 1, APIC) plus the node force balance of Sec. 3.2 in its MLS form:
    grad w_ip is replaced by w_ip * D^-1 (x_i - x_p) with D^-1 = 12 / (dx^2 (b + 1)) =
    4 / dx^2 for b = 2 (the constant Sec. 3.3 gives for the C update). The stress impulse
    and the APIC term then share one 3x3 matrix per particle,
        A_p = m_p C_p - dt V_p (4 / dx^2) tau_p,
    and node momentum accumulates w_ip (m_p v_p + A_p (x_i - x_p)).
  * Grid update (Sec. 3.3 step 2) on nodes with m_i > 0: v_i = p_i / m_i + dt g, then the
    boundary conditions: sticky walls (all components zeroed on nodes within `wall`
    nodes of the domain edge), then an optional moving knife that imposes its velocity.
  * G2P (Sec. 3.3 step 3) on the sample particles: v_p = sum_i w_ip v_i and
    x_p <- x_p + dt v_p. C and F are not advanced: the next step re-infers C and tau
    from the fields (Sec. 5.1).
  * A particle whose stencil leaves the grid is skipped in P2G and G2P (G2P returns
    v = 0, x unchanged) and the DOMAIN flag is raised.
"""
from __future__ import annotations

import itertools
from typing import Tuple

import numpy as np

OFFSETS = np.array(list(itertools.product(range(3), repeat=3)), dtype=np.int64)  # (27, 3)


def bspline_weights(f: np.ndarray) -> np.ndarray:
    """Quadratic B-spline weights of the three stencil nodes, for fractional offsets
    f = x/dx - base in [0.5, 1.5). Returns (..., 3) for nodes base, base+1, base+2."""
    return np.stack([0.5 * (1.5 - f) ** 2, 0.75 - (f - 1.0) ** 2, 0.5 * (f - 0.5) ** 2], axis=-1)


def bspline_kernel(d: np.ndarray) -> np.ndarray:
    """N(d) for a signed distance d in grid units (the 1-D quadratic B-spline)."""
    a = np.abs(d)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def stencil(x: np.ndarray, dx: float):
    """base (n, 3) int, fractional offset f (n, 3), per-axis weights (n, 3, 3)."""
    xs = np.asarray(x, np.float64) / dx
    base = np.floor(xs - 0.5).astype(np.int64)
    f = xs - base
    return base, f, bspline_weights(f)


def in_domain(base: np.ndarray, n: int) -> np.ndarray:
    return np.all((base >= 0) & (base + 2 <= n - 1), axis=1)


def p2g(x: np.ndarray, v: np.ndarray, A: np.ndarray, m: np.ndarray, n: int, dx: float):
    """Scatter mass and momentum. x, v (np, 3); A (np, 3, 3); m (np,).
    Returns grid mass (n^3,), momentum (n^3, 3) flattened as i*n*n + j*n + k, and the
    DOMAIN flag."""
    base, f, w = stencil(x, dx)
    ok = in_domain(base, n)
    mass = np.zeros(n ** 3)
    mom = np.zeros((n ** 3, 3))
    base, f, w, v, A, m = base[ok], f[ok], w[ok], v[ok], A[ok], m[ok]
    for o in OFFSETS:
        wip = w[:, 0, o[0]] * w[:, 1, o[1]] * w[:, 2, o[2]]
        dpos = (o[None, :] - f) * dx
        node = base + o[None, :]
        idx = (node[:, 0] * n + node[:, 1]) * n + node[:, 2]
        np.add.at(mass, idx, wip * m)
        contrib = wip[:, None] * (m[:, None] * v + np.einsum("pab,pb->pa", A, dpos))
        for c in range(3):
            np.add.at(mom[:, c], idx, contrib[:, c])
    return mass, mom, bool(not ok.all())


def node_coords(n: int, dx: float) -> np.ndarray:
    i = np.arange(n)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def grid_update(mass: np.ndarray, mom: np.ndarray, n: int, dx: float, dt: float,
                gravity, wall: int, t_new: float, knife=None) -> np.ndarray:
    """Node velocities at t_{n+1} (n^3, 3); zero where m_i == 0."""
    vel = np.zeros_like(mom)
    has = mass > 0.0
    vel[has] = mom[has] / mass[has, None] + dt * np.asarray(gravity, np.float64)[None, :]
    idx = node_coords(n, dx)
    if wall > 0:
        band = np.any((idx < wall) | (idx >= n - wall), axis=1)
        vel[band & has] = 0.0
    if knife is not None and knife.enabled:
        xi = idx * dx
        nrm = np.asarray(knife.normal, np.float64)
        near = np.abs(xi @ nrm - knife.offset) <= knife.half_thickness
        below_edge = xi[:, 2] >= knife.edge_z0 - knife.edge_speed * t_new
        sel = near & below_edge & has
        vel[sel] = np.asarray(knife.velocity, np.float64)[None, :]
    return vel


def g2p(x: np.ndarray, vel: np.ndarray, n: int, dx: float):
    """Gather node velocities to particles. Returns v (np, 3) and the DOMAIN flag."""
    base, f, w = stencil(x, dx)
    ok = in_domain(base, n)
    v = np.zeros((x.shape[0], 3))
    for o in OFFSETS:
        wip = w[:, 0, o[0]] * w[:, 1, o[1]] * w[:, 2, o[2]]
        node = np.clip(base + o[None, :], 0, n - 1)
        idx = (node[:, 0] * n + node[:, 1]) * n + node[:, 2]
        v += np.where(ok[:, None], wip[:, None] * vel[idx], 0.0)
    return v, bool(not ok.all())


def affine_matrix(C: np.ndarray, tau: np.ndarray, m: np.ndarray, V: np.ndarray,
                  dt: float, dx: float) -> np.ndarray:
    """A_p = m_p C_p - dt V_p (4/dx^2) tau_p (APIC term plus MLS stress impulse)."""
    return m[:, None, None] * C - (dt * 4.0 / (dx * dx)) * V[:, None, None] * tau
