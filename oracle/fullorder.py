"""Full-order explicit MLS-MPM, FP64, to make training snapshots for field fitting.

Paper: Sec. 3.3 (MPM algorithm: P2G with APIC, grid update, G2P with the C and F
updates and the return map) and the supplementary "Elasticity and plasticity details"
(fixed corotated elasticity; von Mises plasticity in log strain).

Readings:
  * MLS form throughout: the stress impulse uses w_ip (4/dx^2)(x_i - x_p) for grad w_ip,
    and the deformation-gradient update uses the particle's affine velocity C_p^{n+1}
    (its MLS estimate of the velocity gradient): F_trial = (I + dt C) F^E.
  * Fixed corotated: tau = 2 mu (F - R) F^T + lambda (J - 1) J I (the identity is missing
    in print).
  * von Mises: with F_trial = U S V^T and eps = log S, eps_hat = dev(eps); the plastic
    multiplier is dgamma = |eps_hat| - tau_y / (2 mu); if positive, eps <- eps -
    dgamma eps_hat / |eps_hat| (the printed normalisation by |eps| is read as |eps_hat|)
    and F^E = U exp(eps) V^T. No hardening.
  * Boundaries: the bottom `wall` node layers are a separating ground (v_z <- max(v_z, 0)),
    all other wall layers are sticky.
This module is test infrastructure like the rest of the oracle; it also writes the
snapshots the fitting example trains on.
"""
from __future__ import annotations

import numpy as np

from . import mpm


def lame(E: float, nu: float):
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    return mu, lam


def fixed_corotated_tau(F: np.ndarray, mu: float, lam: float) -> np.ndarray:
    U, S, Vt = np.linalg.svd(F)
    R = U @ Vt
    J = np.prod(S, axis=-1)
    return 2 * mu * (F - R) @ np.swapaxes(F, -1, -2) + (lam * (J - 1) * J)[:, None, None] * np.eye(3)


def von_mises_return(F: np.ndarray, mu: float, tau_y: float) -> np.ndarray:
    U, S, Vt = np.linalg.svd(F)
    eps = np.log(np.maximum(S, 1e-12))
    eps_hat = eps - eps.mean(axis=1, keepdims=True)
    norm = np.linalg.norm(eps_hat, axis=1)
    dgamma = norm - tau_y / (2 * mu)
    yield_ = dgamma > 0
    safe = np.where(norm > 0, norm, 1.0)
    eps = np.where(yield_[:, None], eps - (dgamma / safe)[:, None] * eps_hat, eps)
    return U @ (np.exp(eps)[:, :, None] * Vt)


def grid_update_ground(mass, mom, n, dx, dt, gravity, wall):
    """v_i = p_i / m_i + dt g; separating ground on the bottom wall layers, sticky walls
    elsewhere."""
    vel = np.zeros_like(mom)
    has = mass > 0.0
    vel[has] = mom[has] / mass[has, None] + dt * np.asarray(gravity, np.float64)[None, :]
    idx = mpm.node_coords(n, dx)
    ground = idx[:, 2] < wall
    other = np.any((idx[:, :2] < wall) | (idx[:, :2] >= n - wall), axis=1) | (idx[:, 2] >= n - wall)
    vel[ground, 2] = np.maximum(vel[ground, 2], 0.0)
    vel[other & ~ground] = 0.0
    vel[other & ground] = 0.0
    return vel


def g2p_affine(x: np.ndarray, vel: np.ndarray, n: int, dx: float):
    """Velocity and APIC affine matrix C = (4/dx^2) sum_i w v_i (x_i - x_p)^T."""
    base, f, w = mpm.stencil(x, dx)
    v = np.zeros((x.shape[0], 3))
    C = np.zeros((x.shape[0], 3, 3))
    for o in mpm.OFFSETS:
        wip = w[:, 0, o[0]] * w[:, 1, o[1]] * w[:, 2, o[2]]
        node = base + o[None, :]
        idx = (node[:, 0] * n + node[:, 1]) * n + node[:, 2]
        vi = vel[idx]
        dpos = (o[None, :] - f) * dx
        v += wip[:, None] * vi
        C += (4.0 / (dx * dx)) * wip[:, None, None] * vi[:, :, None] * dpos[:, None, :]
    return v, C


class FullOrder:
    def __init__(self, X, v0, rho, volume, E, nu, tau_y, n, dt, gravity=(0, 0, -9.8), wall=3):
        self.x = np.array(X, np.float64)
        P = self.x.shape[0]
        self.v = np.broadcast_to(np.asarray(v0, np.float64), (P, 3)).copy()
        self.C = np.zeros((P, 3, 3))
        self.F = np.broadcast_to(np.eye(3), (P, 3, 3)).copy()
        self.V = volume / P
        self.m = rho * self.V
        self.mu, self.lam = lame(E, nu)
        self.tau_y, self.n, self.dx, self.dt = tau_y, n, 1.0 / n, dt
        self.gravity, self.wall = gravity, wall
        self.tau = fixed_corotated_tau(self.F, self.mu, self.lam)

    def step(self):
        P = self.x.shape[0]
        m = np.full(P, self.m)
        A = mpm.affine_matrix(self.C, self.tau, m, np.full(P, self.V), self.dt, self.dx)
        mass, mom, bad = mpm.p2g(self.x, self.v, A, m, self.n, self.dx)
        if bad:
            raise RuntimeError("particle left the grid")
        vel = grid_update_ground(mass, mom, self.n, self.dx, self.dt, self.gravity, self.wall)
        self.v, self.C = g2p_affine(self.x, vel, self.n, self.dx)
        self.x = self.x + self.dt * self.v
        Ftr = (np.eye(3)[None] + self.dt * self.C) @ self.F
        self.F = von_mises_return(Ftr, self.mu, self.tau_y)
        self.tau = fixed_corotated_tau(self.F, self.mu, self.lam)


def voigt(tau: np.ndarray) -> np.ndarray:
    return np.stack([tau[:, 0, 0], tau[:, 1, 1], tau[:, 2, 2], tau[:, 1, 2], tau[:, 0, 2], tau[:, 0, 1]], 1)


def falling_cube(n_particles=50_000, seed=0):
    """Cube of side 0.2 centred at (0.5, 0.5, 0.4), 64^3 grid, dt = 1e-4, rho = 1000,
    E = 5e4, nu = 0.3, von Mises yield 2e3, initial velocity -2 m/s along z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(-0.1, 0.1, size=(n_particles, 3)) + np.array([0.5, 0.5, 0.4])
    return FullOrder(X, (0.0, 0.0, -2.0), rho=1000.0, volume=0.2 ** 3, E=5e4, nu=0.3,
                     tau_y=2e3, n=64, dt=1e-4)


if __name__ == "__main__":
    import argparse
    import time
    ap = argparse.ArgumentParser(description="write full-order snapshots (positions, Voigt "
                                             "stress, affine C) of the falling cube")
    ap.add_argument("--out", required=True)
    ap.add_argument("--particles", type=int, default=50_000)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=25)
    a = ap.parse_args()
    sim = falling_cube(a.particles)
    X = sim.x.copy()
    xs, taus, Cs = [], [], []
    t0 = time.time()
    for s in range(1, a.steps + 1):
        sim.step()
        if s % a.every == 0:
            xs.append(sim.x.astype(np.float32))
            taus.append(voigt(sim.tau).astype(np.float32))
            Cs.append(sim.C.reshape(-1, 9).astype(np.float32))
            print(f"step {s} ({time.time() - t0:.0f} s) z_min {sim.x[:, 2].min():.4f}", flush=True)
    np.savez(a.out, X=X.astype(np.float32), x=np.stack(xs), tau=np.stack(taus), C=np.stack(Cs))
