"""Full-order explicit MLS-MPM, FP64, the model the reduced step is measured against and
the source of the training snapshots for field fitting.

TEST INFRASTRUCTURE, like the rest of the oracle.

Paper: Sec. 3.3 (MPM algorithm: P2G with APIC, grid update, G2P with the C and F
updates and the return map) and the supplementary "Elasticity and plasticity details"
(fixed corotated and StVK-in-log-strain elasticity; von Mises, Drucker-Prager and
Herschel-Bulkley plasticity).

Readings:
  * MLS form throughout: the stress impulse uses w_ip (4/dx^2)(x_i - x_p) for grad w_ip,
    and the deformation-gradient update uses the particle's affine velocity C_p^{n+1}
    (its MLS estimate of the velocity gradient): F_trial = (I + dt C) F^E.
  * Fixed corotated: tau = 2 mu (F - R) F^T + lambda (J - 1) J I (the identity is missing
    in print).
  * StVK in log strain (paired with Drucker-Prager, as in the sand model the paper
    cites): the Kirchhoff stress is U diag(2 mu eps + lambda sum(eps)) U^T. It is printed
    with V^T on the right, which is the first Piola form times Sigma and not a Kirchhoff
    stress; U on both sides is the one that is symmetric and frame-indifferent
    (tau(Q F) = Q tau(F) Q^T, tau(F Q) = tau(F)).
  * von Mises: with F_trial = U S V^T and eps = log S, eps_hat = dev(eps); the plastic
    multiplier is dgamma = |eps_hat| - tau_y / (2 mu); the material yields when
    dgamma > 0 and then eps <- eps - dgamma eps_hat / |eps_hat| (the printed
    normalisation by |eps| is read as |eps_hat|), F^E = U exp(eps) V^T. No hardening.
    The printed elastic branch tests |dev tau| - tau_y <= 0 on the stress; for stress
    that is linear in log strain the two tests coincide (dev tau = 2 mu eps_hat), but
    with fixed corotated stress at finite strain they differ slightly, and only the
    test on dgamma keeps the return consistent: a yielding state moves by exactly
    dgamma >= 0 towards the surface and an elastic state never moves. So the yield test
    is dgamma > 0.
  * Drucker-Prager: dgamma = |eps_hat| + alpha (d lambda + 2 mu) sum(eps) / (2 mu) with
    d = 3 (the "d lambda" of the print is d times lambda) and
    alpha = sqrt(2/3) 2 sin(phi_f) / (3 - sin(phi_f)); sum(eps) > 0 (expansion) returns
    to the stress-free Sigma = 1; dgamma <= 0 with sum(eps) <= 0 is elastic; otherwise
    eps <- eps - dgamma eps_hat / |eps_hat|, which lands on the cone.
  * Herschel-Bulkley (h = 1): s_trial = dev(tau(F_trial)) of the Herschel-Bulkley
    stress tau = kappa/2 (J^2 - 1) I + mu dev(det(b)^(-1/3) b), b = F F^T. If
    |s_trial| > sqrt(2/3) sigma_y it is scaled to
    s = s_trial - (s_trial - sqrt(2/3) sigma_y) / (1 + eta / (2 mu dt)). The paper does not
    say how F^E follows from s; here F^E keeps F_trial's rotations U, V and its volume J,
    and its isochoric part bbar = J^(-2/3) b is the unique s / mu + c I with det = 1, so
    that dev tau(F^E) is exactly s. The flow is then isochoric and leaves the rotation
    alone, as the scalar flow rule on the deviator implies.
  * Boundaries: the bottom `wall` node layers are a separating ground (v_z <- max(v_z, 0)),
    all other wall layers are sticky; a node in both keeps nothing.
"""
from __future__ import annotations

import numpy as np

from . import mpm

MODELS = ("von_mises", "drucker_prager", "herschel_bulkley")


def lame(E: float, nu: float):
    """Shear and Lame moduli (supplementary parameter table)."""
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    return mu, lam


def bulk(E: float, nu: float) -> float:
    """Bulk modulus kappa = E / (3 (1 - 2 nu)) (supplementary parameter table)."""
    return E / (3 * (1 - 2 * nu))


def _svd(F):
    U, S, Vt = np.linalg.svd(F)
    return U, S, Vt


def fixed_corotated_tau(F: np.ndarray, mu: float, lam: float) -> np.ndarray:
    """Supplementary "Fixed corotated elasticity"."""
    U, S, Vt = _svd(F)
    R = U @ Vt
    J = np.prod(S, axis=-1)
    return 2 * mu * (F - R) @ np.swapaxes(F, -1, -2) + (lam * (J - 1) * J)[:, None, None] * np.eye(3)


def hencky_tau(F: np.ndarray, mu: float, lam: float) -> np.ndarray:
    """Supplementary "StVK elasticity" in log strain: U diag(2 mu eps + lam sum(eps)) U^T."""
    U, S, _ = _svd(F)
    eps = np.log(S)
    d = 2 * mu * eps + lam * eps.sum(axis=1, keepdims=True)
    return U @ (d[:, :, None] * np.swapaxes(U, -1, -2))


def hb_tau(F: np.ndarray, mu: float, kappa: float) -> np.ndarray:
    """Supplementary "Herschel-Bulkley plasticity", its stress:
    kappa/2 (J^2 - 1) I + mu dev(det(b)^(-1/3) b) with b = F F^T."""
    b = F @ np.swapaxes(F, -1, -2)
    J = np.linalg.det(F)
    bbar = b * (np.linalg.det(b) ** (-1.0 / 3.0))[:, None, None]
    dev = bbar - (np.trace(bbar, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
    return (kappa / 2 * (J * J - 1))[:, None, None] * np.eye(3) + mu * dev


def von_mises_return(F: np.ndarray, mu: float, tau_y: float) -> np.ndarray:
    """Supplementary "von Mises plasticity" (no hardening), yield test dgamma > 0."""
    U, S, Vt = _svd(F)
    eps = np.log(np.maximum(S, 1e-12))
    eps_hat = eps - eps.mean(axis=1, keepdims=True)
    norm = np.linalg.norm(eps_hat, axis=1)
    dgamma = norm - tau_y / (2 * mu)
    yield_ = dgamma > 0
    safe = np.where(norm > 0, norm, 1.0)
    eps = np.where(yield_[:, None], eps - (dgamma / safe)[:, None] * eps_hat, eps)
    return U @ (np.exp(eps)[:, :, None] * Vt)


def dp_alpha(friction_deg: float) -> float:
    """alpha = sqrt(2/3) 2 sin(phi_f) / (3 - sin(phi_f))."""
    s = np.sin(np.radians(friction_deg))
    return np.sqrt(2.0 / 3.0) * 2.0 * s / (3.0 - s)


def drucker_prager_return(F: np.ndarray, mu: float, lam: float, friction_deg: float) -> np.ndarray:
    """Supplementary "Drucker-Prager plasticity": F^E = U Z(Sigma) V^T."""
    U, S, Vt = _svd(F)
    eps = np.log(np.maximum(S, 1e-12))
    tr = eps.sum(axis=1)
    eps_hat = eps - tr[:, None] / 3.0
    norm = np.linalg.norm(eps_hat, axis=1)
    dgamma = norm + dp_alpha(friction_deg) * (3.0 * lam + 2.0 * mu) * tr / (2.0 * mu)
    Z = np.empty_like(S)
    for p in range(F.shape[0]):
        if tr[p] > 0:
            Z[p] = 1.0
        elif dgamma[p] <= 0:
            Z[p] = S[p]
        else:
            Z[p] = np.exp(eps[p] - dgamma[p] * eps_hat[p] / norm[p])
    return U @ (Z[:, :, None] * Vt)


def _unit_det_shift(a: np.ndarray) -> float:
    """The c with prod(a_i + c) = 1 and every a_i + c > 0, for a with sum(a) = 0: the
    largest real root of c^3 + e2 c + (e3 - 1), e2 = a0 a1 + a0 a2 + a1 a2, e3 = a0 a1 a2."""
    e2 = a[0] * a[1] + a[0] * a[2] + a[1] * a[2]
    e3 = a[0] * a[1] * a[2]
    roots = np.roots([1.0, 0.0, e2, e3 - 1.0])
    real = roots[np.abs(roots.imag) <= 1e-9 * max(1.0, np.abs(roots).max())].real
    return float(real.max())


def herschel_bulkley_return(F: np.ndarray, mu: float, kappa: float, sigma_y: float, eta: float,
                            dt: float) -> np.ndarray:
    """Supplementary "Herschel-Bulkley plasticity" with h = 1 (see the module readings for
    how F^E follows from the returned deviator)."""
    out = F.copy()
    lim = np.sqrt(2.0 / 3.0) * sigma_y
    for p in range(F.shape[0]):
        U, S, Vt = np.linalg.svd(F[p])
        J = np.prod(S)
        bbar = J ** (-2.0 / 3.0) * S * S              # eigenvalues of the isochoric b
        dev = bbar - bbar.mean()
        s_trial = mu * np.linalg.norm(dev)
        if s_trial - lim <= 0:
            continue
        s = s_trial - (s_trial - lim) / (1.0 + eta / (2.0 * mu * dt))
        a = (s / s_trial) * dev                      # new deviator of bbar: s_vec / mu
        c = _unit_det_shift(a)
        sig = J ** (1.0 / 3.0) * np.sqrt(a + c)
        out[p] = U @ np.diag(sig) @ Vt
    return out


def update_deformation(F: np.ndarray, C: np.ndarray, dt: float) -> np.ndarray:
    """Sec. 3.3 G2P: F_trial = (I + dt C_p^{n+1}) F^E_n."""
    return (np.eye(3)[None] + dt * C) @ F


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
    vel[other] = 0.0
    return vel


def g2p_affine(x: np.ndarray, vel: np.ndarray, n: int, dx: float):
    """Sec. 3.3 G2P: v_p = sum_i w v_i and the APIC affine matrix
    C_p = (4/dx^2) sum_i w v_i (x_i - x_p)^T."""
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
    """model: "von_mises" (fixed corotated elasticity, yield stress tau_y),
    "drucker_prager" (StVK in log strain, friction angle in degrees) or
    "herschel_bulkley" (its own stress, yield stress tau_y as sigma_Y, viscosity eta)."""

    def __init__(self, X, v0, rho, volume, E, nu, tau_y, n, dt, gravity=(0, 0, -9.8), wall=3,
                 model="von_mises", friction_angle=30.0, viscosity=0.0):
        if model not in MODELS:
            raise ValueError(f"unknown model {model}")
        self.x = np.array(X, np.float64)
        P = self.x.shape[0]
        self.v = np.broadcast_to(np.asarray(v0, np.float64), (P, 3)).copy()
        self.C = np.zeros((P, 3, 3))
        self.F = np.broadcast_to(np.eye(3), (P, 3, 3)).copy()
        self.V = volume / P
        self.m = rho * self.V
        self.mu, self.lam = lame(E, nu)
        self.kappa = bulk(E, nu)
        self.model, self.friction_angle, self.viscosity = model, friction_angle, viscosity
        self.tau_y, self.n, self.dx, self.dt = tau_y, n, 1.0 / n, dt
        self.gravity, self.wall = gravity, wall
        self.tau = self.stress(self.F)

    def stress(self, F):
        if self.model == "von_mises":
            return fixed_corotated_tau(F, self.mu, self.lam)
        if self.model == "drucker_prager":
            return hencky_tau(F, self.mu, self.lam)
        return hb_tau(F, self.mu, self.kappa)

    def return_map(self, F):
        if self.model == "von_mises":
            return von_mises_return(F, self.mu, self.tau_y)
        if self.model == "drucker_prager":
            return drucker_prager_return(F, self.mu, self.lam, self.friction_angle)
        return herschel_bulkley_return(F, self.mu, self.kappa, self.tau_y, self.viscosity, self.dt)

    def p2g_grid(self):
        """Sec. 3.3 steps 1-2: P2G with APIC and the stress impulse, then the grid update."""
        P = self.x.shape[0]
        m = np.full(P, self.m)
        A = mpm.affine_matrix(self.C, self.tau, m, np.full(P, self.V), self.dt, self.dx)
        mass, mom, bad = mpm.p2g(self.x, self.v, A, m, self.n, self.dx)
        if bad:
            raise RuntimeError("particle left the grid")
        return grid_update_ground(mass, mom, self.n, self.dx, self.dt, self.gravity, self.wall)

    def g2p_update(self, vel):
        """Sec. 3.3 step 3: G2P of v and C at x^n, advection, F update, return map, stress."""
        self.v, self.C = g2p_affine(self.x, vel, self.n, self.dx)
        self.x = self.x + self.dt * self.v
        self.F = self.return_map(update_deformation(self.F, self.C, self.dt))
        self.tau = self.stress(self.F)

    def step(self):
        self.g2p_update(self.p2g_grid())


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
