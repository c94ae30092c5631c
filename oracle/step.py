"""The reduced-order latent time step, FP64 (paper Sec. 5, steps 1-3).

One step from (z_{n-1}, z_n) to z_{n+1}:
  1. Network inference (Sec. 5.1) on the integration particles N_n:
       x_p = X_p + u(X_p, z_n), v_p = (u(X_p, z_n) - u(X_p, z_{n-1})) / dt,
       tau_p = h(X_p, z_n), C_p = l(X_p, z_n).
  2. One MPM step on N_n (Sec. 5.2, Sec. 3.3): P2G with APIC and the MLS stress
     impulse, grid update with gravity and boundary conditions, G2P on S_n.
  3. Network inversion (Sec. 5.3): Gauss-Newton from z_n towards the positions
     x_p + dt v_p^{n+1} of the sample particles.
Then z_{n-1} <- z_n, z_n <- z_{n+1}; decode evaluates X + u(X, z_n) anywhere (Sec. 5.1;
the resolution boost of Sec. 6).

Readings: m_p = rho V_p with V_p = body_volume / |N| (each integration particle stands
for an equal share of the body); z_{-1} = z_0 unless given (zero initial velocity); the
sample set S_n is the first n_sample entries of the step's index list; the step's list is
row (n mod plan_steps) of the plan.

With integration = "closure" the sample set S is the first n_sample entries of the plan's
single row, fixed over time (its size can be reduced between steps, as the paper does
half-way through the cake), and N_n is the closure of S's stencils at the positions
g(X, z_n) of all particles (Sec. 5.4, `closure.py`). Each particle then stands for its own
share of the body, V_p = body_volume / |P|, as in the full-order step it reproduces.
"""
from __future__ import annotations

import numpy as np

from . import closure
from . import fields as F
from . import gn
from . import mpm


class OracleSim:
    FLAG_DOMAIN = 1
    FLAG_NONFINITE = 2
    FLAG_SINGULAR = 4

    def __init__(self, w):
        """w: a synth.Workload (or anything with the same attributes)."""
        self.w = w
        self.X = np.asarray(w.X, np.float64).T          # (P, 3)
        self.z = np.array(w.z0, np.float64)
        self.z_prev = np.array(w.z_prev, np.float64)
        self.n = 0
        self.flags = 0
        self.closure = getattr(w, "integration", "plan") == "closure"
        self.n_sample = int(w.n_sample)
        self.mu = np.array(getattr(w, "mu", ()), np.float64).ravel()

    def set_parameters(self, mu) -> None:
        """Problem parameters of the stress field h(X, z, mu) from the next step on."""
        mu = np.array(mu, np.float64).ravel()
        assert mu.shape == self.mu.shape
        self.mu = mu

    def set_sample_count(self, n_sample: int) -> None:
        """Closure mode: keep the first n_sample sample particles from the next step on."""
        assert self.closure and 3 * n_sample >= self.z.shape[0] and n_sample <= self.w.plan.shape[1]
        self.n_sample = int(n_sample)

    # -- pieces --------------------------------------------------------------------
    def u(self, X, z):
        return F.field(self.w.fields["g"], X, z, self.w.out_scale["g"], self.w.out_shift["g"])

    def jac(self, X, z):
        return F.jacobian_z(self.w.fields["g"], X, z, self.w.out_scale["g"])

    def indices(self, n=None):
        """The step's integration list (S first). Closure mode: at the current latent."""
        if self.closure:
            S = self.w.plan[0][: self.n_sample]
            return closure.integration_set(self.decode(), S, self.w.grid_n, self.w.dx)
        n = self.n if n is None else n
        return self.w.plan[n % self.w.plan.shape[0]]

    def particle_volume(self, n_integration: int) -> float:
        return self.w.body_volume / (self.X.shape[0] if self.closure else n_integration)

    def inference(self, idx):
        """Sec. 5.1 on the integration particles: x, v, tau, C, u (all FP64)."""
        w = self.w
        XN = self.X[idx]
        u_n, tau, C = F.eval_fields(w.fields, XN, self.z, w.out_scale, w.out_shift, self.mu)
        u_prev = self.u(XN, self.z_prev)
        v = (u_n - u_prev) / w.dt
        return XN + u_n, v, tau, C, u_n

    def mpm_step(self, x, v, tau, C, n_sample):
        """Sec. 5.2: one MPM step on N, returning v^{n+1} on S."""
        w = self.w
        nN = x.shape[0]
        V = np.full(nN, self.particle_volume(nN))
        m = w.rho * V
        A = mpm.affine_matrix(C, tau, m, V, w.dt, w.dx)
        mass, mom, bad1 = mpm.p2g(x, v, A, m, w.grid_n, w.dx)
        vel = mpm.grid_update(mass, mom, w.grid_n, w.dx, w.dt, w.gravity, w.wall_nodes,
                              (self.n + 1) * w.dt, w.knife)
        v_new, bad2 = mpm.g2p(x[:n_sample], vel, w.grid_n, w.dx)
        if bad1 or bad2:
            self.flags |= self.FLAG_DOMAIN
        return v_new

    def inversion(self, XS, target_u):
        """Sec. 5.3: K Gauss-Newton iterations from z_n towards target_u on S."""
        z = self.z.copy()
        for _ in range(self.w.gn_iters):
            res = (self.u(XS, z) - target_u).reshape(-1)
            J = self.jac(XS, z).reshape(-1, z.shape[0])
            try:
                z = z + gn.gn_delta(J, res, getattr(self.w, "gn_damping", 0.0))
            except gn.SingularSystem:
                self.flags |= self.FLAG_SINGULAR
                raise
        return z

    # -- the step --------------------------------------------------------------------
    def step(self, n_steps: int = 1):
        for _ in range(n_steps):
            w = self.w
            idx = self.indices()
            nS = self.n_sample
            x, v, tau, C, u_n = self.inference(idx)
            v_new = self.mpm_step(x, v, tau, C, nS)
            target_u = u_n[:nS] + w.dt * v_new
            z_new = self.inversion(self.X[idx[:nS]], target_u)
            if not np.all(np.isfinite(z_new)):
                self.flags |= self.FLAG_NONFINITE
            self.z_prev, self.z = self.z, z_new
            self.n += 1
        return self.z

    def decode(self, X=None) -> np.ndarray:
        """x = X + u(X, z_n), (n, 3). X defaults to all particles."""
        Xq = self.X if X is None else np.asarray(X, np.float64)
        return Xq + self.u(Xq, self.z)

    def state(self):
        return dict(z=self.z.copy(), z_prev=self.z_prev.copy(), n=self.n)

    def restore(self, s):
        self.z, self.z_prev, self.n = s["z"].copy(), s["z_prev"].copy(), int(s["n"])


def relative_error(x: np.ndarray, x_ref: np.ndarray) -> float:
    """delta = sqrt(sum ||x - x*||^2 / sum ||x*||^2), the error measure of Sec. 6."""
    x = np.asarray(x, np.float64)
    x_ref = np.asarray(x_ref, np.float64)
    return float(np.sqrt(np.sum((x - x_ref) ** 2) / np.sum(x_ref ** 2)))
