"""Pins for the full-order generator (paper Sec. 3.3; supplementary elasticity and
plasticity details)."""
import numpy as np
import pytest

from oracle import fullorder as FO


def _rotations(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    d = np.linalg.det(Q)
    Q[d < 0, :, 0] *= -1
    return Q


def test_fixed_corotated_rotation_is_stress_free():
    mu, lam = FO.lame(5e4, 0.3)
    tau = FO.fixed_corotated_tau(_rotations(20, 0), mu, lam)
    assert np.abs(tau).max() < 1e-9


def test_fixed_corotated_small_strain_is_linear_elasticity():
    """For F = I + e (small symmetric e), tau = 2 mu e + lambda tr(e) I + O(e^2)."""
    mu, lam = FO.lame(5e4, 0.3)
    rng = np.random.default_rng(1)
    e = rng.normal(size=(10, 3, 3)) * 1e-6
    e = 0.5 * (e + np.swapaxes(e, 1, 2))
    tau = FO.fixed_corotated_tau(np.eye(3) + e, mu, lam)
    lin = 2 * mu * e + lam * np.trace(e, axis1=1, axis2=2)[:, None, None] * np.eye(3)
    np.testing.assert_allclose(tau, lin, rtol=0, atol=1e-3 * np.abs(lin).max())


def test_lame_parameters():
    mu, lam = FO.lame(5e4, 0.3)
    assert mu == pytest.approx(5e4 / 2.6)
    assert lam == pytest.approx(5e4 * 0.3 / (1.3 * 0.4))


def test_von_mises_projects_onto_the_yield_surface():
    mu = FO.lame(5e4, 0.3)[0]
    tau_y = 2e3
    rng = np.random.default_rng(2)
    F = np.eye(3) + 0.3 * rng.normal(size=(200, 3, 3))
    Fe = FO.von_mises_return(F, mu, tau_y)
    S = np.linalg.svd(Fe, compute_uv=False)
    eps = np.log(S)
    dev = np.linalg.norm(eps - eps.mean(1, keepdims=True), axis=1)
    assert np.all(dev <= tau_y / (2 * mu) + 1e-12)
    # plastic flow is isochoric in log strain: tr(eps) is preserved
    S0 = np.linalg.svd(F, compute_uv=False)
    np.testing.assert_allclose(np.log(S).sum(1), np.log(S0).sum(1), atol=1e-12)
    # and elastic states are left alone
    small = np.eye(3) + 1e-4 * rng.normal(size=(20, 3, 3))
    np.testing.assert_allclose(FO.von_mises_return(small, mu, tau_y), small, atol=1e-14)


def test_free_fall_before_contact():
    """A stress-free cube falling far from the walls keeps its uniform velocity plus dt g
    per step, C stays zero, and mass is conserved."""
    sim = FO.falling_cube(n_particles=500)
    v0 = sim.v.copy()
    for _ in range(3):
        sim.step()
    np.testing.assert_allclose(sim.v, v0 + 3 * sim.dt * np.array([0, 0, -9.8]), atol=1e-10)
    assert np.abs(sim.C).max() < 1e-8
    assert np.abs(sim.F - np.eye(3)).max() < 1e-10
