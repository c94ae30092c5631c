"""Pins for the oracle's whole latent step (paper Sec. 5.1-5.3)."""
import copy

import numpy as np
import pytest

import synth
from oracle.step import OracleSim, relative_error
from tests.helpers import affine_manifold


@pytest.mark.parametrize("gn_iters", [1, 2, 3])
def test_affine_manifold_free_fall_closed_form(gn_iters):
    """With g affine in z (r = 3, invertible latent map), tau = C = 0 and no boundary
    nodes touched, every particle has the same velocity, the grid adds dt*g, and the
    inversion is exact in one Gauss-Newton iteration, so the first-order projection
    (gn_iters = 1) is exact too and further iterations change nothing. Starting at rest
    the decoded positions after n steps are X + u(X, z0) + g dt^2 n (n + 1) / 2
    (symplectic Euler)."""
    w = affine_manifold(synth.small_cube(seed=0, r=3, width=16, n=256))
    w.gn_iters = gn_iters
    sim = OracleSim(w)
    x0 = sim.decode()
    n = 6
    sim.step(n)
    g = np.asarray(w.gravity)
    expect = x0 + g[None, :] * w.dt ** 2 * n * (n + 1) / 2
    np.testing.assert_allclose(sim.decode(), expect, rtol=0, atol=1e-12)
    assert sim.flags == 0


def test_damping_on_the_affine_manifold_is_a_partial_step():
    """Counter-check of the damped solve inside the step: on the affine manifold one
    damped iteration moves the latent by (A^T A + lambda D)^-1 A^T A times the exact
    step, which is not the exact step, while enough damped iterations reach it."""
    w = affine_manifold(synth.small_cube(seed=0, r=3, width=16, n=256))
    exact = OracleSim(w)
    exact.step(1)
    w1 = copy.deepcopy(w)
    w1.gn_iters, w1.gn_damping = 1, 0.5
    one = OracleSim(w1)
    one.step(1)
    d_exact = exact.z - w.z0
    assert np.abs(one.z - exact.z).max() > 0.1 * np.abs(d_exact).max()
    w4 = copy.deepcopy(w)
    w4.gn_iters, w4.gn_damping = 4, 1e-3
    four = OracleSim(w4)
    four.step(1)
    np.testing.assert_allclose(four.z - w.z0, d_exact, rtol=1e-7, atol=1e-14)


def test_mass_and_volume_scale_invariance():
    """Scaling every m_p and V_p by the same factor leaves the trajectory unchanged:
    the stress impulse divides V_p by m_p and the APIC term m_p by m_i."""
    w = synth.small_cube(seed=1, r=6, width=32, n=256, bias_scale=0.1)
    a = OracleSim(w)
    a.step(3)
    w2 = copy.deepcopy(w)
    w2.body_volume *= 7.3
    b = OracleSim(w2)
    b.step(3)
    np.testing.assert_allclose(b.z, a.z, rtol=1e-11, atol=1e-14)


def test_density_changes_stress_response():
    """Counter-check of the invariance test: halving the density doubles the stress
    impulse per unit mass, so the trajectory must change."""
    w = synth.small_cube(seed=1, r=6, width=32, n=256, bias_scale=0.1)
    a = OracleSim(w)
    a.step(2)
    w2 = copy.deepcopy(w)
    w2.rho = 0.5
    b = OracleSim(w2)
    b.step(2)
    assert np.abs(b.z - a.z).max() > 1e-8


def test_resume_is_bit_exact():
    w = synth.small_cube(seed=2, r=6, width=32, n=256, bias_scale=0.1)
    a = OracleSim(w)
    a.step(4)
    b = OracleSim(w)
    b.step(2)
    s = b.state()
    c = OracleSim(w)
    c.restore(s)
    c.step(2)
    np.testing.assert_array_equal(c.z, a.z)
    np.testing.assert_array_equal(c.z_prev, a.z_prev)


def test_small_cube_runs_and_moves():
    w = synth.small_cube(seed=0, r=6, width=64, n=1024, steps=3)
    sim = OracleSim(w)
    x0 = sim.decode()
    sim.step(3)
    x1 = sim.decode()
    assert np.all(np.isfinite(x1))
    assert sim.flags == 0
    d = relative_error(x1, x0)
    assert 0 < d < 1e-2


def test_relative_error_definition():
    x_ref = np.array([[3.0, 4.0, 0.0]])
    assert relative_error(x_ref + np.array([[0.0, 0.0, 0.5]]), x_ref) == pytest.approx(0.1)


def test_problem_parameters_steer_the_stress():
    """With h(X, z, mu) the parameter enters the step through the stress alone: two values
    of mu give different trajectories; zeroing h's mu columns makes them identical."""
    w = synth.small_cube(seed=4, r=6, width=32, n=256, bias_scale=0.1)
    w.fields = synth.make_fields(4, 6, 32, bias_scale=0.1, n_mu=1)
    w.z_prev = w.z0 - 2e-3 * np.random.default_rng(3).normal(size=6)
    w.mu = np.array([0.5])
    a = OracleSim(w)
    a.step(2)
    b = OracleSim(w)
    b.set_parameters([-0.5])
    b.step(2)
    assert np.abs(a.z - b.z).max() > 1e-9
    w0 = copy.deepcopy(w)
    W1, b1 = w0.fields["h"][0]
    W1 = W1.copy()
    W1[:, 3 + 6:] = 0.0
    w0.fields["h"][0] = (W1, b1)
    c, d = OracleSim(w0), OracleSim(w0)
    d.set_parameters([-0.5])
    c.step(2)
    d.step(2)
    np.testing.assert_array_equal(c.z, d.z)
