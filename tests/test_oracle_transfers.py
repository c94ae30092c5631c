"""Pins for the oracle's P2G / grid update / G2P (paper Sec. 3.2 node force balance,
Sec. 3.3 MPM algorithm, APIC transfer)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import mpm


def _particles(seed, n, lo=0.4, hi=0.6):
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=(n, 3))
    v = rng.normal(size=(n, 3))
    A = rng.normal(size=(n, 3, 3))
    m = rng.uniform(0.5, 2.0, size=n)
    return x, v, A, m


def test_p2g_conserves_mass_and_momentum():
    n, dx = 32, 1 / 32
    x, v, A, m = _particles(0, 300)
    mass, mom, bad = mpm.p2g(x, v, A, m, n, dx)
    assert not bad
    assert mass.sum() == pytest.approx(m.sum(), rel=1e-13)
    # the affine/stress term vanishes in the total by linear reproduction
    np.testing.assert_allclose(mom.sum(0), (m[:, None] * v).sum(0), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dx", [1 / 32, 1 / 128])
def test_single_particle_affine_moment(dx):
    """sum_i p_i (x_i - x_p)^T = (dx^2/4) A_p: this fixes the 4/dx^2 constant, the sign of
    (x_i - x_p) and which index of A contracts with it."""
    n = int(round(1 / dx))
    x, v, A, m = _particles(1, 1)
    mass, mom, _ = mpm.p2g(x, v, A, m, n, dx)
    xi = mpm.node_coords(n, dx) * dx
    d = xi - x[0]
    M = (mom[:, :, None] * d[:, None, :]).sum(0)
    np.testing.assert_allclose(M, dx * dx / 4 * A[0], rtol=1e-10, atol=1e-18)


@pytest.mark.parametrize("dx", [1 / 32, 1 / 128])
def test_stress_impulse_first_moment(dx):
    """Node force balance of Sec. 3.2: f_i = -sum_p tau_p grad w_ip V_p. Differentiating
    linear reproduction sum_i w_ip (x_i - x_p) = 0 in x_p gives
    sum_i grad w_ip (x_i - x_p)^T = I for the exact B-spline gradient, so one particle's
    impulse dt f_i has first moment sum_i dt f_i (x_i - x_p)^T = -dt V_p tau_p, whatever dx
    is. The MLS form must reproduce it (this fixes the 4/dx^2 of the stress term)."""
    from oracle.fields import voigt_to_matrix
    n, dt = int(round(1 / dx)), 1e-4
    rng = np.random.default_rng(12)
    x = rng.uniform(0.45, 0.55, size=(1, 3))
    tau = voigt_to_matrix(rng.normal(size=(1, 6)))
    V = np.array([2e-5])
    A = mpm.affine_matrix(np.zeros((1, 3, 3)), tau, V, V, dt, dx)
    _, imp, _ = mpm.p2g(x, np.zeros((1, 3)), A, V, n, dx)
    d = mpm.node_coords(n, dx) * dx - x[0]
    M = (imp[:, :, None] * d[:, None, :]).sum(0)
    np.testing.assert_allclose(M, -dt * V[0] * tau[0], rtol=1e-9, atol=1e-22)


def test_stress_force_sum_and_torque_free():
    """Internal forces (v = 0, C = 0) sum to zero and exert no torque for symmetric tau
    (the angular-momentum property that motivates the affine field, Sec. 4.4)."""
    n, dx, dt = 32, 1 / 32, 1e-4
    rng = np.random.default_rng(5)
    x = rng.uniform(0.4, 0.6, size=(200, 3))
    t6 = rng.normal(size=(200, 6))
    from oracle.fields import voigt_to_matrix
    tau = voigt_to_matrix(t6)
    V = np.full(200, 1e-5)
    m = V.copy()
    A = mpm.affine_matrix(np.zeros((200, 3, 3)), tau, m, V, dt, dx)
    _, f, _ = mpm.p2g(x, np.zeros((200, 3)), A, m, n, dx)
    xi = mpm.node_coords(n, dx) * dx
    scale = np.abs(f).max()
    np.testing.assert_allclose(f.sum(0) / scale, 0.0, atol=1e-12)
    np.testing.assert_allclose(np.cross(xi, f).sum(0) / scale, 0.0, atol=1e-12)


def test_pressure_pushes_outward():
    """A block under compression (tau = -p I, p > 0) must receive an outward grid impulse,
    the sign of the node force balance of Sec. 3.2 (f_i = -sum_p tau_p grad w_ip V_p)."""
    n, dx, dt = 32, 1 / 32, 1e-4
    g = np.linspace(0.42, 0.58, 6)
    x = np.array(list(itertools.product(g, g, g)))
    N = x.shape[0]
    tau = np.broadcast_to(-3.0 * np.eye(3), (N, 3, 3)).copy()
    V = np.full(N, 1e-5)
    A = mpm.affine_matrix(np.zeros((N, 3, 3)), tau, V, V, dt, dx)
    mass, f, _ = mpm.p2g(x, np.zeros((N, 3)), A, V, n, dx)
    xi = mpm.node_coords(n, dx) * dx
    c = x.mean(0)
    radial = np.einsum("ia,ia->i", f, xi - c)
    assert radial.sum() > 0
    # and the closed form: sum_i f_i . (x_i - x_p) summed = (dx^2/4) sum_p tr A_p
    assert radial.sum() == pytest.approx(dx * dx / 4 * np.trace(A, axis1=1, axis2=2).sum(), rel=1e-10)


def test_p2g_brute_force_tiny_grid():
    n, dx = 8, 1 / 8
    x, v, A, m = _particles(7, 5, 2.5 / 8, 4.5 / 8)
    mass, mom, _ = mpm.p2g(x, v, A, m, n, dx)
    xi = mpm.node_coords(n, dx) * dx
    bm = np.zeros(n ** 3)
    bp = np.zeros((n ** 3, 3))
    for i in range(n ** 3):
        for p in range(5):
            d = xi[i] - x[p]
            w = np.prod(mpm.bspline_kernel(d / dx))
            bm[i] += w * m[p]
            bp[i] += w * (m[p] * v[p] + A[p] @ d)
    np.testing.assert_allclose(mass, bm, atol=1e-14)
    np.testing.assert_allclose(mom, bp, atol=1e-13)


def test_g2p_reproduces_affine_grid_field():
    n, dx = 32, 1 / 32
    rng = np.random.default_rng(9)
    M = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    xi = mpm.node_coords(n, dx) * dx
    vel = xi @ M.T + b
    x = rng.uniform(0.2, 0.8, size=(100, 3))
    vp, bad = mpm.g2p(x, vel, n, dx)
    assert not bad
    np.testing.assert_allclose(vp, x @ M.T + b, rtol=1e-12, atol=1e-12)


def test_apic_round_trip_is_exact_for_affine_motion():
    """Particles moving with v = M x + b and C = M (APIC, Sec. 3.3 step 1) give node
    velocities M x_i + b exactly, and G2P gives back M x_p + b (gravity off, tau = 0,
    no boundary nodes involved)."""
    n, dx, dt = 32, 1 / 32, 1e-4
    rng = np.random.default_rng(11)
    M = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    x = rng.uniform(0.4, 0.6, size=(400, 3))
    v = x @ M.T + b
    m = rng.uniform(0.5, 1.5, size=400)
    A = mpm.affine_matrix(np.broadcast_to(M, (400, 3, 3)), np.zeros((400, 3, 3)), m, m, dt, dx)
    mass, mom, _ = mpm.p2g(x, v, A, m, n, dx)
    vel = mpm.grid_update(mass, mom, n, dx, dt, (0, 0, 0), 0, dt)
    xi = mpm.node_coords(n, dx) * dx
    has = mass > 0
    np.testing.assert_allclose(vel[has], xi[has] @ M.T + b, rtol=1e-10, atol=1e-10)
    vp, _ = mpm.g2p(x, vel, n, dx)
    np.testing.assert_allclose(vp, v, rtol=1e-10, atol=1e-10)


def test_grid_update_gravity_walls_knife():
    n, dx, dt = 16, 1 / 16, 1e-3
    mass = np.ones(n ** 3)
    mom = np.zeros((n ** 3, 3))
    mom[:, 0] = 2.0
    knife = synth.Knife(enabled=True, normal=(1, 0, 0), offset=0.5, half_thickness=dx,
                        edge_z0=0.6, edge_speed=10.0, velocity=(0, 0, -0.5))
    t_new = 0.01   # edge at 0.6 - 0.1 = 0.5
    vel = mpm.grid_update(mass, mom, n, dx, dt, (0, 0, -9.8), 3, t_new, knife)
    idx = mpm.node_coords(n, dx)
    xi = idx * dx
    band = np.any((idx < 3) | (idx >= n - 3), axis=1)
    # the knife is applied after the walls, so it also owns wall nodes it passes through
    blade = (np.abs(xi[:, 0] - 0.5) <= dx) & (xi[:, 2] >= 0.5)
    assert np.all(vel[band & ~blade] == 0.0)
    assert (blade & ~band).sum() > 0 and (blade & band).sum() > 0
    np.testing.assert_array_equal(vel[blade], np.broadcast_to([0, 0, -0.5], (blade.sum(), 3)))
    free = ~band & ~blade
    np.testing.assert_allclose(vel[free], np.broadcast_to([2.0, 0, -9.8e-3], (free.sum(), 3)), rtol=1e-15)


def test_domain_violation_is_flagged_and_skipped():
    n, dx = 16, 1 / 16
    x = np.array([[0.5, 0.5, 0.5], [0.01, 0.5, 0.5]])
    v = np.ones((2, 3))
    A = np.zeros((2, 3, 3))
    m = np.ones(2)
    mass, mom, bad = mpm.p2g(x, v, A, m, n, dx)
    assert bad
    assert mass.sum() == pytest.approx(1.0)
    vel = np.ones((n ** 3, 3))
    vp, bad2 = mpm.g2p(x, vel, n, dx)
    assert bad2
    np.testing.assert_allclose(vp[0], 1.0)
    np.testing.assert_array_equal(vp[1], 0.0)
