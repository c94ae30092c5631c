"""Pins for the full-order model (paper Sec. 3.3; supplementary "Elasticity and
plasticity details").

The G2P affine estimate, the deformation-gradient update and the separating ground are
each checked against a closed form, and each check is also run on a copy of its function
with a plausible mistake planted (a transposed C, the F product taken in the wrong order,
a ground that clamps the wrong sign or component) to show that it would catch it.
"""
import numpy as np
import pytest

from oracle import fullorder as FO
from oracle import mpm


def _rotations(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    d = np.linalg.det(Q)
    Q[d < 0, :, 0] *= -1
    return Q


def _affine_grid(n, dx, M, b):
    """Node velocities v_i = M x_i + b on every node of an n^3 grid."""
    xi = mpm.node_coords(n, dx) * dx
    return xi @ M.T + b


# ---- the closed forms, written as checks that take the function under test -------------

def pin_g2p_affine(g2p_affine):
    """Sec. 3.3 G2P on an affine grid velocity v_i = M x_i + b gives v_p = M x_p + b and
    C_p = M exactly: sum_i w (x_i - x_p) = 0 and sum_i w (x_i - x_p)(x_i - x_p)^T =
    dx^2/4 I, so (4/dx^2) sum_i w v_i (x_i - x_p)^T = M. M is not symmetric, so a C built
    as (x_i - x_p) v_i^T (M^T) fails."""
    n, dx = 32, 1 / 32
    rng = np.random.default_rng(7)
    M = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    x = rng.uniform(0.2, 0.8, size=(50, 3))
    v, C = g2p_affine(x, _affine_grid(n, dx, M, b), n, dx)
    np.testing.assert_allclose(v, x @ M.T + b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(C, np.broadcast_to(M, C.shape), rtol=0, atol=1e-11)


def pin_deformation_update(update):
    """F^E after the velocity gradients C_1, C_2, ... is (I + dt C_k) ... (I + dt C_1):
    two non-commuting gradients taken alternately fix the product order."""
    rng = np.random.default_rng(8)
    C1, C2 = rng.normal(size=(3, 3)), rng.normal(size=(3, 3))
    assert np.abs(C1 @ C2 - C2 @ C1).max() > 0.1
    dt = 1e-2
    F = np.broadcast_to(np.eye(3), (2, 3, 3)).copy()
    want = np.eye(3)
    for k in range(6):
        Ck = C1 if k % 2 == 0 else C2
        F = update(F, np.broadcast_to(Ck, (2, 3, 3)), dt)
        want = (np.eye(3) + dt * Ck) @ want
    np.testing.assert_allclose(F, np.broadcast_to(want, F.shape), rtol=0, atol=1e-13)


def pin_ground(grid_update_ground):
    """Hand-built nodes on a 16^3 grid with a 3-node band: the bottom layers keep v_x, v_y
    and v_z only when it points up; side and top walls (and a ground node that is also in
    a side wall) keep nothing; interior nodes get p / m + dt g; empty nodes stay 0."""
    n, dx, dt, wall = 16, 1 / 16, 1e-3, 3
    g = (0.0, 0.0, -9.8)
    mass = np.zeros(n ** 3)
    mom = np.zeros((n ** 3, 3))
    cases = {  # node: (mass, momentum, expected velocity)
        (8, 8, 8): (2.0, (1.0, -2.0, 3.0), (0.5, -1.0, 1.5 - 9.8e-3)),
        (8, 8, 1): (1.0, (0.3, -0.4, -0.5), (0.3, -0.4, 0.0)),       # down into the ground
        (7, 9, 2): (1.0, (0.3, -0.4, 0.5), (0.3, -0.4, 0.5 - 9.8e-3)),  # up, away from it
        (8, 8, 0): (1.0, (0.0, 0.0, 0.005), (0.0, 0.0, 0.0)),        # gravity wins: clamped
        (1, 8, 8): (1.0, (0.3, 0.4, 0.5), (0.0, 0.0, 0.0)),          # side wall x
        (8, 14, 8): (1.0, (0.3, 0.4, 0.5), (0.0, 0.0, 0.0)),         # side wall y
        (8, 8, 13): (1.0, (0.3, 0.4, 0.5), (0.0, 0.0, 0.0)),         # top wall
        (1, 8, 1): (1.0, (0.3, 0.4, 0.5), (0.0, 0.0, 0.0)),          # ground and side wall
    }
    for (i, j, k), (m, p, _) in cases.items():
        node = (i * n + j) * n + k
        mass[node] = m
        mom[node] = p
    vel = grid_update_ground(mass, mom, n, dx, dt, g, wall)
    for (i, j, k), (_, _, want) in cases.items():
        np.testing.assert_allclose(vel[(i * n + j) * n + k], want, rtol=0, atol=1e-15,
                                   err_msg=f"node {(i, j, k)}")
    empty = mass == 0
    assert np.all(vel[empty] == 0.0)


def test_g2p_affine_reproduces_an_affine_field():
    pin_g2p_affine(FO.g2p_affine)


def test_deformation_update_is_left_multiplication():
    pin_deformation_update(FO.update_deformation)


def test_ground_and_walls_on_hand_built_nodes():
    pin_ground(FO.grid_update_ground)


# ---- each pin catches a planted mistake -------------------------------------------------

def _g2p_transposed_C(x, vel, n, dx):
    v, C = FO.g2p_affine(x, vel, n, dx)
    return v, np.swapaxes(C, 1, 2)


def _g2p_missing_constant(x, vel, n, dx):
    v, C = FO.g2p_affine(x, vel, n, dx)
    return v, C * (dx * dx / 4.0) * 3.0 / (dx * dx)   # D^-1 = 3/dx^2 (the cubic-spline value)


def _update_right_multiplied(F, C, dt):
    return F @ (np.eye(3)[None] + dt * C)


def _update_without_identity(F, C, dt):
    return (dt * C) @ F + np.eye(3)[None]


def _ground_clamps_both_signs(mass, mom, n, dx, dt, gravity, wall):
    vel = FO.grid_update_ground(mass, mom, n, dx, dt, gravity, wall)
    idx = mpm.node_coords(n, dx)
    vel[(idx[:, 2] < wall), 2] = 0.0
    return vel


def _ground_sticky(mass, mom, n, dx, dt, gravity, wall):
    vel = FO.grid_update_ground(mass, mom, n, dx, dt, gravity, wall)
    idx = mpm.node_coords(n, dx)
    vel[idx[:, 2] < wall] = 0.0
    return vel


def _ground_before_gravity(mass, mom, n, dx, dt, gravity, wall):
    # clamp v_z on p / m, then add gravity: the ground no longer holds a resting node
    g0 = FO.grid_update_ground(mass, mom, n, dx, dt, (0.0, 0.0, 0.0), wall)
    has = mass > 0
    g0[has] += dt * np.asarray(gravity)[None, :]
    idx = mpm.node_coords(n, dx)
    other = np.any((idx[:, :2] < wall) | (idx[:, :2] >= n - wall), axis=1) | (idx[:, 2] >= n - wall)
    g0[other] = 0.0
    return g0


@pytest.mark.parametrize("pin, bad", [
    (pin_g2p_affine, _g2p_transposed_C),
    (pin_g2p_affine, _g2p_missing_constant),
    (pin_deformation_update, _update_right_multiplied),
    (pin_deformation_update, _update_without_identity),
    (pin_ground, _ground_clamps_both_signs),
    (pin_ground, _ground_sticky),
    (pin_ground, _ground_before_gravity),
])
def test_pin_catches_planted_mistake(pin, bad):
    with pytest.raises(AssertionError):
        pin(bad)


def test_g2p_update_follows_affine_motion():
    """The whole G2P stage (v, C, advection, F update; no yield) against a fixed affine grid
    velocity: x_{k+1} = (I + dt M) x_k + dt b and F^E = (I + dt M)^k."""
    rng = np.random.default_rng(9)
    M = 0.5 * rng.normal(size=(3, 3))
    b = 0.1 * rng.normal(size=3)
    X = rng.uniform(0.45, 0.55, size=(40, 3))
    sim = FO.FullOrder(X, (0, 0, 0), rho=1.0, volume=1e-3, E=1e3, nu=0.3, tau_y=1e30, n=32, dt=1e-3)
    vel = _affine_grid(32, 1 / 32, M, b)
    x, F = X.copy(), np.eye(3)
    for _ in range(5):
        sim.g2p_update(vel)
        x = x @ (np.eye(3) + sim.dt * M).T + sim.dt * b
        F = (np.eye(3) + sim.dt * M) @ F
    np.testing.assert_allclose(sim.x, x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sim.C, np.broadcast_to(M, sim.C.shape), atol=1e-11)
    np.testing.assert_allclose(sim.F, np.broadcast_to(F, sim.F.shape), atol=1e-12)


# ---- elasticity -------------------------------------------------------------------------

def test_lame_parameters():
    mu, lam = FO.lame(5e4, 0.3)
    assert mu == pytest.approx(5e4 / 2.6)
    assert lam == pytest.approx(5e4 * 0.3 / (1.3 * 0.4))
    assert FO.bulk(5e4, 0.3) == pytest.approx(lam + 2 * mu / 3)


def test_fixed_corotated_rotation_is_stress_free():
    mu, lam = FO.lame(5e4, 0.3)
    tau = FO.fixed_corotated_tau(_rotations(20, 0), mu, lam)
    assert np.abs(tau).max() < 1e-9


def _small_strain(seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=(10, 3, 3)) * 1e-6
    return 0.5 * (e + np.swapaxes(e, 1, 2))


def test_fixed_corotated_small_strain_is_linear_elasticity():
    """For F = I + e (small symmetric e), tau = 2 mu e + lambda tr(e) I + O(e^2)."""
    mu, lam = FO.lame(5e4, 0.3)
    e = _small_strain(1)
    tau = FO.fixed_corotated_tau(np.eye(3) + e, mu, lam)
    lin = 2 * mu * e + lam * np.trace(e, axis1=1, axis2=2)[:, None, None] * np.eye(3)
    np.testing.assert_allclose(tau, lin, rtol=0, atol=1e-3 * np.abs(lin).max())


@pytest.mark.parametrize("stress", ["hencky", "hb"])
def test_stress_small_strain_and_frame_indifference(stress):
    """Both stresses reduce to linear elasticity at small strain (Lame lambda, or the bulk
    modulus for the Herschel-Bulkley form), vanish on rotations, and are frame-indifferent:
    tau(Q F) = Q tau(F) Q^T and tau(F Q) = tau(F). The right-rotation check pins U (not V)
    on the right of the log-strain stress."""
    mu, lam = FO.lame(5e4, 0.3)
    kappa = FO.bulk(5e4, 0.3)
    fn = (lambda F: FO.hencky_tau(F, mu, lam)) if stress == "hencky" else (lambda F: FO.hb_tau(F, mu, kappa))
    vol = lam if stress == "hencky" else kappa - 2 * mu / 3   # coefficient of tr(e) I in 2 mu e + . tr(e) I
    e = _small_strain(2)
    lin = 2 * mu * e + vol * np.trace(e, axis1=1, axis2=2)[:, None, None] * np.eye(3)
    np.testing.assert_allclose(fn(np.eye(3) + e), lin, rtol=0, atol=1e-3 * np.abs(lin).max())
    assert np.abs(fn(_rotations(10, 3))).max() < 1e-9
    rng = np.random.default_rng(4)
    F = np.eye(3) + 0.3 * rng.normal(size=(10, 3, 3))
    F[np.linalg.det(F) < 0, :, 0] *= -1
    Q = _rotations(10, 5)
    t = fn(F)
    np.testing.assert_allclose(fn(Q @ F), Q @ t @ np.swapaxes(Q, 1, 2), atol=1e-9 * np.abs(t).max())
    np.testing.assert_allclose(fn(F @ Q), t, atol=1e-9 * np.abs(t).max())


def test_hencky_principal_stress():
    """On a diagonal stretch the log-strain stress is diag(2 mu ln s + lambda sum ln s)."""
    mu, lam = FO.lame(5e4, 0.3)
    s = np.array([[1.2, 0.9, 0.7], [0.5, 1.5, 1.0]])
    tau = FO.hencky_tau(np.stack([np.diag(x) for x in s]), mu, lam)
    want = 2 * mu * np.log(s) + lam * np.log(s).sum(1, keepdims=True)
    np.testing.assert_allclose(np.diagonal(tau, axis1=1, axis2=2), want, rtol=1e-12)
    np.testing.assert_allclose(tau - np.stack([np.diag(w) for w in want]), 0.0, atol=1e-9)


# ---- plasticity -------------------------------------------------------------------------

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


def _diag_F(s, seed):
    """F = U diag(s) V^T with random rotations."""
    U, V = _rotations(len(s), seed), _rotations(len(s), seed + 100)
    return U @ (np.asarray(s)[:, :, None] * np.swapaxes(V, 1, 2)), U, V


def _dp_dgamma(F, mu, lam, phi):
    eps = np.log(np.linalg.svd(F, compute_uv=False))
    tr = eps.sum(1)
    dev = np.linalg.norm(eps - tr[:, None] / 3, axis=1)
    return dev + FO.dp_alpha(phi) * (3 * lam + 2 * mu) * tr / (2 * mu), tr


def test_drucker_prager_cases():
    """Supplementary "Drucker-Prager plasticity": expansion returns to the stress-free
    Sigma = 1 (F^E = U V^T); a compressed state inside the cone is left alone; a compressed
    state outside lands on the cone (dgamma = 0) with its volume sum(eps) and its singular
    vectors kept."""
    mu, lam = FO.lame(3.5e4, 0.3)
    phi = 30.0
    assert FO.dp_alpha(30.0) == pytest.approx(np.sqrt(2 / 3) * 2 * 0.5 / 2.5)
    # expansion
    F, U, V = _diag_F([[1.1, 1.0, 0.95], [1.3, 0.9, 0.9]], 1)
    Fe = FO.drucker_prager_return(F, mu, lam, phi)
    np.testing.assert_allclose(Fe, U @ np.swapaxes(V, 1, 2), atol=1e-12)
    # compression inside the cone
    F, U, V = _diag_F([[0.9, 0.91, 0.92]], 2)
    assert _dp_dgamma(F, mu, lam, phi)[0][0] < 0
    np.testing.assert_allclose(FO.drucker_prager_return(F, mu, lam, phi), F, atol=1e-14)
    # compression outside: onto the cone
    s = np.array([[0.7, 1.3, 1.0], [0.9, 0.8, 1.2], [1.2, 0.75, 1.05]])
    F, U, V = _diag_F(s, 3)
    dg0, tr0 = _dp_dgamma(F, mu, lam, phi)
    assert np.all(dg0 > 0) and np.all(tr0 < 0)
    Fe = FO.drucker_prager_return(F, mu, lam, phi)
    dg1, tr1 = _dp_dgamma(Fe, mu, lam, phi)
    np.testing.assert_allclose(dg1, 0.0, atol=1e-12)
    np.testing.assert_allclose(tr1, tr0, atol=1e-12)
    core = np.swapaxes(U, 1, 2) @ Fe @ V   # diagonal when U and V are kept
    off = core - np.stack([np.diag(np.diagonal(c)) for c in core])
    assert np.abs(off).max() < 1e-12
    # zero friction: the cone is the hydrostatic axis, the whole deviator goes
    Fe0 = FO.drucker_prager_return(F, mu, lam, 0.0)
    S0 = np.linalg.svd(Fe0, compute_uv=False)
    np.testing.assert_allclose(S0, np.exp(tr0 / 3)[:, None] * np.ones(3), rtol=1e-12)


def _hb_dev_norm(F, mu, kappa):
    t = FO.hb_tau(F, mu, kappa)
    d = t - (np.trace(t, axis1=1, axis2=2) / 3)[:, None, None] * np.eye(3)
    return np.linalg.norm(d, axis=(1, 2)), d


@pytest.mark.parametrize("eta", [0.0, 5.0, 1e12])
def test_herschel_bulkley_flow_rule(eta):
    """Supplementary "Herschel-Bulkley plasticity": below the yield limit nothing moves;
    above it the deviatoric stress of F^E has norm
    s_t - (s_t - sqrt(2/3) sigma_y) / (1 + eta / (2 mu dt)) (on the yield surface for
    eta = 0, unchanged as eta grows without bound), keeps its direction, and the volume J
    and the rotations are untouched."""
    mu, _ = FO.lame(1e4, 0.3)
    kappa = FO.bulk(1e4, 0.3)
    sigma_y, dt = 60.0, 1e-3
    lim = np.sqrt(2 / 3) * sigma_y
    F, U, V = _diag_F([[1.05, 0.98, 0.99], [1.2, 0.9, 1.0], [0.8, 1.1, 1.15]], 6)
    s_t, d_t = _hb_dev_norm(F, mu, kappa)
    assert np.all(s_t > lim)
    Fe = FO.herschel_bulkley_return(F, mu, kappa, sigma_y, eta, dt)
    s_n, d_n = _hb_dev_norm(Fe, mu, kappa)
    want = s_t - (s_t - lim) / (1 + eta / (2 * mu * dt))
    np.testing.assert_allclose(s_n, want, rtol=1e-10)
    np.testing.assert_allclose(d_n / s_n[:, None, None], d_t / s_t[:, None, None], atol=1e-10)
    np.testing.assert_allclose(np.linalg.det(Fe), np.linalg.det(F), rtol=1e-12)
    core = np.swapaxes(U, 1, 2) @ Fe @ V
    off = core - np.stack([np.diag(np.diagonal(c)) for c in core])
    assert np.abs(off).max() < 1e-12
    if eta > 1e6:
        np.testing.assert_allclose(Fe, F, atol=1e-8)
    # below the limit
    Fs, _, _ = _diag_F([[1.0001, 0.9999, 1.0]], 7)
    assert _hb_dev_norm(Fs, mu, kappa)[0][0] < lim
    np.testing.assert_allclose(FO.herschel_bulkley_return(Fs, mu, kappa, sigma_y, eta, dt), Fs, atol=1e-15)


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


@pytest.mark.parametrize("model", ["drucker_prager", "herschel_bulkley"])
def test_models_stay_admissible_through_impact(model):
    """A cube dropped on the separating ground: after every step each particle's F^E is
    admissible (inside or on the cone; below or at the Herschel-Bulkley limit for
    eta = 0), and the run stays in the grid with finite state."""
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.uniform(-0.06, 0.06, size=(400, 3)) + np.array([0.5, 0.5, 0.12])
    kw = dict(rho=1000.0, volume=0.12 ** 3, E=2e4, nu=0.3, n=32, dt=2e-4, model=model)
    if model == "drucker_prager":
        sim = FO.FullOrder(X, (0, 0, -2.0), tau_y=0.0, friction_angle=30.0, **kw)
    else:
        sim = FO.FullOrder(X, (0, 0, -2.0), tau_y=80.0, viscosity=0.0, **kw)
    yielded = 0
    for _ in range(40):
        sim.step()
        if model == "drucker_prager":
            dg, tr = _dp_dgamma(sim.F, sim.mu, sim.lam, 30.0)
            assert np.all((dg <= 1e-10) | (np.abs(np.linalg.svd(sim.F, compute_uv=False) - 1) < 1e-10).all(1))
            yielded += int((np.abs(dg) < 1e-10).sum())
        else:
            s, _ = _hb_dev_norm(sim.F, sim.mu, sim.kappa)
            assert np.all(s <= np.sqrt(2 / 3) * 80.0 * (1 + 1e-9))
            yielded += int((np.abs(s - np.sqrt(2 / 3) * 80.0) < 1e-6).sum())
    assert np.isfinite(sim.x).all() and np.isfinite(sim.tau).all()
    assert yielded > 0, "the return map never acted"
