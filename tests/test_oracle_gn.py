"""Pins for the oracle's Gauss-Newton inversion (paper Sec. 5.3)."""
import numpy as np
import pytest

import synth
from oracle import fields as F
from oracle import gn


def test_step_equals_lstsq():
    rng = np.random.default_rng(0)
    J = rng.normal(size=(300, 6))
    r = rng.normal(size=300)
    d = gn.gn_delta(J, r)
    ref = np.linalg.lstsq(J, -r, rcond=None)[0]
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-13)


def test_cholesky_matches_library():
    rng = np.random.default_rng(1)
    B = rng.normal(size=(24, 24))
    H = B @ B.T + 24 * np.eye(24)
    np.testing.assert_allclose(gn.cholesky_lower(H), np.linalg.cholesky(H), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("r", [6, 24])
def test_zero_residual_problem_converges(r):
    """Targets on the manifold: GN from a perturbed start recovers z* (the 2-3 iteration
    convergence the paper reports is for such smooth problems)."""
    fl = synth.make_fields(3, r, 32, bias_scale=0.1)
    X = synth.box_points(4, 200, (0.4, 0.4, 0.4), (0.6, 0.6, 0.6)).T
    scale = np.full(3, 1e-2)
    zs = synth.latent(5, r, 0.1)
    target = F.field(fl["g"], X, zs, scale, np.zeros(3))
    z = zs + 1e-3 * np.random.default_rng(6).normal(size=r)
    for _ in range(3):
        res = (F.field(fl["g"], X, z, scale, np.zeros(3)) - target).ravel()
        J = F.jacobian_z(fl["g"], X, z, scale).reshape(-1, r)
        z = z + gn.gn_delta(J, res)
    assert np.linalg.norm(z - zs) <= 1e-10


def test_singular_system_raises():
    """A latent coordinate the field ignores makes J^T J singular: the pivot is exactly 0."""
    r = 6
    fl = synth.make_fields(3, r, 16)
    W1, b1 = fl["g"][0]
    W1 = W1.copy()
    W1[:, 3 + 2] = 0.0
    fl["g"][0] = (W1, b1)
    X = synth.box_points(4, 50, (0.4, 0.4, 0.4), (0.6, 0.6, 0.6)).T
    z = synth.latent(5, r, 0.1)
    J = F.jacobian_z(fl["g"], X, z, np.ones(3)).reshape(-1, r)
    assert np.all(J[:, 2] == 0.0)
    with pytest.raises(gn.SingularSystem):
        gn.gn_delta(J, np.ones(J.shape[0]))


@pytest.mark.parametrize("lam", [1e-3, 0.5, 10.0])
def test_damped_step_is_augmented_least_squares(lam):
    """(J^T J + lambda D) delta = -J^T r with D = diag(J^T J) is the least-squares solution
    of the stacked system [J; sqrt(lambda D)] delta = [-r; 0] (QR / SVD route of the
    library, not the normal equations). Column scales spread over three decades so the
    diagonal scaling matters."""
    rng = np.random.default_rng(2)
    J = rng.normal(size=(240, 6)) * np.logspace(-2, 1, 6)[None, :]
    r = rng.normal(size=240)
    D = np.diag(J.T @ J)
    A = np.vstack([J, np.diag(np.sqrt(lam * D))])
    rhs = np.concatenate([-r, np.zeros(6)])
    ref = np.linalg.lstsq(A, rhs, rcond=None)[0]
    np.testing.assert_allclose(gn.gn_delta(J, r, lam), ref, rtol=1e-10, atol=1e-14)
    # and it differs from the undamped step
    assert np.abs(gn.gn_delta(J, r, lam) - gn.gn_delta(J, r)).max() > 1e-6 * np.abs(ref).max()


def test_heavy_damping_is_a_scaled_gradient_step():
    """lambda -> infinity: lambda delta -> -D^-1 J^T r, the diagonally scaled steepest
    descent direction of |J z + r|^2 / 2."""
    rng = np.random.default_rng(3)
    J = rng.normal(size=(120, 5))
    r = rng.normal(size=120)
    lam = 1e9
    D = np.diag(J.T @ J)
    np.testing.assert_allclose(lam * gn.gn_delta(J, r, lam), -(J.T @ r) / D, rtol=1e-7, atol=0)


def test_damped_iteration_keeps_the_root():
    """Damping changes the path, not the fixed point: on a well-conditioned zero-residual
    problem r(z) = A z + 0.1 sin(B z) - t the damped iteration converges to z* (linearly,
    about lambda / (1 + lambda) per iteration), while one damped step is only partial."""
    rng = np.random.default_rng(7)
    m, r = 90, 6
    A = rng.normal(size=(m, r))
    B = rng.normal(size=(m, r))
    zs = rng.normal(size=r)
    t = A @ zs + 0.1 * np.sin(B @ zs)
    z = zs + 0.05 * rng.normal(size=r)
    errs = []
    for _ in range(25):
        res = A @ z + 0.1 * np.sin(B @ z) - t
        J = A + 0.1 * np.cos(B @ z)[:, None] * B
        z = z + gn.gn_delta(J, res, 0.1)
        errs.append(np.linalg.norm(z - zs))
    assert errs[0] > 1e-3
    assert errs[-1] <= 1e-12
