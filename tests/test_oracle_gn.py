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
