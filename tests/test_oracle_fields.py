"""Pins for the oracle's neural fields and forward-mode latent Jacobian
(paper Sec. 4.2-4.4; supplementary "Network architecture")."""
import numpy as np
import pytest
import torch

import synth
from oracle import fields as F


def _torch_mlp(layers, X, z):
    """Independent evaluation with torch.nn.functional in float64, input built here."""
    Xt = torch.tensor(np.asarray(X, np.float64))
    zt = torch.tensor(np.asarray(z, np.float64))
    h = torch.cat([Xt, zt.expand(Xt.shape[0], -1)], dim=1)
    for k, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(h, torch.tensor(W, dtype=torch.float64),
                                       torch.tensor(b, dtype=torch.float64))
        if k < len(layers) - 1:
            h = torch.nn.functional.elu(h, alpha=1.0)
    return h.numpy()


@pytest.mark.parametrize("r,width", [(6, 64), (3, 16), (24, 32)])
def test_mlp_matches_torch_functional(r, width):
    fl = synth.make_fields(5, r, width, bias_scale=0.3)
    X = synth.box_points(6, 300, (0.3, 0.3, 0.3), (0.7, 0.7, 0.7)).T
    z = synth.latent(7, r, 0.5)
    for name in synth.FIELD_NAMES:
        ours = F.mlp(fl[name], F.network_input(X, z))
        ref = _torch_mlp(fl[name], X, z)
        assert ours.shape == (300, synth.FIELD_OUT[name])
        np.testing.assert_allclose(ours, ref, rtol=1e-13, atol=1e-14)


def test_elu_and_derivative():
    a = np.linspace(-5, 5, 1001)
    np.testing.assert_allclose(F.elu(a), torch.nn.functional.elu(torch.tensor(a)).numpy(), atol=1e-15)
    h = 1e-6
    fd = (F.elu(a + h) - F.elu(a - h)) / (2 * h)
    np.testing.assert_allclose(F.elu_prime(a), fd, atol=5e-7)  # kink at 0: FD error h/4


@pytest.mark.parametrize("r,width", [(6, 64), (24, 32), (1, 8)])
def test_forward_jacobian_matches_central_fd(r, width):
    fl = synth.make_fields(8, r, width, bias_scale=0.2)
    X = synth.box_points(9, 64, (0.3, 0.3, 0.3), (0.7, 0.7, 0.7)).T
    z = synth.latent(10, r, 0.3)
    scale, shift = np.full(3, 0.7), np.full(3, 0.1)
    J = F.jacobian_z(fl["g"], X, z, scale)
    Jfd = F.jacobian_z_fd(fl["g"], X, z, scale, shift)
    assert J.shape == (64, 3, r)
    err = np.abs(J - Jfd).max() / np.abs(J).max()
    assert err < 1e-7


def test_output_denormalisation_closed_form():
    """With W6 = 0 the field is scale * b6 + shift, independent of X and z; with b6 = 0
    as well the decode returns X exactly."""
    r, width = 6, 16
    fl = synth.make_fields(1, r, width)
    W6, b6 = fl["g"][-1]
    b6 = np.array([0.5, -1.0, 2.0], np.float32)
    fl["g"][-1] = (np.zeros_like(W6), b6)
    X = synth.box_points(2, 50, (0, 0, 0), (1, 1, 1)).T
    z = synth.latent(3, r, 1.0)
    scale, shift = np.array([1e-2, 2.0, 3.0]), np.array([0.1, 0.2, 0.3])
    u = F.field(fl["g"], X, z, scale, shift)
    np.testing.assert_array_equal(u, np.broadcast_to(scale * b6.astype(np.float64) + shift, u.shape))
    fl["g"][-1] = (np.zeros_like(W6), np.zeros(3, np.float32))
    u0 = F.field(fl["g"], X, z, scale, np.zeros(3))
    assert np.all(u0 == 0.0)


def test_voigt_matrix_is_symmetric_and_complete():
    t = np.arange(1.0, 7.0)[None, :]
    M = F.voigt_to_matrix(t)[0]
    np.testing.assert_array_equal(M, M.T)
    assert sorted(np.unique(M).tolist()) == [1, 2, 3, 4, 5, 6]
    np.testing.assert_array_equal(np.diag(M), [1, 2, 3])


def test_stress_field_with_problem_parameters_matches_torch():
    """h(X, z, mu) (Sec. 4.3): eval_fields feeds [X; z; mu] to the stress field only; an
    independent torch evaluation builds the rows [X; z; mu] itself. g and l ignore mu."""
    r, n_mu = 4, 2
    fl = synth.make_fields(7, r, 32, bias_scale=0.1, n_mu=n_mu)
    assert fl["h"][0][0].shape[1] == 3 + r + n_mu and fl["g"][0][0].shape[1] == 3 + r
    X = synth.box_points(8, 50, (0.3, 0.3, 0.3), (0.7, 0.7, 0.7)).T
    z = synth.latent(9, r, 0.2)
    mu = np.array([0.7, -1.3])
    scale, shift = synth.default_scales()
    u, tau, C = F.eval_fields(fl, X, z, scale, shift, mu)
    ref_h = _torch_mlp(fl["h"], X, np.concatenate([z, mu]))
    np.testing.assert_allclose(tau[:, 0, 0], ref_h[:, 0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(tau[:, 1, 2], ref_h[:, 3], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(u, 1e-2 * _torch_mlp(fl["g"], X, z), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(C.reshape(-1, 9), _torch_mlp(fl["l"], X, z), rtol=1e-12, atol=1e-14)
    # zero mu columns: the parameters drop out
    h0 = [(W.copy(), b) for W, b in fl["h"]]
    h0[0][0][:, 3 + r:] = 0.0
    fl0 = dict(fl, h=h0)
    _, tau_a, _ = F.eval_fields(fl0, X, z, scale, shift, mu)
    _, tau_b, _ = F.eval_fields(fl0, X, z, scale, shift, -mu)
    np.testing.assert_array_equal(tau_a, tau_b)
