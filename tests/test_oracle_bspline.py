"""Pins for the oracle's quadratic B-spline stencil (paper Sec. 3.2 weights w_ip = N(x_p - x_i),
Sec. 3.3 constant 12 / (dx^2 (b + 1)))."""
import os

import numpy as np
import pytest

from oracle import mpm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


def test_kernel_tabulated_values():
    tab = _load("bspline_values.txt")
    for d, val in tab:
        assert mpm.bspline_kernel(np.array([d]))[0] == pytest.approx(val, abs=1e-15)
        assert mpm.bspline_kernel(np.array([-d]))[0] == pytest.approx(val, abs=1e-15)


def test_stencil_weights_match_kernel():
    rng = np.random.default_rng(1)
    f = rng.uniform(0.5, 1.5, size=1000)
    w = mpm.bspline_weights(f)
    for k in range(3):
        # node base + k sits at distance (k - f) grid units from the particle
        np.testing.assert_allclose(w[:, k], mpm.bspline_kernel(k - f), atol=1e-15)


@pytest.mark.parametrize("dx", [1 / 32, 1 / 128])
def test_moments(dx):
    """sum w = 1, sum w (x_i - x_p) = 0, sum w (x_i - x_p)(x_i - x_p)^T = (dx^2/4) I, whose
    inverse is the golden constant of Sec. 3.3 at b = 2."""
    tab = _load("apic_dinv.txt")
    dinv = {round(r[1], 12): r[2] for r in tab}[round(dx, 12)]
    rng = np.random.default_rng(2)
    x = rng.uniform(0.3, 0.7, size=(500, 3))
    base, f, w = mpm.stencil(x, dx)
    S0 = np.zeros(500)
    S1 = np.zeros((500, 3))
    S2 = np.zeros((500, 3, 3))
    for o in mpm.OFFSETS:
        wip = w[:, 0, o[0]] * w[:, 1, o[1]] * w[:, 2, o[2]]
        node_x = (base + o) * dx
        d = node_x - x
        S0 += wip
        S1 += wip[:, None] * d
        S2 += wip[:, None, None] * d[:, :, None] * d[:, None, :]
    np.testing.assert_allclose(S0, 1.0, atol=1e-14)
    np.testing.assert_allclose(S1, 0.0, atol=1e-15)
    np.testing.assert_allclose(S2 * dinv, np.broadcast_to(np.eye(3), S2.shape), atol=1e-12)


def test_stencil_vs_brute_force_all_nodes():
    """On an 8^3 grid, the 27-node stencil equals the kernel evaluated at every node."""
    n, dx = 8, 1 / 8
    rng = np.random.default_rng(3)
    x = rng.uniform(2 * dx, 5 * dx, size=(5, 3))
    base, f, w = mpm.stencil(x, dx)
    dense_st = np.zeros((5, n, n, n))
    for o in mpm.OFFSETS:
        wip = w[:, 0, o[0]] * w[:, 1, o[1]] * w[:, 2, o[2]]
        node = base + o
        for p in range(5):
            dense_st[p, node[p, 0], node[p, 1], node[p, 2]] += wip[p]
    i = np.arange(n)
    for p in range(5):
        wx = mpm.bspline_kernel((x[p, 0] - i * dx) / dx)
        wy = mpm.bspline_kernel((x[p, 1] - i * dx) / dx)
        wz = mpm.bspline_kernel((x[p, 2] - i * dx) / dx)
        brute = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
        np.testing.assert_allclose(dense_st[p], brute, atol=1e-15)


def test_tie_gives_zero_weight():
    """At an exact tie (f = 0.5) the far node's weight is exactly zero, so the choice of
    base at a tie cannot change a transfer."""
    w = mpm.bspline_weights(np.array([0.5]))
    assert w[0, 2] == 0.0
    assert w[0, 0] == 0.5 and w[0, 1] == 0.5
