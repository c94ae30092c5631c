"""Batched stepping (nsf_step_batch): each simulation's result is the same alone and in the
mix, also when sims join and leave the batch, and a failing sim does not disturb others.

Sims in a batch share kernels but not state (latents, grids, buffers), and every sum in
the step runs in a fixed order (the field MLPs per tile, P2G per node in particle order,
the Gauss-Newton partials per chunk), so a sim's latent and decoded positions are bit for
bit the same alone and in any mix. The batched FP32 latents are also checked against the
oracle.
"""
import copy

import numpy as np
import pytest
import torch

import synth
from oracle.step import OracleSim
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim, step_batch

pytestmark = pytest.mark.gpu


def _instances(precision):
    out = []
    # well-posed instances: 3|S| >> r and cond(J) <= ~1e4 (checked with the oracle)
    for i, (r, n, ni, grid) in enumerate([(6, 3000, 700, 64), (12, 2000, 600, 64), (24, 2500, 800, 64)]):
        w = synth.cake_slab(seed=10 + i, r=r, width=128, n=n, n_integration=ni, steps=8,
                            grid_n=grid, bias_scale=0.05)
        w.z_prev = w.z0 - 1e-3 * np.random.default_rng(i).normal(size=r)
        out.append(w)
    return out


def _state(sim, s):
    z, zp, st = sim.latent(stream=s)
    x = sim.buffer(A.NSF_BUF_XDEC).double().cpu().numpy()
    return z, x, st


def _close(a, b, w):
    (za, xa, sa), (zb, xb, sb) = a, b
    assert sa == sb
    np.testing.assert_array_equal(za, zb)
    np.testing.assert_array_equal(xa, xb)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "mixed"])
def test_batch_equals_alone(precision):
    print(f"\n[case] batch equals alone {precision}", flush=True)
    s = torch.cuda.Stream()
    ws = _instances(precision)
    alone = []
    for w in ws:
        sim = Sim(w, precision=precision, stream=s)
        sim.step(5, stream=s)
        alone.append(_state(sim, s))
        sim.close()
    sims = [Sim(w, precision=precision, stream=s) for w in ws]
    step_batch(sims, 5, stream=s)
    for w, sim, ref in zip(ws, sims, alone):
        _close(_state(sim, s), ref, w)
        assert sim.flags(stream=s) == (0, 0)
        if precision == "fp32":
            o = OracleSim(w)
            # first-order least-squares perturbation: the FP32 Jacobian's relative error
            # (~1e-6 at width 128) moves each Gauss-Newton step by up to cond(J) times it;
            # taken with a factor 10, and never below 1e-2 of the motion
            idx = o.indices(0)
            J = o.jac(o.X[idx][:w.n_sample], o.z).reshape(-1, w.r)
            tol = max(1e-2, 10 * np.linalg.cond(J) * 1e-6)
            o.step(5)
            z, _, _ = sim.latent(stream=s)
            err = np.abs(z - o.z).max() / np.abs(o.z - w.z0).max()
            print(f"r={w.r}: latent error {err:.2e} of the motion (bound {tol:.2e})", flush=True)
            assert err <= tol


def test_batch_membership_changes():
    """A and B step together; C joins; A leaves; every sim ends where it would alone."""
    print("\n[case] batch membership changes", flush=True)
    s = torch.cuda.Stream()
    wa, wb, wc = _instances("fp32")
    ref = {}
    for key, w, n in (("a", wa, 3), ("b", wb, 6), ("c", wc, 4)):
        sim = Sim(w, stream=s)
        sim.step(n, stream=s)
        ref[key] = _state(sim, s)
        sim.close()
    a, b = Sim(wa, stream=s), Sim(wb, stream=s)
    step_batch([a, b], 2, stream=s)
    c = Sim(wc, stream=s)
    step_batch([a, b, c], 1, stream=s)
    a_state = _state(a, s)
    a.close()
    step_batch([b, c], 3, stream=s)
    _close(a_state, ref["a"], wa)
    _close(_state(b, s), ref["b"], wb)
    _close(_state(c, s), ref["c"], wc)


def test_batch_failure_is_isolated():
    """A non-finite latent in one sim raises only that sim's flag."""
    print("\n[case] batch failure isolation", flush=True)
    s = torch.cuda.Stream()
    ws = _instances("fp32")
    ref = []
    for w in ws[1:]:
        sim = Sim(w, stream=s)
        sim.step(3, stream=s)
        ref.append(_state(sim, s))
        sim.close()
    sims = [Sim(w, stream=s) for w in ws]
    z = np.array(ws[0].z0)
    z[0] = np.nan
    sims[0].set_latent(z, stream=s)
    step_batch(sims, 3, stream=s)
    st, f = sims[0].flags(stream=s)
    assert f & A.NSF_FLAG_NONFINITE
    for w, sim, r in zip(ws[1:], sims[1:], ref):
        assert sim.flags(stream=s) == (0, 0)
        _close(_state(sim, s), r, w)
