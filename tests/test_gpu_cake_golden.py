"""Cake-scale parity over 100 steps against stored FP64 oracle trajectories.

The workload is the benchmark's: 200,000 particles in the slab, 8,192 integration = sample
particles resampled each step, width-128 fields (seed 0), 128^3 grid, dt = 5e-5, knife,
2 Gauss-Newton iterations, run through the same graph-replayed step. The reference
latents and the decoded positions of 2,048 fixed particles after steps 10, 50 and 100 were
written by tests/golden/make_golden.py, which calls only the oracle.

Gates (relative position error delta of the paper's Sec. 6, over the sampled particles):
  FP32: delta_x <= 1e-5 at every checkpoint (FP32 rounding only).
  BF16 hidden layers (velocity as a midpoint JVP and trapezoid Gauss-Newton residuals,
  both O(|dz|^3) from the oracle's exact differences): delta_x <= 1e-4 after 100 steps.
Also printed, not gated: delta_u on displacements (much stricter: |X| dominates |x|),
the largest per-particle position error, and the latent's deviation.
"""
import os

import numpy as np
import pytest
import torch

import synth
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(r):
    path = os.path.join(GOLDEN, f"cake200k_r{r}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path, allow_pickle=False)


def _run(r, precision):
    g = _load(r)
    w = synth.cake_slab(seed=0, r=r, width=128, n=200_000, n_integration=8192, steps=100)
    s = torch.cuda.Stream()
    sim = Sim(w, precision=precision, stream=s)
    idx = torch.from_numpy(g["idx"]).cuda()
    X = w.X[:, g["idx"]].T.astype(np.float64)
    out = {}
    done = 0
    for ck, x_ref in zip(g["steps"], g["x"]):
        sim.step(int(ck) - done, stream=s)
        done = int(ck)
        s.synchronize()
        xg = sim.buffer(A.NSF_BUF_XDEC).reshape(3, -1)[:, idx].double().cpu().numpy().T
        z, _, st = sim.latent(stream=s)
        assert st == ck
        dx = float(np.sqrt(((xg - x_ref) ** 2).sum() / (x_ref ** 2).sum()))
        du = float(np.sqrt(((xg - x_ref) ** 2).sum() / ((x_ref - X) ** 2).sum()))
        emax = float(np.abs(xg - x_ref).max())
        dz = float(np.abs(z - g["z"][ck]).max() / np.abs(g["z"][ck] - g["z"][0]).max())
        out[int(ck)] = (dx, du, emax, dz)
        print(f"[{precision} r={r}] step {ck}: delta_x={dx:.2e} delta_u={du:.2e} "
              f"max|dx|={emax:.2e} dz/motion={dz:.2e}", flush=True)
    assert sim.flags(stream=s) == (0, 0)
    return out


@pytest.mark.parametrize("r", [6, 24])
def test_cake_fp32_100_steps(r):
    res = _run(r, "fp32")
    for dx, du, emax, dz in res.values():
        assert dx <= 1e-5


@pytest.mark.parametrize("r", [6, 24])
def test_cake_bf16_gate_100_steps(r):
    res = _run(r, "bf16")
    assert res[100][0] <= 1e-4
