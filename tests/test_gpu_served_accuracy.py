"""Accuracy of the served mix's own instances against the oracle.

The first eight requests of the served mix (Poisson arrivals at 200/s, seed 4; particle
counts log-uniform in 5k-200k, 4% integration = sample particles, r in {6, 12, 24}, 64^3
or 128^3 grids, width-128 fields from seeds 1000 + i) are stepped together in one batch,
as the server steps them, for 20 steps, then each is compared with the FP64 oracle run of
the same instance: every particle decoded.

Reported per instance: delta_x (the paper's Sec. 6 measure over all particles), delta_u
(the same error relative to the displacement x* - X), the latent's error relative to its
motion max|z - z*| / max|z* - z_0|, and cond(J) of the final inversion.

Gates. Positions: delta_x <= 1e-4 for BF16 (the step's error gate) and <= 1e-5 for FP32;
delta_u <= 5e-2 for BF16 (ten times the error of one BF16 evaluation of u at a fixed
latent, ~2^-8 |u|) and <= 1.5e-4 for FP32 (three times the largest measured, 5.1e-5). The
FP32 latent error is gated at 0.1 of its motion (three times the largest measured, 3.0e-2:
from rest the latent moves little in 20 steps, and the weak directions of J, which the
positions barely see, carry the FP32 rounding). The BF16 latent is printed, not gated: it
differs from the oracle's by 0.5-1 of its small motion, along directions below the BF16
Jacobian's resolution. Also printed: e_u, the largest |x - x_oracle(z)| at the GPU's own
latent (the error of one field evaluation), and cond(J) at the last step.
"""
import numpy as np
import pytest
import torch

import synth
from oracle.step import OracleSim, relative_error
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim, step_batch

pytestmark = pytest.mark.gpu

STEPS = 20


def _instances():
    reqs = synth.served_mix(n_requests=256, seed=4)[:8]
    return [synth.served_instance(q, width=128, steps=STEPS) for q in reqs]


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_served_instances_against_oracle(precision):
    ws = _instances()
    print(f"\n[case] served mix instances 0-7, {precision}, {STEPS} steps in one batch", flush=True)
    s = torch.cuda.Stream()
    sims = [Sim(w, precision=precision, stream=s) for w in ws]
    step_batch(sims, STEPS, stream=s)
    s.synchronize()
    worst = {}
    for i, (w, sim) in enumerate(zip(ws, sims)):
        z, _, st = sim.latent(stream=s)
        assert st == STEPS
        assert sim.flags(stream=s) == (0, 0)
        xg = sim.buffer(A.NSF_BUF_XDEC).reshape(3, -1).double().cpu().numpy().T
        sim.close()
        o = OracleSim(w)
        o.step(STEPS)
        xo = o.decode()
        X = o.X
        dx = relative_error(xg, xo)
        du = relative_error(xg - X, xo - X)
        motion = float(np.abs(o.z - w.z0).max())
        dz = float(np.abs(z - o.z).max() / motion)
        e_u = float(np.abs(xg - (X + o.u(X, z))).max())
        idx = o.indices(STEPS)
        J = o.jac(X[idx][:w.n_sample], o.z).reshape(-1, w.r)
        sv = np.linalg.svd(J, compute_uv=False)
        cond = float(sv[0] / sv[-1])
        print(f"instance {i}: P={X.shape[0]} N=S={w.n_sample} r={w.r} grid={w.grid_n}: "
              f"delta_x={dx:.2e} delta_u={du:.2e} dz/motion={dz:.2e} "
              f"e_u={e_u:.1e} cond(J)={cond:.1e}", flush=True)
        worst = {k: max(worst.get(k, 0.0), v) for k, v in (("dx", dx), ("du", du), ("dz", dz))}
        if precision == "bf16":
            assert dx <= 1e-4
            assert du <= 5e-2
        else:
            assert dx <= 1e-5
            assert du <= 1.5e-4
            assert dz <= 0.1
    print(f"worst over the eight: {worst}", flush=True)
