"""Cake-scale parity against stored FP64 oracle trajectories.

The workload is the benchmark's: 200,000 particles in the slab, 8,192 integration = sample
particles resampled each step, width-128 fields (seed 0), 128^3 grid, dt = 5e-5, knife,
2 Gauss-Newton iterations, run through the same graph-replayed step. The reference
latents, and the decoded positions and Kirchhoff stresses of 2,048 fixed particles after
steps 10, 50 and 100, were written by tests/golden/make_golden.py, which calls only the
oracle.

Gates (relative errors delta of the paper's Sec. 6, over the sampled particles):
  FP32: delta_x <= 1e-5 at every checkpoint; delta_tau <= 2e-2. The stress bound follows
  the Jacobian's conditioning: FP32 Jacobian entries carry ~1e-6 |J| at width 128 (the
  accumulated rounding of four 128-term layers, as the stage-parity test measures), and
  the inversion amplifies that along the weakest latent direction by sigma_max /
  sigma_min (~2e2 at r = 6), per step, and h depends on every latent direction: over
  100 steps 1e-6 x 2e2 x 100 = 2e-2. At r = 24 (up to 7e3 by step 50) the same reasoning
  allows more; the same 2e-2 is kept, well above what it reaches.
  BF16 hidden layers (velocity as a midpoint JVP and trapezoid Gauss-Newton residuals,
  both O(|dz|^3) from the oracle's exact differences): delta_x <= 1e-4 at the last
  checkpoint and delta_u <= 5e-2 at every checkpoint (ten times the error of one BF16
  evaluation of u at a fixed latent, which is 2^-8-sized: ~5e-3 here).
The stress is evaluated at the GPU's latent by the GPU field kernel (nsf_mlp_forward).

What BF16 leaves ungated, and why. Over 100 steps of dt = 5e-5 the slab falls ~1.2e-4 m,
while one BF16 evaluation of u (|u| ~ 5e-3 m) is already off by ~2e-5 m; the latent moves
correspondingly little. With random-init fields the latent Jacobian of g over the slab
has three strong singular values (roughly the three translations of a field that is
smooth at the slab's scale) and r - 3 weak ones, 30x to 3e4x smaller (r = 6: 0.57, 0.38,
0.13, then 6.6e-3, 5.5e-3, 3.1e-3), below the 2^-8 |J| error of BF16 Jacobian entries.
So the BF16 latent differs from the oracle's by a sizeable fraction of its small motion,
and h, which depends on every latent direction, shows it: delta_tau and the latent error
(split with the oracle Jacobian's right singular vectors into the strong subspace,
sigma >= 0.05 sigma_max, and the rest) are printed, not gated.

r = 24 is compared through step 50 only. With random-init weights its latent keeps
accelerating (|z| 0.18 -> 0.93 -> 6.1 at steps 10/50/100, per-step |dz| up to 0.2) and
the Jacobian's conditioning degrades with it (sigma_max / sigma_min 7e3 at step 50, 2.8e4
at step 100); somewhere after step 50 an FP32 Jacobian no longer determines the
Gauss-Newton step (the FP32 run stops with NSF_SINGULAR before step 100) while the FP64
oracle still solves it. The FP64 trajectory itself is well conditioned up to step 50 and
chaotic after it: a 1e-10 change of z0 moves the oracle's positions by 2.9e-12 at step 50,
2.2e-9 at step 75 and 3.4e-4 at step 100 (tests/golden/sensitivity.py,
sensitivity_r24.txt), so at step 100 no arithmetic can match it to a 1e-4 gate.
Also printed: delta_u on displacements (|X| dominates |x|), the largest per-particle
position error, and the latent's deviation.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import fields as F
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim, flatten_mlp
from paper_2310_17790_amd.train import FieldFn

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAST = {6: 100, 24: 50}


def _load(r):
    path = os.path.join(GOLDEN, f"cake200k_r{r}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path, allow_pickle=False)


def _gpu_tau(w, X, z, precision):
    """Kirchhoff stress at positions X (n, 3) and latent z from the GPU field kernel."""
    wt = torch.from_numpy(flatten_mlp(w.fields["h"])).cuda()
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    Z = torch.from_numpy(np.broadcast_to(z.astype(np.float32), (X.shape[0], z.size)).copy()).cuda()
    out = FieldFn.apply(Xt, Z, wt, 128, 6, precision).double().cpu().numpy()
    return w.out_scale["h"] * out + w.out_shift["h"]


def _split_latent_error(w, X, z_ref, z0, z):
    """Latent error relative to the latent's motion, in the span of the oracle Jacobian's
    strong right singular vectors (sigma >= 0.05 sigma_max) and in the rest."""
    J = F.jacobian_z(w.fields["g"], X, z_ref, w.out_scale["g"]).reshape(-1, z_ref.size)
    _, sv, Vt = np.linalg.svd(J, full_matrices=False)
    k = int((sv >= 0.05 * sv[0]).sum())
    Vs, Vw = Vt[:k], Vt[k:]
    e, m = z - z_ref, z_ref - z0
    strong = float(np.linalg.norm(Vs @ e) / np.linalg.norm(Vs @ m))
    weak = float(np.linalg.norm(Vw @ e) / max(np.linalg.norm(Vw @ m), 1e-300)) if k < z.size else 0.0
    return strong, weak


def _run(r, precision):
    g = _load(r)
    w = synth.cake_slab(seed=0, r=r, width=128, n=200_000, n_integration=8192, steps=100)
    s = torch.cuda.Stream()
    sim = Sim(w, precision=precision, stream=s)
    idx = torch.from_numpy(g["idx"]).cuda()
    X = w.X[:, g["idx"]].T.astype(np.float64)
    out = {}
    done = 0
    for ck, x_ref, tau_ref in zip(g["steps"], g["x"], g["tau"]):
        ck = int(ck)
        if ck > LAST[r]:
            break
        sim.step(ck - done, stream=s)
        done = ck
        s.synchronize()
        xg = sim.buffer(A.NSF_BUF_XDEC).reshape(3, -1)[:, idx].double().cpu().numpy().T
        z, _, st = sim.latent(stream=s)
        assert st == ck
        torch.cuda.synchronize()
        tau = _gpu_tau(w, X, z, precision)
        dx = float(np.sqrt(((xg - x_ref) ** 2).sum() / (x_ref ** 2).sum()))
        du = float(np.sqrt(((xg - x_ref) ** 2).sum() / ((x_ref - X) ** 2).sum()))
        dt = float(np.sqrt(((tau - tau_ref) ** 2).sum() / (tau_ref ** 2).sum()))
        emax = float(np.abs(xg - x_ref).max())
        dz = float(np.abs(z - g["z"][ck]).max() / np.abs(g["z"][ck] - g["z"][0]).max())
        strong, weak = _split_latent_error(w, X, g["z"][ck], g["z"][0], z)
        out[ck] = (dx, dt, du, emax, dz, strong, weak)
        print(f"[{precision} r={r}] step {ck}: delta_x={dx:.2e} delta_tau={dt:.2e} "
              f"delta_u={du:.2e} max|dx|={emax:.2e} dz/motion={dz:.2e} "
              f"strong={strong:.2e} weak={weak:.2e}", flush=True)
    assert sim.flags(stream=s) == (0, 0)
    return out


TAU_FP32 = {6: 2e-2, 24: 2e-2}


@pytest.mark.parametrize("r", [6, 24])
def test_cake_fp32(r):
    res = _run(r, "fp32")
    assert max(res) == LAST[r]
    for dx, dt, *_ in res.values():
        assert dx <= 1e-5
        assert dt <= TAU_FP32[r]


@pytest.mark.parametrize("r", [6, 24])
def test_cake_bf16_gate(r):
    res = _run(r, "bf16")
    assert res[LAST[r]][0] <= 1e-4
    for v in res.values():
        assert v[2] <= 5e-2
