"""Fitting the fields to a full-order run with the hand-written backward (Sec. 4.5).

Training data comes from the oracle's full-order MLS-MPM (fixed corotated + von Mises) on
a reduced version of the falling-cube workload: 2,000 particles, 32^3 grid, dt = 5e-4,
400 steps, a snapshot every 20 steps. The Fitter trains g with one latent per snapshot
(r = 12, width 128, BF16 hidden layers, Adam on FP32 masters), then h and l with the
latents frozen. Checks:
  - each field's loss falls by the stated factor;
  - the fitted deformation field reproduces the snapshots' positions to delta_x <= 1e-2
    on average over the snapshots and <= 3e-2 on the worst one (a convergence check of
    2,000 Adam steps on an impact with plastic flow, not a parity bound);
  - the fitted weights deploy unchanged: nsf_decode of a sim built from them, at a
    snapshot's latent, equals the training kernel's output at the same latent.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fullorder as FO
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.fit import Fitter, Snapshots
from paper_2310_17790_amd.sim import Sim

pytestmark = pytest.mark.gpu


def _snapshots():
    rng = np.random.Generator(np.random.PCG64(7))
    X = rng.uniform(-0.1, 0.1, size=(2000, 3)) + np.array([0.5, 0.5, 0.4])
    sim = FO.FullOrder(X, (0.0, 0.0, -2.0), rho=1000.0, volume=0.2 ** 3, E=5e4, nu=0.3,
                       tau_y=2e3, n=32, dt=5e-4)
    xs, taus, Cs = [], [], []
    for s in range(1, 401):
        sim.step()
        if s % 20 == 0:
            xs.append(sim.x.copy())
            taus.append(FO.voigt(sim.tau))
            Cs.append(sim.C.reshape(-1, 9).copy())
    return Snapshots(X=X, x=np.stack(xs), tau=np.stack(taus), C=np.stack(Cs))


@pytest.fixture(scope="module")
def fitted():
    data = _snapshots()
    print(f"\n[case] full-order data: {data.x.shape[0]} snapshots, min z {data.x[..., 2].min():.3f}, "
          f"max |tau| {np.abs(data.tau).max():.3e}", flush=True)
    f = Fitter(data, r=12, width=128, precision="bf16", batch=1 << 14, seed=0)
    losses = {k: f.fit(k, it) for k, it in (("g", 2000), ("h", 1000), ("l", 1000))}
    torch.cuda.synchronize()
    for k, L in losses.items():
        print(f"[fit] {k}: loss {np.mean(L[:10]):.3e} -> {np.mean(L[-20:]):.3e}", flush=True)
    return data, f, losses


def test_losses_fall(fitted):
    _, _, losses = fitted
    for k, factor in (("g", 30.0), ("h", 2.0), ("l", 2.0)):
        L = losses[k]
        assert np.all(np.isfinite(L))
        assert np.mean(L[:10]) / np.mean(L[-20:]) >= factor, k


def test_fitted_positions(fitted):
    data, f, _ = fitted
    errs = [f.relative_error("g", t) for t in range(data.x.shape[0])]
    print(f"[fit] delta_x over snapshots: max {max(errs):.2e}, mean {np.mean(errs):.2e}", flush=True)
    assert np.mean(errs) <= 1e-2 and max(errs) <= 3e-2


def test_fitted_weights_deploy_to_the_sim(fitted):
    """The same flat weights and de-normalisation drive nsf_decode of a reduced sim."""
    data, f, _ = fitted
    ex = f.export()
    w = synth.cake_slab(seed=0, r=12, width=128, n=data.X.shape[0], n_integration=200, steps=4,
                        grid_n=32)
    w.X = np.ascontiguousarray(data.X.T.astype(np.float32))
    w.fields = {k: _unflatten(ex["weights"][k], 12, 128, d) for k, d in (("g", 3), ("h", 6), ("l", 9))}
    w.out_scale = {k: np.asarray(ex["out_scale"][k], np.float64) for k in "ghl"}
    w.out_shift = {k: np.asarray(ex["out_shift"][k], np.float64) for k in "ghl"}
    t = 7
    w.z0 = ex["z"][t].copy()
    w.z_prev = ex["z"][t].copy()
    s = torch.cuda.Stream()
    sim = Sim(w, precision="bf16", stream=s)
    out = torch.empty(3 * w.n_particles, dtype=torch.float32, device="cuda")
    Xd = torch.from_numpy(w.X).cuda()
    A.nsf_decode(sim.handle, Xd.data_ptr(), w.n_particles, out.data_ptr(), s.cuda_stream)
    s.synchronize()
    x_sim = out.reshape(3, -1).double().cpu().numpy().T
    # the training kernel at the same latent
    from paper_2310_17790_amd.train import FieldFn
    Xt = torch.from_numpy(data.X.astype(np.float32)).cuda()
    Z = f.z.detach()[torch.full((w.n_particles,), t, device="cuda", dtype=torch.long)]
    y = FieldFn.apply(Xt, Z, f.w["g"].detach(), 128, 3, "bf16").double().cpu().numpy()
    x_fit = w.out_scale["g"] * y + w.out_shift["g"] + data.X
    err = np.abs(x_sim - x_fit).max()
    print(f"[fit] deploy: max |x_sim - x_fit| = {err:.2e}", flush=True)
    assert err <= 1e-5
    sim.close()


def _unflatten(flat, r, width, d):
    dims = [3 + r, width, width, width, width, width, d]
    out, o = [], 0
    for k in range(6):
        n_in, n_out = dims[k], dims[k + 1]
        W = flat[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = flat[o:o + n_out]
        o += n_out
        out.append((W.astype(np.float32), b.astype(np.float32)))
    return out
