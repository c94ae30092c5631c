"""The GPU full-order MLS-MPM step (nsf_fo_*) against the FP64 oracle's full-order model
(oracle/fullorder.py; Sec. 3.3 with the supplementary return maps: von Mises with fixed
corotated elasticity, Drucker-Prager, Herschel-Bulkley).

The cube falls onto the separating ground, and a low yield stress makes the return map
active once it lands. The GPU keeps x, v and C in FP32 and F^E in FP64, so positions
follow the oracle to FP32 rounding (gate delta_x <= 1e-5, the reduced step's). The
stress follows to the FP32 error of C and x carried through F (gate 1e-3 of its largest
magnitude). Running the oracle again without plasticity must move the positions far more
than the GPU's distance from the plastic run, so the return map is really exercised.
"""
import numpy as np
import pytest
import torch

from oracle import fullorder as FO
from oracle.step import relative_error
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.fullorder import FullOrderSim

pytestmark = pytest.mark.gpu


def _cube(P=3000, seed=11):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-0.1, 0.1, size=(P, 3)) + np.array([0.5, 0.5, 0.15])


def test_full_order_matches_oracle_through_impact():
    X = _cube()
    kw = dict(rho=1000.0, volume=0.2 ** 3, E=5e4, nu=0.3, n=64, dt=1e-4)
    print("\n[case] full-order cube P=3000 grid=64 impact, tau_y=50", flush=True)
    o = FO.FullOrder(X, (0.0, 0.0, -2.0), tau_y=50.0, **kw)
    elastic = FO.FullOrder(X, (0.0, 0.0, -2.0), tau_y=1e12, **kw)
    s = torch.cuda.Stream()
    g = FullOrderSim(X.T.astype(np.float32), (0.0, 0.0, -2.0), 1000.0, 0.2 ** 3, 5e4, 0.3, 50.0, 64, 1e-4,
                     stream=s)
    steps = 30
    for k in range(steps):
        o.step()
        elastic.step()
    g.step(steps, stream=s)
    s.synchronize()
    xg = g.positions().double().cpu().numpy().T
    d = relative_error(xg, o.x)
    apart = relative_error(elastic.x, o.x)
    tau_g = g.buffer(A.NSF_FO_TAU).view(6, -1).double().cpu().numpy().T
    tau_o = FO.voigt(o.tau)
    e_tau = float(np.abs(tau_g - tau_o).max() / np.abs(tau_o).max())
    v_g = g.buffer(A.NSF_FO_V).view(3, -1).double().cpu().numpy().T
    e_v = float(np.abs(v_g - o.v).max() / np.abs(o.v).max())
    print(f"delta_x={d:.2e} (plastic vs elastic {apart:.2e}), v err {e_v:.2e}, tau err {e_tau:.2e}, "
          f"max |tau| {np.abs(tau_o).max():.3e}", flush=True)
    assert d <= 1e-5
    assert apart > 100 * d
    assert e_v < 1e-3
    assert e_tau < 1e-3
    assert g.flags(stream=s) == (0, 0)
    g.close()


@pytest.mark.parametrize("model, kw", [
    ("drucker_prager", dict(friction_angle=30.0, tau_y=0.0)),
    ("herschel_bulkley", dict(tau_y=50.0, viscosity=5.0)),
])
def test_full_order_models_match_oracle_through_impact(model, kw):
    """Drucker-Prager (StVK stress in log strain) and Herschel-Bulkley (its own stress,
    eta / (2 mu dt) ~ 1.3, so the deviator is only partly relaxed each step) through the
    impact on the separating ground, against the oracle's models. Both return maps are
    continuous (a Drucker-Prager state at sum(eps) = 0 is at the cone's tip either way),
    so FP32 positions and velocity gradients move F^E only by their own rounding: the
    gates are those of the von Mises run, with the stress compared in norm over all
    particles. The oracle's final state must hold particles on the yield surface, so the
    return map really acts."""
    X = _cube(P=3000, seed=13)
    print(f"\n[case] full-order cube P=3000 grid=64 impact, model={model} {kw}", flush=True)
    mat = dict(rho=1000.0, volume=0.2 ** 3, E=5e4, nu=0.3, n=64, dt=1e-4)
    fric = kw.get("friction_angle", 30.0)
    visc = kw.get("viscosity", 0.0)
    o = FO.FullOrder(X, (0.0, 0.0, -2.0), tau_y=kw["tau_y"], model=model, friction_angle=fric,
                     viscosity=visc, **mat)
    s = torch.cuda.Stream()
    g = FullOrderSim(X.T.astype(np.float32), (0.0, 0.0, -2.0), 1000.0, 0.2 ** 3, 5e4, 0.3, kw["tau_y"], 64,
                     1e-4, stream=s, model=model, friction_angle=fric, viscosity=visc)
    steps = 30
    for _ in range(steps):
        o.step()
    g.step(steps, stream=s)
    s.synchronize()
    d = relative_error(g.positions().double().cpu().numpy().T, o.x)
    tau_g = g.buffer(A.NSF_FO_TAU).view(6, -1).double().cpu().numpy().T
    tau_o = FO.voigt(o.tau)
    e_tau = float(np.linalg.norm(tau_g - tau_o) / np.linalg.norm(tau_o))
    F_g = g.buffer(A.NSF_FO_F).view(9, -1).cpu().numpy().T.reshape(-1, 3, 3)
    e_F = float(np.abs(F_g - o.F).max())
    v_g = g.buffer(A.NSF_FO_V).view(3, -1).double().cpu().numpy().T
    e_v = float(np.abs(v_g - o.v).max() / np.abs(o.v).max())
    if model == "drucker_prager":
        eps = np.log(np.linalg.svd(o.F, compute_uv=False))
        tr = eps.sum(1)
        dg = np.linalg.norm(eps - tr[:, None] / 3, axis=1) + FO.dp_alpha(fric) * (3 * o.lam + 2 * o.mu) * tr / (2 * o.mu)
        on_surface = int(((np.abs(dg) < 1e-9) & (tr < 0)).sum() + (np.abs(eps).max(1) < 1e-12).sum())
    else:
        t = o.tau
        dev = t - (np.trace(t, axis1=1, axis2=2) / 3)[:, None, None] * np.eye(3)
        on_surface = int((np.linalg.norm(dev, axis=(1, 2)) > np.sqrt(2 / 3) * kw["tau_y"] * 1.001).sum())
    print(f"delta_x={d:.2e}, v err {e_v:.2e}, tau err (norm) {e_tau:.2e}, F^E max err {e_F:.2e}, "
          f"yielding particles {on_surface}", flush=True)
    assert on_surface > 100
    assert d <= 1e-5
    assert e_v < 1e-3
    assert e_tau < 1e-3
    assert e_F < 1e-4
    assert g.flags(stream=s) == (0, 0)
    g.close()


def test_full_order_rest_state_is_exact():
    """No gravity, no velocity: the grid sees only the masses, every velocity stays 0 and
    the positions, C, F^E = I and tau = 0 do not change."""
    X = _cube(P=500, seed=3)
    s = torch.cuda.Stream()
    g = FullOrderSim(X.T.astype(np.float32), (0.0, 0.0, 0.0), 1000.0, 0.2 ** 3, 5e4, 0.3, 2e3, 64, 1e-4,
                     gravity=(0.0, 0.0, 0.0), stream=s)
    g.step(5, stream=s)
    s.synchronize()
    assert float(g.buffer(A.NSF_FO_U).abs().max()) == 0.0
    assert float(g.buffer(A.NSF_FO_V).abs().max()) == 0.0
    assert float(g.buffer(A.NSF_FO_TAU).abs().max()) < 1e-6
    F = g.buffer(A.NSF_FO_F).view(9, -1).cpu().numpy()
    np.testing.assert_allclose(F[[0, 4, 8]], 1.0, atol=1e-12)
    np.testing.assert_allclose(F[[1, 2, 3, 5, 6, 7]], 0.0, atol=1e-12)
    g.close()


def test_full_order_descriptor_validation():
    X = _cube(P=10).T.astype(np.float32)
    with pytest.raises(A.NsfError):
        FullOrderSim(X, (0, 0, 0), 1000.0, 1.0, 5e4, 0.5, 2e3, 64, 1e-4)   # nu = 0.5
    with pytest.raises(A.NsfError):
        FullOrderSim(X, (0, 0, 0), 1000.0, 1.0, 5e4, 0.3, 0.0, 64, 1e-4)   # tau_y = 0


def test_full_order_large_set_allocates_over_bins():
    """Above 32,768 particles the slot allocation walks the bins and a separate pass places
    the particles; 40,000 particles for 5 steps against the oracle (gate as above)."""
    X = _cube(P=40_000, seed=12)
    print("\n[case] full-order cube P=40000 grid=64", flush=True)
    o = FO.FullOrder(X, (0.0, 0.0, -2.0), rho=1000.0, volume=0.2 ** 3, E=5e4, nu=0.3, tau_y=50.0, n=64, dt=1e-4)
    s = torch.cuda.Stream()
    g = FullOrderSim(X.T.astype(np.float32), (0.0, 0.0, -2.0), 1000.0, 0.2 ** 3, 5e4, 0.3, 50.0, 64, 1e-4,
                     stream=s)
    for _ in range(5):
        o.step()
    g.step(5, stream=s)
    s.synchronize()
    d = relative_error(g.positions().double().cpu().numpy().T, o.x)
    print(f"delta_x={d:.2e}", flush=True)
    assert d <= 1e-5
    assert g.flags(stream=s) == (0, 0)
    g.close()
