"""Edge cases of the GPU path against the FP64 oracle: BF16 stage parity at both widths
(the width-64 kernels carry four tangents per wave, the width-128 ones two), and the ABI's
empty calls.

BF16 tolerance. Each of the four hidden layers rounds its weights and its input
activations to BF16 (unit roundoff u = 2^-9), so a layer's output carries up to ~2u of
the sum of its terms' magnitudes. Over four layers that is ~8u = 1.6e-2 of the field's
scale, and 3e-2 of each quantity's largest magnitude is used. The first and output
layers are FP32. The velocity is the directional derivative at the midpoint. Its error is
the Jacobian's BF16 error, plus an O(|dz|^3) truncation that is negligible at
|dz| ~ 2e-3.
"""
import copy

import numpy as np
import pytest
import torch

import synth
from oracle.step import OracleSim
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim

pytestmark = pytest.mark.gpu

TOL_BF16 = 3e-2


def _soa(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("width", [64, 128])
def test_bf16_stage_parity(width):
    r, n = 6, 1000
    w = copy.deepcopy(synth.small_cube(seed=5, r=r, width=width, n=n, bias_scale=0.1))
    w.z_prev = w.z0 - 2e-3 * np.random.default_rng(7).normal(size=r)
    print(f"\n[case] bf16 stage parity width={width}", flush=True)
    s = torch.cuda.Stream()
    sim = Sim(w, precision="bf16", stream=s)
    sim.refresh(stream=s)
    s.synchronize()
    o = OracleSim(w)
    idx = o.indices(0)
    x, v, tau, C, u_n = o.inference(idx)
    N, S = w.n_integration, w.n_sample
    errs = {
        "u": _rel_max(_soa(sim.buffer(A.NSF_BUF_U)).reshape(3, N).T, u_n),
        "v": _rel_max(_soa(sim.buffer(A.NSF_BUF_UPREV)).reshape(3, N).T, v),
        "tau": _rel_max(_soa(sim.buffer(A.NSF_BUF_TAU)).reshape(6, N).T,
                        np.stack([tau[:, 0, 0], tau[:, 1, 1], tau[:, 2, 2], tau[:, 1, 2], tau[:, 0, 2],
                                  tau[:, 0, 1]], 1)),
        "C": _rel_max(_soa(sim.buffer(A.NSF_BUF_C)).reshape(9, N).T, C.reshape(N, 9)),
        "J": _rel_max(_soa(sim.buffer(A.NSF_BUF_JAC)).reshape(3, r, S).transpose(2, 0, 1),
                      o.jac(o.X[idx][:S], o.z)),
        "decode_u": _rel_max(_soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T - o.X, o.decode() - o.X),
    }
    print("errors:", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e < TOL_BF16, (k, e)
    # one step: positions against the oracle's, at the BF16 gate
    sim.step(1, stream=s)
    s.synchronize()
    o.step(1)
    xg = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
    xo = o.decode()
    dx = float(np.sqrt(((xg - xo) ** 2).sum() / (xo ** 2).sum()))
    print(f"delta_x after one step: {dx:.2e}", flush=True)
    assert dx <= 1e-4
    assert sim.flags(stream=s) == (0, 0)
    sim.close()


def test_empty_calls():
    """Zero steps and an empty decode are no-ops; an empty batch is rejected."""
    w = synth.small_cube(seed=1, r=3, width=64, n=64)
    s = torch.cuda.Stream()
    sim = Sim(w, stream=s)
    z0, _, st0 = sim.latent(stream=s)
    A.check(A.lib().nsf_step(sim.handle, 0, s.cuda_stream))
    out = torch.empty(3, dtype=torch.float32, device="cuda")
    A.check(A.lib().nsf_decode(sim.handle, out.data_ptr(), 0, out.data_ptr(), s.cuda_stream))
    z1, _, st1 = sim.latent(stream=s)
    assert st1 == st0 == 0
    np.testing.assert_array_equal(z0, z1)
    import ctypes as C
    arr = (C.c_void_p * 1)()
    assert A.lib().nsf_step_batch(arr, 0, 1, s.cuda_stream) == A.NSF_EINVAL
    sim.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_pipelined_decode_lags_one_step(precision):
    """decode_every_step = 2 decodes the latent each step starts from, concurrently with
    the step: the latent trajectory is bit for bit the synchronous one, and after k steps
    the decoded positions are the synchronous sim's after k - 1 steps; nsf_refresh brings
    them to the current latent."""
    w = synth.cake_slab(seed=2, r=6, width=128, n=20_000, n_integration=2048, steps=8, plan_steps=8)
    s = torch.cuda.Stream()
    ref = Sim(w, precision=precision, decode_every_step=1, stream=s)
    pip = Sim(w, precision=precision, decode_every_step=2, stream=s)
    ref.refresh(stream=s)
    pip.refresh(stream=s)
    s.synchronize()
    prev = _soa(ref.buffer(A.NSF_BUF_XDEC)).copy()
    np.testing.assert_array_equal(_soa(pip.buffer(A.NSF_BUF_XDEC)), prev)
    for k in range(1, 6):
        ref.step(1, stream=s)
        pip.step(1, stream=s)
        s.synchronize()
        zr, _, sr = ref.latent(stream=s)
        zp, _, sp = pip.latent(stream=s)
        assert sr == sp == k
        np.testing.assert_array_equal(zr, zp)
        np.testing.assert_array_equal(_soa(pip.buffer(A.NSF_BUF_XDEC)), prev)
        prev = _soa(ref.buffer(A.NSF_BUF_XDEC)).copy()
    pip.refresh(stream=s)
    s.synchronize()
    np.testing.assert_array_equal(_soa(pip.buffer(A.NSF_BUF_XDEC)), prev)
    assert ref.flags(stream=s) == (0, 0) and pip.flags(stream=s) == (0, 0)
    ref.close()
    pip.close()


def test_fp32_team_group_forms_agree():
    """The FP32 field passes of the cake-size sample set (8,192 samples: one pair of tiles
    per CU) run as team groups of two tiles that also evaluate h, l and the velocity; beside
    a pipelined decode the same passes run as one-tile team groups and separate primal
    groups. Both orders of work give the same bits: the latent trajectories agree exactly."""
    print("\n[case] FP32 team group forms agree", flush=True)
    w = synth.cake_slab(seed=4, r=6, width=128, n=40_000, n_integration=8192, steps=6, plan_steps=6)
    s = torch.cuda.Stream()
    ref = Sim(w, precision="fp32", decode_every_step=1, stream=s)
    pip = Sim(w, precision="fp32", decode_every_step=2, stream=s)
    for k in range(1, 5):
        ref.step(1, stream=s)
        pip.step(1, stream=s)
        s.synchronize()
        zr, zpr, sr = ref.latent(stream=s)
        zp, zpp, sp = pip.latent(stream=s)
        assert sr == sp == k
        np.testing.assert_array_equal(zr, zp)
        np.testing.assert_array_equal(zpr, zpp)
    for b in (A.NSF_BUF_U, A.NSF_BUF_UPREV, A.NSF_BUF_JAC, A.NSF_BUF_TAU, A.NSF_BUF_C):
        np.testing.assert_array_equal(_soa(ref.buffer(b)), _soa(pip.buffer(b)))
    assert ref.flags(stream=s) == (0, 0) and pip.flags(stream=s) == (0, 0)
    ref.close()
    pip.close()


@pytest.mark.parametrize("r", [3, 12])
def test_singular_normal_equations_flagged(r):
    """A latent coordinate the deformation field ignores (its layer-1 column zero) makes
    J^T J singular with an exactly zero pivot: both solve paths (one lane's registers up to
    six latents, the wave's column-parallel factorisation above) raise the SINGULAR flag
    and leave the latent where it was."""
    w = synth.small_cube(seed=2, r=r, width=64, n=512)
    W1, b1 = w.fields["g"][0]
    W1 = W1.copy()
    W1[:, 3 + 1] = 0.0
    w.fields["g"] = [(W1, b1)] + list(w.fields["g"][1:])
    s = torch.cuda.Stream()
    sim = Sim(w, stream=s)
    z0, _, _ = sim.latent(stream=s)
    sim.step(1, stream=s)
    s.synchronize()
    z1, _, st = sim.latent(stream=s)
    status, flags = sim.flags(stream=s)
    print(f"[case] r={r}: status {status}, flags {flags}", flush=True)
    assert flags & A.NSF_FLAG_SINGULAR
    np.testing.assert_array_equal(z1, z0)
    sim.close()
