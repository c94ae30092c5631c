"""Fitting the deformation, stress and affine fields to full-order snapshots.

Training follows the paper's Sec. 4.5 and the supplementary "Training Details": g is fitted
to the snapshot positions first, together with one learnable latent per snapshot (an
auto-decoder in place of the convolutional encoder: the latent table is the encoder's
output for the training snapshots); h and l are then fitted to the snapshot stresses and
affine matrices with those latents frozen. Targets are normalised per channel to mean 0,
variance 1, and the normalisation is returned as the fields' out_scale / out_shift.
Adam updates FP32 master weights; every forward and backward runs in the library's
kernels through FieldFn (BF16 hidden layers with FP32 accumulation, or FP32).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _abi as A
from .fullorder import FullOrderSim
from .train import Adam, FieldFn, PairSquaredError, RowsExpand

OUT_DIM = {"g": 3, "h": 6, "l": 9}
# learning rates of the supplementary "Training Details", one per equal share of the run
LR_STAGES = (1e-3, 5e-4, 2e-4, 1e-4, 5e-5)

# The falling cube whose full-order run is the fitting data: density, body volume (a cube
# of side 0.2), fixed corotated elasticity with von Mises plasticity, initial velocity
# -2 m/s onto the ground, 64^3 grid, dt = 1e-4 (5,000 steps cover the fall, the impact and
# the flow that follows).
FALLING_CUBE = dict(v0=(0.0, 0.0, -2.0), rho=1000.0, body_volume=0.2 ** 3, youngs=5e4, poisson=0.3,
                    yield_stress=2e3, grid_n=64, dt=1e-4)


@dataclasses.dataclass
class Snapshots:
    """Full-order training data: reference positions and T snapshots of positions,
    Kirchhoff stress (Voigt xx yy zz yz xz xy) and affine matrix (row-major)."""
    X: np.ndarray      # (P, 3)
    x: np.ndarray      # (T, P, 3)
    tau: np.ndarray    # (T, P, 6)
    C: np.ndarray      # (T, P, 9)


def falling_cube_sim(X: np.ndarray, stream=None, **overrides) -> FullOrderSim:
    """The GPU full-order sim of the falling cube from reference positions X (n, 3)."""
    kw = dict(FALLING_CUBE)
    kw.update(overrides)
    return FullOrderSim(np.ascontiguousarray(np.asarray(X, np.float32).T), stream=stream, **kw)


def full_order_snapshots(sim: FullOrderSim, n_snapshots: int = 200, every: int = 25,
                         stream=None) -> Snapshots:
    """Step the full-order sim and keep a snapshot (positions, Voigt stress, affine C) after
    every `every` steps; the snapshots stay on the device until the run ends."""
    P = sim.n_particles
    dev = sim.device
    xs = torch.empty(n_snapshots, 3, P, device=dev)
    taus = torch.empty(n_snapshots, 6, P, device=dev)
    Cs = torch.empty(n_snapshots, 9, P, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.stream(s):
        for t in range(n_snapshots):
            sim.step(every, stream=s)
            xs[t].copy_(sim.positions())
            taus[t].copy_(sim.buffer(A.NSF_FO_TAU).view(6, P))
            Cs[t].copy_(sim.buffer(A.NSF_FO_C).view(9, P))
    s.synchronize()
    return Snapshots(X=sim.X.T.double().cpu().numpy(), x=xs.transpose(1, 2).cpu().numpy(),
                     tau=taus.transpose(1, 2).cpu().numpy(), C=Cs.transpose(1, 2).cpu().numpy())


def xavier_flat(r: int, width: int, d: int, gen: torch.Generator) -> torch.Tensor:
    """Xavier-uniform weights (gain 1) and zero biases in the ABI's flat layout."""
    dims = [3 + r, width, width, width, width, width, d]
    parts = []
    for k in range(6):
        fan_in, fan_out = dims[k], dims[k + 1]
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append((torch.rand(fan_out * fan_in, generator=gen, dtype=torch.float64) * 2 - 1) * a)
        parts.append(torch.zeros(fan_out, dtype=torch.float64))
    return torch.cat(parts).float()


class Fitter:
    def __init__(self, data: Snapshots, r: int = 12, width: int = 128, precision: str = "bf16",
                 batch: int = 1 << 18, seed: int = 0, device: Optional[torch.device] = None):
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.dev, self.r, self.width, self.precision, self.batch = dev, r, width, precision, batch
        self.T, self.P = data.x.shape[0], data.x.shape[1]
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        cpu_gen = torch.Generator().manual_seed(seed)
        self.X = torch.as_tensor(np.asarray(data.X, np.float32), device=dev)
        self.XT = self.X.t().contiguous()   # (3, P): a minibatch's positions in one gather
        X64 = np.asarray(data.X, np.float64)
        targets = {"g": np.asarray(data.x, np.float64) - X64[None], "h": np.asarray(data.tau, np.float64),
                   "l": np.asarray(data.C, np.float64)}
        self.scale: Dict[str, np.ndarray] = {}
        self.shift: Dict[str, np.ndarray] = {}
        self.Y: Dict[str, torch.Tensor] = {}
        for f, y in targets.items():
            mu = y.reshape(-1, y.shape[-1]).mean(0)
            sd = y.reshape(-1, y.shape[-1]).std(0)
            sd = np.where(sd > 0, sd, 1.0)
            self.shift[f], self.scale[f] = mu, sd
            # structure of arrays (d, T P), pair (t, p) at column t P + p: a minibatch's targets
            # are one gather along the columns, in the [d][n] order the kernels write
            yn = ((y - mu) / sd).astype(np.float32).reshape(-1, y.shape[-1])
            self.Y[f] = torch.as_tensor(np.ascontiguousarray(yn.T), device=dev)
        self.w = {f: xavier_flat(r, width, OUT_DIM[f], cpu_gen).to(dev).requires_grad_(True)
                  for f in OUT_DIM}
        self.z = torch.zeros(self.T, r, device=dev, requires_grad=True)
        self.history: Dict[str, List[float]] = {f: [] for f in OUT_DIM}
        # A minibatch is stratified over the snapshots: snapshot t holds counts[t] of its
        # pairs (batch / T, the remainder spread over the first snapshots), each with a
        # particle drawn uniformly. Every pair is uniform over (snapshot, particle) up to
        # that remainder, and the pairs come grouped by snapshot, so a snapshot's latent is
        # expanded to its rows and its gradient summed over them without atomics.
        counts = np.full(self.T, batch // self.T, np.int64)
        counts[:batch % self.T] += 1
        self.offsets = torch.as_tensor(np.concatenate([[0], np.cumsum(counts)]), device=dev)
        self.t_rows = torch.repeat_interleave(torch.arange(self.T, device=dev),
                                              torch.as_tensor(counts, device=dev))

    def _batch(self):
        p = torch.randint(0, self.P, (self.batch,), device=self.dev, generator=self.gen)
        return self.t_rows, p

    def loss(self, f: str, t: torch.Tensor, p: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
        """Mean squared error of field f on the normalised targets at pairs (t, p), the
        pairs grouped by snapshot as self.offsets says."""
        zr = RowsExpand.apply(z, self.offsets, self.batch)
        Xp = torch.index_select(self.XT, 1, p).t()   # (n, 3) view of the SoA rows FieldFn takes
        out = FieldFn.apply(Xp, zr, self.w[f], self.width, OUT_DIM[f], self.precision)
        # targets at columns t P + p of the structure-of-arrays table, gathered in the loss
        return PairSquaredError.apply(out, self.Y[f], t, p, self.P)

    def fit(self, f: str, iters: int) -> List[float]:
        """Adam over `iters` minibatches with the staged learning rates. g also trains the
        latent table; h and l see it frozen."""
        params = [self.w[f]] + ([self.z] if f == "g" else [])
        # the library's Adam kernel updates each parameter tensor in one launch; the losses
        # stay on the device until the end, so the host queues iterations ahead of the device
        opt = Adam(params, lr=LR_STAGES[0], betas=(0.9, 0.999), eps=1e-8)
        losses = torch.empty(iters, device=self.dev)
        for it in range(iters):
            opt.lr = LR_STAGES[min(len(LR_STAGES) - 1, it * len(LR_STAGES) // max(iters, 1))]
            t, p = self._batch()
            z = self.z if f == "g" else self.z.detach()
            opt.zero_grad()
            L = self.loss(f, t, p, z)
            L.backward()
            opt.step()
            losses[it] = L.detach()
        out = [float(v) for v in losses.cpu().numpy()]
        self.history[f] += out
        return out

    @torch.no_grad()
    def relative_error(self, f: str, snapshot: int) -> float:
        """sqrt(sum |y - y*|^2 / sum |y*|^2) of the de-normalised field over all particles
        of one snapshot (the paper's relative error, Sec. 6), positions for g."""
        T = torch.full((self.P,), snapshot, device=self.dev, dtype=torch.long)
        out = FieldFn.apply(self.X, self.z[T], self.w[f], self.width, OUT_DIM[f], self.precision)
        sc = torch.as_tensor(self.scale[f], device=self.dev, dtype=torch.float64)
        sh = torch.as_tensor(self.shift[f], device=self.dev, dtype=torch.float64)
        y = out.double() * sc + sh
        ref = self.Y[f][:, snapshot * self.P:(snapshot + 1) * self.P].t().double() * sc + sh
        if f == "g":
            y, ref = y + self.X.double(), ref + self.X.double()
        return float(torch.sqrt(((y - ref) ** 2).sum() / (ref ** 2).sum()))

    def export(self) -> dict:
        """Fitted weights (flat FP32, per field), de-normalisation and the latent table."""
        return dict(weights={f: self.w[f].detach().cpu().numpy() for f in OUT_DIM},
                    out_scale=dict(self.scale), out_shift=dict(self.shift),
                    z=self.z.detach().cpu().numpy().astype(np.float64))
