"""Python face of one reduced simulation (a thin owner around nsf_create_sim & co).

PyTorch provides the device memory (one uint8 arena tensor per sim) and the streams;
all computation happens in libnsf.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi as A

FIELD_OUT = (3, 6, 9)


def flatten_mlp(layers: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    """Concatenate (W row-major, b) for layers 1..6 into the ABI's weight layout."""
    parts = []
    for W, b in layers:
        parts.append(np.ascontiguousarray(W, np.float32).ravel())
        parts.append(np.ascontiguousarray(b, np.float32).ravel())
    return np.concatenate(parts)


def build_desc(w, precision: str, decode_every_step: bool):
    """nsf_sim_desc for a workload; returns (desc, host arrays the desc points into)."""
    keep = []

    def fptr(a):
        a = np.ascontiguousarray(a, np.float32)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def dptr(a):
        a = np.ascontiguousarray(a, np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    d = A.nsf_sim_desc()
    d.r, d.width, d.n_hidden = int(w.r), int(w.width), 5
    precisions = {"fp32": A.NSF_FP32, "bf16": A.NSF_BF16, "mixed": A.NSF_BF16_MIXED}
    if precision not in precisions:
        raise ValueError(f"precision {precision!r}: one of {sorted(precisions)}")
    d.precision = precisions[precision]
    for f, name in enumerate(("g", "h", "l")):
        d.weights[f] = fptr(flatten_mlp(w.fields[name]))
        for c in range(FIELD_OUT[f]):
            d.out_scale[f][c] = float(w.out_scale[name][c])
            d.out_shift[f][c] = float(w.out_shift[name][c])
    d.n_particles = int(w.X.shape[1])
    d.X = fptr(w.X)
    d.rho, d.body_volume = float(w.rho), float(w.body_volume)
    d.grid_n, d.dx, d.dt = int(w.grid_n), float(w.dx), float(w.dt)
    for c in range(3):
        d.gravity[c] = float(w.gravity[c])
    d.wall_nodes = int(w.wall_nodes)
    k = w.knife
    d.knife.enabled = 1 if k.enabled else 0
    for c in range(3):
        d.knife.normal[c] = float(k.normal[c])
        d.knife.velocity[c] = float(k.velocity[c])
    d.knife.offset, d.knife.half_thickness = float(k.offset), float(k.half_thickness)
    d.knife.edge_z0, d.knife.edge_speed = float(k.edge_z0), float(k.edge_speed)
    plan = np.ascontiguousarray(w.plan, np.int32)
    keep.append(plan)
    d.n_integration, d.n_sample = int(plan.shape[1]), int(w.n_sample)
    if getattr(w, "integration", "plan") == "closure":
        # one row of sample indices; n_integration is the capacity of the closure list
        d.integration = A.NSF_INTEGRATION_CLOSURE
        d.n_integration = int(w.closure_cap)
    d.plan_steps = int(plan.shape[0])
    d.sample_plan = plan.ctypes.data_as(C.POINTER(C.c_int32))
    d.gn_iters = int(w.gn_iters)
    d.gn_damping = float(getattr(w, "gn_damping", 0.0))
    mu = np.asarray(getattr(w, "mu", ()), np.float64).ravel()
    d.n_mu = int(mu.shape[0])
    for i, v in enumerate(mu[:4]):
        d.mu[i] = float(v)
    d.decode_every_step = int(decode_every_step)   # 0, 1 (True) or 2 (pipelined)
    d.z0 = dptr(w.z0)
    d.z_prev = dptr(w.z_prev) if w.z_prev is not None else None
    return d, keep


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Sim:
    """One reduced-order simulation resident on the current GPU.

    ``w`` is any object with the attributes of ``synth.Workload`` (fields, X, z0, plan,
    constants). ``precision`` is "fp32", "bf16" or "mixed" (BF16 stress and affine fields
    and decode, FP32 deformation field for the inversion).
    """

    def __init__(self, w, precision: str = "fp32", decode_every_step: bool = True,
                 stream: Optional[torch.cuda.Stream] = None, device: Optional[torch.device] = None):
        self.r = int(w.r)
        self.width = int(w.width)
        self.n_particles = int(w.X.shape[1])
        self.closure = getattr(w, "integration", "plan") == "closure"
        self.n_integration = int(w.closure_cap) if self.closure else int(w.plan.shape[1])
        self.n_sample = int(w.n_sample)
        self.grid_n = int(w.grid_n)
        self.precision = precision
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        d, keep = build_desc(w, precision, decode_every_step)
        nbytes = A.nsf_sim_bytes(d)
        if nbytes == 0:
            raise A.NsfError(A.NSF_EINVAL, A.nsf_last_error())
        self.arena_bytes = nbytes
        self._raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._raw.data_ptr()
        self._off = (-base) % 256
        self.arena = self._raw[self._off:self._off + nbytes]
        self.handle = A.nsf_create_sim(d, self.arena.data_ptr(), nbytes, _stream_handle(stream))
        del keep

    @staticmethod
    def bytes_for(w, precision: str = "fp32", decode_every_step: bool = True) -> int:
        """Device bytes a sim of this workload needs (nsf_sim_bytes), without creating it."""
        d, keep = build_desc(w, precision, decode_every_step)
        n = A.nsf_sim_bytes(d)
        del keep
        if n == 0:
            raise A.NsfError(A.NSF_EINVAL, A.nsf_last_error())
        return n + 256

    # ---- stepping ------------------------------------------------------------------
    def step(self, n: int = 1, stream: Optional[torch.cuda.Stream] = None) -> None:
        A.nsf_step(self.handle, n, _stream_handle(stream))

    def refresh(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        """Evaluate the fields at the current latent (decoded positions and the next step's
        field inference) in one launch."""
        A.nsf_refresh(self.handle, _stream_handle(stream))

    def decode(self, X: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """x = X + u(X, z_n) as a (3, n) float32 tensor; X is a (3, n) float32 device tensor."""
        if X is None:
            n = self.n_particles
            out = torch.empty((3, n), dtype=torch.float32, device=self.device)
            A.nsf_decode(self.handle, None, n, out.data_ptr(), _stream_handle(stream))
        else:
            X = X.contiguous()
            assert X.dtype == torch.float32 and X.dim() == 2 and X.shape[0] == 3
            n = int(X.shape[1])
            out = torch.empty((3, n), dtype=torch.float32, device=self.device)
            A.nsf_decode(self.handle, X.data_ptr(), n, out.data_ptr(), _stream_handle(stream))
        return out

    # ---- state ---------------------------------------------------------------------
    def latent(self, stream=None):
        z, zp, st = A.nsf_get_latent(self.handle, self.r, _stream_handle(stream))
        return np.array(z), np.array(zp), st

    def set_latent(self, z, z_prev=None, step: int = 0, stream=None) -> None:
        A.nsf_set_latent(self.handle, list(z), None if z_prev is None else list(z_prev), step,
                         _stream_handle(stream))

    def set_sample_count(self, n_sample: int, stream=None) -> None:
        """Closure integration: keep the first n_sample sample particles from the next step."""
        A.nsf_set_sample_count(self.handle, int(n_sample), _stream_handle(stream))
        self.n_sample = int(n_sample)

    def set_parameters(self, mu, stream=None) -> None:
        """New problem parameters mu of the stress field h(X, z, mu)."""
        A.nsf_set_parameters(self.handle, [float(v) for v in np.ravel(mu)], _stream_handle(stream))

    def integration_list(self, stream=None) -> np.ndarray:
        """The current integration list (closure: its live part; plan: all rows)."""
        lst = self.buffer(A.NSF_BUF_NLIST)
        if not self.closure:
            return lst.cpu().numpy()
        n = int(self.buffer(A.NSF_BUF_NLIVE).cpu().numpy()[0])
        return lst[:n].cpu().numpy()

    def flags(self, stream=None) -> Tuple[int, int]:
        """(status, flag bits) of the sticky device flags."""
        return A.nsf_status_flags(self.handle, _stream_handle(stream))

    def buffer(self, which: int) -> torch.Tensor:
        """A view of one of the sim's device buffers (see NSF_BUF_*)."""
        ptr, count = A.nsf_sim_buffer(self.handle, which)
        off = ptr - self.arena.data_ptr()
        esize = 8 if which == A.NSF_BUF_Z else 4
        dtype = (torch.float64 if which == A.NSF_BUF_Z else
                 torch.int32 if which in (A.NSF_BUF_NLIST, A.NSF_BUF_NLIVE) else torch.float32)
        return self.arena[off:off + count * esize].view(dtype)

    def close(self) -> None:
        if getattr(self, "handle", None):
            A.nsf_destroy_sim(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(sims: List[Sim], n: int = 1, stream=None) -> None:
    A.nsf_step_batch([s.handle for s in sims], n, _stream_handle(stream))


def mpm_stage(sims: List[Sim], stream=None) -> None:
    """The MPM stage of the current step alone (P2G, grid update, G2P at the samples), one
    launch per kernel over the sims' union; it advances nothing, so repeated calls
    recompute the same grid and velocities."""
    A.nsf_mpm_stage([s.handle for s in sims], _stream_handle(stream))
