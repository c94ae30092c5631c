"""Full-order MLS-MPM on the GPU through the C ABI (nsf_fo_*): every particle integrated
with the same P2G kernels as the reduced step, then G2P with the C and F updates and one
of three return maps with its elasticity: von Mises with fixed corotated stress,
Drucker-Prager with the StVK stress in log strain, Herschel-Bulkley with its own stress
(Sec. 3.3 and the supplementary "Elasticity and plasticity details"). It is the model the
reduced step is measured against.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi as A


MODELS = {"von_mises": A.NSF_FO_VON_MISES, "drucker_prager": A.NSF_FO_DRUCKER_PRAGER,
          "herschel_bulkley": A.NSF_FO_HERSCHEL_BULKLEY}


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class FullOrderSim:
    """X: (3, P) float32 initial positions; material and grid constants as in nsf_fo_desc."""

    def __init__(self, X: np.ndarray, v0: Sequence[float], rho: float, body_volume: float,
                 youngs: float, poisson: float, yield_stress: float, grid_n: int, dt: float,
                 gravity: Sequence[float] = (0.0, 0.0, -9.8), wall_nodes: int = 3,
                 stream: Optional[torch.cuda.Stream] = None, device: Optional[torch.device] = None,
                 model: str = "von_mises", friction_angle: float = 30.0, viscosity: float = 0.0):
        X = np.ascontiguousarray(X, np.float32)
        assert X.ndim == 2 and X.shape[0] == 3
        self.n_particles = int(X.shape[1])
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        d = A.nsf_fo_desc()
        d.n_particles = self.n_particles
        d.X = X.ctypes.data_as(C.POINTER(C.c_float))
        for c in range(3):
            d.v0[c] = float(v0[c])
            d.gravity[c] = float(gravity[c])
        d.rho, d.body_volume = float(rho), float(body_volume)
        d.youngs, d.poisson, d.yield_stress = float(youngs), float(poisson), float(yield_stress)
        d.grid_n, d.dt, d.wall_nodes = int(grid_n), float(dt), int(wall_nodes)
        d.plasticity = MODELS[model]
        d.friction_angle, d.viscosity = float(friction_angle), float(viscosity)
        nbytes = A.lib().nsf_fo_bytes(C.byref(d))
        if nbytes == 0:
            raise A.NsfError(A.NSF_EINVAL, A.nsf_last_error())
        self._raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._raw.data_ptr()) % 256
        self.arena = self._raw[off:off + nbytes]
        h = C.c_void_p()
        A.check(A.lib().nsf_fo_create(C.byref(d), self.arena.data_ptr(), nbytes, _stream_handle(stream),
                                      C.byref(h)))
        self.handle = h.value
        self.X = torch.from_numpy(X).to(self.device)

    def step(self, n: int = 1, stream=None) -> None:
        A.check(A.lib().nsf_fo_step(self.handle, int(n), _stream_handle(stream)))

    def buffer(self, which: int) -> torch.Tensor:
        """View of a state buffer (NSF_FO_*): float32, except F^E in float64."""
        p = C.c_void_p()
        n = C.c_int64()
        A.check(A.lib().nsf_fo_buffer(self.handle, which, C.byref(p), C.byref(n)))
        off = p.value - self.arena.data_ptr()
        esize, dtype = (8, torch.float64) if which == A.NSF_FO_F else (4, torch.float32)
        return self.arena[off:off + int(n.value) * esize].view(dtype)

    def positions(self) -> torch.Tensor:
        """x = X + u, (3, P) float32."""
        return self.X + self.buffer(A.NSF_FO_U).view(3, -1)

    def flags(self, stream=None):
        f = C.c_uint32()
        st = A.lib().nsf_fo_flags(self.handle, C.byref(f), _stream_handle(stream))
        return st, int(f.value)

    def close(self) -> None:
        if getattr(self, "handle", None):
            A.lib().nsf_fo_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
