"""MI355X-native latent-space time step of reduced-order MPM with neural stress fields.

The compute path is libnsf.so (hand-written HIP for gfx950, C ABI in include/nsf.h);
this package marshals arguments to it. Importing Sim loads the library and fails
loudly if it has not been built.
"""
from . import _abi  # noqa: F401

__all__ = ["Sim", "step_batch", "build"]


def __getattr__(name):
    if name in ("Sim", "step_batch"):
        from . import sim
        return getattr(sim, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
