"""Workload builders shared by the tests (inputs only; no method arithmetic)."""
import copy

import numpy as np

import synth


def affine_manifold(w: "synth.Workload", bias1: float = 5.0) -> "synth.Workload":
    """Make g exactly affine in (X, z) and tau = C = 0.

    Layer 1 keeps its random weights but gets a large positive bias so every hidden
    pre-activation stays positive in the unit box; ELU is the identity there. Hidden
    layers 2..5 are the identity. h and l get a zero output layer.
    """
    w = copy.deepcopy(w)
    g = list(w.fields["g"])
    W1, b1 = g[0]
    g[0] = (W1, np.full_like(b1, bias1))
    width = W1.shape[0]
    for k in range(1, 5):
        g[k] = (np.eye(width, dtype=np.float32), np.zeros(width, np.float32))
    w.fields["g"] = g
    for name in ("h", "l"):
        lay = list(w.fields[name])
        W6, b6 = lay[-1]
        lay[-1] = (np.zeros_like(W6), np.zeros_like(b6))
        w.fields[name] = lay
    return w
