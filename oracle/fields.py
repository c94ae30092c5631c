"""Neural fields g (deformation), h (Kirchhoff stress), l (affine momentum), FP64.

Paper: Sec. 4.2 (deformation field g(X, z) ~ phi(X, t)), Sec. 4.3 (stress field
h(X, z) ~ tau), Sec. 4.4 (affine field l(X, z) ~ C); supplementary "Network
architecture": inputs (3 + r), outputs 3 / 6 / 9, five hidden layers, ELU activations.

Readings (where the paper is silent):
  * "5 hidden layers" = 6 affine maps with ELU (alpha = 1) after the first five; the
    output map is linear.
  * Outputs are normalised (supplementary "Training Details": data normalised to mean
    0, variance 1); the physical value is scale * f + shift per channel.
  * g is a displacement field: x = X + u with u = s_g * f_g + c_g.
  * tau's six components are Voigt ordered (xx, yy, zz, yz, xz, xy).
  * C's nine components are row-major, C[a][b] = l[3a + b].
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

Layer = Tuple[np.ndarray, np.ndarray]


def elu(a: np.ndarray) -> np.ndarray:
    """ELU with alpha = 1 (Clevert et al.): a for a > 0, exp(a) - 1 otherwise."""
    return np.where(a > 0.0, a, np.expm1(np.minimum(a, 0.0)))


def elu_prime(a: np.ndarray) -> np.ndarray:
    """d ELU / da: 1 for a > 0, exp(a) otherwise (both sides equal 1 at a = 0)."""
    return np.where(a > 0.0, 1.0, np.exp(np.minimum(a, 0.0)))


def widen(layers: Sequence[Layer]) -> List[Tuple[np.ndarray, np.ndarray]]:
    return [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in layers]


def network_input(X: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Rows [X_p ; z] for each point. X is (n, 3), z is (r,)."""
    X = np.asarray(X, np.float64)
    z = np.asarray(z, np.float64)
    return np.concatenate([X, np.broadcast_to(z, (X.shape[0], z.shape[0]))], axis=1)


def mlp(layers: Sequence[Layer], inp: np.ndarray) -> np.ndarray:
    """f = W6 phi(W5 phi(... phi(W1 inp + b1) ...) + b5) + b6, rows are points."""
    L = widen(layers)
    h = np.asarray(inp, np.float64)
    for k, (W, b) in enumerate(L):
        a = h @ W.T + b
        h = elu(a) if k < len(L) - 1 else a
    return h


def field(layers: Sequence[Layer], X: np.ndarray, z: np.ndarray,
          scale: np.ndarray, shift: np.ndarray) -> np.ndarray:
    """De-normalised field value scale * f(X, z) + shift, shape (n, d)."""
    return np.asarray(scale, np.float64) * mlp(layers, network_input(X, z)) + np.asarray(shift, np.float64)


def voigt_to_matrix(t: np.ndarray) -> np.ndarray:
    """(n, 6) Voigt (xx, yy, zz, yz, xz, xy) -> (n, 3, 3) symmetric."""
    n = t.shape[0]
    M = np.empty((n, 3, 3))
    M[:, 0, 0], M[:, 1, 1], M[:, 2, 2] = t[:, 0], t[:, 1], t[:, 2]
    M[:, 1, 2] = M[:, 2, 1] = t[:, 3]
    M[:, 0, 2] = M[:, 2, 0] = t[:, 4]
    M[:, 0, 1] = M[:, 1, 0] = t[:, 5]
    return M


def eval_fields(fields: Dict[str, Sequence[Layer]], X: np.ndarray, z: np.ndarray,
                scale: Dict[str, np.ndarray], shift: Dict[str, np.ndarray], mu=None):
    """Network inference at one latent (Sec. 5.1): u (n,3), tau (n,3,3), C (n,3,3). With
    problem parameters mu the stress field is h(X, z, mu) (Sec. 4.3), input [X; z; mu]."""
    u = field(fields["g"], X, z, scale["g"], shift["g"])
    zh = z if mu is None or len(mu) == 0 else np.concatenate([np.asarray(z, np.float64), np.asarray(mu, np.float64)])
    tau = voigt_to_matrix(field(fields["h"], X, zh, scale["h"], shift["h"]))
    C = field(fields["l"], X, z, scale["l"], shift["l"]).reshape(-1, 3, 3)
    return u, tau, C


def jacobian_z(layers: Sequence[Layer], X: np.ndarray, z: np.ndarray,
               scale: np.ndarray) -> np.ndarray:
    """Forward-mode latent Jacobian d(scale * f)/dz at each point, shape (n, d, r).

    Tangents are pushed through the network alongside the primal: the first layer's
    tangent is diag(phi'(a1)) W1[:, 3:], each hidden layer maps T -> diag(phi'(a_k)) W_k T,
    and the output map gives W6 T5, scaled per channel. The Gauss-Newton inversion of
    Sec. 5.3 needs this matrix.
    """
    L = widen(layers)
    inp = network_input(X, z)
    n = inp.shape[0]
    r = np.asarray(z).shape[0]
    W1, b1 = L[0]
    a = inp @ W1.T + b1                              # (n, w)
    T = elu_prime(a)[:, :, None] * W1[None, :, 3:]  # (n, w, r)
    h = elu(a)
    for k in range(1, len(L)):
        W, b = L[k]
        a = h @ W.T + b
        # W applied to every tangent column of every point: one matmul over (w_in, n*r)
        WT = (W @ T.transpose(1, 0, 2).reshape(T.shape[1], n * r)).reshape(W.shape[0], n, r)
        WT = WT.transpose(1, 0, 2)
        if k < len(L) - 1:
            T = elu_prime(a)[:, :, None] * WT
            h = elu(a)
        else:
            T = WT
    return np.asarray(scale, np.float64)[None, :, None] * T


def jacobian_z_fd(layers: Sequence[Layer], X: np.ndarray, z: np.ndarray,
                  scale: np.ndarray, shift: np.ndarray, eps: float | None = None) -> np.ndarray:
    """Central finite differences of the field w.r.t. z (test helper)."""
    z = np.asarray(z, np.float64)
    if eps is None:
        eps = 1e-6 * (1.0 + np.linalg.norm(z))
    cols = []
    for j in range(z.shape[0]):
        e = np.zeros_like(z)
        e[j] = eps
        cols.append((field(layers, X, z + e, scale, shift) - field(layers, X, z - e, scale, shift)) / (2 * eps))
    return np.stack(cols, axis=2)
