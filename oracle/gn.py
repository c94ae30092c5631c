"""Gauss-Newton network inversion, FP64 (paper Sec. 5.3, the inversion equation).

z_{n+1} = argmin_z sum_{p in S} || g(X_p, z) - x_p^{n+1} ||^2, solved from z_n by
Gauss-Newton: at each iterate, with residual r (3|S| entries) and Jacobian J (3|S| x r),
solve (J^T J) delta = -J^T r by Cholesky and set z <- z + delta. The paper reports
convergence in 2-3 iterations and offers a first-order (linearised) projection as a
speed-up, which is one such solve with the Jacobian at z_n. The residual is unweighted;
K iterations are a parameter (2 by default). A non-positive pivot raises
SingularSystem.

Damping (a variant for ill-conditioned Jacobians, not in the paper): Levenberg-Marquardt
with Marquardt's diagonal scaling, (J^T J + lambda diag(J^T J)) delta = -J^T r. It is the
minimiser of |J delta + r|^2 + lambda |diag(J^T J)^(1/2) delta|^2.
"""
from __future__ import annotations

import numpy as np


class SingularSystem(ArithmeticError):
    pass


def cholesky_lower(H: np.ndarray) -> np.ndarray:
    """Plain Cholesky H = L L^T, raising on a non-positive pivot."""
    r = H.shape[0]
    L = np.zeros_like(H)
    for i in range(r):
        for j in range(i + 1):
            s = H[i, j] - L[i, :j] @ L[j, :j]
            if i == j:
                if not s > 0.0:
                    raise SingularSystem(f"pivot {i} = {s}")
                L[i, i] = np.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    return L


def normal_equations(J: np.ndarray, res: np.ndarray):
    """H = J^T J, b = J^T r for J (m, r) and r (m,)."""
    J = np.asarray(J, np.float64)
    res = np.asarray(res, np.float64)
    return J.T @ J, J.T @ res


def gn_delta(J: np.ndarray, res: np.ndarray, damping: float = 0.0) -> np.ndarray:
    """The Gauss-Newton step delta solving (J^T J) delta = -J^T r, or with damping
    lambda > 0 the Levenberg-Marquardt step (J^T J + lambda diag(J^T J)) delta = -J^T r."""
    H, b = normal_equations(J, res)
    if damping:
        H = H + damping * np.diag(np.diag(H))
    L = cholesky_lower(H)
    y = np.linalg.solve(L, -b)          # forward substitution
    return np.linalg.solve(L.T, y)      # back substitution
