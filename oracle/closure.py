"""The integration particles N as the closure of the sample particles' stencils, FP64
(paper Sec. 5.4, the construction of sample and integration particles).

Test infrastructure only: the GPU path never imports this module.

Given the positions x_p = g(X_p, z_n) of every particle at step n and the sample set S:
  a. I = the grid nodes i with N_i(x_p) != 0 for some p in S;
  b. N = the particles p whose own stencil meets I.
Then every grid node that G2P reads for a sample particle receives its mass and momentum
from exactly the particles it would receive them from in a full-order step, so x^{n+1} on
S is that of a full-order MPM step (the paper's "no approximation" remark of Sec. 5.2).

Reading: "N_i(x) != 0" is taken as "i is one of the 3 x 3 x 3 stencil nodes base + {0,1,2}^3,
base = floor(x / dx - 0.5)". The quadratic B-spline weight of a stencil node is zero only
on the measure-zero set where the fractional offset is exactly 0.5 or 1.5, and a particle
there contributes nothing to that node either way. A particle whose stencil leaves the
grid is not marked and not a member, except that S is always part of N (the MPM step then
raises DOMAIN for it). The list order is S first, in the given order, then the other
members by ascending particle index.

`stencil_base_f32` is the same decision taken on float32 positions in float32 arithmetic
(x * inv_dx rounded to float32, then minus 0.5 rounded to float32, then floor): it is what
the GPU kernels compute, so a list built from the GPU's own decoded positions can be
compared index for index.
"""
from __future__ import annotations

import numpy as np


def stencil_base(x: np.ndarray, dx: float) -> np.ndarray:
    """base (n, 3) int64 of positions x (n, 3) in FP64."""
    return np.floor(np.asarray(x, np.float64) / dx - 0.5).astype(np.int64)


def stencil_base_f32(x32: np.ndarray, inv_dx32: np.float32) -> np.ndarray:
    """base (n, 3) int64 from float32 positions, each operation rounded to float32."""
    x32 = np.asarray(x32, np.float32)
    xs = (x32 * np.float32(inv_dx32)).astype(np.float32)
    return np.floor((xs - np.float32(0.5)).astype(np.float32)).astype(np.int64)


def _in_grid(base: np.ndarray, n: int) -> np.ndarray:
    return np.all((base >= 0) & (base + 2 <= n - 1), axis=1)


def _node_ids(base: np.ndarray, n: int) -> np.ndarray:
    """The 27 node ids (i n + j) n + k of each stencil, (m, 27)."""
    off = np.array([(a, b, c) for a in range(3) for b in range(3) for c in range(3)], np.int64)
    nodes = base[:, None, :] + off[None, :, :]
    return (nodes[..., 0] * n + nodes[..., 1]) * n + nodes[..., 2]


def integration_set_from_bases(base: np.ndarray, S: np.ndarray, grid_n: int) -> np.ndarray:
    """Sec. 5.4 steps a and b from the stencil bases of all particles (P, 3)."""
    S = np.asarray(S, np.int64)
    ok = _in_grid(base, grid_n)
    marked = np.zeros(grid_n ** 3, bool)
    s_ok = S[ok[S]]
    marked[_node_ids(base[s_ok], grid_n).ravel()] = True                   # step a: I
    member = np.zeros(base.shape[0], bool)
    idx_ok = np.nonzero(ok)[0]
    member[idx_ok] = marked[_node_ids(base[idx_ok], grid_n)].any(axis=1)   # step b: N
    is_s = np.zeros(base.shape[0], bool)
    is_s[S] = True
    rest = np.nonzero(member & ~is_s)[0]
    return np.concatenate([S, rest]).astype(np.int64)


def integration_set(x: np.ndarray, S: np.ndarray, grid_n: int, dx: float) -> np.ndarray:
    """N for FP64 positions x (P, 3): S first, then the other members ascending."""
    return integration_set_from_bases(stencil_base(x, dx), S, grid_n)


def integration_set_f32(x32: np.ndarray, S: np.ndarray, grid_n: int, inv_dx32) -> np.ndarray:
    """N for float32 positions with the float32 stencil decision (see module docstring)."""
    return integration_set_from_bases(stencil_base_f32(x32, inv_dx32), S, grid_n)
