"""Sensitivity of the cake-scale trajectory to its initial latent, in the FP64 oracle.

Runs the oracle twice from z0 and from z0 + 1e-10 (each component) and writes, for the
steps 10, 50, 75 and 100, the relative position error delta between the two runs over
2,048 fixed particles. A run whose own FP64 trajectory moves by more than the precision
gate under a 1e-10 change of z0 cannot be compared at that gate under any arithmetic.

Usage: python tests/golden/sensitivity.py r   (writes sensitivity_r{r}.txt beside it)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.step import OracleSim  # noqa: E402

r = int(sys.argv[1])
w = synth.cake_slab(seed=0, r=r, width=128, n=200_000, n_integration=8192, steps=100)
idx = np.random.default_rng(123).choice(200_000, 2048, replace=False)
a, b = OracleSim(w), OracleSim(w)
b.z = b.z + 1e-10
b.z_prev = b.z_prev + 1e-10
lines = [f"# r = {r}: delta_x between FP64 oracle runs from z0 and z0 + 1e-10 (2,048 particles)",
         "# step delta_x |z_a - z_b|_max"]
for n in range(1, 101):
    a.step(1)
    b.step(1)
    if n in (10, 50, 75, 100):
        xa, xb = a.decode(a.X[idx]), b.decode(b.X[idx])
        d = float(np.sqrt(((xa - xb) ** 2).sum() / (xa ** 2).sum()))
        lines.append(f"{n} {d:.3e} {np.abs(a.z - b.z).max():.3e}")
        print(lines[-1], flush=True)
open(os.path.join(HERE, f"sensitivity_r{r}.txt"), "w").write("\n".join(lines) + "\n")
