"""Write the stored oracle trajectories the GPU tests compare against.

Calls only the FP64 oracle and the seeded input generators. For the cake-scale workload
(200,000 particles in the slab, 8,192 integration = sample particles resampled per step,
width-128 fields from seed 0, 128^3 grid, dt = 5e-5, knife, 2 Gauss-Newton iterations)
at r = 6 and r = 24 it stores the latent after every step, and the decoded positions and
the Kirchhoff stress (Voigt) of 2,048 fixed particles after steps 10, 50, 75 and 100.

Usage: python tests/golden/make_golden.py [r ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import fields as F  # noqa: E402
from oracle.step import OracleSim  # noqa: E402

STEPS = 100
SAMPLE_SEED, N_SAMPLED = 123, 2048
CHECKPOINTS = (10, 50, 75, 100)


def golden_path(r: int) -> str:
    return os.path.join(HERE, f"cake200k_r{r}_oracle.npz")


def workload(r: int):
    return synth.cake_slab(seed=0, r=r, width=128, n=200_000, n_integration=8192, steps=STEPS)


def sampled_particles():
    return np.random.default_rng(SAMPLE_SEED).choice(200_000, N_SAMPLED, replace=False)


def make(r: int) -> None:
    w = workload(r)
    o = OracleSim(w)
    idx = sampled_particles()
    zs = [o.z.copy()]
    xs, taus = {}, {}
    t0 = time.time()
    for n in range(1, STEPS + 1):
        o.step(1)
        zs.append(o.z.copy())
        if n in CHECKPOINTS:
            xs[n] = o.decode(o.X[idx])
            taus[n] = F.field(w.fields["h"], o.X[idx], o.z, w.out_scale["h"], w.out_shift["h"])
        if n % 10 == 0:
            print(f"r={r} step {n} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(golden_path(r), z=np.array(zs), idx=idx.astype(np.int64),
                        steps=np.array(CHECKPOINTS),
                        x=np.stack([xs[c] for c in CHECKPOINTS]),
                        tau=np.stack([taus[c] for c in CHECKPOINTS]), flags=np.array(o.flags))


if __name__ == "__main__":
    for r in [int(a) for a in sys.argv[1:]] or [6, 24]:
        make(r)
