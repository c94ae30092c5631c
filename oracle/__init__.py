"""FP64 CPU oracle for the reduced-order MPM latent step (Neural Stress Fields).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the HIP path is checked against. Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never does, and
this package imports nothing from the product package.

Everything is NumPy float64. Inputs given in float32 (weights, reference positions)
are widened exactly. The steps follow the paper's order and notation:

  fields.py  neural deformation / stress / affine fields (Sec. 4.2-4.4, supplementary
             "Network architecture"), their de-normalisation, and the forward-mode
             latent Jacobian of the deformation field used by the inversion (Sec. 5.3).
  mpm.py     quadratic B-spline weights, P2G with APIC and the MLS stress term,
             grid update with boundary conditions, G2P (Sec. 3.2 node force balance,
             Sec. 3.3 MPM algorithm).
  gn.py      Gauss-Newton network inversion with r x r normal equations (Sec. 5.3, the
             inversion equation).
  step.py    the three-stage latent step: inference, MPM step, inversion (Sec. 5.1-5.3),
             and decode (Sec. 5.1, resolution boost in Sec. 6).
  fullorder.py  full-order explicit MLS-MPM with fixed-corotated elasticity and von
             Mises plasticity (Sec. 3.3; supplementary "Elasticity and plasticity
             details"), used only to make training snapshots for field fitting.

Pins (tests marked "not gpu") check each piece against closed forms, invariants,
brute force and independent library routines; see tests/test_oracle_*.py.
"""
from . import fields, mpm, gn, step  # noqa: F401
