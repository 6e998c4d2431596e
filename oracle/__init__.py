"""FP64 CPU oracle of the IGA-ADS-CRVPINN coupled time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that tests, the round-trip smoke check and
the CPU baseline of the benchmark can compare the HIP path against a plain,
slow and obviously correct implementation written from the paper.  It shares
no code, tables or constants with the HIP library; only the seeded input
arrays (drawn by ``paper_2604_20731_amd.inputs``, which holds no solver
arithmetic) are common, and they are passed in as arguments.

Everything is numpy/scipy in float64.  Each function cites the passage of the
paper (arXiv 2604.20731) it follows; where the paper is silent or ambiguous the
reading taken is stated in the docstring.

Modules
  bspline   open uniform B-spline space, Gauss rules, 1D mass matrices
  pressure  collocation operator, Gram matrix and its inverse, robust loss and
            its gradients, direct solve of the discrete pressure system
  mlp       tanh multilayer perceptron forward/backward and Adam
  ads       L2 projection, Kronecker mass solve, explicit saturation substep
  galerkin  IGA Galerkin pressure system and its sparse direct solve (the
            paper's direct-solver path)
  wells     well discs -> nodal source arrays
  coupled   the IGA-ADS-CRVPINN algorithm (init, pretrain, step, fields)

Parity status: every function is pinned by a test in tests/test_oracle_*.py
except the end-to-end coupled trajectory, which has no worked example in the
paper ("parity unpinned" beyond its components).
"""
from .coupled import Oracle, cfl_dt  # noqa: F401
