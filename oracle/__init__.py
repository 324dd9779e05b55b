"""Double-precision CPU oracle for the differentiable ambiguity function.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2506_22935_amd``) never imports, links or runs anything in here, and
this package imports nothing from the product path.

Layout:
  af_direct.c  -- direct-sum chi and its adjoint (C, fp64, OpenMP), see its header
  reference.py -- energy, magnitude, masks, losses, upstream gradients,
                  gradient assembly, Adam and the MLP, all in float64 numpy
"""
from .reference import *  # noqa: F401,F403
