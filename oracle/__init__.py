"""CPU oracle for BM-Global nuclear-norm matrix completion (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code with the GPU library
(``paper_2204_14067_amd``) and never calls it; the two meet only in the seeded
inputs from ``synth``.

* ``oracle.c``   plain C loops over Omega (sampled residual, sparse products).
* ``core``       the method itself in the paper's order: BM phase, inexact
                 proximal-gradient step (subspace iteration with Rayleigh-Ritz,
                 exact SVD of the projected matrix, singular-value
                 soft-thresholding), warm start and rank safeguard,
                 HMT + Nystrom initialisation, objective and residual.
* ``dense``      small dense references used to pin ``core`` (full-SVD prox,
                 dense proximal gradient, duality gap).
* ``rng``        the counter-based normal generator the method draws from.

Every public function names the passage of the paper it follows.  Parity
status of each function is listed in ``core``'s module docstring.
"""
from . import core, dense, rng  # noqa: F401
