"""FP64 CPU oracle of the disc-galaxy likelihood (arXiv 2205.06819).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  It is a plain,
slow, direct transcription of the paper's model (Sec. 2.1-2.5, 3.1 and
Appendix A, Algorithm 1), written independently of the HIP implementation:
the two share no code, tables or constants generators.

Modules:

* ``special``: Hernquist X, g, h (with exact series where the closed forms
  cancel in FP64), the Freeman disc curve and the NFW mass shape.
* ``model``: frame, components, light-weighted observables, PSF stencil and
  the Gaussian log-likelihood; complex-step and central-difference gradients.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
(closed forms, brute-force quadrature, invariants, textbook values).
"""
from . import special, model  # noqa: F401
