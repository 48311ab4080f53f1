"""Plain, slow, FP64 CPU oracle for IRCUR (Iterated Robust CUR).

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product path (the HIP
library and its Python binding) never imports, calls or links anything here, and
nothing here imports the product path.

Contents
--------
sampler   SplitMix64 + Floyd's sampling of distinct indices (the uniform index
          draw of Algorithm 1 and its optional resampling, section 3.4).
ircur     Algorithm 1 step by step in FP64 NumPy with LAPACK SVD: hard
          thresholding (eq. (4)), the sampled low-rank estimate (eq. (5)), the CUR
          update (eq. (2), (3)), the stopping criterion (eq. (6)); plus a literal
          dense form for tiny inputs and Algorithm 2 (CUR to SVD).
unrolled  The unrolled K-step IRCUR with a gated threshold and its hand-derived
          reverse-mode adjoint.  The paper does not define this variant; its
          readings are stated in the module.
"""
from . import sampler, ircur, unrolled  # noqa: F401
