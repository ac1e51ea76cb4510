"""Reference implementation of PRGD tensor-train completion (test infrastructure).

This package is a plain, slow, float64 CPU implementation of preconditioned
Riemannian gradient descent for low-TT-rank tensor completion, written from
the paper (Bian, Cai, Zhang & Zhang, "Fast and Provable Tensor-Train Format
Tensor Completion via Preconditioned Riemannian Gradient Descent").  It exists
only to check the GPU library: it is imported by the tests, by the smoke
check and by the benchmark's CPU-baseline leg, and by nothing else.  It shares
no code with the GPU path and never loads the compiled library.

Modules
-------
``oracle.tt``    TT algebra of section 2: evaluation, dense form, left/right
                 parts, unfoldings, inner products, TT-SVD (Algorithm 1) and
                 its TT-format form.
``oracle.prgd``  Section 3: the data-driven metric, the preconditioned
                 tangent projection (Lemma 3), the step sizes, the update and
                 retraction of Algorithm 2, and the stopping rules of
                 section 5.

Parity status: every function is pinned by a test in ``tests/`` against
brute force, a closed form or a library routine (see each docstring).
"""

from . import tt, prgd  # noqa: F401
