"""Plain CPU FP64 oracle for the macro-element HDG hot path (arXiv 2402.11361).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with
the HIP library: it computes everything the slow, obvious way (dense NumPy
matrices, complex-step Jacobians, SciPy sparse direct solves) so that a reader
can check it against the paper's equations by eye.

Functions whose result is not fixed by the paper or by mathematics are marked
"parity unpinned" in their docstrings.
"""
