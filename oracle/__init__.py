"""Test infrastructure: CPU oracle for the GLS sequence (see gls_oracle.py).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package; the product path never does.
"""
from .gls_oracle import (gls_sequence, cholesky_lower, whiten, fixed_blocks,  # noqa: F401
                         relative_error, normal_equation_residual)
