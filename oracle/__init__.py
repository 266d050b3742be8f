"""Plain FP64 CPU oracle for the harmonic-balance (HB) GLS Navier-Stokes
residual, its Jacobian-vector products and the Newton-GMRES solve.

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library: it
is imported by the test-suite, by the smoke check and by the CPU-baseline
leg of the benchmark, and by nothing in the product path.  It shares no code
with the HIP library; both consume the same seeded inputs from ``hbinputs``.

The oracle works in the paper's time-sample form (Section 2.1, eq. NS-harm;
Section 2.3, eq. Rmc) with NumPy/SciPy in float64 (complex128 where a
complex-step derivative is taken).  Each module cites the passage it follows.

Parity status: every function is pinned by a test under ``tests/`` (closed
forms, identities, brute force); see ``tests/test_oracle_*.py``.
"""
from . import spectral, fem, residual, tangent, api, solve, march  # noqa: F401
