"""Seeded synthetic inputs for sequences of sparse systems A(t_i) x(t_i) = b(t_i).

This package builds the finite-difference operators and right-hand sides that stand
in for the paper's workloads (Section 1, eq. (seq): a stream of n x n sparse systems
sampled from smooth time-dependent coefficients, cf. Assumption 1 of Section 3).
It holds none of the method's arithmetic: no sketch, basis, projection or Krylov
step lives here.  Both the CPU oracle and the HIP path take their inputs from it.
"""

from .problems import (  # noqa: F401
    CSR,
    SeqProblem,
    config,
    make_problem,
    batch_problems,
)
