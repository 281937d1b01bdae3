"""FP64 CPU oracle of the Flow-Opt safety filter.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with
the HIP implementation.
"""
from .sf import SFOracle, SFResult, bernstein_W, build_operators, solve_problem
from .adjoint import SFAdjoint, SFGrad, loss_value

__all__ = ["SFOracle", "SFResult", "bernstein_W", "build_operators", "solve_problem",
           "SFAdjoint", "SFGrad", "loss_value"]
