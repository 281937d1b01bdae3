"""Seeded synthetic inputs of the SF projection problem (no method arithmetic)."""
from .gen import (WORKLOADS, N_DIM, PackedBatch, Problem, SFConfig, make_batch,
                  make_problem, pack, scaled, straight_coefficients, unpack_coefs)

__all__ = ["WORKLOADS", "N_DIM", "PackedBatch", "Problem", "SFConfig", "make_batch",
           "make_problem", "pack", "scaled", "straight_coefficients", "unpack_coefs"]
