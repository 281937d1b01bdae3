"""MI355X-native safety filter (SF) of Flow-Opt: HIP kernels for gfx950 behind a
C ABI (include/sf.h), with a thin ctypes binding and a torch.autograd.Function."""
from .binding import (EXPORTED, LIB_PATH, SF_OBJECTIVE_ACCEL, SF_OBJECTIVE_PROJECTION, SFError,
                      SFPlan, SFProject, gather_blocks, load_library, rank_residual,
                      select_best, select_candidates, to_device)

__all__ = ["EXPORTED", "LIB_PATH", "SF_OBJECTIVE_ACCEL", "SF_OBJECTIVE_PROJECTION", "SFError", "SFPlan", "SFProject", "gather_blocks",
           "load_library", "rank_residual", "select_best", "select_candidates", "to_device"]
