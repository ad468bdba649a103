"""MI355X (gfx950) implementation of the XM hot path of "Building Rome with
Convex Optimization" (Han & Yang, arXiv 2502.04640).

The compute lives in the HIP library ``libxm.so`` (C ABI in include/xm.h); this
package only marshals torch device tensors and the current HIP stream into it.
Importing the package does not touch the GPU; the first call that needs the
library loads it and raises if it is missing (there is no CPU fallback).
"""
from .api import (XMError, NotTightError, Problem, SolveOptions, XMSolve, align_similarity, build_Q,  # noqa: F401
                  drop_largest, guard_frames, library_path, load_library, memory_info, memory_trim, xm2)

__all__ = ["XMError", "NotTightError", "Problem", "SolveOptions", "XMSolve", "align_similarity", "build_Q",
           "drop_largest", "guard_frames", "library_path", "load_library", "memory_info", "memory_trim", "xm2"]
