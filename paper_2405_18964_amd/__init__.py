"""pintoc: parallel-in-time all-at-once solver for unsteady Stokes/Oseen
distributed optimal control on MI355X (gfx950).

Thin Python binding over the C ABI in ``include/pintoc.h``: argument
marshalling only.  Every step of the computation runs in the HIP library
``libpintoc.so`` built in-tree by ``paper_2405_18964_amd.build``.  Importing
works without a GPU; creating a :class:`Problem` requires the built library
and raises if it is missing (there is no fallback path).

PyTorch supplies device memory (``torch.empty``) and the stream
(``torch.cuda.current_stream()``).
"""
from ._lib import (INNER_GMRES, INNER_LINEAR, INNER_MINRES, OSEEN, OUTER_FGMRES, OUTER_FGMRES_FREQ, OUTER_MINRES, PREC_FP32_INNER, PREC_FP64,
                   SMOOTHER_GLOBAL, SMOOTHER_TILED, STOKES, LibraryMissing, PHASES,
                   Group, Problem, SolveStats, group_bytes, library, library_path, solve_batch)

__all__ = ["Problem", "SolveStats", "library", "library_path", "LibraryMissing", "STOKES", "OSEEN",
           "INNER_LINEAR", "INNER_GMRES", "PREC_FP64", "PREC_FP32_INNER", "OUTER_FGMRES", "OUTER_MINRES", "OUTER_FGMRES_FREQ",
           "SMOOTHER_TILED", "SMOOTHER_GLOBAL", "PHASES",
           "solve_batch", "Group", "group_bytes"]
