"""Plain FP64 CPU oracle for LRR / DFC-LRR (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
from .lrr import (ALMOptions, DFCResult, LRRResult, column_projection, dfc_lrr, dfc_lrr_local, dual_gap,
                  l21_shrink, lrr_alm, objective, svt, trivial_lambda)
from .segment import segment, segmentation_accuracy, oracle_constraints, outlier_flags
from . import adjoint
from . import slr

__all__ = [
    "ALMOptions", "DFCResult", "LRRResult", "column_projection", "dfc_lrr", "dfc_lrr_local", "dual_gap",
    "l21_shrink", "lrr_alm", "objective", "svt", "trivial_lambda", "segment",
    "segmentation_accuracy", "oracle_constraints", "outlier_flags", "adjoint", "slr",
]
