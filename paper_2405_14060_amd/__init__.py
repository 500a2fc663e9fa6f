"""Tensor-network exact inference on one MI355X (gfx950).

The compute path is libtn.so (hand-written HIP kernels behind a C ABI, see
include/tn.h); this package only marshals arguments into it.
"""
from ._capi import (EVIDENCE_INDICATOR, EVIDENCE_NONE, EVIDENCE_SLICED, MAX_PLUS,  # noqa: F401
                    PLANNER_BEST, PLANNER_GREEDY, PLANNER_MINDEG, PLANNER_MINFILL, PLANNER_NATURAL,
                    LAYOUT_AUTO, LAYOUT_INSTANCE_MAJOR, LAYOUT_INTERLEAVED, SUM_PRODUCT, TN_BF16, TN_F16, TN_F32,
                    Network, Plan, TNError, lib, plan_tree_host, tune_clear, tune_load, tune_save)

__all__ = ["Network", "Plan", "TNError", "lib", "plan_tree_host", "tune_clear", "tune_load", "tune_save"]
