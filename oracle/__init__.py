"""Plain FP64 CPU oracle for arXiv:1605.01799 (Darbon & Osher).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the product path never does.
It shares no code with the HIP library in ``paper_1605_01799_amd``.
"""
from .oracle import (  # noqa: F401
    build, available, oracle_eval, oracle_distance_newton, oracle_distance_secular,
    oracle_backward, oracle_control, oracle_max_over_hamiltonians, oracle_eval_linear_control,
    linear_control_weights, OH_WL1, OH_L2, OH_L2_WL1, OH_WL2,
    OH_AL2, OH_LINF,
)
