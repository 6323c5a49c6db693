"""MI355X-native butterfly apply for oscillatory kernels K(x, y) = exp(i Phi(x, y)).

Implements the butterfly algorithm of Poulson, Demanet, Maxwell & Ying, "A
Parallel Butterfly Algorithm" (sequential form, Alg. "alg:serial", with the
analytic Chebyshev interpolation of Sec. 1.4) as HIP kernels for gfx950 behind
the C ABI of include/bfly.h.  This package is the Python binding
(``bfly.py``), the build script (``build.py``) and the seeded synthetic
workloads (``workloads.py``).
"""
from .bfly import (BFLY_FP32, BFLY_FP64, Batch, BatchItem, BflyError, Plan, apply_batched,  # noqa: F401
                   bfly_apply, bfly_apply_adjoint, bfly_apply_autograd, bfly_apply_batched,
                   bfly_apply_batched_autograd, bfly_batch_workspace_size, bfly_contraction_rate, bfly_last_error,
                   bfly_phase_rate, bfly_plan, bfly_plan_destroy, bfly_plan_info, bfly_status_string,
                   bfly_timing_enable, bfly_timing_launches, bfly_timing_read, bfly_tune, bfly_tune_reset,
                   bfly_workspace_size, lib)


def __getattr__(name):
    if name == "BflyApply":
        from . import bfly
        return bfly.BflyApply
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
