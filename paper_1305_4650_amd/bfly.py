"""Python binding of libbfly (include/bfly.h): argument marshalling only.

Every step of the butterfly apply runs in the HIP kernels of libbfly.so;
PyTorch supplies device memory and the stream.  There is no CPU fallback:
importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BFLY_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("BFLY_LIBRARY") or os.path.join(HERE, "libbfly.so")

BFLY_OK, BFLY_EINVAL, BFLY_EUNSUPPORTED, BFLY_ENOMEM, BFLY_EDEVICE, BFLY_EWORKSPACE = range(6)
BFLY_PHASE_FOURIER, BFLY_PHASE_HYPRADON2, BFLY_PHASE_GENRADON3, BFLY_PHASE_SEPARABLE_TEST = range(4)
BFLY_FP64, BFLY_FP32, BFLY_SPLIT32 = 0, 1, 2
BFLY_NOALLOC_MAX_BYTES = 64 << 20  # workspace held by the library for bfly_apply_noalloc

PHASES = {"fourier": 0, "hypradon2": 1, "genradon3": 2, "separable": 3, "genradon3pi": 4}
# "split32" is a valid mode that the library does not build (BFLY_EUNSUPPORTED)
PRECISIONS = {"fp64": BFLY_FP64, "fp32": BFLY_FP32, "split32": BFLY_SPLIT32}

EXPORTS = ("bfly_plan", "bfly_plan_destroy", "bfly_plan_info", "bfly_workspace_size", "bfly_apply",
           "bfly_apply_noalloc", "bfly_apply_adjoint", "bfly_batch_workspace_size", "bfly_apply_batched",
           "bfly_tune", "bfly_tune_reset", "bfly_timing_enable", "bfly_timing_read", "bfly_timing_launches",
           "bfly_phase_rate", "bfly_contraction_rate",
           "bfly_status_string", "bfly_last_error")
STEP_NAMES = ("binning", "first", "second", "final")


class BflyError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {code})")
        self.code = code


_lib = None


class BatchItem(ctypes.Structure):
    """bfly_batch_item of include/bfly.h."""
    _fields_ = [("plan", ctypes.c_void_p), ("adjoint", ctypes.c_int), ("nrhs", ctypes.c_int),
                ("n_in", ctypes.c_int64), ("pts_in", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("ld_in", ctypes.c_int64), ("n_out", ctypes.c_int64), ("pts_out", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("ld_out", ctypes.c_int64)]


def lib() -> ctypes.CDLL:
    """Load libbfly.so (built by ``python -m paper_1305_4650_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1305_4650_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    L.bfly_plan.restype = ctypes.c_int
    L.bfly_plan.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(vp)]
    L.bfly_plan_destroy.restype = ctypes.c_int
    L.bfly_plan_destroy.argtypes = [vp]
    L.bfly_plan_info.restype = ctypes.c_int
    L.bfly_plan_info.argtypes = [vp, ctypes.POINTER(i64)]
    L.bfly_workspace_size.restype = ctypes.c_int
    L.bfly_workspace_size.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.bfly_apply.restype = ctypes.c_int
    L.bfly_apply.argtypes = [vp, i64, vp, vp, i64, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                             ctypes.c_size_t, vp]
    L.bfly_apply_adjoint.restype = ctypes.c_int
    L.bfly_apply_adjoint.argtypes = L.bfly_apply.argtypes
    L.bfly_apply_noalloc.restype = ctypes.c_int
    L.bfly_apply_noalloc.argtypes = [vp, i64, vp, vp, i64, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp]
    L.bfly_batch_workspace_size.restype = ctypes.c_int
    L.bfly_batch_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(BatchItem), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_size_t)]
    L.bfly_apply_batched.restype = ctypes.c_int
    L.bfly_apply_batched.argtypes = [ctypes.c_int, ctypes.POINTER(BatchItem), ctypes.c_int, vp, ctypes.c_size_t,
                                     vp]
    L.bfly_timing_enable.restype = ctypes.c_int
    L.bfly_timing_enable.argtypes = [ctypes.c_int]
    L.bfly_timing_read.restype = ctypes.c_int
    L.bfly_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double)] + [ctypes.POINTER(i64)] * 4
    L.bfly_tune.restype = ctypes.c_int
    L.bfly_tune.argtypes = [vp, ctypes.c_int, i64, vp, vp, i64, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                            ctypes.c_size_t, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
    L.bfly_tune_reset.restype = ctypes.c_int
    L.bfly_tune_reset.argtypes = []
    L.bfly_timing_launches.restype = ctypes.c_int
    ip = ctypes.POINTER(ctypes.c_int)
    L.bfly_timing_launches.argtypes = [ctypes.c_int, ip, ip, ip, ip, ip, ctypes.POINTER(ctypes.c_double)]
    L.bfly_phase_rate.restype = ctypes.c_int
    L.bfly_phase_rate.argtypes = [ctypes.c_int, i64, i64, ctypes.c_double, vp, vp]
    L.bfly_contraction_rate.restype = ctypes.c_int
    L.bfly_contraction_rate.argtypes = [ctypes.c_int, i64, i64, vp, vp]
    L.bfly_status_string.restype = ctypes.c_char_p
    L.bfly_status_string.argtypes = [ctypes.c_int]
    L.bfly_last_error.restype = ctypes.c_char_p
    L.bfly_last_error.argtypes = []
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != BFLY_OK:
        raise BflyError(rc, where, lib().bfly_last_error().decode() or bfly_status_string(rc))


def _darr(v, d):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(d))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------
# the C ABI, one Python function per entry point
# ----------------------------------------------------------------------------

def bfly_plan(d: int, N: int, src_lo, src_hi, tgt_lo, tgt_hi, phase_id: int, q: int) -> int:
    bufs = [_darr(v, d) for v in (src_lo, src_hi, tgt_lo, tgt_hi)]
    out = ctypes.c_void_p()
    _check(lib().bfly_plan(d, N, *[b[1] for b in bufs], phase_id, q, ctypes.byref(out)), "bfly_plan")
    return out.value


def bfly_plan_destroy(plan: int) -> None:
    _check(lib().bfly_plan_destroy(plan), "bfly_plan_destroy")


def bfly_plan_info(plan: int) -> dict:
    out = (ctypes.c_int64 * 5)()
    _check(lib().bfly_plan_info(plan, out), "bfly_plan_info")
    return dict(zip(("d", "N", "q", "r", "switch_level"), list(out)))


def bfly_workspace_size(plan: int, n_in: int, nrhs: int, prec: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().bfly_workspace_size(plan, n_in, nrhs, prec, ctypes.byref(out)), "bfly_workspace_size")
    return out.value


def bfly_apply(plan, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, ws, ws_bytes, stream) -> None:
    _check(lib().bfly_apply(plan, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, ws, ws_bytes, stream),
           "bfly_apply")


def bfly_apply_noalloc(plan, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, stream) -> None:
    _check(lib().bfly_apply_noalloc(plan, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, stream),
           "bfly_apply_noalloc")


def bfly_apply_adjoint(plan, n_tgt, x, f_in, ldf, n_src, y, g_out, ldg, nrhs, prec, ws, ws_bytes,
                       stream) -> None:
    _check(lib().bfly_apply_adjoint(plan, n_tgt, x, f_in, ldf, n_src, y, g_out, ldg, nrhs, prec, ws,
                                    ws_bytes, stream), "bfly_apply_adjoint")


def bfly_batch_workspace_size(items, prec: int) -> int:
    """items: a ctypes array of BatchItem."""
    out = ctypes.c_size_t()
    _check(lib().bfly_batch_workspace_size(len(items), items, prec, ctypes.byref(out)), "bfly_batch_workspace_size")
    return out.value


def bfly_apply_batched(items, prec: int, ws, ws_bytes, stream) -> None:
    _check(lib().bfly_apply_batched(len(items), items, prec, ws, ws_bytes, stream), "bfly_apply_batched")


def bfly_tune(plan, adjoint, n_in, pts_in, vin, ld_in, n_out, pts_out, vout, ld_out, nrhs, prec, ws, ws_bytes,
              max_ms, stream) -> float:
    """Autotune one apply's launch shapes; returns the chosen shapes' ms per apply."""
    best = ctypes.c_double()
    _check(lib().bfly_tune(plan, int(adjoint), n_in, pts_in, vin, ld_in, n_out, pts_out, vout, ld_out, nrhs, prec,
                           ws, ws_bytes, max_ms, ctypes.byref(best), stream), "bfly_tune")
    return best.value


def bfly_tune_reset() -> None:
    _check(lib().bfly_tune_reset(), "bfly_tune_reset")


def bfly_timing_enable(on: bool) -> None:
    _check(lib().bfly_timing_enable(int(bool(on))), "bfly_timing_enable")


def bfly_timing_read() -> dict:
    """{launch kind: {"ms", "launches", "stages", "inits", "switches"}} since the last read."""
    ms = (ctypes.c_double * len(STEP_NAMES))()
    cnt = [(ctypes.c_int64 * len(STEP_NAMES))() for _ in range(4)]
    _check(lib().bfly_timing_read(ms, *cnt), "bfly_timing_read")
    return {k: {"ms": ms[i], "launches": cnt[0][i], "stages": cnt[1][i], "inits": cnt[2][i],
                "switches": cnt[3][i]} for i, k in enumerate(STEP_NAMES)}


def bfly_timing_launches(cap: int = 4096) -> list:
    """[{"kind", "stages", "inits", "switches", "ms"}] of the launches the last
    bfly_timing_read collected, in launch order."""
    cnt = ctypes.c_int()
    arr = [(ctypes.c_int * cap)() for _ in range(4)]
    ms = (ctypes.c_double * cap)()
    _check(lib().bfly_timing_launches(cap, ctypes.byref(cnt), *arr, ms), "bfly_timing_launches")
    return [{"kind": STEP_NAMES[arr[0][i]], "stages": arr[1][i], "inits": arr[2][i], "switches": arr[3][i],
             "ms": ms[i]} for i in range(min(cnt.value, cap))]


def bfly_phase_rate(prec: int, n_threads: int, iters: int, span: float, out, stream) -> None:
    _check(lib().bfly_phase_rate(prec, n_threads, iters, span, out, stream), "bfly_phase_rate")


def bfly_contraction_rate(unit: int, n_threads: int, iters: int, out, stream) -> None:
    _check(lib().bfly_contraction_rate(unit, n_threads, iters, out, stream), "bfly_contraction_rate")


def bfly_status_string(status: int) -> str:
    return lib().bfly_status_string(status).decode()


def bfly_last_error() -> str:
    return lib().bfly_last_error().decode()


# ----------------------------------------------------------------------------
# torch-facing convenience (device buffers and streams from PyTorch)
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _prec_id(prec) -> int:
    return PRECISIONS[prec] if isinstance(prec, str) else int(prec)


def _points(t, d, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or t.shape[1] != d or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({'n'}, {d}) tensor")
    return t


def _values(t, n, name):
    """(nrhs, n) complex128 with unit stride along points -> (tensor, leading dimension)."""
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128):
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2 or t.shape[1] != n or (n > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be (nrhs, {n}) with unit stride along points")
    ld = t.stride(0) if t.shape[0] > 1 else max(n, 1)
    if ld < n:
        raise ValueError(f"{name}: rows overlap")
    return t, max(ld, 1)


class Plan:
    """A butterfly plan: d, N, source box, target box, phase, q."""

    def __init__(self, d: int, N: int, src_box, tgt_box, phase, q: int):
        self.d, self.N, self.q = int(d), int(N), int(q)
        self.phase_id = PHASES[phase] if isinstance(phase, str) else int(phase)
        self.src_box = (np.asarray(src_box[0], float), np.asarray(src_box[1], float))
        self.tgt_box = (np.asarray(tgt_box[0], float), np.asarray(tgt_box[1], float))
        self.handle = bfly_plan(self.d, self.N, self.src_box[0], self.src_box[1], self.tgt_box[0],
                                self.tgt_box[1], self.phase_id, self.q)
        self.info = bfly_plan_info(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.bfly_plan_destroy(h)
            self.handle = None

    def workspace_size(self, n_in: int, nrhs: int, prec="fp64") -> int:
        return bfly_workspace_size(self.handle, n_in, nrhs, _prec_id(prec))

    def workspace(self, n_in: int, nrhs: int, prec="fp64", device=None):
        torch = _torch()
        nbytes = self.workspace_size(n_in, nrhs, prec)
        return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or "cuda")

    def _run(self, adjoint, pin, vin, pout, prec, out, workspace, stream):
        torch = _torch()
        d = self.d
        pin = _points(pin, d, "input points")
        pout = _points(pout, d, "output points")
        n_in, n_out = pin.shape[0], pout.shape[0]
        vin, ldin = _values(vin, n_in, "input values")
        nrhs = vin.shape[0]
        p = _prec_id(prec)
        if out is None:
            out = torch.empty((nrhs, n_out), dtype=torch.complex128, device=pin.device)
        out2, ldout = _values(out, n_out, "output values")
        if out2.shape[0] != nrhs:
            raise ValueError("output has the wrong number of right-hand sides")
        nbytes = self.workspace_size(n_in, nrhs, p)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=pin.device)
        if stream is None:
            stream = torch.cuda.current_stream(pin.device).cuda_stream
        fn = bfly_apply_adjoint if adjoint else bfly_apply
        fn(self.handle, n_in, pin.data_ptr(), vin.data_ptr(), ldin, n_out, pout.data_ptr(),
           out2.data_ptr(), ldout, nrhs, p, workspace.data_ptr(), workspace.numel(), stream)
        return out

    def tune(self, pin, vin, pout, prec="fp64", adjoint=False, max_ms=0.0, out=None, workspace=None, stream=None):
        """Autotune the launch shapes of apply (adjoint=False: pin = sources,
        vin = g, pout = targets) or apply_adjoint (pin = targets) on these
        buffers (bfly_tune); later applies with the same key use the result.
        Returns (outputs of the apply with the chosen shapes, ms per apply)."""
        torch = _torch()
        pin = _points(pin, self.d, "input points")
        pout = _points(pout, self.d, "output points")
        vin, ldin = _values(vin, pin.shape[0], "input values")
        nrhs = vin.shape[0]
        p = _prec_id(prec)
        if out is None:
            out = torch.empty((nrhs, pout.shape[0]), dtype=torch.complex128, device=pin.device)
        out2, ldout = _values(out, pout.shape[0], "output values")
        if workspace is None:
            workspace = torch.empty(max(self.workspace_size(pin.shape[0], nrhs, p), 1), dtype=torch.uint8,
                                    device=pin.device)
        if stream is None:
            stream = torch.cuda.current_stream(pin.device).cuda_stream
        ms = bfly_tune(self.handle, adjoint, pin.shape[0], pin.data_ptr(), vin.data_ptr(), ldin, pout.shape[0],
                       pout.data_ptr(), out2.data_ptr(), ldout, nrhs, p, workspace.data_ptr(), workspace.numel(),
                       float(max_ms), stream)
        return out, ms

    def apply(self, y, g, x, prec="fp64", out=None, workspace=None, stream=None):
        """f = B g: sources y (n_src, d), g (nrhs, n_src) -> f (nrhs, n_tgt) at targets x."""
        return self._run(False, y, g, x, prec, out, workspace, stream)

    def apply_noalloc(self, y, g, x, prec="fp64", out=None, stream=None):
        """f = B g like apply(), with the workspace the library holds on the
        device (bfly_apply_noalloc): nothing is allocated when `out` is given."""
        torch = _torch()
        y = _points(y, self.d, "input points")
        x = _points(x, self.d, "output points")
        g, ldg = _values(g, y.shape[0], "input values")
        nrhs = g.shape[0]
        if out is None:
            out = torch.empty((nrhs, x.shape[0]), dtype=torch.complex128, device=y.device)
        out2, ldf = _values(out, x.shape[0], "output values")
        if out2.shape[0] != nrhs:
            raise ValueError("output has the wrong number of right-hand sides")
        if stream is None:
            stream = torch.cuda.current_stream(y.device).cuda_stream
        bfly_apply_noalloc(self.handle, y.shape[0], y.data_ptr(), g.data_ptr(), ldg, x.shape[0], x.data_ptr(),
                           out2.data_ptr(), ldf, nrhs, _prec_id(prec), stream)
        return out

    def apply_adjoint(self, x, f, y, prec="fp64", out=None, workspace=None, stream=None):
        """g = B' f with B' the butterfly of K^H (roles swapped, phase -Phi)."""
        return self._run(True, x, f, y, prec, out, workspace, stream)


class Batch:
    """Several applies run together by bfly_apply_batched.

    items: sequence of (plan, adjoint, pts_in, vals_in, pts_out), with vals_in
    (nrhs, n_in) complex128 and points as for Plan.apply / apply_adjoint.  The
    outputs (nrhs, n_out) and the workspace are allocated here; run() writes
    the outputs.  Pointers and sizes are fixed at construction, so a run() can
    be captured in a HIP graph and replayed after the inputs are refilled."""

    def __init__(self, items, prec="fp64", device=None):
        torch = _torch()
        self.prec = _prec_id(prec)
        self.items = []
        self.outs = []
        arr = (BatchItem * len(items))()
        for k, (plan, adjoint, pin, vin, pout) in enumerate(items):
            pin = _points(pin, plan.d, f"item {k} input points")
            pout = _points(pout, plan.d, f"item {k} output points")
            vin, ldin = _values(vin, pin.shape[0], f"item {k} input values")
            out = torch.empty((vin.shape[0], pout.shape[0]), dtype=torch.complex128, device=pin.device)
            _, ldout = _values(out, pout.shape[0], f"item {k} output values")
            arr[k] = BatchItem(plan.handle, int(bool(adjoint)), vin.shape[0], pin.shape[0], pin.data_ptr(),
                               vin.data_ptr(), ldin, pout.shape[0], pout.data_ptr(), out.data_ptr(), ldout)
            self.items.append((plan, pin, vin, pout))  # keep every buffer alive
            self.outs.append(out)
        self._arr = arr
        nbytes = bfly_batch_workspace_size(arr, self.prec)
        dev = device or (self.items[0][1].device if self.items else "cuda")
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(self.workspace.device).cuda_stream
        bfly_apply_batched(self._arr, self.prec, self.workspace.data_ptr(), self.workspace.numel(), stream)
        return self.outs


def apply_batched(items, prec="fp64"):
    """Outputs of Batch(items, prec).run() (one call, fresh buffers)."""
    return Batch(items, prec).run()


def _make_autograd():
    torch = _torch()

    class BflyApply(torch.autograd.Function):
        """f = B g with backward grad_g = B' grad_f (the adjoint butterfly).

        The map is linear, so nothing per level is saved; the vector-Jacobian
        product of f = K g for complex g is K^H grad_f, which the adjoint
        butterfly approximates to the same accuracy as B approximates K."""

        @staticmethod
        def forward(ctx, g, plan, y, x, prec="fp64"):
            ctx.plan, ctx.prec = plan, prec
            ctx.save_for_backward(y, x)
            return plan.apply(y, g.contiguous(), x, prec)

        @staticmethod
        def backward(ctx, grad_f):
            y, x = ctx.saved_tensors
            g = ctx.plan.apply_adjoint(x, grad_f.contiguous(), y, ctx.prec)
            return g, None, None, None, None

    return BflyApply


_BflyApply = None
_BflyBatchApply = None


def _make_batch_autograd():
    torch = _torch()

    class BflyBatchApply(torch.autograd.Function):
        """f_k = B_k g_k for every instance k in one batched apply; the
        backward is one batched adjoint apply, grad_g_k = B'_k grad_f_k."""

        @staticmethod
        def forward(ctx, spec, prec, *gs):
            ctx.spec, ctx.prec = spec, prec
            items = [(plan, False, y, g.contiguous(), x) for (plan, y, x), g in zip(spec, gs)]
            return tuple(Batch(items, prec).run())

        @staticmethod
        def backward(ctx, *grads):
            items = [(plan, True, x, gf.contiguous(), y) for (plan, y, x), gf in zip(ctx.spec, grads)]
            return (None, None, *Batch(items, ctx.prec).run())

    return BflyBatchApply


def __getattr__(name):
    """BflyApply: the torch.autograd.Function of a forward apply (backward:
    the adjoint apply), built on first access so that importing this module
    does not import torch."""
    if name == "BflyApply":
        global _BflyApply
        if _BflyApply is None:
            _BflyApply = _make_autograd()
        return _BflyApply
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")


def bfly_apply_autograd(g, plan: Plan, y, x, prec="fp64"):
    """Differentiable forward apply (see BflyApply)."""
    global _BflyApply
    if _BflyApply is None:
        _BflyApply = _make_autograd()
    return _BflyApply.apply(g, plan, y, x, prec)


def bfly_apply_batched_autograd(gs, spec, prec="fp64"):
    """Differentiable batched forward apply: spec = [(plan, y, x), ...], one g per
    instance; returns the tuple of outputs (see BflyBatchApply)."""
    global _BflyBatchApply
    if _BflyBatchApply is None:
        _BflyBatchApply = _make_batch_autograd()
    return _BflyBatchApply.apply(spec, prec, *gs)
