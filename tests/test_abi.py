"""The C ABI without a GPU: the library loads, exports every entry point that
include/bfly.h declares, and rejects invalid arguments on the host before
any HIP call (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1305_4650_amd as P
from paper_1305_4650_amd import bfly as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "bfly.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(bfly_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    syms = header_symbols()
    assert len(syms) >= 8, syms
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in include/bfly.h but not exported"
    assert sorted(B.EXPORTS) == syms


def test_status_strings():
    assert P.bfly_status_string(B.BFLY_OK) == "success"
    assert P.bfly_status_string(B.BFLY_EWORKSPACE) == "workspace too small"
    assert P.bfly_status_string(99) == "unknown status"


BOX2 = (np.array([1.0, 0.0]), np.array([2.0, 1.0]))
TBOX2 = (np.zeros(2), np.ones(2))


def plan_rc(d, N, sbox, tbox, phase, q):
    out = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (*sbox, *tbox)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
    rc = B.lib().bfly_plan(d, N, *ptrs, phase, q, ctypes.byref(out))
    if rc == 0:
        B.lib().bfly_plan_destroy(out)
    return rc


@pytest.mark.parametrize("args,code", [
    ((2, 1024, BOX2, TBOX2, 1, 5), B.BFLY_OK),
    ((4, 8, BOX2, TBOX2, 0, 5), B.BFLY_EINVAL),                       # d
    ((2, 6, BOX2, TBOX2, 1, 5), B.BFLY_EINVAL),                       # N not a power of 2
    ((2, 0, BOX2, TBOX2, 1, 5), B.BFLY_EINVAL),                       # N = 0
    ((2, 1 << 16, BOX2, TBOX2, 1, 5), B.BFLY_EINVAL),                 # N^d >= 2^31
    ((2, 64, BOX2, TBOX2, 1, 1), B.BFLY_EINVAL),                      # q too small
    ((2, 64, BOX2, TBOX2, 1, 17), B.BFLY_EINVAL),                     # q too large
    ((3, 8, (np.zeros(3), np.ones(3)), (np.zeros(3), np.ones(3)), 2, 7), B.BFLY_EINVAL),
    ((2, 64, (np.array([1.0, 0.0]), np.array([1.0, 1.0])), TBOX2, 1, 5), B.BFLY_EINVAL),  # empty box
    ((2, 64, (np.array([np.nan, 0.0]), np.array([2.0, 1.0])), TBOX2, 1, 5), B.BFLY_EINVAL),
    ((2, 64, BOX2, (np.zeros(2), np.array([np.inf, 1.0])), 1, 5), B.BFLY_EINVAL),
    ((2, 64, BOX2, TBOX2, 7, 5), B.BFLY_EINVAL),                      # unknown phase
    ((3, 8, (np.zeros(3), np.ones(3)), (np.zeros(3), np.ones(3)), 1, 4), B.BFLY_EUNSUPPORTED),
    ((2, 8, BOX2, TBOX2, 2, 4), B.BFLY_EUNSUPPORTED),
    ((2, 8, BOX2, TBOX2, 4, 4), B.BFLY_EUNSUPPORTED),                 # GENRADON3_PI needs d = 3
    ((2, 64, BOX2, TBOX2, 5, 5), B.BFLY_EINVAL),                      # unknown phase
    ((3, 8, (np.full(3, -4.0), np.full(3, 4.0)), (np.zeros(3), np.ones(3)), 4, 5), B.BFLY_OK),
    ((1, 1, (np.zeros(1), np.ones(1)), (np.zeros(1), np.ones(1)), 0, 16), B.BFLY_OK),
])
def test_plan_validation(args, code):
    assert plan_rc(*args) == code


def test_plan_info():
    p = P.Plan(3, 64, (np.zeros(3), np.ones(3)), (np.zeros(3), np.ones(3)), "genradon3", 4)
    assert p.info == {"d": 3, "N": 64, "q": 4, "r": 64, "switch_level": 3}
    p = P.Plan(2, 2048, (np.zeros(2), np.ones(2)), (np.zeros(2), np.full(2, 2048.0)), "fourier", 6)
    assert p.info["switch_level"] == 5 and p.info["r"] == 36


def test_apply_rejects_invalid_arguments_on_host():
    """Every argument error is caught before the library touches the device;
    the pointers below are never dereferenced."""
    p = P.Plan(2, 16, BOX2, TBOX2, "hypradon2", 4)
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    base = dict(n_src=256, y=fake, g=fake, ldg=256, n_tgt=256, x=fake, f=fake, ldf=256, nrhs=1, prec=0,
                ws=fake, ws_bytes=1 << 30, stream=None)

    def call(**kw):
        a = dict(base, **kw)
        return L.bfly_apply(p.handle, a["n_src"], a["y"], a["g"], a["ldg"], a["n_tgt"], a["x"], a["f"],
                            a["ldf"], a["nrhs"], a["prec"], a["ws"], a["ws_bytes"], a["stream"])

    assert call(nrhs=0) == B.BFLY_EINVAL
    assert call(nrhs=5000) == B.BFLY_EINVAL
    assert call(prec=9) == B.BFLY_EINVAL
    assert call(ldg=100) == B.BFLY_EINVAL
    assert call(ldf=10) == B.BFLY_EINVAL
    assert call(n_src=-1) == B.BFLY_EINVAL
    assert call(n_tgt=1 << 31) == B.BFLY_EINVAL
    assert call(y=None) == B.BFLY_EINVAL
    assert call(f=None) == B.BFLY_EINVAL
    assert "NULL" in P.bfly_last_error()
    assert L.bfly_apply(None, 1, fake, fake, 1, 1, fake, fake, 1, 1, 0, fake, 1, None) == B.BFLY_EINVAL
    assert L.bfly_apply_adjoint(p.handle, 256, fake, fake, 256, 256, fake, fake, 256, 0, 0, fake, 1,
                                None) == B.BFLY_EINVAL
    out = ctypes.c_size_t()
    assert L.bfly_workspace_size(p.handle, 10, 0, 0, ctypes.byref(out)) == B.BFLY_EINVAL
    assert L.bfly_workspace_size(p.handle, -3, 1, 0, ctypes.byref(out)) == B.BFLY_EINVAL


def test_split32_is_rejected_as_unsupported():
    """The hi/lo split-FP32 mode is a declared precision that the library does
    not build: every entry point taking a precision returns
    BFLY_EUNSUPPORTED for it, on the host, before any HIP call."""
    p = P.Plan(2, 16, BOX2, TBOX2, "hypradon2", 4)
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.bfly_apply(p.handle, 256, fake, fake, 256, 256, fake, fake, 256, 1, B.BFLY_SPLIT32, fake, 1 << 30,
                        None) == B.BFLY_EUNSUPPORTED
    assert "SPLIT32" in P.bfly_last_error()
    assert L.bfly_apply_adjoint(p.handle, 256, fake, fake, 256, 256, fake, fake, 256, 1, B.BFLY_SPLIT32, fake,
                                1 << 30, None) == B.BFLY_EUNSUPPORTED
    out = ctypes.c_size_t()
    assert L.bfly_workspace_size(p.handle, 256, 1, B.BFLY_SPLIT32, ctypes.byref(out)) == B.BFLY_EUNSUPPORTED
    it = B.BatchItem(p.handle, 0, 1, 256, 0x1000, 0x1000, 256, 256, 0x1000, 0x1000, 256)
    arr = (B.BatchItem * 1)(it)
    assert L.bfly_batch_workspace_size(1, arr, B.BFLY_SPLIT32, ctypes.byref(out)) == B.BFLY_EUNSUPPORTED
    assert L.bfly_apply_batched(1, arr, B.BFLY_SPLIT32, fake, 1 << 40, None) == B.BFLY_EUNSUPPORTED
    with pytest.raises(P.BflyError) as ei:
        p.workspace_size(256, 1, "split32")
    assert ei.value.code == B.BFLY_EUNSUPPORTED


def test_batch_workspace_covers_mixed_batches():
    """A batch of small instances (sorted together) and one large instance
    (run as a single apply inside the call): the workspace covers both uses
    of the shared buffers, also where the batched point count sits at the
    sort's tile-size switches (2^14 and 2^18 keys), whose scratch is not
    monotone in the number of keys."""
    small = P.Plan(2, 64, BOX2, TBOX2, "hypradon2", 5)
    big = P.Plan(2, 128, BOX2, TBOX2, "hypradon2", 5)
    fake = 0x1000

    def item(plan, n):
        return B.BatchItem(plan.handle, 0, 1, n, fake, fake, n, n, fake, fake, n)

    def size(items):
        arr = (B.BatchItem * len(items))(*items)
        return B.bfly_batch_workspace_size(arr, B.BFLY_FP64)

    for n_small_each, count, n_big in ((4096, 64, 20000), (5461, 3, 30000), (4096, 4, 16383)):
        only_small = size([item(small, n_small_each)] * count)
        only_big = size([item(big, n_big)])
        mixed = size([item(small, n_small_each)] * count + [item(big, n_big)])
        # the mixed workspace holds both instance sets' weights and the larger
        # of their point, leaf and sort buffers
        weights_big = 128 * 128 * 25 * 16
        assert mixed >= only_small + weights_big, (n_small_each, count, n_big)
        assert mixed >= only_big, (n_small_each, count, n_big)


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        P.Plan(2, 16, BOX2, TBOX2, "hypradon2", 4)


def test_batched_rejects_invalid_arguments_on_host():
    """bfly_apply_batched / bfly_batch_workspace_size validate every item on
    the host before any HIP call; the pointers are never dereferenced."""
    p = P.Plan(2, 16, BOX2, TBOX2, "hypradon2", 4)
    L = B.lib()
    fake = 0x1000

    def item(**kw):
        a = dict(plan=p.handle, adjoint=0, nrhs=1, n_in=256, pts_in=fake, in_=fake, ld_in=256, n_out=256,
                 pts_out=fake, out=fake, ld_out=256)
        a.update(kw)
        return B.BatchItem(**a)

    def call(*its, prec=0, n=None):
        arr = (B.BatchItem * len(its))(*its)
        return L.bfly_apply_batched(len(its) if n is None else n, arr, prec, ctypes.c_void_p(fake), 1 << 40, None)

    assert call(item(nrhs=0)) == B.BFLY_EINVAL
    assert call(item(nrhs=5000)) == B.BFLY_EINVAL
    assert call(item(adjoint=2)) == B.BFLY_EINVAL
    assert call(item(ld_in=10)) == B.BFLY_EINVAL
    assert call(item(ld_out=10)) == B.BFLY_EINVAL
    assert call(item(n_out=-1)) == B.BFLY_EINVAL
    assert call(item(n_in=1 << 31)) == B.BFLY_EINVAL
    assert call(item(pts_in=None)) == B.BFLY_EINVAL
    assert call(item(out=None)) == B.BFLY_EINVAL
    assert call(item(plan=None)) == B.BFLY_EINVAL
    assert call(item(), prec=9) == B.BFLY_EINVAL
    assert call(item(), n=0) == B.BFLY_EINVAL
    assert call(item(), item(nrhs=0)) == B.BFLY_EINVAL
    assert "item 1" in P.bfly_last_error()
    assert L.bfly_apply_batched(1, None, 0, ctypes.c_void_p(fake), 1 << 40, None) == B.BFLY_EINVAL
    arr = (B.BatchItem * 1)(item(nrhs=0))
    out = ctypes.c_size_t()
    assert L.bfly_batch_workspace_size(1, arr, 0, ctypes.byref(out)) == B.BFLY_EINVAL


def test_batch_item_layout_matches_header():
    """The ctypes mirror of bfly_batch_item has the C layout (LP64)."""
    assert ctypes.sizeof(B.BatchItem) == 80
    assert B.BatchItem.n_in.offset == 16 and B.BatchItem.ld_out.offset == 72


def test_tune_rejects_invalid_arguments_on_host():
    """bfly_tune validates like bfly_apply before any HIP call."""
    p = P.Plan(2, 16, BOX2, TBOX2, "hypradon2", 4)
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    best = ctypes.c_double()

    def call(adjoint=0, nrhs=1, prec=0, max_ms=0.0, ws_bytes=1 << 30, plan=p.handle):
        return L.bfly_tune(plan, adjoint, 256, fake, fake, 256, 256, fake, fake, 256, nrhs, prec, fake, ws_bytes,
                           max_ms, ctypes.byref(best), None)

    assert call(adjoint=2) == B.BFLY_EINVAL
    assert call(max_ms=-1.0) == B.BFLY_EINVAL
    assert call(nrhs=0) == B.BFLY_EINVAL
    assert call(prec=7) == B.BFLY_EINVAL
    assert call(prec=B.BFLY_SPLIT32) == B.BFLY_EUNSUPPORTED
    assert call(ws_bytes=16) == B.BFLY_EWORKSPACE
    assert call(plan=None) == B.BFLY_EINVAL
    assert L.bfly_tune_reset() == B.BFLY_OK
