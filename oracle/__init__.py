"""CPU oracle for the butterfly apply -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementations of the direct sum (Eq. 1 of Poulson,
Demanet, Maxwell & Ying, "A Parallel Butterfly Algorithm") and of the
sequential butterfly algorithm (Alg. "alg:serial") with analytic Chebyshev
interpolation (Sec. 1.4, "Avoiding quadratic precomputation").  The arithmetic
lives in ``bfly_oracle.c``; this module only builds, loads and marshals.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1305_4650_amd``) and must never be imported by it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PHASES = {"fourier": 0, "hypradon2": 1, "genradon3": 2, "separable": 3, "genradon3pi": 4}

_CFLAGS = ["-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-D_DEFAULT_SOURCE", "-Wall"]


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    src = os.path.join(HERE, "bfly_oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", *_CFLAGS, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        L.orc_tau.restype = ctypes.c_double
        L.orc_tau.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, dp, dp]
        L.orc_nodes.restype = None
        L.orc_nodes.argtypes = [ctypes.c_int, dp]
        L.orc_bin.restype = None
        L.orc_bin.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, ctypes.c_long, dp, lp]
        L.orc_direct.restype = ctypes.c_int
        L.orc_direct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_int,
                                 ctypes.c_long, dp, dp, ctypes.c_long,
                                 ctypes.c_long, dp, dp, ctypes.c_long,
                                 ctypes.c_int, ctypes.c_int]
        L.orc_butterfly.restype = ctypes.c_int
        L.orc_butterfly.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_int, ctypes.c_int,
                                    dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_long, dp, dp, ctypes.c_long,
                                    ctypes.c_long, dp, dp, ctypes.c_long,
                                    ctypes.c_int, ctypes.c_int, dp]
        L.orc_butterfly_dump.restype = ctypes.c_int
        L.orc_butterfly_dump.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_int, ctypes.c_int,
                                         dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_long, dp, dp, ctypes.c_long,
                                         ctypes.c_long, dp, dp, ctypes.c_long,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pts(p, d):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1, d))
    return p


def _cplx(v, n):
    """(nrhs, n) complex -> contiguous complex128 (nrhs, n)."""
    v = np.asarray(v, dtype=np.complex128)
    if v.ndim == 1:
        v = v[None, :]
    assert v.shape[1] == n
    return np.ascontiguousarray(v)


def _phase_id(phase):
    return PHASES[phase] if isinstance(phase, str) else int(phase)


def tau(phase, N: int, x, y) -> float:
    """Forward phase in turns, tau = Phi / (2 pi)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
    return lib().orc_tau(_phase_id(phase), x.size, N, _dp(x), _dp(y))


def nodes(q: int) -> np.ndarray:
    z = np.zeros(q)
    lib().orc_nodes(q, _dp(z))
    return z


def bin_points(pts, lo, hi, n_per_dim: int) -> np.ndarray:
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    d = lo.size
    pts = _pts(pts, d)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    out = np.zeros((pts.shape[0], d), dtype=np.int64)
    lib().orc_bin(d, n_per_dim, _dp(lo), _dp(hi), pts.shape[0], _dp(pts),
                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return out


def direct(phase, N: int, y, g, x, adjoint: bool = False, nthreads: int = 0) -> np.ndarray:
    """Direct sum.  Forward: f(x) = sum_y e^{i Phi(x,y)} g(y).
    Adjoint: out(y) = sum_x e^{-i Phi(x,y)} g(x) (pass the x points as ``y``
    argument order is always (points of the input, input, points of the output))."""
    d = np.asarray(y).shape[1]  # point arrays are (n, d)
    pin = _pts(y, d)
    pout = _pts(x, d)
    gi = _cplx(g, pin.shape[0])
    nrhs = gi.shape[0]
    out = np.zeros((nrhs, pout.shape[0]), dtype=np.complex128)
    rc = lib().orc_direct(_phase_id(phase), d, N, int(adjoint),
                          pin.shape[0], _dp(pin), _dp(gi.view(np.float64)), pin.shape[0],
                          pout.shape[0], _dp(pout), _dp(out.view(np.float64)), pout.shape[0],
                          nrhs, nthreads)
    if rc:
        raise ValueError(f"orc_direct rejected its arguments (rc={rc})")
    return out


def butterfly(phase, N: int, q: int, src_box, tgt_box, pts_in, vals, pts_out,
              adjoint: bool = False, switch_level: int = -1, nthreads: int = 0,
              return_counts: bool = False):
    """FP64 butterfly apply.  src_box / tgt_box = (lo[d], hi[d]) of the PLAN
    (forward geometry).  Forward: pts_in = sources y, pts_out = targets x.
    Adjoint: pts_in = targets x (values f), pts_out = sources y."""
    slo = np.ascontiguousarray(src_box[0], dtype=np.float64)
    shi = np.ascontiguousarray(src_box[1], dtype=np.float64)
    tlo = np.ascontiguousarray(tgt_box[0], dtype=np.float64)
    thi = np.ascontiguousarray(tgt_box[1], dtype=np.float64)
    d = slo.size
    pin = _pts(pts_in, d)
    pout = _pts(pts_out, d)
    vi = _cplx(vals, pin.shape[0])
    nrhs = vi.shape[0]
    out = np.zeros((nrhs, pout.shape[0]), dtype=np.complex128)
    counts = np.zeros(4)
    rc = lib().orc_butterfly(d, N, q, _phase_id(phase), _dp(slo), _dp(shi), _dp(tlo), _dp(thi),
                             int(adjoint), switch_level,
                             pin.shape[0], _dp(pin), _dp(vi.view(np.float64)), pin.shape[0],
                             pout.shape[0], _dp(pout), _dp(out.view(np.float64)), pout.shape[0],
                             nrhs, nthreads, _dp(counts))
    if rc:
        raise ValueError(f"orc_butterfly rejected its arguments (rc={rc})")
    if return_counts:
        return out, {"phase": counts[0], "mac": counts[1], "cmac": counts[2], "stages": counts[3]}
    return out


def butterfly_weights(phase, N: int, q: int, src_box, tgt_box, pts_in, vals, step: int,
                      adjoint: bool = False, switch_level: int = -1, nthreads: int = 0):
    """The butterfly's weights after one step (orc_butterfly_dump, a test and
    debugging hook): step 0 after the initialisation, k in 1..ls after
    column-space stage k-1, ls+1 after the middle switch, k in ls+2..L+1
    after row-space stage k-2.  Returns complex (N^d pairs, q^d nodes, nrhs)
    indexed [(a << d (L - lvl)) | b][t][rhs] with a, b the target and source
    box indices of the level (dimension j at bits lvl * j, resp. (L - lvl) * j)."""
    slo = np.ascontiguousarray(src_box[0], dtype=np.float64)
    shi = np.ascontiguousarray(src_box[1], dtype=np.float64)
    tlo = np.ascontiguousarray(tgt_box[0], dtype=np.float64)
    thi = np.ascontiguousarray(tgt_box[1], dtype=np.float64)
    d = slo.size
    L = int(N).bit_length() - 1
    if not 0 <= step <= L + 1:
        raise ValueError(f"step {step} outside 0..{L + 1}")
    pin = _pts(pts_in, d)
    vi = _cplx(vals, pin.shape[0])
    nrhs = vi.shape[0]
    P, r = N ** d, q ** d
    dump = np.zeros((P, r, nrhs), dtype=np.complex128)
    pout = np.zeros((0, d))
    out = np.zeros((nrhs, 0), dtype=np.complex128)
    rc = lib().orc_butterfly_dump(d, N, q, _phase_id(phase), _dp(slo), _dp(shi), _dp(tlo), _dp(thi),
                                  int(adjoint), switch_level,
                                  pin.shape[0], _dp(pin), _dp(vi.view(np.float64)), pin.shape[0],
                                  0, _dp(pout), _dp(out.view(np.float64)), 1,
                                  nrhs, nthreads, int(step), _dp(dump.view(np.float64)))
    if rc:
        raise ValueError(f"orc_butterfly_dump rejected its arguments (rc={rc})")
    return dump
