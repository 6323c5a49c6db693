"""Level-by-level parity: the weights after every merge-and-split stage.

A fresh process applies a workload with one stage per launch (BFLY_KSPLIT)
and stops after the first n stages (BFLY_STOP_STAGES, read once per
process), so that the start of the workspace holds the weights of level n;
the oracle's weights after the same step (orc_butterfly_dump) are the
reference.  Workloads: 2-D hyperbolic Radon at N = 128 (dense, sparse
sources, sparse targets) and at full C2 size, 2-D Fourier at C1 size, 3-D
generalized Radon at N = 16, 1-D Fourier at N = 64; forward and adjoint.  Level n's slot of the pair (A, B)
holds A's split bits, coarsest first, in its low n digits and B in Morton
order, finest digit lowest, in the high L - n digits.  Column-space weights
are the equivalent sources themselves; from the switch on the library keeps
them demodulated by the source box's centre, e^{-i Phi(x^A_t, c_B)} delta_t.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W
from parity_norms import assert_parity

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
import paper_1305_4650_amd as P
from paper_1305_4650_amd import workloads as W
w = {make}
plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
y, x, g = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x, w.g))
f = np.load({fpath!r}) if {adjoint} else None
out = {{}}
for prec in {precs}:
    dt = np.complex128 if prec == "fp64" else np.complex64
    ws = plan.workspace((w.x if {adjoint} else w.y).shape[0], 1, prec)
    ws.zero_()
    if {adjoint}:
        plan.apply_adjoint(x, torch.from_numpy(f).cuda(), y, prec, workspace=ws)
    else:
        plan.apply(y, g, x, prec, workspace=ws)
    torch.cuda.synchronize()
    n = w.N ** w.d * w.q ** w.d * np.dtype(dt).itemsize
    out[prec] = ws[:n].cpu().numpy().view(dt).astype(np.complex128)
np.savez({path!r}, **out)
"""


def tau_hypradon2(N, x0, x1, y0, y1):
    """The phase in turns in the oracle's operation order (checked below)."""
    a = y0 * y0
    b = x1 * x1
    c = y1 * y1
    e = b * c
    s = a + e
    m = float(N) * x0
    return m * np.sqrt(s)


def tau_fourier(N, x0, x1, y0, y1):
    """x . y in turns in the oracle's operation order."""
    s = x0 * y0
    return s + x1 * y1


TAU = {"hypradon2": tau_hypradon2, "fourier": tau_fourier}


def level_layout(w, L, lvl, z, tgt_box=None, src_box=None):
    """For every oracle pair index at level lvl: the library's slot, the
    target box's node coordinates and the source box's centre (boxes in the
    roles of the apply: the plan's own, or swapped for the adjoint)."""
    N, q = w.N, w.q
    lb = L - lvl
    p = np.arange(N * N)
    a_lin, b_lin = p >> (2 * lb), p & ((1 << (2 * lb)) - 1)
    a = [(a_lin >> (lvl * j)) & ((1 << lvl) - 1) for j in range(2)]
    b = [(b_lin >> (lb * j)) & ((1 << lb) - 1) for j in range(2)]
    slot = np.zeros(N * N, dtype=np.int64)
    for j in range(2):
        for k in range(lvl):
            slot |= ((a[j] >> (lvl - 1 - k)) & 1) << (2 * k + j)
        for m in range(lb):
            slot |= ((b[j] >> m) & 1) << (2 * (lvl + m) + j)
    tlo, thi = (np.asarray(v, dtype=np.float64) for v in (w.tgt_box if tgt_box is None else tgt_box))
    slo, shi = (np.asarray(v, dtype=np.float64) for v in (w.src_box if src_box is None else src_box))
    wa = (thi - tlo) / 2 ** lvl
    wb = (shi - slo) / 2 ** lb
    t = np.arange(q * q)
    t0, t1 = t % q, t // q
    ca = [tlo[j] + (a[j] + 0.5) * wa[j] for j in range(2)]
    x0 = ca[0][:, None] + (0.5 * wa[0]) * z[t0][None, :]
    x1 = ca[1][:, None] + (0.5 * wa[1]) * z[t1][None, :]
    cb = [slo[j] + (b[j] + 0.5) * wb[j] for j in range(2)]
    return slot, x0, x1, cb[0][:, None], cb[1][:, None]


BOTH = (("fp64", 1e-12), ("fp32", 1e-5))
CASES = [
    ("hypradon2_N128_q5", "W.hypradon2(128, q=5)", False, BOTH),
    ("hypradon2_N128_q5", "W.hypradon2(128, q=5)", True, BOTH),
    ("C1_fourier2d_N64_q5", "W.C1()", False, BOTH),
    ("C1_fourier2d_N64_q5", "W.C1()", True, BOTH),
    ("hypradon2_srccurve_N128_q5", "W.hypradon2_curve(128, q=5)", False, BOTH),
    ("hypradon2_tgtcurve_N128_q5", "W.hypradon2_curve(128, q=5, curve_targets=True)", False, BOTH),
    ("C2_hypradon2_N1024_q5", "W.C2()", False, BOTH),
]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("name, make, adjoint, precs", CASES,
                         ids=[f"{c[0]}-{'adj' if c[2] else 'fwd'}" for c in CASES])
def test_weights_after_every_stage_match_oracle(orc, tmp_path, name, make, adjoint, precs):
    """Forward: the switch after floor(L/2) stages; adjoint (roles swapped,
    phase -Phi(x, y)): after L - floor(L/2), and its row-space weights are
    demodulated by e^{+i Phi(c_B, x^A_t)} with c_B in the plan's target box."""
    w = eval(make, {"W": W})
    N, q = w.N, w.q
    tau = TAU[w.phase]
    L = N.bit_length() - 1
    ls = L - L // 2 if adjoint else L // 2
    z = orc.nodes(q)
    fpath = str(tmp_path / "f.npy")
    f = None
    if adjoint:
        rng = np.random.default_rng(31)
        f = rng.standard_normal((1, w.x.shape[0])) + 1j * rng.standard_normal((1, w.x.shape[0]))
        np.save(fpath, f)
    roles = (w.src_box, w.tgt_box) if adjoint else (w.tgt_box, w.src_box)
    # leaves of the target role that hold an output point: with sparse
    # outputs a launch skips target boxes without one, whose slots then
    # hold no defined value
    tpts = w.y if adjoint else w.x
    leaf = orc.bin_points(tpts, roles[0][0], roles[0][1], N)
    for stop in range(1, L + 1):
        print(f"[case] {name} {'adjoint' if adjoint else 'forward'}: weights after {stop} of {L} stages "
              f"(switch after {ls})", flush=True)
        path = str(tmp_path / f"stop{stop}.npz")
        env = {k: v for k, v in os.environ.items() if not k.startswith("BFLY_")}
        env.update(BFLY_KSPLIT=",".join(["1"] * L), BFLY_STOP_STAGES=str(stop))
        code = CODE.format(root=ROOT, path=path, make=make, adjoint=adjoint, fpath=fpath,
                           precs=[p for p, _ in precs])
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        with np.load(path) as data:
            got = {k: data[k] for k in data.files}
        os.remove(path)
        step = stop if stop < ls else stop + 1
        if adjoint:
            delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.x, f, step, adjoint=True)[:, :, 0]
        else:
            delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.y, w.g, step)[:, :, 0]
        slot, x0, x1, cb0, cb1 = level_layout(w, L, stop, z, *roles)
        want = delta
        if stop >= ls:
            if adjoint:  # tau of the adjoint's roles: -tau_fwd(c_B, x^A_t)
                t = tau(N, cb0, cb1, x0, x1)
                chk = lambda a, k: orc.tau(w.phase, N, [cb0[a, 0], cb1[a, 0]], [x0[a, k], x1[a, k]])
                sign = 1.0
            else:
                t = tau(N, x0, x1, cb0, cb1)
                chk = lambda a, k: orc.tau(w.phase, N, [x0[a, k], x1[a, k]], [cb0[a, 0], cb1[a, 0]])
                sign = -1.0
            for i in (0, 7, t.size // 2, t.size - 1):
                a, k = divmod(i, q * q)
                assert t[a, k] == chk(a, k)
            want = delta * np.exp(sign * 2j * np.pi * (t - np.rint(t)))
        anc = leaf >> (L - stop)
        live = np.zeros(1 << (2 * stop), dtype=bool)
        live[anc[:, 0] | (anc[:, 1] << stop)] = True
        keep = live[np.arange(N * N) >> (2 * (L - stop))]
        for prec, tol in precs:
            g = got[prec].reshape(N * N, q * q)
            assert_parity(g[slot][keep], want[keep], tol, what=f"{name} level {stop} {prec} ({keep.sum()} pairs)")


def level_layout_nd(w, L, lvl, z, d, tgt_box, src_box):
    """level_layout in d dimensions: slot, target nodes [pair][t][j] and
    source centres [pair][j] (t = sum_j t_j q^j)."""
    N, q = w.N, w.q
    lb = L - lvl
    p = np.arange(N ** d)
    a_lin, b_lin = p >> (d * lb), p & ((1 << (d * lb)) - 1)
    a = [(a_lin >> (lvl * j)) & ((1 << lvl) - 1) for j in range(d)]
    b = [(b_lin >> (lb * j)) & ((1 << lb) - 1) for j in range(d)]
    slot = np.zeros(N ** d, dtype=np.int64)
    for j in range(d):
        for k in range(lvl):
            slot |= ((a[j] >> (lvl - 1 - k)) & 1) << (d * k + j)
        for m in range(lb):
            slot |= ((b[j] >> m) & 1) << (d * (lvl + m) + j)
    tlo, thi = (np.asarray(v, dtype=np.float64) for v in tgt_box)
    slo, shi = (np.asarray(v, dtype=np.float64) for v in src_box)
    wa, wb = (thi - tlo) / 2 ** lvl, (shi - slo) / 2 ** lb
    t = np.arange(q ** d)
    x = np.empty((N ** d, q ** d, d))
    cb = np.empty((N ** d, d))
    for j in range(d):
        t_j = (t // q ** j) % q
        x[:, :, j] = (tlo[j] + (a[j] + 0.5) * wa[j])[:, None] + (0.5 * wa[j]) * z[t_j][None, :]
        cb[:, j] = slo[j] + (b[j] + 0.5) * wb[j]
    return slot, x, cb


ND_CASES = [("genradon3_N16_q4", "W.genradon3(16, q=4)", False), ("genradon3_N16_q4", "W.genradon3(16, q=4)", True),
            ("fourier1d_N64_q8", "W.fourier_grid(64, d=1, q=8)", False)]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("name, make, adjoint", ND_CASES, ids=[f"{c[0]}-{'adj' if c[2] else 'fwd'}" for c in ND_CASES])
def test_nd_weights_after_every_stage_match_oracle(orc, tmp_path, name, make, adjoint):
    """3-D (generalized Radon; demodulation factors from the oracle's own
    phase, node by node) and 1-D (Fourier), every level."""
    w = eval(make, {"W": W})
    N, q, d = w.N, w.q, w.d
    L = N.bit_length() - 1
    ls = L - L // 2 if adjoint else L // 2
    r = q ** d
    z = orc.nodes(q)
    fpath = str(tmp_path / "f.npy")
    f = None
    if adjoint:
        rng = np.random.default_rng(37)
        f = rng.standard_normal((1, w.x.shape[0])) + 1j * rng.standard_normal((1, w.x.shape[0]))
        np.save(fpath, f)
    roles = (w.src_box, w.tgt_box) if adjoint else (w.tgt_box, w.src_box)
    for stop in range(1, L + 1):
        print(f"[case] {name} {'adjoint' if adjoint else 'forward'}: weights after {stop} of {L} stages "
              f"(switch after {ls})", flush=True)
        path = str(tmp_path / f"stop{stop}.npz")
        env = {k: v for k, v in os.environ.items() if not k.startswith("BFLY_")}
        env.update(BFLY_KSPLIT=",".join(["1"] * L), BFLY_STOP_STAGES=str(stop))
        code = CODE.format(root=ROOT, path=path, make=make, adjoint=adjoint, fpath=fpath,
                           precs=[p for p, _ in BOTH])
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        assert res.returncode == 0, res.stderr[-2000:]
        with np.load(path) as data:
            got = {k: data[k] for k in data.files}
        os.remove(path)
        step = stop if stop < ls else stop + 1
        if adjoint:
            delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.x, f, step, adjoint=True)[:, :, 0]
        else:
            delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.y, w.g, step)[:, :, 0]
        slot, x, cb = level_layout_nd(w, L, stop, z, d, *roles)
        want = delta
        if stop >= ls:
            if adjoint:
                t = np.array([[orc.tau(w.phase, N, cb[a], x[a, k]) for k in range(r)] for a in range(N ** d)])
                want = delta * np.exp(2j * np.pi * (t - np.rint(t)))
            else:
                t = np.array([[orc.tau(w.phase, N, x[a, k], cb[a]) for k in range(r)] for a in range(N ** d)])
                want = delta * np.exp(-2j * np.pi * (t - np.rint(t)))
        for prec, tol in BOTH:
            assert_parity(got[prec].reshape(N ** d, r)[slot], want, tol, what=f"{name} level {stop} {prec}")
