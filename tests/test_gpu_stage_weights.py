"""Stage-level parity: the library's last-level weights against the oracle's.

After an apply the weight buffer at the start of the workspace holds the
weights of the last level, before the final evaluation: for target leaf A
and node t, e^{-i Phi(x^A_t, c_Y)} delta^{AY}_t (the row-space form,
demodulated by the root source box's centre c_Y), in slot order ([slot][node],
one right-hand side; the slot interleaves the bits of A's index, coarsest
split first).  The oracle returns delta^{AY}_t after its last stage
(orc_butterfly_dump, step L + 1).  The two are compared vector by vector,
with the same FP64 / FP32 bars as the outputs: a mistake that the final
evaluation's interpolation smooths over would still show here.
"""
import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W
from parity_norms import assert_parity

pytestmark = pytest.mark.gpu


def tau_hypradon2(N, x0, x1, y0, y1):
    """The hyperbolic-Radon phase in turns, in the oracle's operation order
    (checked bit for bit against the oracle's own below)."""
    a = y0 * y0
    b = x1 * x1
    c = y1 * y1
    e = b * c
    s = a + e
    m = float(N) * x0
    return m * np.sqrt(s)


def tau_fourier(N, x0, x1, y0, y1):
    """x . y in turns, in the oracle's operation order."""
    s = x0 * y0
    return s + x1 * y1


TAU = {"hypradon2": tau_hypradon2, "fourier": tau_fourier}


def leaf_nodes(w, L, z, box=None):
    """Target-role leaf nodes x^A_t, indexed [a0 + N a1][t0 + q t1], with the
    library's box arithmetic (centre + half width times node); the target
    role is the plan's target box, or the given box (the adjoint's)."""
    N, q = w.N, w.q
    tlo, thi = w.tgt_box if box is None else box
    wd = (np.asarray(thi) - np.asarray(tlo)) / N
    a = np.arange(N)
    c0 = tlo[0] + (a + 0.5) * wd[0]
    c1 = tlo[1] + (a + 0.5) * wd[1]
    h0, h1 = 0.5 * wd[0], 0.5 * wd[1]
    x0 = c0[:, None] + h0 * z[None, :]          # [a0][t0]
    x1 = c1[:, None] + h1 * z[None, :]          # [a1][t1]
    X0 = np.broadcast_to(x0[None, :, None, :], (N, N, q, q))  # [a1][a0][t1][t0]
    X1 = np.broadcast_to(x1[:, None, :, None], (N, N, q, q))
    return X0.reshape(N * N, q * q), X1.reshape(N * N, q * q)


def slots(N, L):
    """Slot of target leaf A = (a0, a1) at the last level, for A's oracle
    index a0 + N a1: bit k of the slot's digit d is bit L-1-k of a_d."""
    a = np.arange(N * N)
    a0, a1 = a % N, a // N
    s = np.zeros(N * N, dtype=np.int64)
    for k in range(L):
        s |= ((a0 >> (L - 1 - k)) & 1) << (2 * k)
        s |= ((a1 >> (L - 1 - k)) & 1) << (2 * k + 1)
    return s


CASES = [
    ("C1_fourier2d_N64_q5", lambda: W.C1(), "fp64", 1e-12),
    ("C1_fourier2d_N64_q5", lambda: W.C1(), "fp32", 1e-5),
    ("hypradon2_N128_q5", lambda: W.hypradon2(128, q=5), "fp64", 1e-12),
    ("hypradon2_N128_q5", lambda: W.hypradon2(128, q=5), "fp32", 1e-5),
    ("C2_hypradon2_N1024_q5", lambda: W.C2(), "fp64", 1e-12),
    ("C2_hypradon2_N1024_q5", lambda: W.C2(), "fp32", 1e-5),
]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name, make, prec, tol", CASES, ids=[f"{c[0]}-{c[2]}" for c in CASES])
def test_last_level_weights_match_oracle(orc, name, make, prec, tol):
    import torch
    import paper_1305_4650_amd as P
    w = make()
    N, q = w.N, w.q
    L = N.bit_length() - 1
    r = q * q
    print(f"[case] last-level weights {name} {prec}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x, w.g))
    ws = plan.workspace(w.y.shape[0], 1, prec)
    plan.apply(y, g, x, prec, workspace=ws)
    torch.cuda.synchronize()
    dt = np.complex128 if prec == "fp64" else np.complex64
    nbytes = N * N * r * np.dtype(dt).itemsize
    got = ws[:nbytes].cpu().numpy().view(dt).reshape(N * N, r).astype(np.complex128)
    del ws

    delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.y, w.g, L + 1)[:, :, 0]
    z = orc.nodes(q)
    X0, X1 = leaf_nodes(w, L, z)
    slo, shi = (np.asarray(b, dtype=np.float64) for b in w.src_box)
    cy = slo + 0.5 * (shi - slo)  # the root source box's centre, as the library forms it
    t = TAU[w.phase](N, X0, X1, cy[0], cy[1])
    # the phase as written here is the oracle's, bit for bit
    rng = np.random.default_rng(5)
    for i in rng.choice(t.size, 200, replace=False):
        a, k = divmod(int(i), r)
        assert t[a, k] == orc.tau(w.phase, N, [X0[a, k], X1[a, k]], cy)
    want = delta * np.exp(-2j * np.pi * (t - np.rint(t)))
    assert_parity(got[slots(N, L)], want, tol, what=f"{name} {prec} last-level weights")


ADJ_CASES = [
    ("C1_fourier2d_N64_q5", lambda: W.C1(), "fp64", 1e-12),
    ("hypradon2_N128_q5", lambda: W.hypradon2(128, q=5), "fp64", 1e-12),
    ("C2_hypradon2_N1024_q5", lambda: W.C2(), "fp64", 1e-12),
    ("C2_hypradon2_N1024_q5", lambda: W.C2(), "fp32", 1e-5),
]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name, make, prec, tol", ADJ_CASES, ids=[f"{c[0]}-{c[2]}" for c in ADJ_CASES])
def test_adjoint_last_level_weights_match_oracle(orc, name, make, prec, tol):
    """The adjoint apply (roles swapped, phase -Phi(x, y), mirror switch
    level): its last level lives on the leaves of the plan's source box, and
    is demodulated by the plan's target-box centre c_X, i.e. multiplied by
    e^{+i Phi(c_X, y_t)}."""
    import torch
    import paper_1305_4650_amd as P
    w = make()
    N, q = w.N, w.q
    L = N.bit_length() - 1
    r = q * q
    rng = np.random.default_rng(17)
    f = rng.standard_normal((1, w.x.shape[0])) + 1j * rng.standard_normal((1, w.x.shape[0]))
    print(f"[case] adjoint last-level weights {name} {prec}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, fd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x, f))
    ws = plan.workspace(w.x.shape[0], 1, prec)
    plan.apply_adjoint(x, fd, y, prec, workspace=ws)
    torch.cuda.synchronize()
    dt = np.complex128 if prec == "fp64" else np.complex64
    nbytes = N * N * r * np.dtype(dt).itemsize
    got = ws[:nbytes].cpu().numpy().view(dt).reshape(N * N, r).astype(np.complex128)
    del ws

    delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.x, f, L + 1, adjoint=True)[:, :, 0]
    z = orc.nodes(q)
    Y0, Y1 = leaf_nodes(w, L, z, box=w.src_box)
    tlo, thi = (np.asarray(b, dtype=np.float64) for b in w.tgt_box)
    cx = tlo + 0.5 * (thi - tlo)
    t = TAU[w.phase](N, cx[0], cx[1], Y0, Y1)
    for i in rng.choice(t.size, 200, replace=False):
        a, k = divmod(int(i), r)
        assert t[a, k] == orc.tau(w.phase, N, cx, [Y0[a, k], Y1[a, k]])
    want = delta * np.exp(2j * np.pi * (t - np.rint(t)))
    assert_parity(got[slots(N, L)], want, tol, what=f"{name} {prec} adjoint last-level weights")


def leaf_nodes_nd(box, N, q, d, z):
    """Leaf nodes of a box in d dimensions, [a_lin][t][j] with a_lin =
    sum_j a_j N^j and t = sum_j t_j q^j (the library's box arithmetic)."""
    lo, hi = (np.asarray(b, dtype=np.float64) for b in box)
    wd = (hi - lo) / N
    out = np.empty((N ** d, q ** d, d))
    for j in range(d):
        a_j = (np.arange(N ** d) // N ** j) % N
        t_j = (np.arange(q ** d) // q ** j) % q
        c = lo[j] + (a_j + 0.5) * wd[j]
        out[:, :, j] = c[:, None] + (0.5 * wd[j]) * z[t_j][None, :]
    return out


def slots_nd(N, L, d):
    a = np.arange(N ** d)
    s = np.zeros(N ** d, dtype=np.int64)
    for j in range(d):
        a_j = (a // N ** j) % N
        for k in range(L):
            s |= ((a_j >> (L - 1 - k)) & 1) << (d * k + j)
    return s


CASES_ND = [
    ("genradon3_N16_q4", lambda: W.genradon3(16, q=4), "fp64", 1e-12, False),
    ("genradon3_N16_q4", lambda: W.genradon3(16, q=4), "fp32", 1e-5, False),
    ("genradon3_N16_q4", lambda: W.genradon3(16, q=4), "fp64", 1e-12, True),
    ("fourier1d_N64_q8", lambda: W.fourier_grid(64, d=1, q=8), "fp64", 1e-12, False),
    ("fourier1d_N64_q8", lambda: W.fourier_grid(64, d=1, q=8), "fp32", 1e-5, False),
    ("fourier1d_N64_q8", lambda: W.fourier_grid(64, d=1, q=8), "fp64", 1e-12, True),
]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name, make, prec, tol, adjoint", CASES_ND,
                         ids=[f"{c[0]}-{c[2]}-{'adj' if c[4] else 'fwd'}" for c in CASES_ND])
def test_nd_last_level_weights_match_oracle(orc, name, make, prec, tol, adjoint):
    """Other dimensions: the 3-D generalized-Radon phase (its sine and
    cosine terms make the demodulation factors come from the oracle's own
    phase, node by node) and the 1-D Fourier phase (slot = bit-reversed leaf
    index)."""
    import torch
    import paper_1305_4650_amd as P
    w = make()
    N, q, d = w.N, w.q, w.d
    L = N.bit_length() - 1
    r = q ** d
    rng = np.random.default_rng(23)
    print(f"[case] last-level weights {name} {prec} {'adjoint' if adjoint else 'forward'}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x))
    if adjoint:
        f = rng.standard_normal((1, w.x.shape[0])) + 1j * rng.standard_normal((1, w.x.shape[0]))
        ws = plan.workspace(w.x.shape[0], 1, prec)
        plan.apply_adjoint(x, torch.from_numpy(f).cuda(), y, prec, workspace=ws)
    else:
        ws = plan.workspace(w.y.shape[0], 1, prec)
        plan.apply(y, torch.from_numpy(np.ascontiguousarray(w.g)).cuda(), x, prec, workspace=ws)
    torch.cuda.synchronize()
    dt = np.complex128 if prec == "fp64" else np.complex64
    got = ws[:N ** d * r * np.dtype(dt).itemsize].cpu().numpy().view(dt).reshape(N ** d, r).astype(np.complex128)
    del ws
    z = orc.nodes(q)
    if adjoint:
        delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.x, f, L + 1, adjoint=True)[:, :, 0]
        nodes = leaf_nodes_nd(w.src_box, N, q, d, z)
        lo, hi = (np.asarray(b, dtype=np.float64) for b in w.tgt_box)
        c = lo + 0.5 * (hi - lo)
        t = np.array([[orc.tau(w.phase, N, c, nodes[a, k]) for k in range(r)] for a in range(N ** d)])
        want = delta * np.exp(2j * np.pi * (t - np.rint(t)))
    else:
        delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.y, w.g, L + 1)[:, :, 0]
        nodes = leaf_nodes_nd(w.tgt_box, N, q, d, z)
        lo, hi = (np.asarray(b, dtype=np.float64) for b in w.src_box)
        c = lo + 0.5 * (hi - lo)
        t = np.array([[orc.tau(w.phase, N, nodes[a, k], c) for k in range(r)] for a in range(N ** d)])
        want = delta * np.exp(-2j * np.pi * (t - np.rint(t)))
    assert_parity(got[slots_nd(N, L, d)], want, tol, what=f"{name} {prec} last-level weights")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec, tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_chunked_rhs_last_level_weights_match_oracle(orc, prec, tol):
    """Three right-hand sides: a chunk of two ([slot][node][2]) and one more
    chunk of one, which starts at 2 N^d r values."""
    import torch
    import paper_1305_4650_amd as P
    w = W.hypradon2(128, q=5, nrhs=3)
    N, q = w.N, w.q
    L = N.bit_length() - 1
    r = q * q
    print(f"[case] last-level weights, 3 rhs, {prec}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x, w.g))
    ws = plan.workspace(w.y.shape[0], 3, prec)
    plan.apply(y, g, x, prec, workspace=ws)
    torch.cuda.synchronize()
    dt = np.complex128 if prec == "fp64" else np.complex64
    flat = ws[:3 * N * N * r * np.dtype(dt).itemsize].cpu().numpy().view(dt).astype(np.complex128)
    del ws
    got = np.empty((N * N, r, 3), dtype=np.complex128)
    got[:, :, 0:2] = flat[:2 * N * N * r].reshape(N * N, r, 2)
    got[:, :, 2] = flat[2 * N * N * r:].reshape(N * N, r)
    delta = orc.butterfly_weights(w.phase, N, q, w.src_box, w.tgt_box, w.y, w.g, L + 1)
    X0, X1 = leaf_nodes(w, L, orc.nodes(q))
    slo, shi = (np.asarray(b, dtype=np.float64) for b in w.src_box)
    cy = slo + 0.5 * (shi - slo)
    t = tau_hypradon2(N, X0, X1, cy[0], cy[1])
    want = delta * np.exp(-2j * np.pi * (t - np.rint(t)))[:, :, None]
    assert_parity(got[slots(N, L)], want, tol, what=f"3 rhs {prec} last-level weights")
