"""The many-right-hand-side Fourier configuration (d = 2, Phi = 2 pi x.y on
uniform grids, q = 6, 64 right-hand sides).

At full size (N = 2048, 4,194,304 points) the GPU applies all 64 right-hand
sides in both modes, as bench.py times them, and right-hand sides 0 and 1 are
compared with the oracle's FP64 butterfly (the oracle needs about 10 GB and a
minute or two for those two).  On uniform grids the direct sum is an
unnormalised inverse DFT, so numpy's FFT also gives the exact result, which
the butterfly matches within its own error at q = 6 (the oracle measures
7.3e-4 to 7.9e-4 for N = 64..256, decreasing with N); FP32 is checked against
FP64 on all 64 right-hand sides.

FP64 bar at full size: the phase tau = x.y reaches 4096 turns, where one
rounding of tau is about 4.5e-13 turns.  The oracle evaluates every switch
factor from the canonical tau; the library's Fourier switch evaluates the
same factor as a product over dimensions of exp(2 pi i x_j (y_j - c_j))
(Sec. 1.4: a tensor-product phase makes the switch a Kronecker product),
whose arguments are far smaller and round far less.  The oracle run both ways
differs from itself by L2 3.3e-13 / sup 5.0e-13 at N = 1024 and about twice
that at N = 2048 (linear in N, the size of tau); the L2 bar stays 1e-12 and
the sup bar is 2e-12, twice that measured self-noise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1305_4650_amd as P
from paper_1305_4650_amd import workloads as W
from parity_norms import assert_parity

pytestmark = pytest.mark.gpu
EPS_Q6 = 1.5e-3  # twice the oracle's q = 6 Fourier butterfly error at N = 64..256


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c4_geometry_oracle_parity(orc):
    w = W.fourier_grid(256, d=2, q=6, nrhs=4, config_id=4, name="C4_geometry_N256")
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(a).cuda() for a in (w.y, w.x, w.g))
    print("[case] oracle C4 geometry at N = 256, 4 rhs", flush=True)
    ref = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        assert_parity(plan.apply(y, g, x, prec).cpu().numpy(), ref, tol, what=prec)


@pytest.fixture(scope="module")
def c4_full(orc):
    """C4 inputs and the oracle's butterfly on right-hand sides 0 and 1."""
    w = W.C4()
    print(f"[case] oracle C4 full size, rhs 0-1 ({w.N ** 2} points)", flush=True)
    ref = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g[:2], w.x)
    return w, ref


@pytest.mark.timeout(1000)
def test_c4_full_size(c4_full):
    w, ref = c4_full
    N = w.N
    print(f"[case] C4 full size: {N * N} points x {w.nrhs} rhs", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x = torch.from_numpy(w.y).cuda(), torch.from_numpy(w.x).cuda()
    g = torch.from_numpy(w.g).cuda()
    f32 = plan.apply(y, g, x, "fp32")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    f64 = plan.apply(y, g, x, "fp64")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    d = float(torch.linalg.vector_norm(f32 - f64) / torch.linalg.vector_norm(f64))
    print(f"  fp32 vs fp64 over 64 rhs: {d:.3e}", flush=True)
    assert d < 1e-5
    got64, got32 = f64[:2].cpu().numpy(), f32[:2].cpu().numpy()
    assert_parity(got64, ref, 1e-12, sup_tol=2e-12, what="fp64 rhs 0-1 vs oracle")
    assert_parity(got32, ref, 1e-5, what="fp32 rhs 0-1 vs oracle")
    for s in range(2):
        exact = N * N * np.fft.ifftn(w.g[s].reshape(N, N)).reshape(-1)
        e = rel(got64[s], exact)
        print(f"  rhs {s}: fp64 butterfly vs exact DFT {e:.3e}", flush=True)
        assert e < EPS_Q6
