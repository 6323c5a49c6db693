"""Differentiation through the butterfly: torch.autograd with the adjoint
butterfly as backward (GPU).

For f = B g and a real loss L, PyTorch's gradient for complex g is
B^H dL/df; the backward uses the adjoint butterfly B' (the butterfly of
K^H = exp(-i Phi), roles of x and y swapped), which approximates K^H to the
same accuracy as B approximates K and, with its middle switch at the mirror
level L - floor(L/2), is B^H exactly.  Checks:
  * the gradient equals the oracle's adjoint butterfly applied to f - d
    (FP64, 1e-12);
  * <h, B g> = <B' h, g> on the GPU's own outputs at odd L (where a switch at
    floor(L/2) would miss it by the interpolation error);
  * central finite differences of L agree with the gradient to rounding at
    odd L and q = 4 (interpolation error ~1e-3 there, so an adjoint that is
    only close to B^H would fail).
"""
import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _setup(w):
    import torch

    import paper_1305_4650_amd as P
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(w.y).to(dev)
    x = torch.from_numpy(w.x).to(dev)
    return torch, P, plan, y, x, dev


def test_autograd_backward_is_adjoint_butterfly(orc):
    w = W.hypradon2(32, q=5, nrhs=2)
    torch, P, plan, y, x, dev = _setup(w)
    print("[case] autograd backward vs oracle adjoint, hypradon2 N=32 q=5", flush=True)
    dat = torch.from_numpy(W.random_rhs(W.rng(w.config_id, 2), 2, w.x.shape[0])).to(dev)
    g = torch.from_numpy(w.g).to(dev).requires_grad_(True)
    f = P.bfly_apply_autograd(g, plan, y, x, "fp64")
    loss = 0.5 * (f - dat).abs().pow(2).sum()
    loss.backward()
    torch.cuda.synchronize()
    resid = (f - dat).detach().cpu().numpy()
    ref = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.x, resid, w.y, adjoint=True)
    e = rel(g.grad.cpu().numpy(), ref)
    print(f"  rel err {e:.3e}", flush=True)
    assert e < 1e-12


def test_bflyapply_function_name():
    """The autograd Function is reachable as paper_1305_4650_amd.BflyApply and
    gives the same gradient as bfly_apply_autograd."""
    w = W.hypradon2(16, q=4, nrhs=1)
    torch, P, plan, y, x, dev = _setup(w)
    print("[case] BflyApply.apply", flush=True)
    g1 = torch.from_numpy(w.g).to(dev).requires_grad_(True)
    g2 = torch.from_numpy(w.g).to(dev).requires_grad_(True)
    P.BflyApply.apply(g1, plan, y, x, "fp64").abs().pow(2).sum().backward()
    P.bfly_apply_autograd(g2, plan, y, x, "fp64").abs().pow(2).sum().backward()
    assert torch.equal(g1.grad, g2.grad)


def test_gradient_matches_finite_differences():
    w = W.hypradon2(32, q=4, nrhs=1)
    torch, P, plan, y, x, dev = _setup(w)
    print("[case] finite differences, hypradon2 N=32 q=4", flush=True)
    dat = torch.from_numpy(W.random_rhs(W.rng(w.config_id, 2), 1, w.x.shape[0])).to(dev)
    g0 = torch.from_numpy(w.g).to(dev)

    def loss_of(gv):
        f = plan.apply(y, gv, x, "fp64")
        return 0.5 * float((f - dat).abs().pow(2).sum())

    g = g0.clone().requires_grad_(True)
    f = P.bfly_apply_autograd(g, plan, y, x, "fp64")
    (0.5 * (f - dat).abs().pow(2).sum()).backward()
    grad = g.grad.cpu().numpy()[0]
    idx = W.sample_indices(w.y.shape[0], 16, 77)
    h = 1e-4  # the loss is quadratic in g: central differences are exact up to rounding
    fd = np.zeros(len(idx), complex)
    for k, j in enumerate(idx):
        for part, unit in ((0, 1.0), (1, 1j)):
            gp = g0.clone()
            gm = g0.clone()
            gp[0, j] += h * unit
            gm[0, j] -= h * unit
            dv = (loss_of(gp) - loss_of(gm)) / (2 * h)
            if part == 0:
                fd[k] += dv
            else:
                fd[k] += 1j * dv
    scale = np.abs(grad).max()
    err = np.abs(fd - grad[idx]).max() / scale
    print(f"  fd max err / max|grad| = {err:.3e}", flush=True)
    assert err < 1e-7


@pytest.mark.parametrize("name,prec,tol", [
    ("hypradon2_N32_q5", "fp64", 1e-13), ("genradon3_N8_q4", "fp64", 1e-13),
    ("fourier1d_N32_q6", "fp64", 1e-13), ("genradon3pi_N8_q4", "fp64", 1e-13),
    ("hypradon2_N32_q5", "fp32", 1e-5)])
def test_adjoint_is_exact_transpose(name, prec, tol):
    """<h, B g> = <B' h, g> with both applies from the GPU (odd L)."""
    w = {"hypradon2_N32_q5": lambda: W.hypradon2(32, q=5), "genradon3_N8_q4": lambda: W.genradon3(8, q=4),
         "fourier1d_N32_q6": lambda: W.fourier_grid(32, d=1, q=6),
         "genradon3pi_N8_q4": lambda: W.genradon3pi(8, q=4)}[name]()
    torch, P, plan, y, x, dev = _setup(w)
    print(f"[case] transpose identity {name} {prec}", flush=True)
    hv = W.random_rhs(W.rng(w.config_id, 2), 1, w.x.shape[0])
    Bg = plan.apply(y, torch.from_numpy(w.g).to(dev), x, prec).cpu().numpy()
    Bh = plan.apply_adjoint(x, torch.from_numpy(hv).to(dev), y, prec).cpu().numpy()
    lhs, rhs = np.vdot(hv, Bg), np.vdot(Bh, w.g)
    e = abs(lhs - rhs) / (np.linalg.norm(hv) * np.linalg.norm(Bg))
    print(f"  |<h,Bg> - <B'h,g>| / (|h||Bg|) = {e:.3e}", flush=True)
    assert e < tol


def test_adjoint_matches_direct_KH(orc):
    """The adjoint butterfly against the direct sum K^H f on sampled outputs."""
    w = W.hypradon2(64, q=8, nrhs=1)
    torch, P, plan, y, x, dev = _setup(w)
    print("[case] adjoint vs direct K^H, hypradon2 N=64 q=8", flush=True)
    fv = W.random_rhs(W.rng(w.config_id, 2), 1, w.x.shape[0])
    gb = plan.apply_adjoint(x, torch.from_numpy(fv).to(dev), y, "fp64")
    torch.cuda.synchronize()
    idx = W.sample_indices(w.y.shape[0], 512, 78)
    gd = orc.direct(w.phase, w.N, w.x, fv, w.y[idx], adjoint=True)
    gref = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.x, fv, w.y, adjoint=True)
    eps_q = rel(gref[:, idx], gd)
    e = rel(gb.cpu().numpy()[:, idx], gd)
    print(f"  gap gpu {e:.3e} oracle {eps_q:.3e}", flush=True)
    assert e <= eps_q + 1e-12
