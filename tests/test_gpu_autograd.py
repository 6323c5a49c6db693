"""Differentiation through the butterfly: torch.autograd with the adjoint
butterfly as backward (GPU).

For f = B g and a real loss L, PyTorch's gradient for complex g is
B^H dL/df; the backward uses the adjoint butterfly B' (the butterfly of
K^H = exp(-i Phi), roles of x and y swapped), which approximates K^H to the
same accuracy as B approximates K, but is not exactly B^H.  Checks:
  * the gradient equals the oracle's adjoint butterfly applied to f - d
    (FP64, 1e-12);
  * central finite differences of L agree with it to O(eps_q): at q = 10
    (eps_q ~ 1e-8 here) that is a tight check of signs and conjugations.
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


def test_gradient_matches_finite_differences():
    w = W.hypradon2(16, q=10, nrhs=1)
    torch, P, plan, y, x, dev = _setup(w)
    print("[case] finite differences, hypradon2 N=16 q=10", flush=True)
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
    h = 1e-6
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
    assert err < 1e-5


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
