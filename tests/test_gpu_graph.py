"""A single apply captured in a HIP graph: the apply launches kernels only
(the leaf sort, the offsets, the empty-leaf flag and the target occupancy are
kernels; no memset, allocation or synchronisation), so it can be captured.
The graph is replayed several times with fresh inputs and eager work and
synchronisations between replays; every replay must equal an eager apply on
the same inputs bit for bit.  Cases: an evenly filled apply and one with
sparse targets (occupancy pyramid built and cleared inside the graph), both
precisions, forward and adjoint."""
import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "hypradon2_N64_q5_2rhs": lambda: W.hypradon2(64, q=5, nrhs=2),
    "tgtcurve_N64_q5": lambda: W.hypradon2_curve(64, q=5, curve_targets=True),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_single_apply_graph_replays(name, prec, adjoint):
    import torch

    import paper_1305_4650_amd as P
    w = CASES[name]()
    print(f"[case] graph replays {name} {prec} adjoint={adjoint}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(w.y).to(dev)
    x = torch.from_numpy(w.x).to(dev)
    pin, pout = (x, y) if adjoint else (y, x)
    gen = np.random.default_rng(21)
    vin = torch.from_numpy(W.random_rhs(gen, w.nrhs, pin.shape[0])).to(dev)
    out = torch.empty((w.nrhs, pout.shape[0]), dtype=torch.complex128, device=dev)
    ws = plan.workspace(pin.shape[0], w.nrhs, prec, device=dev)

    def run(o, wsp):
        if adjoint:
            plan.apply_adjoint(pin, vin, pout, prec, out=o, workspace=wsp)
        else:
            plan.apply(pin, vin, pout, prec, out=o, workspace=wsp)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(out, ws)  # warm-up: kernels loaded, LDS attributes set
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run(out, ws)
    ref = torch.empty_like(out)
    ws_e = plan.workspace(pin.shape[0], w.nrhs, prec, device=dev)
    for rep in range(3):
        vin.copy_(torch.from_numpy(W.random_rhs(gen, w.nrhs, pin.shape[0])).to(dev))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        run(ref, ws_e)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
