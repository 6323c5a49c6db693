"""Batched applies (bfly_apply_batched): many instances of uneven size, in
both directions, binned in one sort and run level-synchronously.  Every
instance must give exactly what its own bfly_apply / bfly_apply_adjoint gives
(the arithmetic per weight vector is the same), the oracle agrees to the
usual tolerance, a captured HIP graph replays correctly, and the batched
autograd function equals the per-instance one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1305_4650_amd as P
from paper_1305_4650_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _instances():
    """Uneven mix: hyperbolic Radon at N = 8..64 (nrhs 1, 3, 5: chunked and
    remainder right-hand sides), one adjoint, one Fourier instance (another
    group), one N = 1 instance (no stages)."""
    out = []
    for i, (N, nrhs) in enumerate([(8, 1), (32, 3), (16, 5), (64, 2), (32, 1)]):
        w = W.hypradon2(N, q=5, nrhs=nrhs, config_id=900 + i)
        out.append((w, False))
    out.append((W.hypradon2(16, q=5, nrhs=2, config_id=910), True))
    out.append((W.fourier_grid(32, d=2, q=5, nrhs=2, config_id=911), False))
    out.append((W.hypradon2(1, q=3, nrhs=1, config_id=912), False))
    return out


def _plan(w):
    return P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)


def _items(insts, gen):
    items, ref = [], []
    for w, adj in insts:
        plan = _plan(w)
        y, x = _dev(w.y), _dev(w.x)
        if adj:
            f = W.random_rhs(gen, w.nrhs, x.shape[0])
            items.append((plan, True, x, _dev(f), y))
        else:
            items.append((plan, False, y, _dev(w.g), x))
        ref.append(plan)
    return items


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_equals_single_applies_bitwise(prec):
    insts = _instances()
    items = _items(insts, np.random.default_rng(7))
    outs = P.apply_batched(items, prec)
    torch.cuda.synchronize()
    for k, (plan, adj, pin, vin, pout) in enumerate(items):
        single = (plan.apply_adjoint(pin, vin, pout, prec) if adj else plan.apply(pin, vin, pout, prec))
        torch.cuda.synchronize()
        assert torch.equal(outs[k], single), f"instance {k} (N={plan.N}, adjoint={adj})"


def test_batched_matches_oracle(orc):
    insts = _instances()[:3]
    items = _items(insts, np.random.default_rng(8))
    outs = P.apply_batched(items, "fp64")
    for k, ((w, adj), out) in enumerate(zip(insts, outs)):
        ref = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x)
        got = out.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12, k


def test_batched_graph_replays(prec="fp32"):
    """Capture one batched apply in a HIP graph; refill the inputs and replay
    it several times, with eager work and synchronisations in between; every
    replay equals an eager batched apply on the same inputs."""
    insts = _instances()[:5]
    gen = np.random.default_rng(9)
    items = _items(insts, gen)
    batch = P.Batch(items, prec)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.run()  # warm-up (library attributes, kernels loaded)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run()
    eager = P.Batch(items, prec)  # same input tensors, its own outputs and workspace
    for rep in range(3):
        for (plan, adj, pin, vin, pout) in items:
            vin.copy_(_dev(W.random_rhs(gen, vin.shape[0], vin.shape[1])))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ref = eager.run()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert torch.equal(batch.outs[k], ref[k]), f"replay {rep}, instance {k}"


def test_batched_autograd_equals_per_instance():
    """The least-squares gradient through the batched apply (backward = one
    batched adjoint apply) equals the per-instance autograd gradients."""
    insts = [(W.hypradon2(N, q=5, nrhs=2, config_id=920 + i), False) for i, N in enumerate([8, 16, 32])]
    spec, gs, ds = [], [], []
    gen = np.random.default_rng(10)
    for w, _ in insts:
        plan = _plan(w)
        y, x = _dev(w.y), _dev(w.x)
        spec.append((plan, y, x))
        gs.append(_dev(w.g).requires_grad_(True))
        ds.append(_dev(W.random_rhs(gen, w.nrhs, x.shape[0])))
    fs = P.bfly_apply_batched_autograd(gs, spec, "fp64")
    loss = sum(0.5 * (f - d).abs().pow(2).sum() for f, d in zip(fs, ds))
    loss.backward()
    for (plan, y, x), g, d in zip(spec, gs, ds):
        g1 = g.detach().clone().requires_grad_(True)
        f1 = P.bfly_apply_autograd(g1, plan, y, x, "fp64")
        (0.5 * (f1 - d).abs().pow(2).sum()).backward()
        assert torch.equal(g.grad, g1.grad)


@pytest.mark.parametrize("prec", ["fp32"])
def test_c5_batch_equals_single_applies(prec):
    """The uneven batch at its real shape: 48 hyperbolic-Radon instances with
    N drawn from {128, 256, 512, 1024}, q = 5, 8 right-hand sides, in one
    batched apply; each instance equals its own apply bit for bit (checked on
    every instance)."""
    sizes = W.C5_sizes()
    insts = [(W.C5_instance(i, int(N)), False) for i, N in enumerate(sizes)]
    items = _items(insts, np.random.default_rng(11))
    print(f"[c5] {len(items)} instances, {int(sum(int(N) ** 2 for N in sizes))} points x 8 rhs", flush=True)
    outs = P.apply_batched(items, prec)
    torch.cuda.synchronize()
    for k, (plan, adj, pin, vin, pout) in enumerate(items):
        single = plan.apply(pin, vin, pout, prec)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], single), f"instance {k} (N={plan.N})"
    del outs


def _instances_other_dims():
    """d = 1 and d = 3 groups beside a d = 2 one: Fourier 1-D (forward and
    adjoint), the 3-D generalized-Radon workload form (right-hand-side chunks
    and a remainder), the printed 3-D phase, and a 3-D adjoint."""
    return [
        (W.fourier_grid(64, d=1, q=8, nrhs=2, config_id=930), False),
        (W.fourier_grid(16, d=1, q=5, nrhs=1, config_id=931), True),
        (W.genradon3(8, q=4, nrhs=3, config_id=932), False),
        (W.genradon3pi(4, q=5, config_id=933), False),
        (W.separable(4, d=3, q=2, config_id=934), True),
        (W.hypradon2(8, q=5, nrhs=1, config_id=935), False),
        # sparse sources (blocks of empty source boxes skip their work in the
        # batched launches too) and sparse targets (computed in full there)
        (W.hypradon2_curve(32, q=5, nrhs=2, config_id=936), False),
        (W.hypradon2_curve(32, q=5, config_id=937, curve_targets=True), False),
    ]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_other_dims_equal_single_and_oracle(orc, prec):
    """Batched groups for d = 1 and d = 3: each instance equals its own apply
    bit for bit, and (FP64) the oracle to 1e-12."""
    insts = _instances_other_dims()
    items = _items(insts, np.random.default_rng(12))
    print(f"[case] batched d = 1, 2, 3 mix, {prec}", flush=True)
    outs = P.apply_batched(items, prec)
    torch.cuda.synchronize()
    for k, ((w, adj), (plan, _, pin, vin, pout)) in enumerate(zip(insts, items)):
        single = plan.apply_adjoint(pin, vin, pout, prec) if adj else plan.apply(pin, vin, pout, prec)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], single), f"instance {k} (d={w.d}, N={w.N}, adjoint={adj})"
        if prec == "fp64":
            v = vin.cpu().numpy()
            ref = (orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.x, v, w.y, adjoint=True) if adj
                   else orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, v, w.x))
            got = outs[k].cpu().numpy()
            e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print(f"  instance {k} d={w.d} N={w.N} adjoint={adj}: rel err {e:.3e}", flush=True)
            assert e < 1e-12, k


def test_c5_gradient_matches_finite_differences():
    """The least-squares problem at its real shape: 4 C5 instances (N from
    {128, ..., 1024}, q = 5, 8 right-hand sides), data d = B g_true + 1%
    complex Gaussian noise (scaled by the rms of B g_true), loss
    1/2 sum ||B g - d||^2 at g_0 ~ N(0,1) + iN(0,1), gradient from the batched
    autograd function (backward: one batched adjoint apply, which is B^H).
    Central differences on 16 seeded coordinates x {re, im} per instance; the
    loss is quadratic in g, so they are exact for any step and h = 1 keeps
    the difference far above the rounding of a loss of order 1e12."""
    sizes = W.C5_sizes()[:4]
    insts = [W.C5_instance(i, int(N)) for i, N in enumerate(sizes)]
    spec, gs, ds = [], [], []
    for w in insts:
        plan = _plan(w)
        y, x = _dev(w.y), _dev(w.x)
        f_true = plan.apply(y, _dev(w.g), x, "fp64")
        rms = float(f_true.abs().pow(2).mean().sqrt())
        noise = W.random_rhs(W.rng(w.config_id, 2), w.nrhs, w.x.shape[0]) / np.sqrt(2.0)
        ds.append(f_true + _dev(0.01 * rms * noise))
        spec.append((plan, y, x))
        gs.append(_dev(W.random_rhs(W.rng(w.config_id, 3), w.nrhs, w.y.shape[0])).requires_grad_(True))
    print(f"[case] C5 finite differences, N = {list(map(int, sizes))}", flush=True)
    fs = P.bfly_apply_batched_autograd(gs, spec, "fp64")
    sum(0.5 * (f - d).abs().pow(2).sum() for f, d in zip(fs, ds)).backward()
    h = 1.0
    for k, ((plan, y, x), g, d, w) in enumerate(zip(spec, gs, ds, insts)):
        grad = g.grad.cpu().numpy()
        g0 = g.detach()

        def loss(gv):
            return 0.5 * float((plan.apply(y, gv, x, "fp64") - d).abs().pow(2).sum())

        coords = W.rng(w.config_id, 3).integers(0, [w.nrhs, w.y.shape[0]], size=(16, 2))
        err = 0.0
        for (rr, j) in coords:
            fd = 0.0 + 0.0j
            for unit in (1.0, 1j):
                gp, gm = g0.clone(), g0.clone()
                gp[rr, j] += h * unit
                gm[rr, j] -= h * unit
                fd += unit * (loss(gp) - loss(gm)) / (2 * h)
            err = max(err, abs(fd - grad[rr, j]))
        scale = np.abs(grad).max()
        print(f"  instance {k} N={w.N}: fd max err / max|grad| = {err / scale:.3e}", flush=True)
        assert err / scale < 1e-7, k


@pytest.mark.parametrize("count, n_each, n_big", [(3, 5461, 30000), (64, 4096, 20000), (4, 4095, 70000)])
def test_mixed_batch_at_sort_tile_switches(count, n_each, n_big):
    """Small instances (N = 64: sorted together) with a batched point total
    just below or at the sort's tile-size switches (2^14 = 16384 and 2^18 =
    262144 keys), plus one large instance (N = 128 with more points than
    leaves: run as a single apply inside the call, which uses the shared
    sort scratch for its own sort).  Every output equals the instance's own
    single apply bit for bit."""
    gen = np.random.default_rng([count, n_each, n_big])
    box = (np.array([1.0, 0.0]), np.array([2.0, 1.0]))
    tbox = (np.zeros(2), np.ones(2))
    small = P.Plan(2, 64, box, tbox, "hypradon2", 4)
    big = P.Plan(2, 128, box, tbox, "hypradon2", 4)
    print(f"[case] mixed batch {count} x {n_each} + {n_big} (batched points {count * n_each})", flush=True)
    items = []
    for k in range(count + 1):
        plan, n = (big, n_big) if k == count else (small, n_each)
        y = box[0] + gen.random((n, 2)) * (box[1] - box[0])
        x = gen.random((257, 2))
        g = W.random_rhs(gen, 1, n)
        items.append((plan, False, _dev(y), _dev(g), _dev(x)))
    outs = P.apply_batched(items, "fp64")
    torch.cuda.synchronize()
    for k, (plan, _, y, g, x) in enumerate(items):
        single = plan.apply(y, g, x, "fp64")
        torch.cuda.synchronize()
        assert torch.equal(outs[k], single), f"instance {k}"
