#!/usr/bin/env python3
"""Throughput of the butterfly apply on one MI355X.

A step is one full apply (binning, leaf initialisation, the log2 N stages with
the middle switch, final evaluation) of the 2-D hyperbolic-Radon workload:
N = 1024 (1,048,576 jittered sources in [1,2) x [0,1), 1,048,576 grid
targets in [0,1)^2), q = 5 (r = 25), one right-hand side, inputs resident in
HBM.  Both precision modes are timed; the headline `value` is the FP32 mode,
the FP64 mode is reported beside it with the speedup.  Relative errors are
measured against the FP64 CPU oracle (the same run times the oracle on the
host cores as `cpu_baseline`).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "Mpoints/s per butterfly apply (2D N=1024, q=5); FP32-MFMA vs FP64 at 1e-5 rel err"
PEAK_VALU_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, non-packed VALU issue rate

# Flops charged per evaluation of tau (sqrt, sin and cos as below), see the design doc.
SINCOS_FLOPS = 28  # sin + cos pair of a reduced argument (two Horner polynomials)
TAU_FLOPS = {"fourier": lambda d: 2 * d - 1, "hypradon2": lambda d: 6, "genradon3": lambda d: 80,
             "separable": lambda d: 5 * d}


def phase_flops(phase: str, d: int) -> int:
    """tau + reduction modulo 1 (2) + sine/cosine pair."""
    return TAU_FLOPS[phase](d) + 2 + SINCOS_FLOPS


def algorithmic_flops(step: str, phase: str, d: int, N: int, q: int, nrhs: int, n_src: int, n_tgt: int):
    """Algorithmic flops of ONE launch of a step (tensor-factored contraction
    counts, phase evaluations at a fixed cost, complex multiply = 6 flops,
    real x complex multiply-add = 4 flops)."""
    r, nc, P = q ** d, 2 ** d, N ** d
    cphi = phase_flops(phase, d)
    if step == "stage_src":
        evals = P * (nc + 1) * r
        macs = P * (2 ** (d + 1) - 2) * q ** (d + 1)
        return evals * cphi + evals * nrhs * 6 + macs * nrhs * 4
    if step == "stage_tgt":
        evals = P * (nc + 1) * r
        macs = P * nc * d * q ** (d + 1)
        return evals * cphi + evals * nrhs * 6 + macs * nrhs * 4
    if step == "switch":
        evals = P * r * r
        return evals * cphi + evals * nrhs * 8
    if step == "init":
        evals = n_src + P * r
        return evals * cphi + evals * nrhs * 6 + n_src * r * nrhs * 4
    if step == "final":
        evals = n_tgt + P * r
        return evals * cphi + evals * nrhs * 6 + n_tgt * r * nrhs * 4
    return 0


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def time_steps(fn, torch, steps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (no rel err either)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (default: all in affinity)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the apply does not shard across GPUs.", file=sys.stderr)
        return 2

    import torch

    import paper_1305_4650_amd as P
    from paper_1305_4650_amd import workloads as W

    t0 = time.time()
    w = W.C2()
    print(f"[bench] workload {w.name}: {w.y.shape[0]} sources, {w.x.shape[0]} targets "
          f"({time.time() - t0:.1f}s to generate)", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(w.y).to(dev)
    x = torch.from_numpy(w.x).to(dev)
    g = torch.from_numpy(w.g).to(dev)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    n = w.y.shape[0]
    npts = w.N ** w.d * w.nrhs

    res = {}
    for prec in ("fp64", "fp32"):
        ws = plan.workspace(n, w.nrhs, prec, device=dev)
        f = torch.empty((w.nrhs, w.x.shape[0]), dtype=torch.complex128, device=dev)

        def step():
            plan.apply(y, g, x, prec, out=f, workspace=ws)

        ms = time_steps(step, torch, args.steps, args.warmup)
        # instrumented pass: per-step-kind HIP event timing on the apply's stream
        P.bfly_timing_enable(True)
        P.bfly_timing_read()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        tim = P.bfly_timing_read()
        P.bfly_timing_enable(False)
        res[prec] = {"ms": ms, "out": f.cpu().numpy(), "timing": tim}
        print(f"[bench] {prec}: {ms:.3f} ms/apply  {npts / ms / 1e3:.1f} Mpoints/s  "
              + " ".join(f"{k}={v[0] / max(v[1], 1):.3f}ms" for k, v in tim.items()),
              file=sys.stderr, flush=True)
        del ws

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = args.cpu_threads or len(os.sched_getaffinity(0))
        t0 = time.time()
        ref = oracle.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x, nthreads=cores)
        t_cpu = time.time() - t0
        cpu = {"value": npts / t_cpu / 1e6, "unit": "Mpoints/s", "cores": cores, "kind": "oracle",
               "sample": "the full workload: one FP64 oracle butterfly apply of all 1,048,576 sources "
                         f"and targets ({t_cpu:.1f} s)"}
        for prec in res:
            res[prec]["rel_err"] = rel(res[prec]["out"], ref)
        print(f"[bench] oracle {t_cpu:.1f}s on {cores} threads; rel err fp64 "
              f"{res['fp64']['rel_err']:.2e} fp32 {res['fp32']['rel_err']:.2e}", file=sys.stderr, flush=True)

    head = "fp32"
    tim = res[head]["timing"]
    dom = max(tim, key=lambda k: tim[k][0])
    launches = max(tim[dom][1], 1)
    avg_ms = tim[dom][0] / launches
    flops = algorithmic_flops(dom, w.phase, w.d, w.N, w.q, w.nrhs, n, w.x.shape[0])
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_VALU_TFLOPS, 4), "traffic": None, "kernel": dom,
                "avg_launch_ms": round(avg_ms, 5), "algorithmic_flops_per_launch": flops}
    out = {
        "metric": METRIC,
        "value": round(npts / res[head]["ms"] / 1e3, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[head]["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: 2-D hyperbolic-Radon phase N*x0*sqrt(y0^2+x1^2*y1^2), N=1024, q=5 (r=25), "
                               "1,048,576 jittered sources in [1,2)x[0,1), 1,048,576 grid targets in [0,1)^2, "
                               "1 right-hand side",
                   "d": w.d, "N": w.N, "q": w.q, "nrhs": w.nrhs, "prec": head,
                   "contraction_unit": "valu"},
        "rel_err_vs_oracle": res[head].get("rel_err"),
        "fp64": {"value": round(npts / res["fp64"]["ms"] / 1e3, 3), "ms_per_step": round(res["fp64"]["ms"], 4),
                 "rel_err_vs_oracle": res["fp64"].get("rel_err")},
        "speedup_fp32_over_fp64": round(res["fp64"]["ms"] / res[head]["ms"], 3),
        "step_ms": {p: {k: round(v[0] / max(v[1], 1), 5) for k, v in res[p]["timing"].items()} for p in res},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
