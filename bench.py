#!/usr/bin/env python3
"""Throughput of the butterfly apply on one MI355X.

A step is one full apply (binning, leaf initialisation, the log2 N stages with
the middle switch, final evaluation) of the 2-D hyperbolic-Radon workload:
N = 1024 (1,048,576 jittered sources in [1,2) x [0,1), 1,048,576 grid
targets in [0,1)^2), q = 5 (r = 25), one right-hand side, inputs resident in
HBM.  Both precision modes are timed; the headline `value` is the FP64 mode
(the paper computes in double precision), the FP32 mode is reported beside it
with the speedup.  Relative errors are measured against the FP64 CPU oracle
(the same run times the oracle on the host cores as `cpu_baseline`).  Each
mode carries its roofline: algorithmic flops per launch over the launch's
event-timed duration against the VALU peak, a sine/cosine evaluation charged
at the cost the phase-rate microkernel measures in the same run.

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
ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_1305_4650_amd", "csrc")
# MI355X published vector peaks: FP64 78.6 TFLOP/s (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz), FP32
# 157.3 TFLOP/s.  The FP32 mode runs its contraction and sine/cosine in FP32 and its phase arguments
# in FP64; its roofline is taken against the FP32 peak, an FP64 operation counting as two FP32 ones
# (half the rate).  (The contraction-rate microkernel measures non-packed v_fma_f32 at about 73% of
# 157.3 on this part, the same fraction FP64 FMAs reach of 78.6, so 78.6 would not bound FP32.)
HBM_PEAK_TBPS = 8.0  # MI355X HBM3E, published
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# Flops charged per evaluation of tau: the operations of its definition, a
# square root counted as one operation (the kernels' correctly rounded FP64
# square root takes about ten, and they share it where the definition allows).
TAU_FLOPS = {"fourier": lambda d: 2 * d - 1, "hypradon2": lambda d: 6, "genradon3": lambda d: 80,
             "genradon3pi": lambda d: 78,
             "separable": lambda d: 5 * d}
# Harness operations of the phase-rate microkernel per factor (an FP64
# argument step, two additions into the sum in the working precision), in
# flops at the precision's own rate, taken off its measured per-factor cost.
PHASE_RATE_HARNESS_FLOPS = {"fp64": 3, "fp32": 4}
# FP64 operations (the phase arguments) in flop equivalents of each mode.
FP64_WEIGHT = {"fp64": 1, "fp32": 2}


def affine_x0(prec: str, phase: str, d: int, adjoint: bool) -> bool:
    """The FP32 kernels factor phases that are affine in the target-role
    coordinate x0 along node lines (1 + q/2 sine/cosine pairs per line of q
    factors); FP64 keeps tau's canonical operation order and evaluates every
    factor."""
    return prec == "fp32" and (phase == "fourier" or (phase == "hypradon2" and d == 2 and not adjoint))


def evaluated(kind: str, prec: str, phase: str, d: int, q: int, adjoint: bool = False):
    """(sine/cosine evaluations, tau evaluations, factor applications) that
    the kernels perform per output weight vector of one column-space stage
    ("col"), row-space stage ("row") or middle switch ("switch"), counted from
    the kernels' loops.  Where they evaluate every factor, these are the
    algorithmic counts: column space (2^d + 1) r, row space 2^d r factors of a
    phase difference and r taus alone, switch r^2 factors and r taus alone.
    Not modelled (the algorithmic count stands): the hyperbolic-Radon
    adjoint's factorisations."""
    r, nc, rm = q ** d, 2 ** d, q ** (d - 1)
    half = 1 + q // 2
    aff = affine_x0(prec, phase, d, adjoint)
    fourier32 = prec == "fp32" and phase == "fourier"
    if kind == "col":
        if fourier32:  # per line job: pass 0 two centre factors and q/2 line factors; demodulation 1 + q/2
            n = (nc // 2) * rm * (2 + q // 2) + rm * half
            return n, n, (nc + 1) * r
        return (nc + 1) * r, (nc + 1) * r, (nc + 1) * r
    if kind == "row":
        if fourier32:  # per line job: q/2 line factors shared by the children (conjugate), one per child
            return rm * (nc + q // 2), rm * (nc + 1), nc * r
        if aff:  # per line job: one tau for the parent centre, per child one tau and 1 + q/2 pairs
            return rm * nc * half, rm * (nc + 1), nc * r
        return nc * r, nc * r + r, nc * r
    if kind == "switch":
        if phase == "fourier":  # Kronecker product of d q x q factor matrices
            return d * q * q, d * q * q, d * q ** (d + 1)
        if aff:  # per line job and source node: one tau and 1 + q/2 pairs
            return rm * r * half, rm * (r + 1), r * r
        return r * r, r * r + r, r * r
    raise ValueError(kind)


def tensor_macs(d: int, q: int) -> int:
    """Real x complex multiply-adds per output vector of one merge-and-split
    stage in tensor form: along each dimension a q x q transform onto both
    halves, (2^(d+1) - 2) q^(d+1) in total (both halves of the algorithm)."""
    return (2 ** (d + 1) - 2) * q ** (d + 1)


def flop_model(prec: str, c_cs: float, phase: str, d: int, N: int, q: int, nrhs: int, n_src: int, n_tgt: int,
               adjoint: bool = False) -> dict:
    """Flops charged per unit of work, all N^d output vectors at once: one
    "stage" of each half, one leaf initialisation, one switch, one final
    evaluation.  A sine/cosine evaluation costs c_cs (measured: the vector
    peak over the phase-rate microkernel's factors per second, less its
    harness), and a phase difference one flop more; tau its TAU_FLOPS (FP64
    operations, counted twice in the FP32 mode); applying a
    factor to a complex value 6 flops (complex multiply) or 8 (complex
    multiply-add, row space and switch); a real x complex multiply-add 4 (the
    tensor-form interpolation, Sec. 1.4)."""
    r, P = q ** d, N ** d
    tf = TAU_FLOPS[phase](d) * FP64_WEIGHT[prec]
    macs = P * tensor_macs(d, q) * nrhs * 4

    def cost(kind, apply_flops, diff):
        n_cs, n_tau, n_app = evaluated(kind, prec, phase, d, q, adjoint)
        return P * (n_cs * (c_cs + diff) + n_tau * tf + n_app * nrhs * apply_flops)

    evals_init = n_src + P * r
    return {
        "col": cost("col", 6, 0) + macs,
        "row": cost("row", 8, 1) + macs,
        "switch": cost("switch", 8, 1),
        "init": evals_init * (c_cs + tf) + evals_init * nrhs * 6 + n_src * r * nrhs * 4,
        "final": n_tgt * (c_cs + tf) + n_tgt * r * nrhs * 4 + n_tgt * nrhs * 6,
    }


def kind_flops(kind: str, t: dict, fm: dict) -> float:
    """Flops of all launches of one kind, from the work counts the library
    reports for them (stages, initialisations, switches, launches)."""
    if kind == "first":
        return t["stages"] * fm["col"] + t["inits"] * fm["init"] + t["switches"] * fm["switch"]
    if kind == "second":
        return t["stages"] * fm["row"]
    if kind == "final":
        return t["launches"] * fm["final"]
    return 0.0


def measure_phase_cost(torch, P, dev) -> dict:
    """Factors per second of the phase-rate microkernel (the kernels' own
    reduction and sine/cosine) in each precision, and the per-factor cost in
    flops at the VALU peak."""
    from paper_1305_4650_amd import bfly as B
    n, iters = 256 * 1024 * 4, 256
    out = torch.empty(n, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()
    res = {}
    for prec, pid in (("fp64", B.BFLY_FP64), ("fp32", B.BFLY_FP32)):
        def run():
            B.bfly_phase_rate(pid, n, iters, 2048.0, out.data_ptr(), stream.cuda_stream)
        run()
        torch.cuda.synchronize()
        ms = time_steps(run, torch, 10, 2)
        rate = n * iters / (ms * 1e-3)
        res[prec] = {"factors_per_s": rate, "ms": round(ms, 4),
                     "c_cs_flops": round(PEAK_TFLOPS[prec] * 1e12 / rate - PHASE_RATE_HARNESS_FLOPS[prec], 2)}
        print(f"[bench] phase rate {prec}: {rate / 1e9:.0f} G factors/s -> c_cs = "
              f"{res[prec]['c_cs_flops']:.1f} flops per sine/cosine pair", file=sys.stderr, flush=True)
    return res


def measure_contraction_units(torch, P, dev) -> dict:
    """FP32 multiply-add rates of the two contraction units (VALU v_fma_f32,
    matrix cores v_mfma_f32_4x4x1_16b_f32), alone and interleaved in one
    instruction stream: the measured basis of running the interpolation
    contractions on the VALU."""
    from paper_1305_4650_amd import bfly as B
    n, iters = 256 * 1024 * 2, 2048
    out = torch.empty(n, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    waves = n // 64
    macs = {0: 32 * 64, 1: 8 * 256, 2: 32 * 64 + 8 * 256}  # per wave per iteration
    res = {}
    for unit, name in ((0, "valu_fma_f32"), (1, "mfma_4x4x1_f32"), (2, "both_interleaved")):
        ms = time_steps(lambda: B.bfly_contraction_rate(unit, n, iters, out.data_ptr(), stream.cuda_stream), torch,
                        5, 1)
        res[name] = {"ms": round(ms, 4), "tflops": round(2 * macs[unit] * waves * iters / (ms * 1e-3) / 1e12, 2)}
    res["interleaved_over_sum_of_alone"] = round(res["both_interleaved"]["ms"] / (res["valu_fma_f32"]["ms"]
                                                                                 + res["mfma_4x4x1_f32"]["ms"]), 3)
    print(f"[bench] contraction units: VALU {res['valu_fma_f32']['tflops']} TFLOP/s, MFMA 4x4x1 "
          f"{res['mfma_4x4x1_f32']['tflops']} TFLOP/s, interleaved / sum of alone "
          f"{res['interleaved_over_sum_of_alone']}", file=sys.stderr, flush=True)
    return res


def kernel_sources_sha256() -> str:
    """Hash of the device-code sources (.hip, .inc, .h under csrc/): the
    counter summary is valid while they are unchanged (host-only .cpp files
    do not affect the kernels' traffic)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".inc", ".h")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + fh.read())
    return h.hexdigest()


def traffic_per_launch(kernel_family: str, prec: str):
    """HBM bytes per launch of a kernel family in one precision from the
    committed counter summary, or None if the kernel sources changed since it
    was taken."""
    path = os.path.join(ROOT, "profiles", "c2_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    fam = rec.get("kernels", {}).get(f"{kernel_family} {prec}")
    return None if fam is None else fam.get("hbm_bytes_per_launch")


TRAFFIC_BENCH = ("python3 bench.py --steps 2 --warmup 1 --no-tune --no-cpu-baseline --no-c5 --no-c4 --no-3d "
                 "--no-sparse --no-c1 --no-adjoint --no-rhs")


def summarize_traffic(d: str) -> int:
    """Write profiles/c2_hbm_traffic.json from four rocprofv3 counter runs
    under d: fetch/ and write/ (FETCH_SIZE, WRITE_SIZE of the C2 bench legs,
    TRAFFIC_BENCH) and copy_fetch/, copy_write/ (the same counters of
    --copy-calibration).  The counters are KiB per dispatch; each is scaled
    by what it reads for the plain 1 GiB copy, and the level kernels' values
    are averaged per kernel family and precision."""
    import csv
    import glob
    import re

    def rows(sub):
        paths = glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True)
        if len(paths) != 1:
            raise SystemExit(f"expected one counter_collection.csv under {os.path.join(d, sub)}, found {len(paths)}")
        with open(paths[0]) as fh:
            return list(csv.DictReader(fh))

    def per_dispatch(sub, counter):
        out = {}
        for r in rows(sub):
            if r["Counter_Name"] == counter:
                out.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        return out

    def copy_kib(sub, counter):
        vals = [v for name, v in per_dispatch(sub, counter).values() if "copy" in name.lower()]
        if not vals:
            raise SystemExit(f"no copy kernel in {sub}")
        return max(vals)

    copy_bytes = 1 << 30
    fk, wk = copy_kib("copy_fetch", "FETCH_SIZE"), copy_kib("copy_write", "WRITE_SIZE")
    ff, wf = copy_bytes / (fk * 1024.0), copy_bytes / (wk * 1024.0)
    fetch, write = per_dispatch("fetch", "FETCH_SIZE"), per_dispatch("write", "WRITE_SIZE")
    fams = {}
    for table, key in ((fetch, "fetch"), (write, "write")):
        for name, v in table.values():
            m = re.search(r"\b(k_first|k_second|k_final)<\d+, \d+, (float|double),", name)
            if m:
                fam = f"{m.group(1)} {'fp64' if m.group(2) == 'double' else 'fp32'}"
                fams.setdefault(fam, {"fetch": [], "write": []})[key].append(v)
    kernels = {}
    for fam, v in sorted(fams.items()):
        f, w_ = float(np.mean(v["fetch"])), float(np.mean(v["write"]))
        kernels[fam] = {"fetch_kib_raw_per_launch": round(f, 1), "write_kib_raw_per_launch": round(w_, 1),
                        "hbm_bytes_per_launch": int(round((f * ff + w_ * wf) * 1024)),
                        "launches_sampled": min(len(v["fetch"]), len(v["write"]))}
    rec = {"what": "HBM bytes per launch of the level kernels on the C2 workload (2-D hyperbolic Radon, N=1024, "
                   "q=5, 1 RHS, built-in launch shapes), from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per "
                   f"dispatch) scaled by a 1 GiB plain device copy: fetch factor {ff:.4f}, write factor {wf:.4f}.",
           "commands": ["cd /tmp && export TMPDIR=/tmp",
                        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <d>/fetch -o c2 -- {TRAFFIC_BENCH}",
                        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <d>/write -o c2 -- {TRAFFIC_BENCH}",
                        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <d>/copy_fetch -o copy -- "
                        "python3 bench.py --copy-calibration",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <d>/copy_write -o copy -- "
                        "python3 bench.py --copy-calibration",
                        "python3 bench.py --summarize-traffic <d>"],
           "copy_calibration": {"bytes_copied": copy_bytes, "fetch_kib_raw": fk, "write_kib_raw": wk,
                                "fetch_factor": ff, "write_factor": wf},
           "source_sha256": kernel_sources_sha256(), "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "c2_hbm_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(kernels, indent=1))
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


def time_each(fn, torch, n: int) -> dict:
    """n applies timed one by one with HIP events on the current stream:
    median and interquartile range in ms."""
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    q1, med, q3 = np.percentile(t, [25, 50, 75])
    return {"n": n, "median_ms": round(float(med), 4), "iqr_ms": round(float(q3 - q1), 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure_c5(torch, P, W, dev, steps: int, warmup: int, tune: bool = True) -> dict:
    """The uneven batch: 48 hyperbolic-Radon instances (N from {128, 256,
    512, 1024}, q = 5, 8 right-hand sides) in one batched apply, eagerly and
    as a replayed HIP graph, against the 48 applies issued one after another."""
    t0 = time.time()
    sizes = W.C5_sizes()
    plans = {int(N): P.Plan(2, int(N), ([1.0, 0.0], [2.0, 1.0]), ([0.0, 0.0], [1.0, 1.0]), "hypradon2", 5)
             for N in set(sizes.tolist())}
    items = []
    for i, N in enumerate(sizes):
        w = W.C5_instance(i, int(N))
        items.append((plans[int(N)], False, torch.from_numpy(w.y).to(dev), torch.from_numpy(w.g).to(dev),
                      torch.from_numpy(w.x).to(dev)))
    pts = int(sum(int(N) ** 2 for N in sizes)) * 8
    print(f"[bench] C5: {len(items)} instances, {pts // 8} points x 8 rhs ({time.time() - t0:.1f}s to generate)",
          file=sys.stderr, flush=True)
    out = {"workload": "48 hyperbolic-Radon instances, N drawn from {128,256,512,1024}, q=5, 8 right-hand sides",
           "instances": len(items), "points_x_rhs": pts, "unit": "Mpoints/s"}
    for prec in ("fp32", "fp64"):
        if tune:  # one tuning per distinct N (the instances of one N share the key)
            t0 = time.time()
            done = set()
            for (plan, _, y, g, x) in items:
                if plan.N not in done:
                    done.add(plan.N)
                    plan.tune(y, g, x, prec)
            torch.cuda.synchronize()
            out[f"tune_s_{prec}"] = round(time.time() - t0, 2)
        batch = P.Batch(items, prec)
        ms_b = time_steps(batch.run, torch, steps, warmup)
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            batch.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            batch.run()
        ms_g = time_steps(graph.replay, torch, steps, warmup)
        singles = []
        for (plan, _, y, g, x) in items:
            ws = plan.workspace(y.shape[0], g.shape[0], prec, device=dev)
            singles.append((plan, y, g, x, torch.empty_like(g), ws))

        def seq():
            for plan, y, g, x, f, ws in singles:
                plan.apply(y, g, x, prec, out=f, workspace=ws)

        ms_s = time_steps(seq, torch, steps, warmup)
        out[prec] = {"batched_ms": round(ms_b, 3), "graph_ms": round(ms_g, 3), "sequential_ms": round(ms_s, 3),
                     "value": round(pts / ms_g / 1e3, 3)}
        print(f"[bench] C5 {prec}: batched {ms_b:.2f} ms, graph {ms_g:.2f} ms, 48 single applies {ms_s:.2f} ms "
              f"-> {pts / ms_g / 1e3:.1f} Mpoints/s", file=sys.stderr, flush=True)
        del batch, graph, singles
        torch.cuda.empty_cache()
    return out


def measure_c4(torch, P, W, dev, nrhs: int = 0) -> dict:
    """The many-right-hand-side Fourier configuration: d = 2, N = 2048, q = 6,
    64 right-hand sides (nrhs > 0: only that many, for profiling runs), one
    apply per precision (after one warm-up)."""
    t0 = time.time()
    w = W.C4()
    if nrhs > 0:
        w.g = np.ascontiguousarray(w.g[:nrhs])
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(a).to(dev) for a in (w.y, w.x, w.g))
    pts = w.N ** 2 * w.nrhs
    print(f"[bench] C4: {w.N ** 2} points x {w.nrhs} rhs ({time.time() - t0:.1f}s to generate)", file=sys.stderr,
          flush=True)
    out = {"workload": "Fourier phase on uniform grids, d=2, N=2048, q=6 (r=36), 64 right-hand sides",
           "points_x_rhs": pts, "unit": "Mpoints/s"}
    for prec in ("fp32", "fp64"):
        ws = plan.workspace(w.y.shape[0], w.nrhs, prec, device=dev)
        f = torch.empty_like(g)
        ms = time_steps(lambda: plan.apply(y, g, x, prec, out=f, workspace=ws), torch, 1, 1)
        out[prec] = {"ms": round(ms, 2), "value": round(pts / ms / 1e3, 3)}
        print(f"[bench] C4 {prec}: {ms:.1f} ms -> {pts / ms / 1e3:.1f} Mpoints/s", file=sys.stderr, flush=True)
        del ws, f
        torch.cuda.empty_cache()
    return out


def measure_c1(torch, P, W, dev, steps: int) -> dict:
    """The small Fourier configuration (d = 2, N = 64, q = 5, 4096 points):
    launch-latency bound, so it is timed eagerly and as a captured HIP graph
    replayed steps times."""
    w = W.C1()
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(a).to(dev) for a in (w.y, w.x, w.g))
    out = {"workload": "C1: Fourier phase on uniform grids, d=2, N=64, q=5 (r=25), 4096 points, 1 RHS",
           "unit": "us per apply"}
    for prec in ("fp32", "fp64"):
        ws = plan.workspace(w.y.shape[0], w.nrhs, prec, device=dev)
        f = torch.empty((w.nrhs, w.x.shape[0]), dtype=torch.complex128, device=dev)

        def run():
            plan.apply(y, g, x, prec, out=f, workspace=ws)

        eager = time_steps(run, torch, steps, 5)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            run()
        replay = time_steps(graph.replay, torch, steps, 5)
        out[prec] = {"eager_us": round(eager * 1e3, 1), "graph_us": round(replay * 1e3, 1)}
        print(f"[bench] C1 {prec}: eager {eager * 1e3:.1f} us, graph {replay * 1e3:.1f} us per apply",
              file=sys.stderr, flush=True)
    return out


def measure_sparse(torch, P, W, dev, steps: int) -> dict:
    """Sparse sets in the C2 geometry (N = 1024, q = 5): 4096 sources on a
    curve with all 1,048,576 grid targets, and 4096 targets on the curve with
    all 1,048,576 jittered sources.  Blocks whose source boxes hold no point
    or whose target boxes hold no target skip their work; reported as time
    per apply (the dense C2 apply is the comparison)."""
    out = {"unit": "ms per apply"}
    for key, w, what in (
            ("sources_on_curve", W.hypradon2_curve(1024, q=5),
             "4096 sources on the curve y = (1+u, 0.5+0.4 sin 2 pi u), 1,048,576 grid targets"),
            ("targets_on_curve", W.hypradon2_curve(1024, q=5, curve_targets=True),
             "1,048,576 jittered sources, 4096 targets on the curve x = (u, 0.5+0.4 sin 2 pi u)")):
        plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
        y, x, g = (torch.from_numpy(a).to(dev) for a in (w.y, w.x, w.g))
        rec = {"workload": "C2 geometry, N=1024, q=5, 1 right-hand side: " + what}
        for prec in ("fp32", "fp64"):
            ws = plan.workspace(w.y.shape[0], w.nrhs, prec, device=dev)
            f = torch.empty((w.nrhs, w.x.shape[0]), dtype=torch.complex128, device=dev)
            ms = time_steps(lambda: plan.apply(y, g, x, prec, out=f, workspace=ws), torch, steps, 2)
            rec[prec] = {"ms": round(ms, 4)}
            print(f"[bench] sparse {key} {prec}: {ms:.3f} ms/apply", file=sys.stderr, flush=True)
        out[key] = rec
    return out


def measure_adjoint(torch, P, w, plan, dev, steps: int, cores) -> dict:
    """The adjoint apply g = B' f of the C2 plan (targets in, sources out,
    phase negated, switch at L - L/2), with f = the C2 input values placed on
    the 1,048,576 targets.  Timed per precision; with the oracle enabled, its
    FP64 adjoint butterfly gives the relative errors."""
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    fin = torch.from_numpy(w.g).to(dev)  # (nrhs, n_tgt): n_tgt = n_src in C2
    out = {"workload": "C2 adjoint: f on the 1,048,576 grid targets -> g at the 1,048,576 jittered sources, "
                       "N=1024, q=5, 1 right-hand side", "unit": "Mpoints/s"}
    npts = w.N ** w.d * w.nrhs
    got = {}
    for prec in ("fp32", "fp64"):
        ws = plan.workspace(w.x.shape[0], w.nrhs, prec, device=dev)
        g = torch.empty((w.nrhs, w.y.shape[0]), dtype=torch.complex128, device=dev)
        ms = time_steps(lambda: plan.apply_adjoint(x, fin, y, prec, out=g, workspace=ws), torch, steps, 2)
        got[prec] = g.cpu().numpy()
        out[prec] = {"ms": round(ms, 4), "value": round(npts / ms / 1e3, 3)}
        print(f"[bench] adjoint {prec}: {ms:.3f} ms/apply  {npts / ms / 1e3:.1f} Mpoints/s", file=sys.stderr,
              flush=True)
        del ws
    if cores:
        import oracle
        ref = oracle.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.x, w.g, w.y, adjoint=True,
                               nthreads=cores)
        for prec in got:
            out[prec]["rel_err_vs_oracle"] = rel(got[prec], ref)
        print(f"[bench] adjoint rel err vs oracle: fp64 {out['fp64']['rel_err_vs_oracle']:.2e} "
              f"fp32 {out['fp32']['rel_err_vs_oracle']:.2e}", file=sys.stderr, flush=True)
    return out


def measure_rhs(torch, P, W, dev, steps: int, tune: bool = True) -> dict:
    """The C2 geometry with 8 right-hand sides in one apply (chunks of 2
    share their phase factors), timed with events; reported per right-hand
    side."""
    w = W.hypradon2(1024, q=5, nrhs=8)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(a).to(dev) for a in (w.y, w.x, w.g))
    pts = w.N ** w.d * w.nrhs
    out = {"workload": "C2 geometry (2-D hyperbolic Radon, N=1024, q=5), 8 right-hand sides in one apply",
           "unit": "Mpoints/s"}
    for prec in ("fp32", "fp64"):
        ws = plan.workspace(w.y.shape[0], w.nrhs, prec, device=dev)
        f = torch.empty((w.nrhs, w.x.shape[0]), dtype=torch.complex128, device=dev)
        ms_b = time_steps(lambda: plan.apply(y, g, x, prec, out=f, workspace=ws), torch, steps, 2)
        if tune:
            plan.tune(y, g, x, prec, out=f, workspace=ws)
        ms = time_steps(lambda: plan.apply(y, g, x, prec, out=f, workspace=ws), torch, steps, 2)
        out[prec] = {"ms": round(ms, 3), "ms_per_rhs": round(ms / w.nrhs, 4), "value": round(pts / ms / 1e3, 3),
                     "builtin_shapes_ms": round(ms_b, 3)}
        print(f"[bench] C2 8 rhs {prec}: {ms:.2f} ms ({ms / w.nrhs:.3f} ms per rhs) -> {pts / ms / 1e3:.1f} Mpoints/s",
              file=sys.stderr, flush=True)
        del ws
    return out


def measure_3d(torch, P, W, dev, steps: int) -> dict:
    """The 3-D generalized-Radon configurations: the workload form (N = 64,
    q = 4, r = 64) and the phase as printed (N = 64, q = 5, r = 125), one
    right-hand side, timed per precision over a few applies."""
    out = {"unit": "Mpoints/s"}
    for key, w, what in (
            ("c3_genradon3", W.C3(), "3-D generalized-Radon analogue N (x.y + sqrt(...)), N=64, q=4 (r=64)"),
            ("genradon3pi", W.genradon3pi(64, q=5), "3-D generalized Radon as printed, pi (x.p + sqrt(...)), "
                                                     "N=64, q=5 (r=125), p in [-32, 32)^3")):
        plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
        y, x, g = (torch.from_numpy(a).to(dev) for a in (w.y, w.x, w.g))
        pts = w.N ** 3 * w.nrhs
        rec = {"workload": what, "points": pts}
        for prec in ("fp32", "fp64"):
            ws = plan.workspace(w.y.shape[0], w.nrhs, prec, device=dev)
            f = torch.empty_like(g)
            ms = time_steps(lambda: plan.apply(y, g, x, prec, out=f, workspace=ws), torch, steps, 2)
            rec[prec] = {"ms": round(ms, 3), "value": round(pts / ms / 1e3, 3)}
            print(f"[bench] {key} {prec}: {ms:.2f} ms -> {pts / ms / 1e3:.1f} Mpoints/s", file=sys.stderr,
                  flush=True)
        out[key] = rec
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (no rel err either)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (default: all in affinity)")
    ap.add_argument("--no-c5", action="store_true", help="skip the batched 48-instance measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the 64-right-hand-side Fourier measurement")
    ap.add_argument("--c4-rhs", type=int, default=0, help="C4 with only this many right-hand sides (profiling)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D generalized-Radon measurements")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse source / target measurements")
    ap.add_argument("--no-c1", action="store_true", help="skip the small (launch-bound) Fourier measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the C2 adjoint measurement")
    ap.add_argument("--no-rhs", action="store_true", help="skip the C2 8-right-hand-side measurement")
    ap.add_argument("--no-tune", action="store_true", help="time the built-in launch shapes only (no autotuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one plain device copy of 1 GiB (scales the HBM byte counters)")
    ap.add_argument("--summarize-traffic", metavar="DIR",
                    help="only write profiles/c2_hbm_traffic.json from the rocprofv3 counter runs under DIR")
    args = ap.parse_args()
    if args.summarize_traffic:
        return summarize_traffic(args.summarize_traffic)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return 0
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (got --gpus {args.gpus}); "
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

    phase_cost = measure_phase_cost(torch, P, dev)
    units = measure_contraction_units(torch, P, dev)
    P.bfly_tune_reset()
    res = {}
    for prec in ("fp64", "fp32"):
        ws = plan.workspace(n, w.nrhs, prec, device=dev)
        f = torch.empty((w.nrhs, w.x.shape[0]), dtype=torch.complex128, device=dev)

        def step():
            plan.apply(y, g, x, prec, out=f, workspace=ws)

        # built-in launch shapes, then the autotuner's (its time is not in the timed region)
        ms_builtin = time_steps(step, torch, args.steps, args.warmup)
        tune_s = None
        if not args.no_tune:
            t0 = time.time()
            plan.tune(y, g, x, prec, out=f, workspace=ws)
            torch.cuda.synchronize()
            tune_s = time.time() - t0
        ms = time_steps(step, torch, args.steps, args.warmup)
        dist = time_each(step, torch, 20)
        # instrumented pass: per-step-kind HIP event timing on the apply's stream
        P.bfly_timing_enable(True)
        P.bfly_timing_read()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        tim = P.bfly_timing_read()
        recs = P.bfly_timing_launches()
        P.bfly_timing_enable(False)
        one = []  # the launches of the first instrumented apply
        for rec in recs:
            one.append(rec)
            if rec["kind"] == "final":
                break
        res[prec] = {"ms": ms, "out": f.cpu().numpy(), "timing": tim, "dist": dist, "launches": one,
                     "builtin_ms": ms_builtin, "tune_s": tune_s}
        print(f"[bench] {prec}: {ms:.3f} ms/apply  {npts / ms / 1e3:.1f} Mpoints/s (built-in shapes {ms_builtin:.3f} ms) "
              + " ".join(f"{k}={v['ms'] / args.steps:.3f}ms/{v['launches'] // args.steps}"
                         for k, v in tim.items()), file=sys.stderr, flush=True)
        del ws

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = args.cpu_threads or len(os.sched_getaffinity(0))
        runs = []
        for _ in range(3):
            t0 = time.time()
            ref = oracle.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x, nthreads=cores)
            runs.append(time.time() - t0)
        t_cpu = float(np.median(runs))
        # one thread on a smaller sample of the same geometry (N = 256)
        ws1 = W.hypradon2(256, q=w.q, config_id=2)
        t0 = time.time()
        oracle.butterfly(ws1.phase, ws1.N, ws1.q, ws1.src_box, ws1.tgt_box, ws1.y, ws1.g, ws1.x, nthreads=1)
        t_one = time.time() - t0
        cpu = {"value": npts / t_cpu / 1e6, "unit": "Mpoints/s", "cores": cores, "kind": "oracle",
               "sample": "the full workload: FP64 oracle butterfly applies of all 1,048,576 sources and targets, "
                         f"median of 3 ({', '.join(f'{t:.1f}' for t in runs)} s)",
               "cpu_model": cpu_model(),
               "single_thread": {"value": round(ws1.N ** 2 / t_one / 1e6, 4), "unit": "Mpoints/s",
                                 "sample": f"same geometry at N = 256 (65,536 points), 1 thread ({t_one:.1f} s)"}}
        for prec in res:
            res[prec]["rel_err"] = rel(res[prec]["out"], ref)
        print(f"[bench] oracle {t_cpu:.1f}s on {cores} threads; rel err fp64 "
              f"{res['fp64']['rel_err']:.2e} fp32 {res['fp32']['rel_err']:.2e}", file=sys.stderr, flush=True)

    adj = None if args.no_adjoint else measure_adjoint(
        torch, P, w, plan, dev, 10, None if args.no_cpu_baseline else (args.cpu_threads or len(os.sched_getaffinity(0))))
    rhs8 = None if args.no_rhs else measure_rhs(torch, P, W, dev, 10, not args.no_tune)
    c5 = None if args.no_c5 else measure_c5(torch, P, W, dev, max(3, args.steps // 4), 1, not args.no_tune)
    c4 = None if args.no_c4 else measure_c4(torch, P, W, dev, args.c4_rhs)
    r3d = None if args.no_3d else measure_3d(torch, P, W, dev, 5)
    sparse = None if args.no_sparse else measure_sparse(torch, P, W, dev, 10)
    c1 = None if args.no_c1 else measure_c1(torch, P, W, dev, 200)

    def roofline_for(prec: str) -> dict:
        """The dominant launch kind's algorithmic flops per launch over its
        average event-timed duration, every launch of one apply beside it,
        and the whole apply."""
        tim = res[prec]["timing"]
        fm = flop_model(prec, phase_cost[prec]["c_cs_flops"], w.phase, w.d, w.N, w.q, w.nrhs, n, w.x.shape[0])
        dom = max(tim, key=lambda k: tim[k]["ms"])
        launches = max(tim[dom]["launches"], 1)
        avg_ms = tim[dom]["ms"] / launches
        flops = kind_flops(dom, tim[dom], fm) / launches
        achieved = flops / (avg_ms * 1e-3) / 1e12
        fam = {"first": "k_first", "second": "k_second", "final": "k_final"}.get(dom, dom)
        per = []
        for rec in res[prec]["launches"]:
            fl = kind_flops(rec["kind"], dict(rec, launches=1), fm)
            per.append({"kind": rec["kind"], "stages": rec["stages"], "init": rec["inits"],
                        "switch": rec["switches"], "ms": round(rec["ms"], 4),
                        "frac": round(fl / (rec["ms"] * 1e-3) / 1e12 / PEAK_TFLOPS[prec], 4) if fl else None})
        total_flops = sum(kind_flops(k, tim[k], fm) for k in tim)
        total_s = sum(t["ms"] for t in tim.values()) * 1e-3
        traffic = traffic_per_launch(fam, prec)
        # the other roofline of the same launches: measured HBM bytes per
        # launch over their duration, against the 8 TB/s peak
        hbm = None if traffic is None else traffic / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[prec], 4), "traffic": traffic,
                "hbm_tb_per_s": None if hbm is None else round(hbm, 3),
                "hbm_frac": None if hbm is None else round(hbm / HBM_PEAK_TBPS, 4),
                "kernel": fam, "avg_launch_ms": round(avg_ms, 5), "algorithmic_flops_per_launch": round(flops),
                "c_cs_flops": phase_cost[prec]["c_cs_flops"], "launches_of_one_apply": per,
                "apply": {"achieved": round(total_flops / total_s / 1e12, 3),
                          "frac": round(total_flops / total_s / 1e12 / PEAK_TFLOPS[prec], 4),
                          "algorithmic_flops_per_apply": round(total_flops / args.steps)}}

    head = "fp64"
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C2: 2-D hyperbolic-Radon phase N*x0*sqrt(y0^2+x1^2*y1^2), N=1024, q=5 (r=25), "
                               "1,048,576 jittered sources in [1,2)x[0,1), 1,048,576 grid targets in [0,1)^2, "
                               "1 right-hand side",
                   "d": w.d, "N": w.N, "q": w.q, "nrhs": w.nrhs, "prec": head,
                   "contraction_unit": "valu"},
        "rel_err_vs_oracle": res[head].get("rel_err"),
        "per_apply": res[head]["dist"],
        "launch_shapes": "autotuned (bfly_tune) before timing" if not args.no_tune else "built-in",
        "builtin_shapes_ms": round(res[head]["builtin_ms"], 4),
        "tune_s": res[head]["tune_s"],
        "roofline": roofline_for("fp64"),
        "fp32": {"value": round(npts / res["fp32"]["ms"] / 1e3, 3), "ms_per_step": round(res["fp32"]["ms"], 4),
                 "rel_err_vs_oracle": res["fp32"].get("rel_err"), "per_apply": res["fp32"]["dist"],
                 "builtin_shapes_ms": round(res["fp32"]["builtin_ms"], 4), "tune_s": res["fp32"]["tune_s"],
                 "roofline": roofline_for("fp32")},
        "speedup_fp32_over_fp64": round(res["fp64"]["ms"] / res["fp32"]["ms"], 3),
        "launch_ms": {p: {k: round(v["ms"] / args.steps, 5) for k, v in res[p]["timing"].items()} for p in res},
        "phase_rate": phase_cost,
        "contraction_units": units,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "c2_8rhs": rhs8,
        "c5_batched": c5,
        "c4_many_rhs": c4,
        "genradon_3d": r3d,
        "sparse_sets": sparse,
        "c1_small": c1,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
