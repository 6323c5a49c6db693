"""The autotuner (bfly_tune): every candidate shape computes the same result,
so the tuned apply equals the built-in one bit for bit; the recorded shapes
are what later applies launch (checked through the per-launch timing
records); the JSON cache named by BFLY_TUNE_CACHE carries them to a fresh
process."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _launch_split(P, run):
    """Stages per launch of the level launches of one apply."""
    P.bfly_timing_enable(True)
    P.bfly_timing_read()
    run()
    P.bfly_timing_read()
    recs = P.bfly_timing_launches()
    P.bfly_timing_enable(False)
    return [r["stages"] for r in recs if r["kind"] in ("first", "second")]


@pytest.mark.parametrize("prec, nrhs", [("fp64", 1), ("fp32", 1), ("fp32", 4)])
def test_tuned_apply_equals_builtin_and_is_used(prec, nrhs):
    import torch
    import paper_1305_4650_amd as P
    P.bfly_tune_reset()
    w = W.hypradon2(128, q=5, nrhs=nrhs)
    print(f"[case] tune {prec} nrhs={nrhs}", flush=True)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = _dev(torch, w.y), _dev(torch, w.x), _dev(torch, w.g)
    ref = plan.apply(y, g, x, prec)
    torch.cuda.synchronize()
    builtin = _launch_split(P, lambda: plan.apply(y, g, x, prec))
    out, ms = plan.tune(y, g, x, prec)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(out, ref)
    after = plan.apply(y, g, x, prec)
    torch.cuda.synchronize()
    assert torch.equal(after, ref)
    tuned = _launch_split(P, lambda: plan.apply(y, g, x, prec))
    print(f"  built-in launches {builtin}, tuned {tuned}, {ms:.3f} ms", flush=True)
    assert sum(tuned) == sum(builtin)
    P.bfly_tune_reset()
    assert _launch_split(P, lambda: plan.apply(y, g, x, prec)) == builtin


def test_tune_cache_file_is_read_by_a_fresh_process(tmp_path):
    import torch
    import paper_1305_4650_amd as P
    cache = str(tmp_path / "tune.json")
    os.environ["BFLY_TUNE_CACHE"] = cache
    try:
        P.bfly_tune_reset()
        w = W.hypradon2(64, q=5, nrhs=1)
        plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
        y, x, g = _dev(torch, w.y), _dev(torch, w.x), _dev(torch, w.g)
        print("[case] tune cache write", flush=True)
        plan.tune(y, g, x, "fp64")
        torch.cuda.synchronize()
        rec = json.load(open(cache))["records"]
        assert len(rec) == 1 and rec[0]["log2N"] == 6 and rec[0]["q"] == 5 and rec[0]["prec"] == 0
        tuned = _launch_split(P, lambda: plan.apply(y, g, x, "fp64"))
    finally:
        del os.environ["BFLY_TUNE_CACHE"]
        P.bfly_tune_reset()
    # a fresh process with the cache set launches the recorded shapes
    code = (
        "import sys, json, numpy as np, torch; sys.path.insert(0, %r)\n"
        "import paper_1305_4650_amd as P\n"
        "from paper_1305_4650_amd import workloads as W\n"
        "w = W.hypradon2(64, q=5, nrhs=1)\n"
        "plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)\n"
        "y, x, g = (torch.from_numpy(a).cuda() for a in (w.y, w.x, w.g))\n"
        "P.bfly_timing_enable(True); P.bfly_timing_read(); plan.apply(y, g, x, 'fp64'); P.bfly_timing_read()\n"
        "print(json.dumps([r['stages'] for r in P.bfly_timing_launches() if r['kind'] in ('first', 'second')]))\n"
    ) % ROOT
    print("[case] tune cache read in a fresh process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, BFLY_TUNE_CACHE=cache),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert json.loads(r.stdout.strip().splitlines()[-1]) == tuned
