"""Launch shapes do not change results.

A block's shape (fusion units per workgroup, threads, stages per launch)
decides which jobs share a wavefront and which lines the half-in-place
tensor passes overwrite while others read them; every shape must still give
the same result bit for bit, because each line takes the same operations in
the same order.  A fresh process applies the 2-D hyperbolic-Radon workload
(N = 128, q = 5: three column-space and four row-space stages) with launch
shapes forced through the tuning overrides BFLY_UB and BFLY_KSPLIT, which
are read once per process, and this process compares its outputs with the
built-in shapes' (one right-hand side, and three: a chunk of two plus one).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1305_4650_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import sys, json, numpy as np, torch
sys.path.insert(0, {root!r})
import paper_1305_4650_amd as P
from paper_1305_4650_amd import workloads as W
out = {{}}
splits = {{}}
for nrhs in (1, 3):
    w = W.hypradon2(128, q=5, nrhs=nrhs)
    plan = P.Plan(w.d, w.N, w.src_box, w.tgt_box, w.phase, w.q)
    y, x, g = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w.y, w.x, w.g))
    for prec in ("fp64", "fp32"):
        P.bfly_timing_enable(True); P.bfly_timing_read()
        f = plan.apply(y, g, x, prec)
        torch.cuda.synchronize(); P.bfly_timing_read()
        splits[f"{{prec}} {{nrhs}}"] = [r["stages"] for r in P.bfly_timing_launches() if r["kind"] in ("first", "second")]
        P.bfly_timing_enable(False)
        b = plan.apply_adjoint(x, f, y, prec)
        torch.cuda.synchronize()
        out[f"{{prec}} {{nrhs}} fwd"] = f.cpu().numpy()
        out[f"{{prec}} {{nrhs}} adj"] = b.cpu().numpy()
np.savez({path!r}, **out)
print(json.dumps(splits))
"""

OVERRIDES = [
    {"BFLY_UB": "1"},
    {"BFLY_UB": "2"},
    {"BFLY_UB": "5"},
    {"BFLY_KSPLIT": "1,2,2,2"},
    {"BFLY_KSPLIT": "3,1,3"},
    {"BFLY_KSPLIT": "2,1,3,1", "BFLY_UB": "3"},
]


def _run(tmp_path, env_extra, tag):
    path = str(tmp_path / f"{tag}.npz")
    env = {k: v for k, v in os.environ.items() if not k.startswith("BFLY_")}
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", CODE.format(root=ROOT, path=path)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    splits = json.loads(r.stdout.strip().splitlines()[-1])
    data = np.load(path)
    return {k: data[k] for k in data.files}, splits


@pytest.mark.timeout(900)
def test_forced_shapes_give_identical_results(tmp_path):
    print("[case] built-in shapes, N = 128, q = 5, 1 and 3 rhs, both directions", flush=True)
    ref, ref_splits = _run(tmp_path, {}, "builtin")
    print(f"  built-in launch splits {ref_splits}", flush=True)
    for i, ov in enumerate(OVERRIDES):
        print(f"[case] forced shapes {ov}", flush=True)
        got, splits = _run(tmp_path, ov, f"forced{i}")
        print(f"  launch splits {splits}", flush=True)
        if "BFLY_KSPLIT" in ov:
            want = [int(k) for k in ov["BFLY_KSPLIT"].split(",")]
            # FP32 fits every split; FP64 at least those of up to 3 stages
            assert splits["fp32 1"] == want
            assert splits["fp64 1"] == want
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (ov, k)
