"""CPU checks of the benchmark's contract that need no GPU: a run on more
than one GPU is refused with one JSON line, the percentile helper, and the
rule that counter traffic is reported only for the kernel sources it was
measured on."""
import json
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_percentiles():
    import bench
    xs = np.random.Generator(np.random.PCG64(3)).permutation(np.arange(1, 102, dtype=np.float64))
    assert bench.pct(xs, 50) == 51.0
    assert bench.pct(xs, 0) == 1.0 and bench.pct(xs, 100) == 101.0
    assert bench.pct(xs, 99) == 100.0


def test_traffic_only_for_the_measured_sources(monkeypatch):
    import bench
    with open(bench.TRAFFIC_PROFILE) as fh:
        d = json.loads(re.search(r"```json\n(.*?)\n```", fh.read(), re.S).group(1))
    names = list(d["kernels"])
    want = sum(float(d["kernels"][k]["traffic_bytes_per_launch"]) for k in names)
    monkeypatch.setattr(bench, "edt_source_hash", lambda: d["source_sha256"])
    assert bench.measured_traffic(names) == want
    assert bench.measured_traffic(names + ["no_such_kernel"]) is None
    monkeypatch.setattr(bench, "edt_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(names) is None
