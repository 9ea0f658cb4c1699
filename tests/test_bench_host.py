"""Host-side pieces of bench.py, CPU only: the profiled-traffic lookup reads
every committed profile summary without error, and the command line refuses
more than one GPU before it touches a device."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_profile_records_parse(bench):
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        for block in re.findall(r"```json\n(.*?)\n```", text, re.S):
            rec = json.loads(block)
            if "kernels" in rec:          # one record per kernel of the run
                assert rec["kernels"] and all("avg_us" in k for k in rec["kernels"].values()), name
            else:
                assert "kernel" in rec and "avg_us" in rec, name


@pytest.mark.parametrize("workload", ["gauss3_8d", "ridge_4d", "gauss_prod_4d", "corr_gauss_16d", "genz_batch",
                                      "no_such_workload"])
def test_profiled_traffic_lookup(bench, workload):
    t = bench.profiled_traffic(workload)
    assert t is None or (isinstance(t, float) and t > 0)


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("kernel", ["k_flow_sample", "k_flow_grad", "no_such_kernel"])
def test_profiled_traffic_per_kernel(bench, kernel):
    """The warp's summary holds one record per kernel, keyed by the sources
    of both kernels."""
    t = bench.profiled_traffic("corr_gauss_16d", "k_flow", bench.FLOW_SOURCES, kernel=kernel)
    assert t is None or (isinstance(t, float) and t > 0)
    if kernel == "no_such_kernel":
        assert t is None
