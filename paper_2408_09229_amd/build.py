"""Build the HIP library libvegas_hip.so for gfx950 (in-tree).

Each .hip source compiles to an object in parallel, then one shared library
is linked.  Contraction is off so that the parity-relevant FP64 arithmetic
follows the written order (hot FP32 code writes its fma explicitly); packed
FP32 instructions are disabled.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libvegas_hip.so")
UBENCH_OUT = os.path.join(HERE, "libvegas_issue_rates.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("VEGAS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fill.hip", "update.hip", "ordered.hip", "batch.hip", "flow.hip", "flow_train.hip", "api.hip", "batch_api.hip"]

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(HERE, "..", "include"),
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    # instruction issue-rate probe used by bench.py --issue-rates (not the path)
    ub = _compile("issue_rates.hip", verbose)
    subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", UBENCH_OUT + ".tmp", ub], check=True)
    os.replace(UBENCH_OUT + ".tmp", UBENCH_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
