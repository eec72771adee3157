"""Build libcpdmi.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2103_04081_amd.build

Every call compiles from source: one hipcc process per translation unit (run
in parallel), then one link; the shared library lands next to this file.
"""

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcpdmi.so")

SOURCES = ["cpd_api.hip", "step_kernel.hip", "layout_fit.hip", "batch_serve.hip", "serve.hip", "variance.hip",
           "wide_step.hip", "rescale.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unused-command-line-argument",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _jobs():
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 1), 16))


def build(verbose=True):
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="cpdmi_build_") as tmpd:
        def compile_one(s):
            obj = os.path.join(tmpd, s.replace(".hip", ".o"))
            cmd = [hipcc()] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return s, obj, r
        with ThreadPoolExecutor(_jobs()) as ex:
            results = list(ex.map(compile_one, srcs))
        failed = False
        for s, _, r in results:
            out = (r.stdout + r.stderr).strip()
            if r.returncode != 0:
                failed = True
                print(f"--- {s} failed:\n{out}", file=sys.stderr, flush=True)
            elif verbose and out:
                # hipcc's host pass does not know the packed-FP32 feature switch
                lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
                if lines:
                    print("\n".join(lines), flush=True)
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc")
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + \
            [obj for _, obj, _ in results] + ["-o", tmp, "-lpthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
