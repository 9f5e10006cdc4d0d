"""Build the gfx950 HIP library (liblbm_hip.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
# one translation unit per storage format (each holds every tuning variant of
# its step kernel), the reductions and dispatch, and the host runtime / C ABI
SOURCES = ["lbm_step_f32.hip", "lbm_step_f64.hip", "lbm_step_f16.hip", "lbm_step_f32g16.hip",
           "lbm_kernels.hip", "lbm_api.hip"]
HEADERS = ["lbm_device.hpp", "lbm_params.hpp", "lbm_launch.hpp", "lbm_step.hpp"]

# Packed FP32 instructions are kept out of the generated code.  Multiply-adds
# are fused only within one source expression (-ffp-contract=on): with the
# default cross-statement fusion the compiler fused differently in different
# inlined copies of the same node update, so a node at a work item's first
# row could round differently from the same node inside another item, and
# results depended on the launch configuration at the last-bit level.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile every HIP source for gfx950 (in parallel) and link liblbm_hip.so."""
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc()] + HIPFLAGS + [f"-D{d}" for d in defines] + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, obj))

    def compile_one(job):
        cmd, _ = job
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS") or os.cpu_count() or 1), 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(compile_one, jobs))
    objs = [o for _, o in jobs]
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
