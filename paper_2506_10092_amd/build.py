"""Build libccq.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled to its own object in parallel (the
persistent-kernel instances in ccq_inst.hip once per RLE-column bound and
kernel kind), then linked into one shared library."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libccq.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]

# (source, extra defines, object name)
UNITS = [("ccq_api.cpp", [], "ccq_api"), ("ccq_batch.cpp", [], "ccq_batch"),
         ("ccq_server.cpp", [], "ccq_server"), ("ccq_kernels.hip", [], "ccq_kernels"),
         ("ccq_encode.hip", [], "ccq_encode"), ("ccq_join.hip", [], "ccq_join")]
UNITS += [("ccq_inst.hip", ["-DCCQ_KMAX=%d" % k, "-DCCQ_BATCH=%d" % b], "ccq_inst_k%d_%s" % (k, "batch" if b else "fused"))
          for k in (2, 4, 8) for b in (0, 1)]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(u):
        src, defs, name = u
        obj = os.path.join(OBJDIR, name + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + inc + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, msg))
        if msg.strip() and verbose:
            print(msg, flush=True)
        return obj

    n = jobs or min(len(UNITS), os.cpu_count() or 4, 16)
    with ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(compile_one, UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
