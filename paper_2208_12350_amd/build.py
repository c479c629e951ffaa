"""Build libswalign.so (the gfx950 HIP library) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswalign.so")
PROBE_LIB = os.path.join(HERE, "libswprobe.so")
STENCIL_LIB = os.path.join(HERE, "libswstencil.so")
SOURCES = ["sw_plan.hip", "sw_queue_i16_w16.hip", "sw_queue_i16_w16b.hip", "sw_queue_i16_w32.hip",
           "sw_queue_i16_w32b.hip", "sw_queue_i16_w64.hip", "sw_queue_i16_w64_long.hip", "sw_queue_i16_w256.hip",
           "sw_queue_i32.hip", "sw_trace.hip", "sw_runtime.hip", "sw_server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link the shared
    library.  Always recompiles."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + text)
        if verbose and text.strip():
            print(text)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    # the VALU issue-rate probe, a separate library outside the alignment path
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-shared", os.path.join(CSRC, "sw_probe.hip"), "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, PROBE_LIB)
    # the grid diffusion library (the second workload), also separate
    tmp = STENCIL_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-shared", os.path.join(CSRC, "sw_stencil.hip"), "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, STENCIL_LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0))
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
