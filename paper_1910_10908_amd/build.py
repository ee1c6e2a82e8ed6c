"""Build libtffr.so (HIP, gfx950) in-tree with hipcc (one object per source, compiled in
parallel, then linked)."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtffr.so")
SOURCES = ["tffr_host.hip"]
# kernel sources: one object per compute type (FP32 / FP64 instantiations), built in parallel
KERNEL_SOURCES = ["tffr_range.hip", "tffr_azimuth.hip", "tffr_entstep.hip", "tffr_coord.hip", "tffr_ffr.hip", "tffr_rma.hip",
                  "tffr_misc.hip"]
ARCH = "gfx950"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose=False):
    """Compile every source for gfx950 and link libtffr.so next to this file."""
    objs = []
    flags = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
             # keep FP32 arithmetic on the unpacked VALU path
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds = []
    jobs = [(src, src.replace(".hip", ".o"), []) for src in SOURCES]
    for src in KERNEL_SOURCES:
        for tag, define in (("f32", "TFFR_REAL_F32"), ("f64", "TFFR_REAL_F64")):
            jobs.append((src, src.replace(".hip", f"_{tag}.o"), ["-D" + define]))
    for src, oname, extra in jobs:
        obj = os.path.join(bdir, oname)
        cmds.append([hipcc()] + flags + extra + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
        if verbose:
            print(" ".join(cmds[-1]), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for r in list(ex.map(lambda c: subprocess.run(c), cmds)):
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, r.args)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
