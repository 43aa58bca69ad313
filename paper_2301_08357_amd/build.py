"""Build the HIP library libpressure.so for gfx950 (in-tree, with hipcc)."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUTDIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUTDIR, "libpressure.so")

SOURCES = ["pressure.hip", "layout.cpp", "tune.cpp"]
PROBE_SOURCE = "stream_probe.hip"          # the benchmark's bandwidth probe (libstream_probe.so)
PROBE_LIB = os.path.join(OUTDIR, "libstream_probe.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False):
    """Compile every source to an object file (in parallel), then link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OUTDIR, exist_ok=True)
    tag = ".tmp%d" % os.getpid()
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OUTDIR, src + tag + ".o")
        objs.append(obj)
        cmds.append(["/opt/rocm/bin/hipcc"] + compile_flags + ["-I", INCLUDE, "-I", CSRC, "-c",
                                                               os.path.join(CSRC, src), "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    probe_tmp = PROBE_LIB + tag
    cmds.append(["/opt/rocm/bin/hipcc"] + HIPCC_FLAGS + [os.path.join(CSRC, PROBE_SOURCE), "-o", probe_tmp])
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            list(ex.map(run, cmds))
        os.replace(probe_tmp, PROBE_LIB)
        tmp = LIB + tag
        run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
        os.replace(tmp, LIB)
    finally:
        for o in objs + [probe_tmp]:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
