"""Builds the HIP library libsubsmc.so in-tree for gfx950 with hipcc.

The translation units (the C ABI with the per-stage kernels, and one launcher
unit per family of particle kernels) compile in parallel to objects under
_build/ and link into one shared library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
UNITS = ["subsmc.hip", "launch_narrow.hip", "launch_wide.hip", "launch_resident.hip", "launch_persist_f32.hip",
         "launch_persist_f64.hip"]
LIB = os.path.join(HERE, "libsubsmc.so")
OBJ_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    hs.append(os.path.join(ROOT, "include", "subsmc.h"))
    return max(os.path.getmtime(h) for h in hs)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every unit and link. incremental=True skips a unit whose object
    is newer than the unit and every header (a development shortcut)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    procs, objs = [], []
    newest_h = _newest_header()
    for u in UNITS:
        obj = os.path.join(OBJ_DIR, os.path.splitext(u)[0] + ".o")
        objs.append(obj)
        src = os.path.join(CSRC, u)
        if (incremental and os.path.exists(obj)
                and os.path.getmtime(obj) > max(os.path.getmtime(src), newest_h)):
            continue
        cmd = [HIPCC, *FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((u, subprocess.Popen(cmd)))
    failed = [u for u, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed for {', '.join(failed)}")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
