"""Build libtsf.so (HIP kernels for gfx950 + the host C-ABI) in-tree.

The walk kernels are instantiated in four translation units (32/64-bit masks x
ternary/Z2) that compile in parallel; the host part is plain C++.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "tsf")
LIB = os.path.join(PKG, "libtsf.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             # packed FP32 instructions stay off in every HIP build
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _units():
    units = []
    for wide in (0, 1):
        for z2 in (0, 1):
            units.append(([HIPCC] + HIP_FLAGS + ["-DTSFK_WIDE=%d" % wide, "-DTSFK_Z2=%d" % z2,
                                                  "-c", os.path.join(CSRC, "walk_inst.hip")],
                          "walk_inst_w%d_z%d.o" % (wide, z2)))
    for src in ("walk.hip", "mlp.hip", "lift.hip"):
        path = os.path.join(CSRC, src)
        if os.path.exists(path):
            units.append(([HIPCC] + HIP_FLAGS + ["-c", path], src.replace(".hip", ".o")))
    units.append((["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-c",
                   os.path.join(CSRC, "host.cpp")], "host.o"))
    return units


def _compile(unit):
    cmd, obj = unit
    out = os.path.join(OBJ, obj)
    proc = subprocess.run(cmd + ["-o", out], capture_output=True, text=True)
    msgs = "\n".join(l for l in (proc.stdout + proc.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if proc.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), msgs))
    return out


def build(force: bool = True, jobs: int = 6) -> str:
    """Compile every HIP/C++ source and link paper_2511_20317_amd/libtsf.so."""
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, _units()))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
