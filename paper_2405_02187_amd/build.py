"""Build libxslam.so for gfx950 with hipcc (in-tree, no JIT cache).

Each (precision, D, Q) shape listed in csrc/combos.hpp is one translation unit
of csrc/inst.hip; the C ABI is csrc/api.cpp.  FP contraction is off so real
parts (the decision path) are evaluated exactly as written, and packed FP32
instructions are disabled.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libxslam.so")
ARCH = os.environ.get("XSLAM_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", f"-I{os.path.join(HERE, '..', 'include')}"]


def combos():
    src = open(os.path.join(CSRC, "combos.hpp")).read()
    return re.findall(r"X\((\w+),\s*(\d+),\s*(\d+),\s*(\w+)\)", src)


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _stale(obj: str, deps: list) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every unit (incremental=True: only units older than a source)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    units = [(os.path.join(CSRC, "api.cpp"), os.path.join(BUILD, "api.o"), ["-x", "hip"]),
             (os.path.join(CSRC, "cnn.hip"), os.path.join(BUILD, "cnn.o"), [])]
    for T, D, Q, name in combos():
        units.append((os.path.join(CSRC, "inst.hip"), os.path.join(BUILD, f"inst_{name}.o"),
                      [f"-DXS_T={T}", f"-DXS_D={D}", f"-DXS_Q={Q}", f"-DXS_NAME={name}"]))
    hdr = os.path.join(HERE, "..", "include", "xslam.h")
    eng = [os.path.join(CSRC, f) for f in ("jet.hpp", "common.hpp", "kernels.hpp", "newton.hpp", "reloc.hpp", "surfel.hpp", "group.hpp", "engine.hpp", "ctx.hpp",
                                           "inst.hip")] + [hdr]
    deps = {"api.cpp": eng + [os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "combos.hpp")],
            "inst.hip": eng, "cnn.hip": [os.path.join(CSRC, "cnn.hip"), hdr]}
    cmds = [["hipcc", *FLAGS, *extra, "-c", src, "-o", obj] for src, obj, extra in units
            if not incremental or _stale(obj, deps[os.path.basename(src)])]
    with ThreadPoolExecutor(jobs) as ex:
        for r in ex.map(_run, cmds):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp, *[u[1] for u in units]])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
