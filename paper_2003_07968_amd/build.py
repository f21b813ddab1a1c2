"""Compile the HIP library (liblbm.so) for gfx950 with hipcc.

The device code is split into translation units that compile in parallel:
csrc/lbm_inst.hip once per storage mode and kernel family (the single-step
sweeps, and the two-step pass), csrc/lbm.hip (host runtime and C ABI) and
csrc/server.cpp (the serving loop).  Objects go to _build/ beside this file;
the library is linked in-tree so that it travels with the source tree.

Run as `python -m paper_2003_07968_amd.build`.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")
INCLUDE = os.path.join(ROOT, "include")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no implicit multiply-add contraction: the kernels spell their fma()s out,
    # so results do not depend on how the compiler schedules inlined copies
    "-ffp-contract=off",
    # packed FP32 instructions stay disabled in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no mixed-precision fma: folded into a conversion to binary16 it rounds
    # once where the source rounds twice (to FP32, then to binary16), and the
    # compiler folds some unrolled copies of a row body and not others, which
    # made binary16 results depend on the launch shape
    "-Xclang", "-target-feature", "-Xclang", "-fma-mix-insts",
    f"-I{INCLUDE}",
]

# (object name, source, extra defines)
UNITS = [("lbm_host", "lbm.hip", [])] + [
    (f"lbm_st{st}_k{fam}", "lbm_inst.hip", [f"-DLBM_INST_ST={st}", f"-DLBM_INST_FAMILY={fam}"])
    for fam in (2, 1) for st in (0, 1, 2, 3)
] + [("server", "server.cpp", [])]

# hipcc's host pass does not know the two GPU features and says so
_NOISE = ("packed-fp32-ops", "fma-mix-insts")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if not any(n in ln for n in _NOISE)]
    return res.returncode, msgs


def _jobs() -> int:
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        if os.environ.get(var, "").isdigit():
            return max(1, int(os.environ[var]))
    return max(1, min(len(UNITS), os.cpu_count() or 1))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)

    def compile_unit(unit):
        name, src, defines = unit
        obj = os.path.join(OBJDIR, name + ".o")
        cmd = [hipcc(), *FLAGS, *defines, "-c", "-o", obj, os.path.join(CSRC, src)]
        return cmd, obj, _run(cmd)

    with ThreadPoolExecutor(max_workers=_jobs()) as pool:
        results = list(pool.map(compile_unit, UNITS))
    objs = []
    for cmd, obj, (rc, msgs) in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            sys.stderr.write("\n".join(msgs) + "\n")
            raise RuntimeError(f"hipcc failed with exit code {rc}: {' '.join(cmd)}")
        if verbose and msgs:
            print("\n".join(msgs))
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    rc, msgs = _run(cmd)
    if rc != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError(f"linking liblbm.so failed with exit code {rc}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
