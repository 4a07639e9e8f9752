"""Build libmpfc.so (HIP, gfx950) in-tree with hipcc.

The library is linked from several translation units compiled in parallel:
csrc/mpfc.hip (host code of every entry point and the per-step kernels) and
csrc/launch_inst.hip once per operator group (-DMPFC_GROUP=k: the fused tile
kernels and persistent coarse kernels of that group's operators).  Objects go
to paper_1208_2643_amd/_build/, the library next to this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SRC = os.path.join(CSRC, "mpfc.hip")
INST = os.path.join(CSRC, "launch_inst.hip")
NGROUPS = 8
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpfc.so")
ARCH = os.environ.get("MPFC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP64 atomic add (all atomics target coarse-grained hipMalloc memory)
    "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".hpp", ".h"))] + [os.path.join(ROOT, "include", "mpfc.h")]


def _units():
    units = [(SRC, os.path.join(BUILD, "mpfc.o"), [])]
    for k in range(NGROUPS):
        units.append((INST, os.path.join(BUILD, f"launch_{k}.o"), [f"-DMPFC_GROUP={k}"]))
    return units


def _compile(unit, verbose):
    src, obj, extra = unit
    cmd = ["hipcc", *FLAGS, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, r


def _report(r, verbose):
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    elif verbose and r.stderr.strip():
        # hipcc's host pass notes that it does not know the packed-fp32 feature
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose), units))
    failed = False
    for _, r in results:
        _report(r, verbose)
        failed |= r.returncode != 0
    if failed:
        raise RuntimeError("hipcc failed compiling libmpfc.so")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC",
           *[u[1] for u in units], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libmpfc.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
