"""Build the HIP library libdwos.so for gfx950 (in-tree, next to this file).

Each source is compiled to an object of its own (in parallel, under _build/),
then the objects are linked into the shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdwos.so")
SOURCES = ["dwos.hip", "mlp.hip", "opt.hip", "probe.hip", "bvh_build.cpp", "remesh.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def build(verbose: bool = False, out: str = LIB, csrc: str = CSRC, defines=()) -> str:
    """Compile libdwos.so.  `defines` are extra -D knobs (e.g. DWOS_LEAF_MAX_3D=2)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in HIPCC_FLAGS if f != "-shared"]
    tag = os.path.splitext(os.path.basename(out))[0]

    def compile_one(src):
        obj = os.path.join(objdir, f"{tag}.{src}.o")
        cmd = [hipcc, *cflags, *[f"-D{d}" for d in defines], "-c", "-o", obj, os.path.join(csrc, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, cwd=csrc, capture_output=True, text=True)
        return obj, r

    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    for obj, r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed compiling {os.path.basename(obj)}")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp] + [obj for obj, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=csrc, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libdwos.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
