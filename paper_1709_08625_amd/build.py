"""Compile the hcov HIP library for gfx950 (in-tree: paper_1709_08625_amd/libhcov.so)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhcov.so")
SOURCES = ["plan.cpp", "nm.cpp", "tree.hip", "kernels.hip", "aca_big.hip", "hcov.hip", "server.hip"]
FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for s in SOURCES:
        src = os.path.join(SRC, s)
        obj = os.path.join(objdir, s + ".o")
        cmd = [hipcc] + FLAGS + ["-c", src, "-o", obj]
        if s.endswith(".cpp"):
            cmd = [hipcc, "-std=c++17", "-O3", "-fPIC", "-x", "c++", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the translation units are independent: compile them concurrently
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(subprocess.run, c, check=True) for c in cmds]:
            f.result()
    tmp = OUT + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
