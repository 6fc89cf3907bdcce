"""Build libfm.so in-tree with hipcc for gfx950.

    python -m paper_2005_05398_amd.build      (or build() from Python)

Every call recompiles every source.  Objects go to paper_2005_05398_amd/_build/,
the library to paper_2005_05398_amd/libfm.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["basis.cpp", "linalg.cpp", "setup.cpp", "coupled.cpp", "coupling.cpp", "api.cpp", "eigs.cpp", "host_api.cpp", "serve.cpp", "noalloc.cpp", "kernels.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
# gfx950 only; packed-FP32 instructions disabled in device code
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose=False, jobs=None):
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmds.append([HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", obj])
        objs.append(obj)
    # the kernels file first: it takes most of the time
    order = sorted(range(len(cmds)), key=lambda i: not SOURCES[i].endswith(".hip"))
    with ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 1)) as ex:
        outs = list(ex.map(lambda i: _run(cmds[i]), order))
    if verbose:
        for out in outs:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
