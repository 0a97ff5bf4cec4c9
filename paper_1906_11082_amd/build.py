"""Build libnmodes.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 with packed FP32 instructions disabled,
then linked against the HIP runtime, rocBLAS and rocSOLVER that PyTorch
ships (same sonames as /opt/rocm), so a process that has imported torch
holds exactly one HIP runtime.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnmodes.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["nm_ref.cpp", "nm_assemble.hip", "nm_groups.hip", "nm_ops.hip", "nm_eig.hip", "nm_slices.hip",
           "nm_rotation.hip", "nm_api.hip", "nm_server.hip", "nm_noalloc.hip",
           "nm_selfgrav.hip", "nm_gemm.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _torch_lib() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return "/opt/rocm/lib"
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-4000:]))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tl = _torch_lib()
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp,
           "-L" + tl, "-lrocblas", "-lrocsolver", "-lamdhip64", "-Wl,-rpath," + tl]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
