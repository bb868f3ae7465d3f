"""Build the HIP library for gfx950 with hipcc (in-tree, no JIT cache).

Produces ``paper_2607_01338_amd/libiris_rt.so`` from ``csrc/*.hip``. Every
call recompiles (objects go to ``_build/``, which is not committed).
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libiris_rt.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wall",
    "-Wno-unused-result",
    # Packed FP32 instructions are kept out of every kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


# Sources whose host code validates arguments, folds constants, carves
# workspaces, reads molecular data and sets up plans: the checking build
# compiles their host side with AddressSanitizer and UBSan.
HOST_SOURCES = ("api.hip", "host_common.hip", "plan.hip", "levels.hip", "checks.hip",
                "noalloc.hip")
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _compile(src: str, extra=(), obj_dir: str = OBJ) -> str:
    obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_host_sanitized(out: str, verbose: bool = False) -> str:
    """A checking variant of the library at ``out``: the host code of
    HOST_SOURCES with AddressSanitizer and UBSan (the process must preload
    clang's ASan runtime), the other objects as built by build()."""
    os.makedirs(OBJ, exist_ok=True)
    san_dir = os.path.join(OBJ, "san")
    os.makedirs(san_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host = [x for x in srcs if os.path.basename(x) in HOST_SOURCES]
    rest = [x for x in srcs if os.path.basename(x) not in HOST_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda x: _compile(x, SANITIZE_HOST, san_dir), host))
        for x in rest:
            o = os.path.join(OBJ, os.path.basename(x) + ".o")
            objs.append(o if os.path.exists(o) and os.path.getmtime(o) >= os.path.getmtime(x)
                        else ex.submit(_compile, x).result())
    # The sanitizer runtime is not linked in: the process preloads it.
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
