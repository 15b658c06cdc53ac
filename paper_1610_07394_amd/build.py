"""Build libsmx.so (all HIP sources, gfx950) in-tree with hipcc.

    python -m paper_1610_07394_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsmx.so")
# the same sources with device checks compiled in (SMX_CHECKED=1)
OBJDIR_CHECKED = os.path.join(HERE, "_build_checked")
LIB_CHECKED = os.path.join(HERE, "libsmx_checked.so")

ARCH = os.environ.get("SMX_OFFLOAD_ARCH", "gfx950")
# -packed-fp32-ops: keep the compiler from forming v_pk_*_f32 from scalar float code.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, checked: bool = False) -> str:
    obj = os.path.join(OBJDIR_CHECKED if checked else OBJDIR, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *(["-DSMX_CHECKED=1"] if checked else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, checked: bool = False) -> str:
    """Compile and link libsmx.so, or libsmx_checked.so with checked=True."""
    lib = LIB_CHECKED if checked else LIB
    os.makedirs(OBJDIR_CHECKED if checked else OBJDIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, checked), srcs))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    build(verbose=True, checked=True)
    sys.exit(0)
