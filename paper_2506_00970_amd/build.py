"""Build libgs2d.so (the gfx950 HIP kernels and their C ABI) in-tree with hipcc.

Usage: ``python -m paper_2506_00970_amd.build`` or ``build()`` from Python.  Every
call recompiles; objects go to ``paper_2506_00970_amd/_build`` and the library
to ``paper_2506_00970_amd/libgs2d.so``.

Two debug variants build beside it (load one with ``GS2D_LIB=<path>``):

* ``--device-checks`` -> ``libgs2d_checked.so``: kernels check their tile rectangles,
  pair keys and slots, sorted keys and blended ranges, and record failures in
  ``gs2d_counts.device_checks`` (no trap);
* ``--sanitize-host`` -> ``libgs2d_hostsan.so``: the host code with AddressSanitizer and
  UndefinedBehaviorSanitizer (device code unchanged); the process must preload clang's
  ASan runtime (``asan_runtime()``).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgs2d.so")
SOURCES = ["api.hip", "preprocess.hip", "sort.hip", "blend.hip", "loss_pose.hip", "warmstart.hip", "mapstate.hip", "mapping_loss.hip",
           "image_loss_noalloc.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",              # every fused multiply-add is an explicit fmaf
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",  # no packed FP32 math
    "-Wall", "-Wno-unused-function",
    "-fvisibility=hidden",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libgs2d.so)")


# host-only sanitizers: every -fsanitize= goes to the host compilation alone
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]
VARIANTS = {
    "release": ("_build", "libgs2d.so", []),
    "device_checks": ("_build_checked", "libgs2d_checked.so", ["-DGS2D_DEVICE_CHECKS"]),
    "sanitize_host": ("_build_hostsan", "libgs2d_hostsan.so", HOST_SANITIZE),
}


def asan_runtime() -> str:
    """Path of clang's shared ASan runtime (with the UBSan handlers) that a process loading
    the host-sanitized library must preload."""
    cc = hipcc()
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(cc)), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's shared ASan runtime was not found")
    return path


def _compile(src: str, cc: str, verbose: bool, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [cc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and verbose:
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = False, variant: str = "release") -> str:
    """Compile every HIP source for gfx950 and link the library of ``variant`` (release:
    libgs2d.so); returns its path."""
    sub, name, extra = VARIANTS[variant]
    build_dir, lib = os.path.join(HERE, sub), os.path.join(HERE, name)
    cc = hipcc()
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, cc, verbose, build_dir, extra), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    # the host-sanitized objects leave the sanitizer runtime's symbols undefined; the
    # preloaded runtime supplies them
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    variant = "device_checks" if "--device-checks" in sys.argv else (
        "sanitize_host" if "--sanitize-host" in sys.argv else "release")
    print(build(verbose="-v" in sys.argv, variant=variant))
