"""Build libagsplat.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled to an object in parallel, then linked into one shared
library next to this file.  Packed FP32 instructions are disabled for all device code
(`-Xclang -target-feature -Xclang -packed-fp32-ops`); float atomics use the hardware
instruction (`-munsafe-fp-atomics`, device memory is coarse-grained).

`build(sanitize=True)` makes a second library, `_build_san/libagsplat_san.so`, whose host code
carries AddressSanitizer and UndefinedBehaviorSanitizer checks (device code unchanged; each
sanitizer flag applies to the host side only); load it with the sanitizer runtime preloaded
(`sanitizer_runtime()`).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libagsplat.so")
BUILD_SAN = os.path.join(ROOT, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libagsplat_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
             "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ARCH = os.environ.get("AGS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "project.hip", "sortscan.hip", "bin.hip", "raster.hip", "loss.hip",
           "project_bwd.hip", "optim.hip", "ssim.hip", "lifecycle.hip", "map.hip"]

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
          "-Wno-unused-variable", f"-I{INCLUDE}"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm is required to build libagsplat)")
    return exe


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *CFLAGS, *(SAN_FLAGS if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(_filter_warnings(r.stderr))
    return obj


def _filter_warnings(text: str) -> str:
    # the host pass does not know the device-only feature flag; that warning is harmless
    keep = [ln for ln in text.splitlines(keepends=True) if "packed-fp32-ops" not in ln
            and "is not a recognized feature" not in ln]
    return "".join(keep)


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every HIP translation unit and link libagsplat.so (or, with sanitize, the
    host-sanitized libagsplat_san.so); returns its path."""
    out = LIB_SAN if sanitize else LIB
    os.makedirs(BUILD_SAN if sanitize else BUILD, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if sanitize:
        cmd[2:2] = [*SAN_FLAGS, "-Xarch_host", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def sanitizer_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload for libagsplat_san.so)."""
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin",
                                     "clang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        import glob
        found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        if not found:
            raise RuntimeError("the AddressSanitizer runtime of the ROCm compiler was not found")
        path = found[-1]
    return path


if __name__ == "__main__":
    build()
