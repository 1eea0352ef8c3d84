"""Host-sanitizer build of libpdhg (AddressSanitizer + UndefinedBehaviorSanitizer
on the host code only; the gfx950 device code is built as usual).  Used by the
CPU test of the ABI's host validation, with clang's ASan runtime preloaded."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

from paper_2512_06715_amd import build as hipbuild

BUILD = os.path.join(hipbuild.ROOT, "_build_san")
LIB = os.path.join(BUILD, "libpdhg_san.so")
# each sanitizer flag applies to the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]


def asan_runtime() -> str:
    """clang's shared ASan runtime that the sanitized library links."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's ASan runtime not found")
    return hits[-1]


def build() -> str:
    srcs = [os.path.join(hipbuild.CSRC, s) for s in hipbuild.SOURCES]
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) > os.path.getmtime(s) for s in
                                   srcs + glob.glob(os.path.join(hipbuild.CSRC, "*.h")) +
                                   [os.path.join(hipbuild.INCLUDE, "pdhg.h")]):
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    hipcc = hipbuild._hipcc()
    flags = [f for f in hipbuild.HIPCC_FLAGS if f != "-O3"] + ["-O1"] + HOST_SAN

    def one(src):
        obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
        r = subprocess.run([hipcc, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-3000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(one, srcs))
    # the host link (no device link is needed: each object carries its own
    # device code) with clang, the sanitizer runtimes shared
    clang = "/opt/rocm/llvm/bin/clang++"
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [clang, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libasan", "-o", tmp,
           *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-3000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
