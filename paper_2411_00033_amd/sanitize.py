"""Host sanitizer build of the library: AddressSanitizer and UndefinedBehaviorSanitizer on
the host pass of every source (the device code is built as in the product), for the
host-only tests (argument checking, plan cache, tuning tables, allocation bookkeeping).

    python -m paper_2411_00033_amd.sanitize     # builds _build/asan/libleg2cheb_hostasan.so

The library is loaded into a Python process with the ASan runtime preloaded (see
tests/test_host_sanitizer.py).  GPU code is never built with a sanitizer.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess

from . import build as hipbuild

OUT = os.path.join(hipbuild.OBJ, "asan")
LIB = os.path.join(OUT, "libleg2cheb_hostasan.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """Path of the ASan runtime of hipcc's clang (empty if it is not installed)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipbuild.HIPCC)), "..", "llvm", "bin", "clang")
    try:
        d = subprocess.run([clang, "--print-runtime-dir"], stdout=subprocess.PIPE, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return ""
    for cand in (os.path.join(d, "libclang_rt.asan.so"), os.path.join(d, "libclang_rt.asan-x86_64.so"),
                 os.path.join(os.path.dirname(d), "linux", "libclang_rt.asan-x86_64.so")):
        if os.path.exists(cand):
            return cand
    return ""


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = hipbuild.sources() + [os.path.join(hipbuild.PKG, "csrc", f) for f in os.listdir(os.path.join(hipbuild.PKG, "csrc"))]
    deps.append(os.path.join(hipbuild.ROOT, "include", "leg2cheb.h"))
    return any(os.path.getmtime(p) > t for p in deps)


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = hipbuild.sources()
    objs = [os.path.join(OUT, os.path.basename(s)[:-4] + ".o") for s in srcs]
    cmds = [[hipbuild.HIPCC, *hipbuild.FLAGS, *HOST_SAN, "-I", os.path.join(hipbuild.ROOT, "include"), "-c", s, "-o", o]
            for s, o in zip(srcs, objs)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1, 16)) as ex:
        results = list(ex.map(lambda c: hipbuild._run(c, verbose), cmds))
    for (rc, out), src in zip(results, srcs):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, out))
    tmp = LIB + ".tmp%d" % os.getpid()
    rc, out = hipbuild._run([hipbuild.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", *HOST_SAN,
                             *objs, "-o", tmp], verbose)
    if rc != 0:
        raise RuntimeError("hipcc link failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
