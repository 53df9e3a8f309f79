"""Build libfock.so in-tree with hipcc for gfx950.

Every call recompiles.  Object files go to paper_1111_0716_amd/_build/, the
shared library to paper_1111_0716_amd/libfock.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfock.so")
SOURCES = ["kernels.hip", "pair_fused.hip", "overlap_mfma.hip", "pass_reg.hip", "pw_fft.hip", "plan.cpp", "api.cpp"]
ARCH = os.environ.get("FOCK_OFFLOAD_ARCH", "gfx950")

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 arithmetic stays off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


# ---- host-code sanitizer build ------------------------------------------
# A variant for checking the host code (planner, C ABI, launch set-up) on
# the CPU: host code built with AddressSanitizer and UndefinedBehaviorSanitizer
# (-Xarch_host: the device code is compiled as usual, at -O1), into
# _build/sanitize/.  Load it by setting FOCK_LIBRARY to its path with the ASan
# runtime preloaded (asan_runtime()).
SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libfock_host_sanitized.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime():
    """Path of the compiler's shared ASan runtime (to preload)."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError(f"ASan runtime not found ({path!r})")
    return path


def _sources_digest():
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)) + ["../../include/fock.h"]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    with open(os.path.abspath(__file__), "rb") as f:  # the commands themselves
        h.update(f.read())
    return h.hexdigest()


def build_host_sanitized(verbose=False):
    """Build (or reuse, when the sources are unchanged) the sanitizer variant."""
    os.makedirs(SAN_DIR, exist_ok=True)
    stamp = os.path.join(SAN_DIR, "sources.sha256")
    digest = _sources_digest()
    if os.path.exists(SAN_LIB) and os.path.exists(stamp) and open(stamp).read() == digest:
        return SAN_LIB

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O1", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument", *SAN_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitizer compile of {src} failed:\n{' '.join(cmd)}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_FLAGS, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    with open(stamp, "w") as f:
        f.write(digest)
    if verbose:
        print(f"built {SAN_LIB}", file=sys.stderr)
    return SAN_LIB


if __name__ == "__main__":
    if sys.argv[1:] == ["sanitize"]:
        build_host_sanitized(verbose=True)
    else:
        build()
