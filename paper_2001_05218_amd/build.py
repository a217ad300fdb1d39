"""Build the HIP shared library in-tree with hipcc for gfx950.

    python -m paper_2001_05218_amd.build      (or __graft_entry__.build())
    python -m paper_2001_05218_amd.build --sanitize   (host ASan/UBSan build, see SANITIZE)

Every source under csrc/ is compiled to an object in csrc/_build/ (in
parallel) and linked into paper_2001_05218_amd/libwilson_mi355x.so. The
build always recompiles: it is also the "does it build" check.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB_NAME = "libwilson_mi355x.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
# device code: no packed-FP32 instructions (see DESIGN notes on v_pk_*_f32)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the library needs ROCm's hipcc to build")
    return path


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name.endswith(".cpp"):
            out.append(os.path.join(CSRC, name))
    return out


# Host-code sanitizers for the checking build (--sanitize): AddressSanitizer
# and UndefinedBehaviorSanitizer on the host side only (device code is built
# as usual). The result is a separate library, loaded by setting
# WILSON_MI355X_LIB to its path and preloading the ASan runtime.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_LIB_PATH = os.path.join(SAN_BUILD, "libwilson_mi355x_sanitize.so")


def _compile(src: str, sanitize: bool = False) -> str:
    out_dir = SAN_BUILD if sanitize else BUILD
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, "-c", src, "-o", obj]
    cmd[1:1] = ["-x", "hip"]
    cmd += DEVICE
    if sanitize:
        cmd += SANITIZE
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    out_dir = SAN_BUILD if sanitize else BUILD
    lib = SAN_LIB_PATH if sanitize else LIB_PATH
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}", file=sys.stderr)
    return lib


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
