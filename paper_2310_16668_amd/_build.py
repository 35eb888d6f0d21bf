"""Compile the C-ABI library libskelfmm.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libskelfmm.so")
OBJ = os.path.join(HERE, "_build")

HOST_SOURCES = ["capi.cpp", "host/tree.cpp", "host/skel.cpp", "device/layout.cpp"]
# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build (CPU tests only;
# device code stays uninstrumented: each -fsanitize applies to the host pass).
SAN_LIB = os.path.join(HERE, "libskelfmm_san.so")
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-shared-libasan",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
DEVICE_SOURCES = ["device/sweep_lap3.hip", "device/sweep_helm3.hip", "device/sweep_lap2.hip", "device/sweep_helm2.hip", "device/exec.hip",
                  "device/build_gpu.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-mavx2", "-mfma"]
# No packed-FP32 instructions in device code (v_pk_*_f32 are avoided on purpose).
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, sanitize: bool = False) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(SAN_OBJ if sanitize else OBJ, src.replace("/", "_") + ".o")
    flags = COMMON + (DEVICE_FLAGS if src.endswith(".hip") else HOST_FLAGS) + (SAN_FLAGS if sanitize else [])
    cmd = [HIPCC, *flags, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link libskelfmm.so (always recompiles).
    sanitize: the host-side ASan + UBSan library libskelfmm_san.so instead (load it
    with SKELFMM_LIB and the ASan runtime preloaded; see tests/run_sanitized.sh)."""
    out, objdir = (SAN_LIB, SAN_OBJ) if sanitize else (LIB, OBJ)
    os.makedirs(objdir, exist_ok=True)
    srcs = DEVICE_SOURCES + HOST_SOURCES
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda x: _compile(x, sanitize), srcs))
    tmp = out + ".tmp"
    extra = ["-shared-libasan", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"] if sanitize else []
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *extra, "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
