"""Build the HIP library in-tree: paper_2012_01968_amd/libntt_mi355x.so (gfx950).

Each translation unit is compiled by hipcc into _build/ in parallel, then linked into a
shared library next to this file.  Run ``python paper_2012_01968_amd/build.py`` (as a
script: importing the package needs the library this builds).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("NTT_BUILD_DIR") or os.path.join(ROOT, "_build", "ntt")
LIB = os.environ.get("NTT_BUILD_OUT") or os.path.join(HERE, "libntt_mi355x.so")
SOURCES = ["kernels_fwd_fast.hip", "kernels_inv_fast.hip", "kernels_fwd_wide.hip", "kernels_inv_wide.hip",
           "kernels_mul_fast.hip", "kernels_mul_wide.hip",
           "fused_fwd.hip", "fused_inv.hip", "kernels.hip", "permute.hip", "stages.hip", "kernels32.hip", "crt.hip",
           "calib.hip", "capi.cpp"]
# (object name, source, defines): the row-pass instances, one unit per direction (forward,
# inverse, key product), arithmetic policy and range of row lengths
ROW_RANGES = ((1, 7), (8, 10), (11, 13))
UNITS = [(os.path.splitext(src)[0], src, []) for src in SOURCES] + [
    (f"rows_{d}_{'fast' if fast else 'wide'}_{lo}_{hi}", "kernels_rows.hip",
     [f"-DNTTK_ROWS_DIR={d}", f"-DNTTK_ROWS_FAST={'true' if fast else 'false'}", f"-DNTTK_ROWS_LO={lo}",
      f"-DNTTK_ROWS_HI={hi}"])
    for d in (0, 1, 2) for fast in (1, 0) for lo, hi in ROW_RANGES]
ARCH = os.environ.get("NTT_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
    # packed-FP32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
] + os.environ.get("NTT_EXTRA_FLAGS", "").split()


# Host-only sources: they decide which launches happen but hold no device code, so a change
# there leaves every kernel's measured time (and the counters taken of it) valid.
HOST_ONLY_SOURCES = ("capi.cpp", "plan_math.hpp", "plan_life.hpp", "tune_file.hpp", "crt_math.hpp")
# Device code that no plan launches (the calibration copy): outside the hash as well.
UNHASHED_DEVICE_SOURCES = ("calib.hip",)


def source_hash() -> str:
    """Hash of the device-code sources the kernels are built from (the .hip and .hpp files
    other than the host-only ones).  The library is built with it, and the tuner keys its
    cache by it: a measured choice or counter stays valid while it is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")) and name not in HOST_ONLY_SOURCES + UNHASHED_DEVICE_SOURCES:
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _compile(unit) -> str:
    name, src, defines = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, *defines, f'-DNTT_SOURCE_HASH="{source_hash()}"', "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {name} ({src}):\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # the longest units first, at most one compiler per CPU (each takes a few GB)
    order = sorted(UNITS, key=lambda u: (u[1] != "kernels_rows.hip", -int(u[2][3].split("=")[1]) if u[2] else 0))
    with ThreadPoolExecutor(max(1, min(len(order), os.cpu_count() or 1))) as ex:
        objs = list(ex.map(_compile, order))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
