"""Build libqw.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2307_01571_amd.build          # or build() from Python

Each translation unit compiles in its own hipcc process (in parallel), then
one link step writes paper_2307_01571_amd/libqw.so.  Always rebuilds.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqw.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
# the slowest translation units first
SOURCES = ["qw_batch_f32.hip", "qw_kernels_f32.hip", "qw_batch_f64.hip", "qw_kernels_f64.hip", "qw_common.hip",
           "qw_mlp_kernels.hip", "qw_api.cpp", "qw_batch.cpp", "qw_mlp.cpp"]
# per-file flags: the batched kernels are built without machine loop-invariant
# code motion (see qw_batch_f32.hip)
SOURCE_FLAGS = {
    "qw_batch_f32.hip": ["-mllvm", "-disable-machine-licm"],
    "qw_batch_f64.hip": ["-mllvm", "-disable-machine-licm"],
}
COMMON_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed FP32 instructions stay off (see the kernels' build notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return p


def _compile(src: str, extra=(), build_dir=BUILD_DIR) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON_FLAGS, *SOURCE_FLAGS.get(src, []), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra_flags=(), out: str = OUT) -> str:
    """Compile and link; extra_flags (e.g. -D tuning macros) and out allow variant builds."""
    build_dir = BUILD_DIR if out == OUT else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, tuple(extra_flags), build_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="build libqw.so for gfx950")
    ap.add_argument("--split-rotations", action="store_true",
                    help="FP32 radix rotation constants as hi + lo float pairs (QW_F32_SPLIT_ROTATIONS=1): "
                         "no per-bin drift from their rounding over long runs, about 3%% slower")
    a = ap.parse_args()
    build(verbose=True, extra_flags=["-DQW_F32_SPLIT_ROTATIONS=1"] if a.split_rotations else ())
    sys.exit(0)
