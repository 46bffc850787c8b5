"""Build the HIP library ``libfwi.so`` in-tree for gfx950.

Every ``csrc/*.hip`` translation unit is compiled with hipcc in parallel and
linked into ``paper_2102_00755_amd/libfwi.so``.  Packed-FP32 instructions are
disabled for device code (``-Xclang -target-feature -Xclang -packed-fp32-ops``).

    python -m paper_2102_00755_amd.build            # build
    python -m paper_2102_00755_amd.build --jobs 8
    python -m paper_2102_00755_amd.build --define FWI_AXIS_TILE_BYTES=128 --out /tmp/libfwi_t128.so

``--define`` sets a tuning macro of the kernels (see the top of
csrc/kernels.h); ``--out`` writes such a variant elsewhere (load it with
``FWI_LIBRARY=<path>``) and leaves the in-tree library alone.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwi.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("FWI_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str, objdir: str, defines) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, defines=(), out: str | None = None) -> str:
    lib = out or LIB
    objdir = OBJDIR if not defines and out is None else os.path.join(
        OBJDIR, "variant_" + "_".join(d.replace("=", "-") for d in defines) if defines else "variant")
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not srcs:
        raise RuntimeError("no HIP sources found")
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, defines), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--define", action="append", default=[], help="NAME=VALUE tuning macro")
    ap.add_argument("--out", default=None, help="library path (default: in-tree libfwi.so)")
    args = ap.parse_args(argv)
    build(args.jobs, verbose=True, defines=args.define, out=args.out)


if __name__ == "__main__":
    sys.exit(main())
