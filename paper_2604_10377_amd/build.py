"""Build libfmap.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2604_10377_amd.build

Every .hip file under csrc/ is compiled to an object in _build/ (in
parallel), then linked into paper_2604_10377_amd/libfmap.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfmap.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed fp32 instructions are disabled (known-bad forms on this target).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The register-resident row solves rely on full unrolling of their static loops
# (a partially unrolled loop would index the register array dynamically and
# spill it to scratch); the build fails if any kernel ends up using scratch.
CFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Wno-unknown-warning-option", "-mllvm", "-pragma-unroll-threshold=200000",
          "-Rpass-analysis=kernel-resource-usage"] + DEVICE_FLAGS


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build_id() -> str:
    """Hash of every kernel source and header (keys the plan's tuning cache to this build)."""
    import hashlib
    h = hashlib.sha256()
    files = sources() + sorted(glob.glob(os.path.join(CSRC, "*.h"))) + [os.path.join(os.path.dirname(HERE), "include",
                                                                                    "fmap.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    usage, warn, fn = [], [], None
    for line in r.stderr.splitlines():
        if "kernel-resource-usage" in line:
            body = line.split("remark:", 1)[-1].replace("[-Rpass-analysis=kernel-resource-usage]", "").strip()
            if body.startswith("Function Name:"):
                fn = body.split(":", 1)[1].strip()
            elif body.startswith("ScratchSize") and not body.endswith(": 0"):
                raise RuntimeError(f"{fn} uses scratch memory ({body}); a register array is not fully unrolled")
            usage.append(body)
        elif "packed-fp32-ops" in line or not line.strip() or re.match(r"^\s*\d*\s*\|", line):
            continue  # feature notice of the host pass, or source context of a remark
        else:
            warn.append(line)
    with open(obj + ".usage.txt", "w") as f:
        f.write("\n".join(usage) + "\n")
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")
    return obj


def build(extra=(), jobs: int = 8) -> str:
    """Compile every HIP source for gfx950 and link libfmap.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    extra = list(extra) + [f'-DFMAP_BUILD_ID="{build_id()}"']
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
