"""Build libnndtw.so (HIP for gfx950) in-tree with hipcc.

Every .hip file under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_1808_09617_amd/libnndtw.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnndtw.so")
ARCH = os.environ.get("NNDTW_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",                       # FP64 sums/products round exactly as written
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Task counters are advanced by whole-wave LDS atomics whose addend is
    # non-zero in lane 0 only (so that no lane branch surrounds the deal):
    # issue them as they are, not through a wave scan, which would hold
    # whole-wave registers across the engines' register-bound loops.
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


RESOURCES = os.path.join(BUILD, "kernel_resources.txt")


# Per-file flags.  The bound kernels and the DTW engines take minima and
# maxima of loaded or lane-shifted values; inputs are finite (a precondition
# of the C ABI) and no operation of these kernels makes a NaN from finite
# values and infinities (no inf - inf, no 0 * inf), so the compiler need not
# quiet NaNs before each of them (a canonicalising max per term, and per
# shifted FP64 value on the engine's dependency chain).
NO_NANS = ["-fno-honor-nans"]
EXTRA = {f: NO_NANS for f in ("bounds.hip", "compare.hip", "search.hip", "dtw.hip", "batch.hip", "grad.hip",
                               "envelopes.hip")}


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    # a compilation-unit ID of the file's name (not of its path), so that the
    # device code does not depend on where the tree is built
    cuid = "nndtw_" + os.path.splitext(os.path.basename(src))[0]
    cmd = [HIPCC, *CFLAGS, *EXTRA.get(os.path.basename(src), []), f"-cuid={cuid}",
           "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj, _resources(r.stderr)


def _resources(remarks: str):
    """(kernel, VGPRs, AGPRs, scratch bytes per lane) from the compiler's
    kernel-resource-usage remarks."""
    out, cur = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            continue
        if cur is None:
            continue
        for key, pat in (("v", r"VGPRs: (\d+)"), ("a", r"AGPRs: (\d+)"), ("s", r"ScratchSize \[bytes/lane\]: (\d+)")):
            m = re.search(pat, line)
            if m:
                cur[key] = int(m.group(1))
        if all(k in cur for k in "vas"):
            out.append((cur["name"], cur["v"], cur["a"], cur["s"]))
            cur = None
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    with open(RESOURCES, "w") as f:
        f.write("# kernel VGPRs AGPRs scratch_bytes_per_lane (gfx950)\n")
        for _, res in done:
            for name, v, a, sc in res:
                f.write(f"{name} {v} {a} {sc}\n")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(out: str) -> str:
    """A build of the library whose host code (argument validation, planning,
    launch sequencing: api.hip and the host halves of the launchers) is
    instrumented with AddressSanitizer and UndefinedBehaviorSanitizer; the
    device code is the same.  For the CPU sanitizer test, which loads it with
    clang's ASan runtime preloaded."""
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    flags = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def comp(src):
        obj = os.path.join(san, os.path.basename(src) + ".o")
        cuid = "nndtw_" + os.path.splitext(os.path.basename(src))[0]
        cmd = [HIPCC, *CFLAGS, *EXTRA.get(os.path.basename(src), []), f"-cuid={cuid}", *flags, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(comp, srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *flags, "-o", out, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
