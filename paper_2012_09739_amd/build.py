"""Builds libmlmc.so (the HIP kernels and the C-ABI) and libvalurates.so (the VALU issue-rate
probes behind the issue roofline) for gfx950, in-tree.

    python -m paper_2012_09739_amd.build        (or build() from Python)

Every translation unit is compiled with hipcc for gfx950 only, with floating-point
contraction off (the method's operations are separately rounded; explicit fma() calls in
the binary64 inverse CDF stay fused) and packed-FP32 instruction selection disabled.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmlmc.so")
# issue rates of single VALU opcodes (the weights of the level kernels' issue roofline):
# a separate library, not part of the method's C-ABI
RATES_SOURCE = "valu_rates.hip"
RATES_LIB = os.path.join(HERE, "libvalurates.so")

HIP_SOURCES = ["level_f64.hip", "level_f32.hip", "level_f16.hip", "level_bf16.hip",
               "level_milstein_f64.hip", "level_milstein_f32.hip", "level_milstein_f16.hip",
               "level_milstein_bf16.hip", "level_coop.hip", "kernels_misc.hip", "batch.hip", "mlp_train.hip", "abi.cpp"]
CXX_SOURCES = ["tables.cpp"]
# the binary16 instances evaluate each path's variable with scalar binary16 operations, which
# issue two per clock like binary32 ones; the SLP vectorizer would pack the two paths of a lane
# into v_pk_* operations (same rate) plus a v_perm per coefficient pair (one slot each)
EXTRA_FLAGS = {"level_f16.hip": ["-fno-slp-vectorize"], "level_milstein_f16.hip": ["-fno-slp-vectorize"],
               "batch.hip": ["-fno-slp-vectorize"], "level_coop.hip": ["-fno-slp-vectorize"]}

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I" + os.path.join(ROOT, "include"),
          "-I" + CSRC, "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]
# matrix instructions (the learned variable's 16 x 16 layer) read and write VGPRs directly,
# with no copies out of accumulation registers
HIP_FLAGS = ["--offload-arch=gfx950", "-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fno-gpu-rdc", "-mllvm", "-amdgpu-mfma-vgpr-form"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def build(verbose=False, jobs=None):
    """Compile every source and link libmlmc.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        cmds.append([hipcc, "-c", *COMMON, *HIP_FLAGS, *EXTRA_FLAGS.get(src, []), os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        cmds.append(["g++", "-c", *COMMON, os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    rates_tmp = RATES_LIB + ".tmp"
    cmds.append([hipcc, "-shared", *COMMON, *HIP_FLAGS, os.path.join(CSRC, RATES_SOURCE), "-o", rates_tmp])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    os.replace(rates_tmp, RATES_LIB)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


# Host sanitizers: the host side of every translation unit (argument validation, tables,
# launch code) with AddressSanitizer and UndefinedBehaviorSanitizer, the device code as
# usual; for the CPU tests of the C-ABI (tests/test_abi.py), loaded through MLMC_LIBRARY with
# the sanitizer runtime preloaded into the interpreter.
SANITIZED_LIB = os.path.join(BUILD, "libmlmc_sanitized.so")
_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
        "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libasan"]


def sanitizer_runtime():
    """Path of the AddressSanitizer runtime of the HIP compiler (to LD_PRELOAD)."""
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(_clangxx())), "clang++"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def _clangxx():
    for cand in ("/opt/rocm/llvm/bin/clang++", "/opt/rocm/lib/llvm/bin/clang++"):
        if os.path.exists(cand):
            return cand
    return "clang++"


def build_sanitized(verbose=False, jobs=None):
    """libmlmc with host sanitizers (in the build folder, not the product library)."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, "san_" + src.replace(".", "_") + ".o")
        cmds.append([hipcc, "-c", *COMMON, *HIP_FLAGS, *EXTRA_FLAGS.get(src, []), *_SAN, os.path.join(CSRC, src),
                     "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, "san_" + src.replace(".", "_") + ".o")
        cmds.append([_clangxx(), "-c", *COMMON, "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                     "-fno-omit-frame-pointer", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *_SAN, "-o", SANITIZED_LIB, *objs], verbose)
    return SANITIZED_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
        print(sanitizer_runtime())
    else:
        print(build(verbose="-v" in sys.argv))
