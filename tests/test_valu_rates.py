"""CPU tests of the VALU issue-rate probe library (libvalurates.so): it loads, exports the
entry point include/valu_rates.h declares, and rejects invalid arguments before any HIP call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2012_09739_amd", "libvalurates.so")
HEADER = os.path.join(ROOT, "include", "valu_rates.h")


def _lib():
    if not os.path.exists(LIB):
        pytest.fail("libvalurates.so is not built: run python -m paper_2012_09739_amd.build")
    lib = ctypes.CDLL(LIB)
    lib.valu_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]
    return lib


def test_exports_declared_entry_point():
    names = re.findall(r"^\s*int\s+(valu_\w+)\s*\(", open(HEADER).read(), re.M)
    assert names == ["valu_rate"]
    assert hasattr(_lib(), "valu_rate")


def test_op_list_matches_bench():
    import bench
    ops = re.search(r"enum \{(.*?)\};", open(HEADER).read(), re.S).group(1)
    n = len(re.findall(r"^\s*VALU_(?!N_OPS)\w+", ops, re.M))
    assert n == len(bench.VALU_OPS)


def test_roofline_counts_belong_to_the_current_sources():
    # bench.py's issue counts (slots per path-step) and counter traffic were taken from the
    # roofline kernels' sources as they are now; a change to any of those files must re-count
    # the step loop's assembly (or show it unchanged) and refresh the hashes, else the bench
    # line reports those figures as null
    import bench
    assert bench.sources_sha256(bench.ISA_SOURCES) == bench.ISA_SOURCES_SHA256
    assert bench.kernel_sources_sha256() == bench.TRAFFIC_SOURCES_SHA256


@pytest.mark.parametrize("op,waves,iters", [(-1, 8, 16), (99, 8, 16), (0, 0, 16), (0, 9, 16), (0, 8, 0),
                                            (0, 8, (1 << 20) + 1)])
def test_invalid_arguments(op, waves, iters):
    r = ctypes.c_double()
    assert _lib().valu_rate(op, waves, iters, ctypes.byref(r), None) == -1
    assert _lib().valu_rate(0, 8, 16, None, None) == -1
