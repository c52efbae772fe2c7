"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11) and of its counter layout.

External pin: rocRAND's Philox4x32-10 engine header, compiled for the host, is an
independent library implementation of the same published generator.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

PIN_SRC = os.path.join(os.path.dirname(__file__), "pins", "rocrand_philox_pin.cpp")


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("host compiler or rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("pin") / "pin")
    subprocess.run([gxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-o", exe, PIN_SRC], check=True)

    def run(rows):
        text = "".join(" ".join(str(int(v)) for v in r) + "\n" for r in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(rocrand_pin):
    rng = np.random.default_rng(1234)
    M = 0xFFFFFFFF
    rows = [[0] * 6, [M] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1], [M, M, 0, 0, 0, 0]]
    rows += rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64).tolist()
    rows = np.array(rows, dtype=np.uint64)
    want = rocrand_pin(rows)
    got = np.stack(philox.philox4x32_10(*rows.T), axis=1)
    np.testing.assert_array_equal(got, want)


def test_counter_layout_matches_scalar_definition():
    seed, stream, level, pset = 0x0123456789ABCDEF, 3, 7, 5
    paths = np.array([0, 1, 2 ** 31, 2 ** 32 - 1, 977], dtype=np.uint64)
    w = philox.words(seed, stream, level, pset, paths, 11)
    for i, p in enumerate(paths):
        for n in range(11):
            c = philox.philox4x32_10(n >> 2, int(p), (stream << 16) | level, pset,
                                     seed & 0xFFFFFFFF, seed >> 32)
            assert int(w[i, n]) == int(c[n & 3])
            assert int(w[i, n]) == philox.word(seed, stream, level, pset, int(p), n)


@pytest.mark.parametrize("level", [0, 1])
def test_coarse_levels_share_calls_across_paths(level):
    # levels 0 and 1: one call (0, path div G, ...) for G = 4 / 2^level consecutive paths,
    # its four words dealt out in path order, every word used once
    seed, stream, pset = 0xFEDCBA9876543210, 5, 9
    S, G = 2 ** level, 4 // 2 ** level
    paths = np.arange(4096, 4096 + 4 * G, dtype=np.uint64)
    w = philox.words(seed, stream, level, pset, paths, S)
    for m in range(4):
        c = philox.philox4x32_10(0, (4096 + m * G) // G, (stream << 16) | level, pset,
                                 seed & 0xFFFFFFFF, seed >> 32)
        np.testing.assert_array_equal(w[m * G:(m + 1) * G].ravel(), np.array([int(x) for x in c], dtype=np.uint32))
        for j in range(G):
            for n in range(S):
                assert int(w[m * G + j, n]) == philox.word(seed, stream, level, pset, 4096 + m * G + j, n)
    # unaligned first path: the same words (they depend on the path, not on the slice)
    np.testing.assert_array_equal(philox.words(seed, stream, level, pset, paths[1:], S), w[1:])
    with pytest.raises(ValueError):
        philox.words(seed, stream, level, pset, paths, S + 1)


def test_words_prefix_independent_of_length():
    a = philox.words(0, 0, 5, 0, np.arange(8), 32)
    b = philox.words(0, 0, 5, 0, np.arange(8), 5)
    np.testing.assert_array_equal(a[:, :5], b)


def test_uniform_map_is_exact_and_symmetric():
    x = np.array([0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 2, 2 ** 32 - 1], dtype=np.uint64)
    u = philox.uniform(x)
    assert u.min() > 0 and u.max() < 1
    np.testing.assert_array_equal(philox.uniform(np.uint64(2 ** 32 - 1) - x), 1.0 - u)
    assert u[0] == 2.0 ** -33


def test_uniform_moments():
    w = philox.words(42, 0, 10, 0, np.arange(4096), 64).ravel()
    u = philox.uniform(w)
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
