"""The bfloat16 storage of the SW_MIXED_FP16 inner CG's direction
(csrc/sw_bf16.h, built with g++ for the CPU) against PyTorch's float32 ->
bfloat16 conversion, which rounds to nearest with ties to even: random
values over the whole exponent range, exact ties (both parities), values
that round up into the next binade and to infinity, subnormals, zeros,
infinities and NaN; and the way back is exact (the upper half of the FP32
pattern)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_17754_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("bf16") / "libbf16_check.so"
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, os.path.join(HERE, "bf16_check.cpp"),
                    "-o", str(out)], check=True)
    return C.CDLL(str(out))


def _to(lib, x):
    x = np.ascontiguousarray(x, np.float32)
    h = np.zeros(x.size, np.uint16)
    lib.to_bf16(C.c_int64(x.size), C.c_void_p(x.ctypes.data), C.c_void_p(h.ctypes.data))
    return h


def _torch_bits(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(
        np.uint16)


def test_rounding_matches_round_to_nearest_even(lib):
    rng = np.random.default_rng(7)
    bits = rng.integers(0, 2**32, 200000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    # exact ties: a kept part of either parity with the dropped half 0x8000
    kept = rng.integers(0, 2**16, 2000, dtype=np.uint32) & 0x7f7f
    ties = ((kept << 16) | 0x8000).astype(np.uint32).view(np.float32)
    edge = np.array([0.0, -0.0, 1.0, -1.0, np.float32(3.4028235e38), np.float32(-3.4028235e38),
                     np.float32(1e-45), np.float32(-1e-45), np.float32(1.1754942e-38), np.float32(1.0039062),
                     np.float32(1.9999999), np.float32(65504.0), np.inf, -np.inf], np.float32)
    for v in (x, ties, edge):
        np.testing.assert_array_equal(_to(lib, v), _torch_bits(v))


def test_nan_stays_nan_and_way_back_is_exact(lib):
    nan = np.array([np.nan, -np.nan, np.float32(np.uint32(0x7f800001).view(np.float32))], np.float32)
    h = _to(lib, nan)
    back = np.zeros(h.size, np.float32)
    lib.from_bf16(C.c_int64(h.size), C.c_void_p(h.ctypes.data), C.c_void_p(back.ctypes.data))
    assert np.all(np.isnan(back))
    allh = np.arange(2**16, dtype=np.uint16)
    back = np.zeros(allh.size, np.float32)
    lib.from_bf16(C.c_int64(allh.size), C.c_void_p(allh.ctypes.data), C.c_void_p(back.ctypes.data))
    np.testing.assert_array_equal(back.view(np.uint32), allh.astype(np.uint32) << 16)
    # every finite bfloat16 value converts to itself
    fin = np.isfinite(back)
    np.testing.assert_array_equal(_to(lib, back[fin]), allh[fin])
