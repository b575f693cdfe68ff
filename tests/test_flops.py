"""The algorithmic flops per tetrahedron that bench.py's ALU roofline uses
are the element arithmetic's own count: sw_elem.h's element_apply is
compiled with g++ on a counting number type (tests/flop_count.cpp), and the
count of the CG operator pass (stiffness and mass together) must equal the
element term of bench.FLOPS_PER_TET."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_17754_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("flops")
    (d / "hip").mkdir()
    (d / "hip" / "hip_runtime.h").write_text("// stand-in: the element arithmetic needs no HIP runtime\n")
    out = d / "libflop_count.so"
    subprocess.run([gxx, "-O0", "-std=c++17", "-shared", "-fPIC", "-I", str(d), "-I", CSRC,
                    os.path.join(HERE, "flop_count.cpp"), "-o", str(out)], check=True)
    lib = C.CDLL(str(out))
    lib.element_flops.restype = C.c_int64
    lib.element_flops.argtypes = [C.c_int, C.c_int]
    return lib


def test_element_flops_match_the_benchmark_constant(lib):
    both = lib.element_flops(1, 1)
    assert both == bench.ELEMENT_FLOPS
    # the terms are separate: stiffness alone and mass alone each cost less
    assert 0 < lib.element_flops(1, 0) < both and 0 < lib.element_flops(0, 1) < both
    assert lib.element_flops(0, 0) == 0 or lib.element_flops(0, 0) < 10
