"""The C-ABI library loads and exports every entry point that include/sw.h
declares (no compute calls: runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2404_17754_amd", "libsw.so")


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^SW_API\s+[\w\s\*]+?\b(sw_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("sw_ctx_create", "sw_mesh_create", "sw_case_create", "sw_case_step", "sw_case_waveforms",
              "sw_misfit", "sw_batch_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_declares_every_symbol():
    from paper_2404_17754_amd import _lib as L
    assert set(_declared()) <= set(L.SIGNATURES)
    lib = L.load()
    assert lib.sw_version().decode().startswith("sw ")


def test_product_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_2404_17754_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, flags=re.M), f
                assert "casegen" not in txt, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_mlp_initial_parameters():
    """Host-side initializer: Glorot-uniform hidden weights within their
    bounds, zero biases and output layer, deterministic per seed."""
    import numpy as np
    from paper_2404_17754_amd import _lib as L
    lib = L.load()

    def init(seed):
        p = np.zeros(L.MLP_NPARAM, np.float32)
        L.check(lib.sw_mlp_init_params(seed, p.ctypes.data_as(C.c_void_p)))
        return p

    p = init(7)
    W1, b1, W2, b2, w3, b3 = p[:640], p[640:704], p[704:4800], p[4800:4864], p[4864:4928], p[4928:]
    a1, a2 = np.sqrt(6.0 / 74), np.sqrt(6.0 / 128)
    assert np.all(np.abs(W1) <= a1) and np.all(np.abs(W2) <= a2)
    # uniform over [-a, a): mean near 0, variance near a^2 / 3
    assert abs(W2.mean()) < 0.05 * a2 and abs(W2.var() / (a2 * a2 / 3) - 1) < 0.1
    assert not b1.any() and not b2.any() and not w3.any() and not b3.any()
    assert np.array_equal(p, init(7)) and not np.array_equal(p, init(8))
