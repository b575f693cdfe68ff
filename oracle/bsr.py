"""Assembled-sparse oracle for meshes too large for the SciPy oracle: a
C++/OpenMP symmetric 3x3 block-sparse (upper triangle, FP64) assembly of
K, M and the dashpot matrix, and the Newmark march with every step solved
by 3x3 block-Jacobi preconditioned CG to a true relative residual
(oracle/native/bsr_march.cpp).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The element integrals follow the same definitions as oracle/fem.py (whose
reference-element tables it takes from there: the quadrature points' shape
gradients, the reference mass and the triangle tables), and the march the
same Newmark average-acceleration step as oracle/march.py (Section 3).  It
is pinned against the SciPy oracle in tests/test_oracle_bsr.py: the
assembled products with K, M and C_abs, the input basis and marched
receiver records on small meshes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import fem

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "bsr_march.cpp")
LIB = os.path.join(HERE, "native", "liboracle_bsr.so")

_lib = None


def build(verbose=False):
    """Compile the native oracle with g++ (OpenMP); always recompiles."""
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.oracle_bsr_create.restype = vp
    lib.oracle_bsr_create.argtypes = [i64, i64, vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.oracle_bsr_destroy.argtypes = [vp]
    lib.oracle_bsr_threads.restype = i32
    lib.oracle_bsr_threads.argtypes = [vp]
    lib.oracle_bsr_blocks.restype = i64
    lib.oracle_bsr_blocks.argtypes = [vp]
    lib.oracle_bsr_apply.argtypes = [vp, f64, f64, f64, vp, vp]
    lib.oracle_bsr_input_basis.argtypes = [vp, vp]
    lib.oracle_bsr_march.restype = i32
    lib.oracle_bsr_march.argtypes = [vp, f64, f64, f64, vp, i64, i32, vp, vp, vp, vp, f64, i32, i32, vp, vp, vp, vp]
    _lib = lib
    return lib


def reference_tables():
    """Reference-element data from oracle/fem.py: stiffness rule (points'
    shape gradients in reference coordinates, weights summing to 1/6),
    reference mass int N_a N_b, and per-unit-area triangle mass and load."""
    L, w = fem.tet_rule(2)
    gref = np.array([[[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]])
    dN = fem.tet10_dshape(L, gref)[0]                 # (m,10,3)
    Lm, wm = fem.tet_rule(3)
    N = fem.tet10_shape(Lm)
    Mref = np.einsum("m,ma,mb->ab", wm, N, N)
    Lt, wt = fem.tri_rule(3)
    Nt = fem.tri6_shape(Lt)
    Sref = 2.0 * np.einsum("m,ma,mb->ab", wt, Nt, Nt)
    Lref = 2.0 * np.einsum("m,ma->a", wt, Nt)
    return (np.ascontiguousarray(dN), np.ascontiguousarray(w), np.ascontiguousarray(Mref),
            np.ascontiguousarray(Sref), np.ascontiguousarray(Lref))


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


class System:
    """K, M, C_abs and the input basis of one mesh and material map."""

    def __init__(self, mesh, mat, tet_mat):
        lib = load()
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64), np.ascontiguousarray(mesh.tet10, np.int32),
                      np.ascontiguousarray(mesh.tri6, np.int32), np.ascontiguousarray(mesh.face_tet, np.int32),
                      np.ascontiguousarray(mesh.face_role, np.uint8), np.ascontiguousarray(mat, np.float64),
                      np.ascontiguousarray(tet_mat, np.uint8)]
        xyz, tet10, tri6, ft, fr, m, tm = self._keep
        dN, w, Mref, Sref, Lref = self._tables = reference_tables()
        self.n_nodes = mesh.n_nodes
        self.h = lib.oracle_bsr_create(mesh.n_nodes, mesh.n_tets, _ptr(xyz), _ptr(tet10), mesh.n_faces, _ptr(tri6),
                                       _ptr(ft), _ptr(fr), m.shape[0], _ptr(m), _ptr(tm), len(w), _ptr(dN),
                                       _ptr(w), _ptr(Mref), _ptr(Sref), _ptr(Lref))
        if not self.h:
            raise ValueError("native oracle rejected the mesh (non-positive element volume)")
        self._lib = lib

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.oracle_bsr_destroy(self.h)
            self.h = None

    @property
    def threads(self):
        return int(self._lib.oracle_bsr_threads(self.h))

    @property
    def blocks(self):
        return int(self._lib.oracle_bsr_blocks(self.h))

    def apply(self, x, cK=0.0, cM=0.0, cC=0.0):
        """(cK K + cM M + cC C_abs) x."""
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty(3 * self.n_nodes)
        self._lib.oracle_bsr_apply(self.h, cK, cM, cC, _ptr(x), _ptr(y))
        return y

    def input_basis(self):
        out = np.empty((3, 3 * self.n_nodes))
        self._lib.oracle_bsr_input_basis(self.h, _ptr(out))
        return out

    def march(self, dt, alpha, beta, v_in, n_steps, rec_node, u0=None, v0=None, a0=None, rtol=1e-12,
              max_iter=100000, guess="previous"):
        """Newmark march of n_steps from (u0, v0, a0) (zero by default).
        Returns dict(rec_v (n_steps, n_rec, 3), u, v, a, iters, relres,
        secs (wall time per step))."""
        n3 = 3 * self.n_nodes
        u = np.zeros(n3) if u0 is None else np.array(u0, np.float64)
        v = np.zeros(n3) if v0 is None else np.array(v0, np.float64)
        a = np.zeros(n3) if a0 is None else np.array(a0, np.float64)
        v_in = np.ascontiguousarray(v_in[:n_steps + 1], np.float64)
        rec = np.ascontiguousarray(rec_node, np.int32)
        rec_v = np.zeros((n_steps, len(rec), 3))
        iters = np.zeros(n_steps, np.int32)
        relres = np.zeros(n_steps)
        secs = np.zeros(n_steps)
        rc = self._lib.oracle_bsr_march(self.h, dt, alpha, beta, _ptr(v_in), n_steps, len(rec), _ptr(rec), _ptr(u),
                                        _ptr(v), _ptr(a), rtol, max_iter, 1 if guess == "previous" else 0,
                                        _ptr(rec_v), _ptr(iters), _ptr(relres), _ptr(secs))
        if rc != 0:
            raise RuntimeError("native oracle CG did not converge")
        return dict(rec_v=rec_v, u=u, v=v, a=a, iters=iters, relres=relres, secs=secs)
