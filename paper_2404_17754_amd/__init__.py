"""MI355X implicit seismic-wave analysis: Python binding of libsw.

Argument marshalling only: every step of the analysis runs in the HIP
kernels of libsw.so.  PyTorch supplies device memory (caller-owned
workspaces) and the stream.  Importing this package does not load the
library; the first object created does, and fails loudly if the library is
not built or no HIP device is present.

Typical use::

    ctx = Context()
    mesh = Mesh(ctx, m)            # m: xyz, tet10, tri6, face_tet, face_role arrays
    case = Case(ctx, mesh, c)      # c: mat, tet_mat, rec_node, v_in, dt, ray_alpha, ray_beta
    case.step(c.n_steps)
    w = case.waveforms()           # (n_steps, n_rec, 3) receiver velocities
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import SwError  # noqa: F401

PRECISIONS = {"fp64": L.SW_FP64, "mixed": L.SW_MIXED_FP32, "mixed_fp32": L.SW_MIXED_FP32,
              "flex": L.SW_MIXED_FP32_FLEX, "fp16": L.SW_MIXED_FP16}
GUESSES = {"zero": L.SW_GUESS_ZERO, "poly": L.SW_GUESS_POLY, "mlp": L.SW_GUESS_MLP, "proj": L.SW_GUESS_PROJ,
           "proj_mlp": L.SW_GUESS_PROJ_MLP}
OPS = {"M": L.SW_OP_M, "K": L.SW_OP_K, "Cabs": L.SW_OP_CABS, "A": L.SW_OP_A}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the analysis runs only on the GPU")
    return torch


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(a.data_ptr())


def _workspace(nbytes, device):
    torch = _torch()
    # 256-byte aligned base (torch's caching allocator aligns to >= 512 B)
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Context:
    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        L.check(self.lib.sw_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def set_graphs(self, enable):
        """Replay CG iterations from captured HIP graphs (default) or launch
        every kernel directly."""
        L.check(self.lib.sw_ctx_set_graphs(self.h, 1 if enable else 0))

    def set_grid_cap(self, max_workgroups):
        """Cap the workgroups of the persistent FP32 passes (0: default)."""
        L.check(self.lib.sw_ctx_set_grid_cap(self.h, int(max_workgroups)))

    def profile(self, enable=True, kinds=None, every=1):
        """Start (reset) or stop per-kernel HIP-event timing of the CG kernels:
        all classes, or only those named in `kinds` (see profile_read), one
        launch in `every` of each."""
        if kinds is None and every == 1:
            L.check(self.lib.sw_ctx_profile(self.h, 1 if enable else 0))
        else:
            names = L.PROF_KINDS if kinds is None else kinds
            mask = sum(1 << L.PROF_KINDS[k] for k in names) if enable else 0
            L.check(self.lib.sw_ctx_profile_kinds(self.h, mask, int(every)))

    def profile_read(self, kind):
        """(total ms, launches, mean ms of full launches, full launches) of one
        kernel class: tile_f64, tile_f32, update_f64, update_f32, dir_f64,
        dir_f32.  Full launches are those lasting at least half the longest."""
        t, fm = C.c_double(), C.c_double()
        n, fn = C.c_int64(), C.c_int64()
        L.check(self.lib.sw_ctx_profile_read(self.h, L.PROF_KINDS[kind], C.byref(t), C.byref(n), C.byref(fm),
                                             C.byref(fn)))
        return t.value, n.value, fm.value, fn.value

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.sw_ctx_destroy(self.h)
            self.h = None


class Mesh:
    """Device layout of a mesh (sw_mesh_create).  tile_nodes / tile_elems:
    tile capacity (0 = the library's default 1280 / 512); deterministic:
    also build the node incidence lists deterministic cases need."""

    def __init__(self, ctx: Context, m, tile_nodes=0, tile_elems=0, deterministic=False):
        self.ctx = ctx
        lib = ctx.lib
        self._xyz = np.ascontiguousarray(m.xyz, np.float64)
        self._tet = np.ascontiguousarray(m.tet10, np.int32)
        self._tri = np.ascontiguousarray(m.tri6, np.int32).reshape(-1, 6)
        self._ft = np.ascontiguousarray(m.face_tet, np.int32)
        self._fr = np.ascontiguousarray(m.face_role, np.uint8)
        self.n_nodes, self.n_tets, self.n_faces = len(self._xyz), len(self._tet), len(self._tri)
        d = L.MeshDesc(self.n_nodes, self.n_tets, self.n_faces, _ptr(self._xyz), _ptr(self._tet),
                       _ptr(self._tri), _ptr(self._ft), _ptr(self._fr), tile_nodes, tile_elems,
                       int(bool(deterministic)))
        nb = C.c_size_t()
        L.check(lib.sw_mesh_workspace_bytes(C.byref(d), C.byref(nb)))
        self.ws = _workspace(nb.value, ctx.device)
        h = C.c_void_p()
        L.check(lib.sw_mesh_create(ctx.h, C.byref(d), C.c_void_p(self.ws.data_ptr()), nb.value, C.byref(h)))
        self.h = h
        del self._xyz, self._tet, self._tri, self._ft, self._fr

    def info(self):
        """(tiles, largest tile's node count) of the device layout."""
        nt, mx = C.c_int32(), C.c_int32()
        L.check(self.ctx.lib.sw_mesh_info(self.h, C.byref(nt), C.byref(mx)))
        return nt.value, mx.value

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.sw_mesh_destroy(self.h)
            self.h = None


class Case:
    """One analysis on ``mesh``.  ``c`` provides mat, tet_mat, rec_node,
    v_in ((n_steps+1) x 3), dt, ray_alpha, ray_beta (and n_steps)."""

    def __init__(self, ctx: Context, mesh: Mesh, c, rtol=1e-8, max_iter=10000, precision="fp64",
                 guess="zero", poly_order=2, inner_rtol=0.0, n_steps=None, proj_dim=6, deterministic=False):
        self.ctx, self.mesh = ctx, mesh
        lib = ctx.lib
        v_in = np.ascontiguousarray(c.v_in, np.float64)
        n_steps = (len(v_in) - 1) if n_steps is None else int(n_steps)
        if len(v_in) < n_steps + 1:
            raise ValueError("v_in shorter than n_steps + 1")
        v_in = np.ascontiguousarray(v_in[: n_steps + 1])
        mat = np.ascontiguousarray(c.mat, np.float64)
        tet_mat = np.ascontiguousarray(c.tet_mat, np.uint8)
        rec = np.ascontiguousarray(c.rec_node, np.int32)
        self.n_rec, self.n_steps = len(rec), n_steps
        self.n_dof = 3 * mesh.n_nodes
        d = L.CaseDesc(float(c.dt), float(c.ray_alpha), float(c.ray_beta), float(rtol), int(max_iter),
                       PRECISIONS[precision], GUESSES[guess], int(poly_order), float(inner_rtol),
                       len(mat), _ptr(mat), _ptr(tet_mat), len(rec), _ptr(rec), n_steps, _ptr(v_in),
                       int(proj_dim), int(bool(deterministic)))
        nb = C.c_size_t()
        L.check(lib.sw_case_workspace_bytes(mesh.h, C.byref(d), C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = _workspace(nb.value, ctx.device)
        h = C.c_void_p()
        L.check(lib.sw_case_create(ctx.h, mesh.h, C.byref(d), C.c_void_p(self.ws.data_ptr()), nb.value,
                                   C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.sw_case_destroy(self.h)
            self.h = None

    # -- march
    def step(self, n=1):
        L.check(self.ctx.lib.sw_case_step(self.h, int(n)))

    def stats(self):
        s = L.CaseStats()
        L.check(self.ctx.lib.sw_case_stats_get(self.h, C.byref(s)))
        return dict(steps=s.steps, cg_iters=s.cg_iters, ir_outer=s.ir_outer,
                    max_true_rel_res=s.max_true_rel_res, flags=s.flags)

    def step_log(self, step0=0, n=None):
        n = self.stats()["steps"] - step0 if n is None else n
        it = np.zeros(n, np.int32)
        rel = np.zeros(n, np.float64)
        L.check(self.ctx.lib.sw_case_step_log(self.h, step0, n, _ptr(it), _ptr(rel)))
        return it, rel

    def waveforms(self, step0=0, n=None):
        n = self.stats()["steps"] - step0 if n is None else n
        out = np.zeros((n, self.n_rec, 3))
        L.check(self.ctx.lib.sw_case_waveforms(self.h, step0, n, _ptr(out)))
        return out

    def waveform_device(self):
        """Device waveform buffer as a torch tensor view (n_steps, n_rec, 3)."""
        torch = _torch()
        p = C.c_void_p()
        L.check(self.ctx.lib.sw_case_waveform_device(self.h, C.byref(p)))
        base = self.ws.data_ptr()
        off = p.value - base
        n = self.n_steps * self.n_rec * 3
        return self.ws[off: off + 8 * n].view(torch.float64).view(self.n_steps, self.n_rec, 3)

    # -- state
    def set_state(self, u=None, v=None, a=None, step=0):
        arr = [None if x is None else np.ascontiguousarray(x, np.float64) for x in (u, v, a)]
        ptrs = [C.c_void_p(0) if x is None else _ptr(x) for x in arr]
        L.check(self.ctx.lib.sw_case_set_state(self.h, *ptrs, int(step)))

    def get_state(self):
        u, v, a = (np.zeros(self.n_dof) for _ in range(3))
        st = C.c_int64()
        L.check(self.ctx.lib.sw_case_get_state(self.h, _ptr(u), _ptr(v), _ptr(a), C.byref(st)))
        return u, v, a, st.value

    # -- operators (device tensors)
    def _vec(self, x, dtype):
        torch = _torch()
        x = x.to(self.ctx.device, dtype).contiguous().reshape(-1)
        if x.numel() != self.n_dof:
            raise ValueError(f"vector has {x.numel()} entries, expected {self.n_dof}")
        return x

    def apply(self, op, x):
        torch = _torch()
        x = self._vec(x, torch.float64)
        y = torch.empty_like(x)
        mask = op if isinstance(op, int) else sum(OPS[o] for o in op.split("+"))
        L.check(self.ctx.lib.sw_case_apply(self.h, mask, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def apply_f32(self, op, x):
        torch = _torch()
        x = self._vec(x, torch.float32)
        y = torch.empty_like(x)
        mask = op if isinstance(op, int) else sum(OPS[o] for o in op.split("+"))
        L.check(self.ctx.lib.sw_case_apply_f32(self.h, mask, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def autotune(self, reps=5):
        """Pick the fastest workgroup count of the FP32 pass
        (sw_case_autotune); returns (choice, mean ms of the 3 candidates)."""
        ch = C.c_int32()
        ms = np.zeros(3)
        L.check(self.ctx.lib.sw_case_autotune(self.h, int(reps), C.byref(ch), _ptr(ms)))
        return ch.value, ms

    def rhs(self):
        torch = _torch()
        y = torch.empty(self.n_dof, dtype=torch.float64, device=self.ctx.device)
        L.check(self.ctx.lib.sw_case_rhs(self.h, C.c_void_p(y.data_ptr())))
        return y

    def guess(self):
        """Initial guess the next step would start from (device, user order)."""
        torch = _torch()
        y = torch.empty(self.n_dof, dtype=torch.float64, device=self.ctx.device)
        L.check(self.ctx.lib.sw_case_guess(self.h, C.c_void_p(y.data_ptr())))
        return y

    def diag_blocks(self):
        torch = _torch()
        y = torch.empty(self.mesh.n_nodes * 6, dtype=torch.float64, device=self.ctx.device)
        L.check(self.ctx.lib.sw_case_diag_blocks(self.h, C.c_void_p(y.data_ptr())))
        return y.view(-1, 6)

    # -- learned guess
    def attach_mlp(self, mlp):
        L.check(self.ctx.lib.sw_case_attach_mlp(self.h, mlp.h if mlp is not None else C.c_void_p(0)))
        self._mlp = mlp

    def set_sampler(self, capacity, per_step, seed=0):
        """Record training rows into a new device buffer; returns it."""
        torch = _torch()
        buf = torch.zeros((int(capacity), L.MLP_ROW), dtype=torch.float32, device=self.ctx.device)
        L.check(self.ctx.lib.sw_case_set_sampler(self.h, C.c_void_p(buf.data_ptr()), int(capacity), int(per_step),
                                                 int(seed)))
        self._samp = buf
        return buf

    def samples(self):
        n = C.c_int64()
        L.check(self.ctx.lib.sw_case_samples(self.h, C.byref(n)))
        return self._samp[: n.value]

    def misfit(self, obs):
        """ERR of the recorded waveforms against obs (device tensor)."""
        torch = _torch()
        obs = obs.to(self.ctx.device, torch.float64).contiguous()
        need = self.stats()["steps"] * self.n_rec * 3
        if obs.numel() < need or (obs.dim() == 3 and obs.shape[1:] != (self.n_rec, 3)):
            raise ValueError(f"obs must hold at least {need} values laid out (steps, {self.n_rec}, 3)")
        e = C.c_double()
        n = C.c_int32()
        L.check(self.ctx.lib.sw_case_misfit(self.h, C.c_void_p(obs.data_ptr()), C.byref(e), C.byref(n)))
        return e.value, n.value


class Mlp:
    """Initial-guess network (see sw_mlp_* in include/sw.h).  params: 4929
    floats packed W1[64][10], b1, W2[64][64], b2, w3, b3."""

    def __init__(self, ctx: Context, params=None, seed=0):
        self.ctx = ctx
        if params is None:
            params = self.initial_params(ctx, seed)
        p = np.ascontiguousarray(params, np.float32).ravel()
        if p.size != L.MLP_NPARAM:
            raise ValueError(f"expected {L.MLP_NPARAM} parameters, got {p.size}")
        nb = C.c_size_t()
        L.check(ctx.lib.sw_mlp_workspace_bytes(C.byref(nb)))
        self.ws = _workspace(nb.value, ctx.device)
        h = C.c_void_p()
        L.check(ctx.lib.sw_mlp_create(ctx.h, _ptr(p), C.c_void_p(self.ws.data_ptr()), nb.value, C.byref(h)))
        self.h = h

    @staticmethod
    def initial_params(ctx: Context, seed=0):
        """Untrained parameters (sw_mlp_init_params): the guess they give is
        the quadratic extrapolation."""
        p = np.zeros(L.MLP_NPARAM, np.float32)
        L.check(ctx.lib.sw_mlp_init_params(int(seed), _ptr(p)))
        return p

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.sw_mlp_destroy(self.h)
            self.h = None

    def params(self):
        out = np.zeros(L.MLP_NPARAM, np.float32)
        L.check(self.ctx.lib.sw_mlp_get_params(self.h, _ptr(out)))
        return out

    def forward(self, X):
        torch = _torch()
        X = X.to(self.ctx.device, torch.float32).contiguous()
        if X.dim() != 2 or X.shape[1] != 10:
            raise ValueError("X must be (n, 10)")
        y = torch.empty(X.shape[0], dtype=torch.float32, device=self.ctx.device)
        L.check(self.ctx.lib.sw_mlp_forward(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                            X.shape[0]))
        return y

    @staticmethod
    def _rows(S, device):
        torch = _torch()
        S = S.to(device, torch.float32).contiguous()
        if S.dim() != 2 or S.shape[1] != L.MLP_ROW:
            raise ValueError(f"sample rows must be (n, {L.MLP_ROW})")
        return S

    def gradient(self, S):
        S = self._rows(S, self.ctx.device)
        g = np.zeros(L.MLP_NPARAM)
        loss = C.c_double()
        L.check(self.ctx.lib.sw_mlp_gradient(self.h, C.c_void_p(S.data_ptr()), S.shape[0], _ptr(g),
                                             C.byref(loss)))
        return g, loss.value

    def train(self, S, steps, batch=4096, lr=1e-3, seed=0):
        S = self._rows(S, self.ctx.device)
        losses = np.zeros(steps, np.float32)
        L.check(self.ctx.lib.sw_mlp_train(self.h, C.c_void_p(S.data_ptr()), S.shape[0], int(steps), int(batch),
                                          float(lr), int(seed), _ptr(losses)))
        return losses


def misfit(ctx: Context, U, obs):
    """ERR of Eq. (eqerr) between device waveforms U and obs, (n_steps, n_rec, 3)."""
    torch = _torch()
    U = U.to(ctx.device, torch.float64).contiguous()
    obs = obs.to(ctx.device, torch.float64).contiguous()
    if U.dim() != 3 or U.shape != obs.shape or U.shape[2] != 3:
        raise ValueError("U and obs must both be (n_steps, n_rec, 3)")
    n_steps, n_rec = U.shape[0], U.shape[1]
    nb = C.c_size_t()
    L.check(ctx.lib.sw_misfit_workspace_bytes(n_rec, C.byref(nb)))
    ws = _workspace(nb.value, ctx.device)
    e = C.c_double()
    n = C.c_int32()
    L.check(ctx.lib.sw_misfit(ctx.h, n_rec, n_steps, C.c_void_p(U.data_ptr()), C.c_void_p(obs.data_ptr()),
                              C.c_void_p(ws.data_ptr()), nb.value, C.byref(e), C.byref(n)))
    return e.value, n.value


def fit_input(ctx: Context, green, obs, stride, n_shift, rel_cut=1e-6, return_response=False):
    """Input estimation and ERR of Section 2 (sw_fit_input).  green: three
    device tensors (n_steps, n_rec, 3), the Green's records for the impulse
    along x1, x2, x3; obs: device tensor of the same shape.  Returns
    (c (3, n_shift), ERR, pairs used, rank[, fitted response])."""
    torch = _torch()
    green = [g.to(ctx.device, torch.float64).contiguous() for g in green]
    obs = obs.to(ctx.device, torch.float64).contiguous()
    n_steps, n_rec = int(obs.shape[0]), int(obs.shape[1])
    for g in green:
        if tuple(g.shape) != (n_steps, n_rec, 3):
            raise ValueError("Green's records must have the shape of obs")
    nb = C.c_size_t()
    L.check(ctx.lib.sw_fit_workspace_bytes(n_rec, n_steps, int(stride), int(n_shift), C.byref(nb)))
    ws = _workspace(nb.value, ctx.device)
    ptrs = (C.c_void_p * 3)(*[g.data_ptr() for g in green])
    c = np.zeros((3, int(n_shift)))
    e, used, rank = C.c_double(), C.c_int32(), C.c_int32()
    U = torch.empty_like(obs) if return_response else None
    L.check(ctx.lib.sw_fit_input(ctx.h, n_rec, n_steps, ptrs, C.c_void_p(obs.data_ptr()), int(stride), int(n_shift),
                                 float(rel_cut), C.c_void_p(ws.data_ptr()), nb.value, _ptr(c), C.byref(e),
                                 C.byref(used), C.byref(rank), C.c_void_p(U.data_ptr() if U is not None else 0)))
    out = (c, e.value, used.value, rank.value)
    return out + (U,) if return_response else out


def fit_events(ctx: Context, green, events, stride, n_shift, rel_cut=1e-6):
    """One model's misfit over several observed events (sw_fit_events): the
    Green's records are the model's, the input is estimated per event, and
    the model's misfit is its worst event's.  Returns the list of
    (c (3, n_shift), ERR, pairs, rank) per event, the largest ERR and the
    index of that event."""
    torch = _torch()
    green = [g.to(ctx.device, torch.float64).contiguous() for g in green]
    events = [o.to(ctx.device, torch.float64).contiguous() for o in events]
    n_steps, n_rec = int(events[0].shape[0]), int(events[0].shape[1])
    for t in green + events:
        if tuple(t.shape) != (n_steps, n_rec, 3):
            raise ValueError("Green's and observed records must all have the same (n_steps, n_rec, 3) shape")
    ne = len(events)
    nb = C.c_size_t()
    L.check(ctx.lib.sw_fit_workspace_bytes(n_rec, n_steps, int(stride), int(n_shift), C.byref(nb)))
    ws = _workspace(nb.value, ctx.device)
    gp = (C.c_void_p * 3)(*[g.data_ptr() for g in green])
    op = (C.c_void_p * ne)(*[o.data_ptr() for o in events])
    c = np.zeros((ne, 3, int(n_shift)))
    err = np.zeros(ne)
    used = np.zeros(ne, np.int32)
    rank = np.zeros(ne, np.int32)
    emax, worst = C.c_double(), C.c_int32()
    L.check(ctx.lib.sw_fit_events(ctx.h, n_rec, n_steps, gp, ne, op, int(stride), int(n_shift), float(rel_cut),
                                  C.c_void_p(ws.data_ptr()), nb.value, _ptr(c), _ptr(err), _ptr(used), _ptr(rank),
                                  C.byref(emax), C.byref(worst)))
    fits = [(c[e], float(err[e]), int(used[e]), int(rank[e])) for e in range(ne)]
    return fits, emax.value, worst.value


class Batch:
    """Several cases marched together (see sw_batch_* in include/sw.h)."""

    def __init__(self, ctx: Context, cases):
        self.ctx, self.cases = ctx, list(cases)
        arr = (C.c_void_p * len(self.cases))(*[c.h.value for c in self.cases])
        nb = C.c_size_t()
        L.check(ctx.lib.sw_batch_workspace_bytes(arr, len(self.cases), C.byref(nb)))
        self.ws = _workspace(nb.value, ctx.device)
        h = C.c_void_p()
        L.check(ctx.lib.sw_batch_create(ctx.h, arr, len(self.cases), C.c_void_p(self.ws.data_ptr()), nb.value,
                                        C.byref(h)))
        self.h = h

    def step(self, n=1):
        L.check(self.ctx.lib.sw_batch_step(self.h, int(n)))

    def autotune(self, reps=5):
        """Pick the fastest lane-pass schedule (sw_batch_autotune); returns
        (choice, mean ms of each of the 4 candidates)."""
        ch = C.c_int32()
        ms = np.zeros(4)
        L.check(self.ctx.lib.sw_batch_autotune(self.h, int(reps), C.byref(ch), _ptr(ms)))
        return ch.value, ms

    def stats(self):
        """Statistics of every lane (sw_batch_stats), in lane order."""
        out = (L.CaseStats * len(self.cases))()
        L.check(self.ctx.lib.sw_batch_stats(self.h, out))
        return [{"steps": s.steps, "cg_iters": s.cg_iters, "ir_outer": s.ir_outer,
                 "max_true_rel_res": s.max_true_rel_res, "flags": s.flags} for s in out]

    def apply_f32(self, xs):
        """Lane pass y_l = A_l x_l (FP32 device vectors, one per case)."""
        torch = _torch()
        xs = [c._vec(x, torch.float32) for c, x in zip(self.cases, xs)]
        ys = [torch.empty_like(x) for x in xs]
        xa = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        ya = (C.c_void_p * len(ys))(*[y.data_ptr() for y in ys])
        L.check(self.ctx.lib.sw_batch_apply_f32(self.h, xa, ya))
        return ys

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.sw_batch_destroy(self.h)
            self.h = None
