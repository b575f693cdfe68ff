"""Seeded synthetic inputs for the wave-propagation analyses.

This module produces *inputs only*: meshes, per-case material maps, the
incident wavelet and receiver lists.  It holds none of the method's
arithmetic (no element matrices, no time march, no solver) and is shared
by the CPU oracle, the tests and the benchmark.

What it stands in for: the paper's candidate models are octree meshes of
second-order tetrahedra built from 120 borehole depths, driven by KiK-net
borehole records (Section 3).  Neither the records nor the depths are
available, so the cases here are boxes of hexahedral cells, each split into
six quadratic tetrahedra, with a two-layer material law whose interface
depth is a seeded smooth random field, driven by a Ricker wavelet.

Conventions (also the library's conventions):
  * x3 (z) points up; the free surface is z = 0, the base is z = -Lz.
  * tet10 node order: vertices 0..3, then edge nodes 01, 12, 02, 03, 13, 23;
    every tetrahedron has positive volume.
  * tri6 node order: vertices 0..2, then edge nodes 01, 12, 20.
  * face_role: 1 = absorbing side face, 2 = absorbing base face that also
    carries the input force.
  * material table rows are (Vp, Vs, rho).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# VTK quadratic-tetrahedron edge order
TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))

SOFT = (1600.0, 150.0, 1800.0)   # Vp, Vs, rho of the sedimentary layer
ROCK = (2000.0, 500.0, 2000.0)   # Vp, Vs, rho of the bedrock


@dataclass
class Mesh:
    xyz: np.ndarray        # (n_nodes, 3) float64
    tet10: np.ndarray      # (n_tets, 10) int32
    tri6: np.ndarray       # (n_faces, 6) int32
    face_tet: np.ndarray   # (n_faces,) int32
    face_role: np.ndarray  # (n_faces,) uint8
    box: tuple = (0.0, 0.0, 0.0)
    cell: float = 0.0
    ncell: tuple = (0, 0, 0)

    @property
    def n_nodes(self):
        return int(self.xyz.shape[0])

    @property
    def n_tets(self):
        return int(self.tet10.shape[0])

    @property
    def n_faces(self):
        return int(self.tri6.shape[0])


@dataclass
class Case:
    """Per-analysis inputs on a given mesh."""
    mat: np.ndarray        # (n_mat, 3) float64 rows (Vp, Vs, rho)
    tet_mat: np.ndarray    # (n_tets,) uint8
    rec_node: np.ndarray   # (n_rec,) int32
    v_in: np.ndarray       # (n_steps + 1, 3) incident velocity at t = n dt
    dt: float
    n_steps: int
    ray_alpha: float
    ray_beta: float
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------- mesh

def _kuhn_cell():
    """Six tetrahedra of the unit cell split along its (0,0,0)-(1,1,1)
    diagonal, as half-lattice offsets in {0,1,2}^3 for all ten nodes."""
    tets = []
    for perm in itertools.permutations(range(3)):
        e = np.eye(3, dtype=np.int64) * 2
        v = [np.zeros(3, np.int64), e[perm[0]], e[perm[0]] + e[perm[1]],
             np.full(3, 2, np.int64)]
        d = np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]).astype(float))
        if d < 0:
            v[1], v[2] = v[2], v[1]
        nodes = list(v) + [(v[a] + v[b]) // 2 for a, b in TET_EDGES]
        tets.append(np.stack(nodes))
    return np.stack(tets)  # (6, 10, 3)


def graded_levels(Lz, h_top, ratio):
    """Vertex depths from -Lz up to 0 of layers whose thickness is h_top at
    the surface and grows by ``ratio`` per layer downwards (the last layer
    takes what is left, merged into the one above when thinner than half of
    it): a mesh refined towards the surface, as the paper's are near the
    soft layer."""
    th, z = [], 0.0
    t = h_top
    while z + t < Lz - 1e-9:
        th.append(t)
        z += t
        t *= ratio
    rest = Lz - z
    if th and rest < 0.5 * th[-1]:
        th[-1] += rest
    else:
        th.append(rest)
    levels = -np.concatenate([[0.0], np.cumsum(th)])      # 0 at the top, downwards
    return levels[::-1].copy()                             # -Lz .. 0


def box_mesh(Lx, Ly, Lz, h, jitter=0.0, seed=12345, z_levels=None) -> Mesh:
    """Structured box [0,Lx]x[0,Ly]x[-Lz,0] of cubic cells of edge h, each
    split into six 10-node tetrahedra (conforming Kuhn split).

    ``z_levels`` (optional): the vertex depths, increasing from -Lz to 0,
    of layers of varying thickness (x and y spacing stays h), e.g. from
    graded_levels.

    ``jitter`` > 0 moves every interior vertex node by a seeded uniform
    offset of at most jitter times the local spacing per coordinate; every
    edge node is then put back at the middle of its (straight) edge.  The
    result is a mesh with no lattice structure left in its geometry, for
    tests that must not rely on one.
    """
    nx, ny = int(round(Lx / h)), int(round(Ly / h))
    assert abs(nx * h - Lx) < 1e-9 and abs(ny * h - Ly) < 1e-9
    if z_levels is None:
        nz = int(round(Lz / h))
        assert abs(nz * h - Lz) < 1e-9
        zv = -Lz + np.arange(nz + 1, dtype=np.float64) * h
    else:
        zv = np.asarray(z_levels, np.float64)
        nz = len(zv) - 1
        assert nz >= 1 and abs(zv[0] + Lz) < 1e-9 and abs(zv[-1]) < 1e-9 and np.all(np.diff(zv) > 0)
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    I = np.arange(NX, dtype=np.float64) * (h / 2)
    J = np.arange(NY, dtype=np.float64) * (h / 2)
    K = np.empty(NZ)
    K[0::2] = zv
    K[1::2] = 0.5 * (zv[:-1] + zv[1:])
    xyz = np.empty((NZ, NY, NX, 3), np.float64)
    xyz[..., 0] = I[None, None, :]
    xyz[..., 1] = J[None, :, None]
    xyz[..., 2] = K[:, None, None]
    xyz = xyz.reshape(-1, 3)

    loc = _kuhn_cell()  # (6,10,3)
    loc_off = (loc[..., 2] * NY + loc[..., 1]) * NX + loc[..., 0]  # (6,10)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # cell-major order, x fastest
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    base = ((2 * ck) * NY + 2 * cj) * NX + 2 * ci  # (ncell,)
    tet10 = (base[:, None, None] + loc_off[None]).reshape(-1, 10).astype(np.int32)

    if jitter > 0:
        rng = np.random.default_rng(seed)
        g = np.stack(np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij"), -1).reshape(-1, 3)
        gk, gj, gi = g[:, 0], g[:, 1], g[:, 2]
        is_vert = (gi % 2 == 0) & (gj % 2 == 0) & (gk % 2 == 0)
        interior = (gi > 0) & (gi < NX - 1) & (gj > 0) & (gj < NY - 1) & (gk > 0) & (gk < NZ - 1)
        mv = is_vert & interior
        off = rng.uniform(-jitter, jitter, (int(mv.sum()), 3))
        # local vertical spacing: the thinner of the two layers at the vertex
        kk = gk[mv] // 2
        hz = np.minimum(zv[kk] - zv[kk - 1], zv[kk + 1] - zv[kk])
        off[:, :2] *= h
        off[:, 2] *= hz
        xyz[mv] += off
        mid = ~is_vert
        d = np.stack([gi % 2, gj % 2, gk % 2], -1)[mid]
        p = np.stack([gi, gj, gk], -1)[mid]
        lo, hi = p - d, p + d
        ilo = (lo[:, 2] * NY + lo[:, 1]) * NX + lo[:, 0]
        ihi = (hi[:, 2] * NY + hi[:, 1]) * NX + hi[:, 0]
        xyz[mid] = 0.5 * (xyz[ilo] + xyz[ihi])

    tri6, face_tet, face_role = _boundary_faces(tet10, xyz, nx, ny, nz, Lx, Ly, Lz)
    return Mesh(xyz=xyz, tet10=tet10, tri6=tri6, face_tet=face_tet, face_role=face_role,
                box=(float(Lx), float(Ly), float(Lz)), cell=float(h), ncell=(nx, ny, nz))


def refined_levels(Lz, z_int, h_fine, h_coarse, ratio=1.5):
    """Vertex depths from -Lz to 0: spacing h_fine at depth z_int (below the
    surface), growing by ``ratio`` per layer upwards and downwards up to
    h_coarse: layers refined towards a layer interface."""
    up, down = [], []
    h, z = h_fine, -z_int
    while z + h < -1e-9:
        z += h
        up.append(z)
        h = min(h * ratio, h_coarse)
    h, z = h_fine, -z_int
    while z - h > -Lz + 1e-9:
        z -= h
        down.append(z)
        h = min(h * ratio, h_coarse)
    return np.array(sorted([-Lz] + down + [-z_int] + up + [0.0]))


def delaunay_mesh(Lx, Ly, Lz, z_int, h_fine, h_coarse, ratio=1.5, jitter=0.3, seed=0) -> Mesh:
    """Unstructured 10-node tetrahedral mesh of the box [0,Lx]x[0,Ly]x[-Lz,0],
    refined towards depth z_int (e.g. a layer interface): seeded points on
    layers of refined_levels, each layer a grid whose spacing is the local
    layer thickness, every point moved by a seeded uniform offset of up to
    ``jitter`` times the local spacing (points on a box face stay on it),
    tetrahedralised by scipy.spatial.Delaunay; edge nodes at the edge
    midpoints.  Element sizes vary about fourfold and no lattice is left
    in the connectivity.  ncell is (0, 0, 0) (no cell grid)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng([seed, 5])
    zl = refined_levels(Lz, z_int, h_fine, h_coarse, ratio)
    dz = np.diff(zl)
    pts = []
    for k, z in enumerate(zl):
        hz = min(dz[max(k - 1, 0)], dz[min(k, len(dz) - 1)])
        nx, ny = max(1, int(round(Lx / hz))), max(1, int(round(Ly / hz)))
        X, Y = np.meshgrid(np.linspace(0.0, Lx, nx + 1), np.linspace(0.0, Ly, ny + 1), indexing="ij")
        P = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1)
        off = rng.uniform(-jitter, jitter, P.shape) * np.array([Lx / nx, Ly / ny, hz])
        off[(np.abs(P[:, 0]) < 1e-9) | (np.abs(P[:, 0] - Lx) < 1e-9), 0] = 0.0
        off[(np.abs(P[:, 1]) < 1e-9) | (np.abs(P[:, 1] - Ly) < 1e-9), 1] = 0.0
        if k == 0 or k == len(zl) - 1:
            off[:, 2] = 0.0
        pts.append(P + off)
    pts = np.concatenate(pts)
    T = Delaunay(pts).simplices.astype(np.int64)
    X = pts[T]
    vol = np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))
    T = T[vol != 0.0]
    neg = np.einsum("ij,ij->i", *(lambda X: (X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])))(pts[T])) < 0
    T[neg, 1], T[neg, 2] = T[neg, 2].copy(), T[neg, 1].copy()
    nv = len(pts)
    # edge nodes
    E = np.stack([np.sort(T[:, [a, b]], 1) for a, b in TET_EDGES], 1)         # (n, 6, 2)
    key = E[..., 0] * nv + E[..., 1]
    ukey, inv = np.unique(key.ravel(), return_inverse=True)
    ea, eb = ukey // nv, ukey % nv
    xyz = np.concatenate([pts, 0.5 * (pts[ea] + pts[eb])])
    tet10 = np.concatenate([T, nv + inv.reshape(-1, 6)], 1).astype(np.int32)
    # boundary faces: faces of one tet only, all on the sides or the base
    tri, own, role = [], [], []
    tol = 1e-9 * max(Lx, Ly, Lz)
    allf = np.concatenate([np.sort(tet10[:, list(v)], 1) for v, _ in _TET_FACES])
    fkey = (allf[:, 0].astype(np.int64) * nv + allf[:, 1]) * nv + allf[:, 2]
    uk, cnt = np.unique(fkey, return_counts=True)
    single = set(uk[cnt == 1].tolist())
    n = tet10.shape[0]
    for fi, (verts, edges) in enumerate(_TET_FACES):
        fv = tet10[:, list(verts)]
        k3 = np.sort(fv, 1).astype(np.int64)
        kk = (k3[:, 0] * nv + k3[:, 1]) * nv + k3[:, 2]
        on_b = np.fromiter((int(v) in single for v in kk), bool, n)
        P = xyz[fv]
        for m, r in ((np.all(np.abs(P[..., 0]) < tol, 1), 1), (np.all(np.abs(P[..., 0] - Lx) < tol, 1), 1),
                     (np.all(np.abs(P[..., 1]) < tol, 1), 1), (np.all(np.abs(P[..., 1] - Ly) < tol, 1), 1),
                     (np.all(np.abs(P[..., 2] + Lz) < tol, 1), 2)):
            sel = np.nonzero(m & on_b)[0]
            if sel.size:
                tri.append(np.concatenate([fv[sel], tet10[sel][:, list(edges)]], 1))
                own.append(sel)
                role.append(np.full(sel.size, r, np.uint8))
    tri6 = np.concatenate(tri).astype(np.int32)
    face_tet = np.concatenate(own).astype(np.int32)
    face_role = np.concatenate(role)
    o = np.lexsort((face_tet, face_role))
    return Mesh(xyz=xyz, tet10=tet10, tri6=tri6[o], face_tet=face_tet[o], face_role=face_role[o],
                box=(float(Lx), float(Ly), float(Lz)), cell=float(h_coarse), ncell=(0, 0, 0))


# faces of a tet: (vertex triple, the tet-local edge slots of edges 01,12,20)
_TET_FACES = (
    ((0, 1, 2), (4, 5, 6)),
    ((0, 1, 3), (4, 8, 7)),
    ((1, 2, 3), (5, 9, 8)),
    ((0, 2, 3), (6, 9, 7)),
)


def _boundary_faces(tet10, xyz, nx, ny, nz, Lx, Ly, Lz):
    """Side and base faces.  Only tets of boundary cells are examined; a face
    is on a boundary plane when its three vertices share that plane."""
    ncell = nx * ny * nz
    c = np.arange(ncell)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    bc = np.nonzero((i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1) | (k == 0))[0]
    tets = (bc[:, None] * 6 + np.arange(6)[None]).ravel()
    T = tet10[tets]
    tri, own, role = [], [], []
    tol = 1e-9 * max(Lx, Ly, Lz)
    for verts, edges in _TET_FACES:
        fv = T[:, list(verts)]
        P = xyz[fv]  # (m,3,3)
        planes = (
            (np.all(np.abs(P[..., 0]) < tol, 1), 1),
            (np.all(np.abs(P[..., 0] - Lx) < tol, 1), 1),
            (np.all(np.abs(P[..., 1]) < tol, 1), 1),
            (np.all(np.abs(P[..., 1] - Ly) < tol, 1), 1),
            (np.all(np.abs(P[..., 2] + Lz) < tol, 1), 2),
        )
        for m, r in planes:
            sel = np.nonzero(m)[0]
            if sel.size == 0:
                continue
            tri.append(np.concatenate([fv[sel], T[sel][:, list(edges)]], 1))
            own.append(tets[sel])
            role.append(np.full(sel.size, r, np.uint8))
    tri6 = np.concatenate(tri).astype(np.int32)
    face_tet = np.concatenate(own).astype(np.int32)
    face_role = np.concatenate(role)
    o = np.lexsort((face_tet, face_role))
    return tri6[o], face_tet[o], face_role[o]


# ------------------------------------------------------------ materials

def interface_field(seed, amp, corr, nmodes=256):
    """Smooth random field g(x, y) as a sum of random Fourier features with
    Gaussian covariance exp(-r^2/corr^2).  Returns (kx, ky, phase) so the
    field can be evaluated anywhere; the amplitude is applied by
    ``interface_depth``."""
    rng = np.random.default_rng(seed)
    k = rng.normal(0.0, math.sqrt(2.0) / corr, (nmodes, 2))
    ph = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    return k, ph


def _rff_eval(k, ph, x, y, chunk=1 << 18):
    out = np.empty(x.shape, np.float64)
    xf, yf, of = x.ravel(), y.ravel(), out.ravel()
    for s in range(0, xf.size, chunk):
        arg = np.outer(xf[s:s + chunk], k[:, 0]) + np.outer(yf[s:s + chunk], k[:, 1]) + ph[None]
        of[s:s + chunk] = np.cos(arg).sum(1)
    return out


def interface_depth(mesh: Mesh, seed, h0, amp, corr):
    """Returns a callable depth(x, y) = h0 + g(x, y), where g is scaled so
    that its largest magnitude over the centres of the surface cell grid (on
    a mesh without one, a grid of the mesh's coarse spacing) is ``amp``."""
    k, ph = interface_field(seed, amp, corr)
    nx, ny, _ = mesh.ncell
    Lx, Ly, _ = mesh.box
    if nx == 0:  # no cell grid: columns of the mesh's coarse spacing
        nx, ny = max(1, int(round(Lx / mesh.cell))), max(1, int(round(Ly / mesh.cell)))
    xc = (np.arange(nx) + 0.5) * (Lx / nx)
    yc = (np.arange(ny) + 0.5) * (Ly / ny)
    X, Y = np.meshgrid(xc, yc, indexing="ij")
    g = _rff_eval(k, ph, X, Y)
    scale = amp / max(np.max(np.abs(g)), 1e-300)

    def depth(x, y):
        return h0 + scale * _rff_eval(k, ph, np.asarray(x, float), np.asarray(y, float))

    return depth


def tet_centroids(mesh: Mesh, chunk=1 << 20):
    out = np.empty((mesh.n_tets, 3), np.float64)
    for s in range(0, mesh.n_tets, chunk):
        out[s:s + chunk] = mesh.xyz[mesh.tet10[s:s + chunk, :4]].mean(1)
    return out


def two_layer_materials(mesh: Mesh, depth_fn):
    """Material id per tet: 0 (soft) if the centroid lies above the
    interface (depth below surface < h(x, y)), else 1 (bedrock)."""
    c = tet_centroids(mesh)
    # evaluate the field once per distinct (x, y) centroid position
    q = np.rint(c[:, :2] * 1e6).astype(np.int64)
    key = (q[:, 0] - q[:, 0].min()) * (int(q[:, 1].max() - q[:, 1].min()) + 1) + (q[:, 1] - q[:, 1].min())
    ukey, first, inv = np.unique(key, return_index=True, return_inverse=True)
    d = depth_fn(c[first, 0], c[first, 1])[inv.ravel()]
    return np.where(-c[:, 2] < d, 0, 1).astype(np.uint8)


def material_table():
    return np.array([SOFT, ROCK], np.float64)


# ----------------------------------------------------------- wavelets

def ricker(t, fp, t0):
    """Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0."""
    a = (math.pi * fp * (np.asarray(t, float) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def incident_velocity(n_steps, dt, freqs, t0, direction=0):
    """Incident velocity at t = n dt, n = 0..n_steps; a sum of unit Ricker
    wavelets with common delay t0, along ``direction`` (0 = x1 gives a
    vertically incident SV wave)."""
    t = np.arange(n_steps + 1) * dt
    w = sum(ricker(t, f, t0) for f in freqs)
    v = np.zeros((n_steps + 1, 3))
    v[:, direction] = w
    return v


def hann_impulse(n_steps, stride):
    """Unit impulse p of the input parametrisation, sampled at the time
    steps n = 0..n_steps: a Hann pulse sin^2(pi n / (2 stride)) on
    0 <= n <= 2 stride (peak 1 at n = stride), zero elsewhere.  Copies
    shifted by multiples of the stride sum to one (partition of unity)."""
    n = np.arange(n_steps + 1, dtype=float)
    p = np.sin(np.pi * n / (2.0 * stride)) ** 2
    p[n > 2 * stride] = 0.0
    return p


def impulse_inputs(n_steps, stride):
    """The three inputs of the Green's-function runs: the unit impulse along
    x1, x2 and x3 ((n_steps + 1) x 3 each)."""
    p = hann_impulse(n_steps, stride)
    out = []
    for j in range(3):
        v = np.zeros((n_steps + 1, 3))
        v[:, j] = p
        out.append(v)
    return out


def rayleigh_coefficients(xi, f1, f2):
    """Mass/stiffness-proportional coefficients giving damping ratio xi at
    frequencies f1 and f2 (Hz)."""
    w1, w2 = 2 * math.pi * f1, 2 * math.pi * f2
    return 2 * xi * w1 * w2 / (w1 + w2), 2 * xi / (w1 + w2)


# ----------------------------------------------------------- receivers

def surface_receivers(mesh: Mesh, n):
    """n x n grid of surface nodes at ((i+1/2) Lx/n, (j+1/2) Ly/n, 0); on a
    mesh without a cell grid, the surface nodes nearest to those points."""
    Lx, Ly, _ = mesh.box
    xs = (np.arange(n) + 0.5) * (Lx / n)
    ys = (np.arange(n) + 0.5) * (Ly / n)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    target = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    if mesh.ncell == (0, 0, 0):
        top = np.nonzero(np.abs(mesh.xyz[:, 2]) < 1e-9)[0]
        d = ((mesh.xyz[top][None, :, :2] - target[:, None, :2]) ** 2).sum(-1)
        return top[np.argmin(d, 1)].astype(np.int32)
    nx, ny, nz = mesh.ncell
    NX, NY = 2 * nx + 1, 2 * ny + 1
    hh = mesh.cell / 2
    gi = np.rint(target[:, 0] / hh).astype(np.int64)
    gj = np.rint(target[:, 1] / hh).astype(np.int64)
    ids = ((2 * nz) * NY + gj) * NX + gi
    if not np.allclose(mesh.xyz[ids], target, atol=1e-6 * mesh.cell):
        raise ValueError("receiver grid does not land on mesh nodes")
    return ids.astype(np.int32)


# ----------------------------------------------------------- configs

@dataclass(frozen=True)
class BoxConfig:
    name: str
    box: tuple            # (Lx, Ly, Lz) metres
    cell: float           # hex cell edge, metres
    h0: float             # mean interface depth
    amp: float            # interface amplitude (or range for batches)
    corr: float           # interface correlation length (or range)
    freqs: tuple          # Ricker peak frequencies (summed)
    t0: float             # Ricker delay
    dt: float
    n_steps: int
    n_rec: int            # receivers per side
    seed: int


CONFIGS = {
    # plain FP64 single case, 3000 tets, 14,553 DOF
    "small": BoxConfig("small", (100.0, 100.0, 50.0), 10.0, 20.0, 8.0, 40.0, (2.0,), 0.5, 0.01, 50, 10, 0),
    # single large case, 9.6 M tets, 39.07 M DOF
    "large": BoxConfig("large", (1000.0, 1000.0, 200.0), 5.0, 40.0, 15.0, 150.0, (2.5,), 0.4, 0.005, 400, 20, 1),
    # batched uneven cases (first of the three sizes; the others differ in box)
    "batch200": BoxConfig("batch200", (200.0, 200.0, 100.0), 5.0, 30.0, (5.0, 20.0), (50.0, 200.0), (2.0,), 0.5, 0.005, 1000, 20, 1000),
    "batch300": BoxConfig("batch300", (300.0, 300.0, 100.0), 5.0, 30.0, (5.0, 20.0), (50.0, 200.0), (2.0,), 0.5, 0.005, 1000, 20, 1000),
    "batch400": BoxConfig("batch400", (400.0, 400.0, 100.0), 5.0, 30.0, (5.0, 20.0), (50.0, 200.0), (2.0,), 0.5, 0.005, 1000, 20, 1000),
    # full selection sweep mesh, 4.8 M tets, 19.78 M DOF
    "sweep": BoxConfig("sweep", (1000.0, 1000.0, 100.0), 5.0, 30.0, (5.0, 20.0), (50.0, 200.0), (1.0, 2.0, 4.0), 1.0, 0.005, 2000, 50, 3000),
}


def config_mesh(cfg: BoxConfig, jitter=0.0) -> Mesh:
    return box_mesh(*cfg.box, cfg.cell, jitter=jitter)


def make_case(mesh: Mesh, cfg: BoxConfig, seed=None, n_steps=None, xi=0.02, damp_f=(1.0, 5.0),
              n_rec=None) -> Case:
    """Case on ``mesh`` following ``cfg``.  For batch configs (amp and corr
    given as ranges) the case seed also draws the amplitude and correlation
    length uniformly from those ranges."""
    seed = cfg.seed if seed is None else seed
    n_steps = cfg.n_steps if n_steps is None else n_steps
    amp, corr = cfg.amp, cfg.corr
    if isinstance(amp, tuple):
        r = np.random.default_rng([seed, 7])
        amp = float(r.uniform(*amp))
        corr = float(r.uniform(*corr))
    depth = interface_depth(mesh, seed, cfg.h0, amp, corr)
    tet_mat = two_layer_materials(mesh, depth)
    a, b = rayleigh_coefficients(xi, *damp_f)
    return Case(mat=material_table(), tet_mat=tet_mat,
                rec_node=surface_receivers(mesh, cfg.n_rec if n_rec is None else n_rec),
                v_in=incident_velocity(n_steps, cfg.dt, cfg.freqs, cfg.t0),
                dt=cfg.dt, n_steps=n_steps, ray_alpha=a, ray_beta=b,
                meta=dict(seed=seed, amp=amp, corr=corr, h0=cfg.h0))


def smooth_field(mesh: Mesh, seed, corr, amp, nmodes=32, chunk=1 << 18):
    """Seeded smooth random vector field at the nodes (3 * n_nodes values,
    node-major): per component a sum of random Fourier features in 3D with
    Gaussian covariance exp(-r^2/corr^2), scaled so that its largest
    magnitude over the nodes is ``amp``.  Used as an initial velocity that
    sets every element of a large mesh in motion from the first step."""
    rng = np.random.default_rng([seed, 11])
    out = np.empty((mesh.n_nodes, 3))
    for c in range(3):
        k = rng.normal(0.0, math.sqrt(2.0) / corr, (nmodes, 3))
        ph = rng.uniform(0.0, 2.0 * math.pi, nmodes)
        for s in range(0, mesh.n_nodes, chunk):
            out[s:s + chunk, c] = np.cos(mesh.xyz[s:s + chunk] @ k.T + ph[None]).sum(1)
    out *= amp / max(np.abs(out).max(), 1e-300)
    return out.ravel()


def random_vector(n, seed, dtype=np.float64):
    """Seeded standard-normal vector for operator parity tests."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)
