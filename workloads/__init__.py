"""Seeded synthetic inputs for the node-patch Poisson-Boltzmann solver.

This module only *makes inputs*: closed triangulated surfaces, atom positions,
charges and radii, and the physical parameters of each workload.  It holds none
of the solver's arithmetic (no kernels, no patch geometry, no quadrature), so
that both the FP64 CPU oracle and the GPU path can read the same inputs while
sharing no code.

Workloads (stand-ins for the paper's molecules; the paper's PQR files and
TMSmesh meshes are not available):

* ``born_ion``      -- one +1 e charge at the centre of an icosphere of radius
                       2 A (level 4: 2,562 nodes / 5,120 triangles); the
                       paper's analytic sphere test (Section 5) at small size.
* ``globular``      -- 5,000 atoms by a seeded self-avoiding walk inside
                       25 A, Gaussian-density isosurface meshed by marching
                       tetrahedra on a 1.25 A grid (~100k triangles).
* ``star_request``  -- the serving stream's star-shaped molecules
                       r(x) = R max(0.3, 1 + sum a_lm Y_lm(x)).
* ``complex_100k``  -- 100,000 atoms inside 90 A, same generator.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` with a fixed
draw order.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Molecule", "icosphere", "born_ion", "saw_atoms", "gaussian_surface",
    "gaussian_surface_native", "shell_atoms", "globular", "complex_100k",
    "capsid_shell", "star_request", "check_closed_manifold", "random_rigid_motion",
]

# grid spacing of the capsid-scale shell's isosurface (A)
CAPSID_H_GRID = 2.5


@dataclass
class Molecule:
    """One solve request: surface mesh + atoms + physical parameters."""
    name: str
    xyz: np.ndarray          # float64 [N,3] mesh nodes (A)
    tri: np.ndarray          # int32  [M,3] triangles, CCW seen from the solvent
    atom_xyz: np.ndarray     # float64 [K,3] (A)
    charge: np.ndarray       # float64 [K]   (e)
    radius: np.ndarray       # float64 [K]   (A), used only to make the surface
    eps_p: float = 2.0
    eps_s: float = 80.0
    kappa: float = 0.1       # 1/A
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_unknowns(self) -> int:
        return 2 * self.n_nodes


# ---------------------------------------------------------------------------
# Icosphere
# ---------------------------------------------------------------------------

def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a, b in itertools.product((-1.0, 1.0), repeat=2):
        v.append((0.0, a, b * phi))
        v.append((a, b * phi, 0.0))
        v.append((b * phi, 0.0, a))
    v = np.array(v, dtype=np.float64)
    # Faces: all triples of mutually nearest vertices (edge length 2).
    n = len(v)
    d2 = ((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)
    adj = np.abs(d2 - 4.0) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    c = v[f].mean(0)
                    nrm = np.cross(v[j] - v[i], v[k] - v[i])
                    if nrm @ c < 0:
                        f = [i, k, j]
                    faces.append(f)
    assert len(faces) == 20
    return v, np.array(faces, dtype=np.int64)


def icosphere(level: int, radius: float = 1.0):
    """Icosahedron subdivided ``level`` times by edge midpoints, projected
    onto the sphere of the given radius.  V = 10*4^L + 2, T = 20*4^L."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        cache = {}
        newf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                pa, pb = verts[a], verts[b]
                verts.append(((pa[0] + pb[0]) / 2, (pa[1] + pb[1]) / 2,
                              (pa[2] + pb[2]) / 2))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(newf, dtype=np.int64)
    vv = np.array(verts, dtype=np.float64)
    vv /= np.linalg.norm(vv, axis=1, keepdims=True)
    return vv * radius, f.astype(np.int32)


def born_ion(level: int = 4, radius: float = 2.0, charge: float = 1.0,
             eps_p: float = 2.0, eps_s: float = 80.0, kappa: float = 0.1):
    """Config 'Born ion': one charge at the centre of an icosphere."""
    xyz, tri = icosphere(level, radius)
    return Molecule(
        name=f"born_ion_L{level}", xyz=xyz, tri=tri,
        atom_xyz=np.zeros((1, 3)), charge=np.array([charge]),
        radius=np.array([radius]), eps_p=eps_p, eps_s=eps_s, kappa=kappa,
        meta={"level": level, "sphere_radius": radius})


# ---------------------------------------------------------------------------
# Self-avoiding walk atoms
# ---------------------------------------------------------------------------

def _unit_vectors(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def saw_atoms(n: int, r_max: float, seed: int, step: float = 1.5,
              min_sep: float = 1.2, max_reject: int = 64):
    """Atoms by a seeded self-avoiding random walk inside a ball.

    Each step proposes x_{i-1} + step*u (u uniform on the sphere) and accepts
    it if |x| <= r_max and every other atom is at least ``min_sep`` away
    (grid hash).  After ``max_reject`` rejections the walk restarts from a
    uniformly chosen earlier atom.  Radii ~ U(1.2, 2.0); charges ~ N(0, 0.4)
    shifted to net charge 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cell = min_sep
    grid: dict[tuple, list] = {}
    pos = np.zeros((n, 3))

    def key(p):
        return (int(math.floor(p[0] / cell)), int(math.floor(p[1] / cell)),
                int(math.floor(p[2] / cell)))

    def ok(p):
        if p @ p > r_max * r_max:
            return False
        k = key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((k[0] + dx, k[1] + dy, k[2] + dz), ()):
                        d = pos[j] - p
                        if d @ d < min_sep * min_sep:
                            return False
        return True

    grid.setdefault(key(pos[0]), []).append(0)
    cur = 0
    count = 1
    rejects = 0
    while count < n:
        u = _unit_vectors(rng, 1)[0]
        p = pos[cur] + step * u
        if ok(p):
            pos[count] = p
            grid.setdefault(key(p), []).append(count)
            cur = count
            count += 1
            rejects = 0
        else:
            rejects += 1
            if rejects >= max_reject:
                cur = int(rng.integers(0, count))
                rejects = 0
    radius = rng.uniform(1.2, 2.0, n)
    q = rng.normal(0.0, 0.4, n)
    q -= q.mean()
    return pos, radius, q


# ---------------------------------------------------------------------------
# Gaussian-density isosurface by marching tetrahedra
# ---------------------------------------------------------------------------

# Freudenthal (Kuhn) split of the unit cube into 6 tetrahedra sharing the
# main diagonal (0,0,0)-(1,1,1).  Adjacent cubes split their shared face along
# the same diagonal, so the tetrahedra form one conforming complex and the
# zero set of the piecewise-linear interpolant is a closed surface.
def _kuhn_tets():
    tets = []
    for perm in itertools.permutations(range(3)):
        c = [0, 0, 0]
        t = [tuple(c)]
        for ax in perm:
            c[ax] = 1
            t.append(tuple(c))
        tets.append(t)
    return np.array(tets, dtype=np.int64)  # [6,4,3]


def _density(atoms, radii, lo, h, shape, beta, trunc=3.0):
    """rho(x) = sum_k exp(-beta (|x-r_k|^2 / R_k^2 - 1)), truncated at 3 R_k."""
    rho = np.zeros(shape, dtype=np.float64)
    gx = lo[0] + h * np.arange(shape[0])
    gy = lo[1] + h * np.arange(shape[1])
    gz = lo[2] + h * np.arange(shape[2])
    for (ax, ay, az), r in zip(atoms, radii):
        rc = trunc * r
        i0 = max(0, int(math.floor((ax - rc - lo[0]) / h)))
        i1 = min(shape[0], int(math.ceil((ax + rc - lo[0]) / h)) + 1)
        j0 = max(0, int(math.floor((ay - rc - lo[1]) / h)))
        j1 = min(shape[1], int(math.ceil((ay + rc - lo[1]) / h)) + 1)
        k0 = max(0, int(math.floor((az - rc - lo[2]) / h)))
        k1 = min(shape[2], int(math.ceil((az + rc - lo[2]) / h)) + 1)
        dx2 = (gx[i0:i1] - ax) ** 2
        dy2 = (gy[j0:j1] - ay) ** 2
        dz2 = (gz[k0:k1] - az) ** 2
        d2 = dx2[:, None, None] + dy2[None, :, None] + dz2[None, None, :]
        inv = 1.0 / (r * r)
        val = np.exp(-beta * (d2 * inv - 1.0))
        val[d2 > rc * rc] = 0.0
        rho[i0:i1, j0:j1, k0:k1] += val
    return rho


def gaussian_surface(atoms, radii, h_grid: float, beta: float = 2.0,
                     pad: float = 5.0, level: float = 1.0, clamp: float = 0.25):
    """Closed, outward-oriented triangulation of {rho = level}.

    Marching tetrahedra over the Freudenthal split of the grid cubes; mesh
    vertices sit on grid edges (welded by edge id) with the interpolation
    parameter clamped to [0.25, 0.75]: every vertex stays a quarter edge away
    from the grid points, which bounds the triangle quality from below
    (slivers from vertices next to a grid point make the node-patch system
    ill-conditioned and inaccurate).
    Triangles are oriented toward decreasing density (out of the molecule).
    """
    atoms = np.asarray(atoms, dtype=np.float64)
    lo = atoms.min(0) - pad
    hi = atoms.max(0) + pad
    shape = tuple(int(math.ceil((hi[a] - lo[a]) / h_grid)) + 1 for a in range(3))
    rho = _density(atoms, radii, lo, h_grid, shape, beta)
    F = rho - level
    F[F == 0.0] = 1e-300          # no grid value exactly on the level set
    inside = F > 0.0
    nx, ny, nz = shape
    # cubes with mixed signs
    c000 = inside[:-1, :-1, :-1]
    anyin = np.zeros((nx - 1, ny - 1, nz - 1), bool)
    allin = np.ones((nx - 1, ny - 1, nz - 1), bool)
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        s = inside[dx:nx - 1 + dx, dy:ny - 1 + dy, dz:nz - 1 + dz]
        anyin |= s
        allin &= s
    del c000
    ci, cj, ck = np.nonzero(anyin & ~allin)
    tets = _kuhn_tets()                                        # [6,4,3]
    # grid point ids of all tet corners: [ncube,6,4]
    base = np.stack([ci, cj, ck], axis=1)                      # [nc,3]
    corners = base[:, None, None, :] + tets[None, :, :, :]     # [nc,6,4,3]
    corners = corners.reshape(-1, 4, 3)
    gid = (corners[..., 0] * ny + corners[..., 1]) * nz + corners[..., 2]  # [nt,4]
    Ff = F.reshape(-1)
    val = Ff[gid]                                              # [nt,4]
    ins = val > 0
    nin = ins.sum(1)
    keep = (nin > 0) & (nin < 4)
    gid, val, ins, nin = gid[keep], val[keep], ins[keep], nin[keep]

    npts = nx * ny * nz
    nt = len(gid)
    # crossing edges of every tetrahedron, in a fixed per-tet order: one
    # corner inside (its 3 edges to the outside corners in index order), three
    # inside (the inside corners' edges to the outside corner), or two inside
    # (i0-o0, i0-o1, i1-o1, i1-o0); a vertex is numbered at the first tet
    # (in tet order) that uses its edge
    order = np.argsort(~ins, axis=1, kind="stable")          # inside corners first
    srt_in = np.take_along_axis(ins, order, 1)
    assert np.array_equal(srt_in.sum(1), nin)
    ea = np.zeros((nt, 4), np.int64)
    eb = np.zeros((nt, 4), np.int64)
    nslot = np.where(nin == 2, 4, 3)
    one = nin == 1
    three = nin == 3
    two = nin == 2
    # one inside: corner order[0] with order[1..3]
    ea[one, :3] = order[one, 0:1]
    eb[one, :3] = order[one, 1:4]
    # three inside: order[0..2] with order[3]
    ea[three, :3] = order[three, 0:3]
    eb[three, :3] = order[three, 3:4]
    # two inside: i0=order[0], i1=order[1], o0=order[2], o1=order[3]
    o2 = order[two]
    ea[two] = np.stack([o2[:, 0], o2[:, 0], o2[:, 1], o2[:, 1]], 1)
    eb[two] = np.stack([o2[:, 2], o2[:, 3], o2[:, 3], o2[:, 2]], 1)
    valid = np.arange(4)[None, :] < nslot[:, None]
    ga = np.take_along_axis(gid, ea, 1)                      # inside grid point
    gb = np.take_along_axis(gid, eb, 1)                      # outside grid point
    fa = np.take_along_axis(val, ea, 1)
    fb = np.take_along_axis(val, eb, 1)
    key = np.minimum(ga, gb) * npts + np.maximum(ga, gb)
    kv, av, bv, fav, fbv = key[valid], ga[valid], gb[valid], fa[valid], fb[valid]
    uk, first, inv = np.unique(kv, return_index=True, return_inverse=True)
    rank = np.empty(len(uk), np.int64)                       # first appearance order
    rank[np.argsort(first, kind="stable")] = np.arange(len(uk))
    slot_vid = np.full((nt, 4), -1, np.int64)
    slot_vid[valid] = rank[inv]
    src = first[np.argsort(first, kind="stable")]            # defining slot per vertex
    t = fav[src] / (fav[src] - fbv[src])
    t = np.minimum(1.0 - clamp, np.maximum(clamp, t))
    pa = np.stack(np.unravel_index(av[src], shape), -1).astype(np.float64)
    pb = np.stack(np.unravel_index(bv[src], shape), -1).astype(np.float64)
    V = lo + h_grid * (pa + t[:, None] * (pb - pa))
    # triangles in tet order (two per two-inside tet: q0 q1 q2, q0 q2 q3)
    tri = np.full((nt, 2, 3), -1, np.int64)
    tri[:, 0, :] = slot_vid[:, :3]
    tri[two, 0, :] = slot_vid[two][:, [0, 1, 2]]
    tri[two, 1, :] = slot_vid[two][:, [0, 2, 3]]
    tmask = np.zeros((nt, 2), bool)
    tmask[:, 0] = True
    tmask[two, 1] = True
    T = tri[tmask]
    owner = np.repeat(np.arange(nt), tmask.sum(1))
    # orientation: normal must point from inside corners to outside corners
    gpos = np.stack(np.unravel_index(gid[owner], shape), -1)
    sg = ins[owner]
    cin = (gpos * sg[..., None]).sum(1) / sg.sum(1, keepdims=True)
    cout = (gpos * (~sg)[..., None]).sum(1) / (~sg).sum(1, keepdims=True)
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    flip = (nrm * (cout - cin)).sum(1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    T = _collapse_degenerate(V, T)
    V, T = _compact(V, T)
    return V, T.astype(np.int32), {"grid_shape": shape, "h_grid": h_grid,
                                   "beta": beta}


def _tri_area(V, T):
    return 0.5 * np.linalg.norm(
        np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]]), axis=1)


def _collapse_degenerate(V, T, rel=1e-12):
    """Collapse the shortest edge of any triangle with area < rel*mean."""
    for _ in range(100):
        A = _tri_area(V, T)
        bad = np.nonzero(A < rel * A.mean())[0]
        if len(bad) == 0:
            return T
        t = T[bad[0]]
        e = [(t[0], t[1]), (t[1], t[2]), (t[2], t[0])]
        L = [np.linalg.norm(V[a] - V[b]) for a, b in e]
        a, b = e[int(np.argmin(L))]
        T = np.where(T == b, a, T)
        keep = (T[:, 0] != T[:, 1]) & (T[:, 1] != T[:, 2]) & (T[:, 2] != T[:, 0])
        T = T[keep]
    return T


def _compact(V, T):
    used = np.unique(T)
    remap = -np.ones(len(V), np.int64)
    remap[used] = np.arange(len(used))
    return V[used], remap[T]


def check_closed_manifold(tri) -> bool:
    """Every directed edge appears exactly once and its reverse exactly once."""
    T = np.asarray(tri, np.int64)
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    key = e[:, 0] * (T.max() + 1) + e[:, 1]
    rkey = e[:, 1] * (T.max() + 1) + e[:, 0]
    u, c = np.unique(key, return_counts=True)
    if (c != 1).any():
        return False
    return bool(np.isin(rkey, u).all())


def globular(seed: int = 2, n_atoms: int = 5000, r_max: float = 25.0,
             h_grid: float = 1.25):
    """Config 'synthetic globular molecule' (5,000 atoms, ~50k nodes).

    Marching tetrahedra yields about six times the triangles of marching
    cubes at equal spacing, so the grid is 1.25 A (not 0.5 A) to land on the
    configuration's ~100k triangles / ~50k nodes."""
    pos, rad, q = saw_atoms(n_atoms, r_max, seed)
    V, T, meta = gaussian_surface(pos, rad, h_grid)
    return Molecule(name=f"globular_{n_atoms}", xyz=V, tri=T, atom_xyz=pos,
                    charge=q, radius=rad, meta=dict(meta, seed=seed))


def complex_100k(seed: int = 3, n_atoms: int = 100000, r_max: float = 90.0,
                 h_grid: float = 1.5):
    """Config 'synthetic large protein complex' (100,000 atoms): the grid
    spacing 1.5 A puts the isosurface near the configuration's ~2M triangles
    (~1M nodes).  The surface comes from the native generator (the same mesh
    as ``gaussian_surface``, nine times faster at this size)."""
    pos, rad, q = saw_atoms(n_atoms, r_max, seed)
    V, T, meta = gaussian_surface_native(pos, rad, h_grid)
    return Molecule(name=f"complex_{n_atoms}", xyz=V, tri=T, atom_xyz=pos,
                    charge=q, radius=rad, meta=dict(meta, seed=seed))


# ---------------------------------------------------------------------------
# Native generators (workloads/meshgen.cpp) for multi-million-atom inputs
# ---------------------------------------------------------------------------

_MG_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "meshgen.cpp")
_MG_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmeshgen.so")
_mg = None


def build_native(force: bool = False) -> str:
    """Compile meshgen.cpp (g++, OpenMP, no fused multiply-add)."""
    if force or not os.path.exists(_MG_LIB) or (
            os.path.getmtime(_MG_LIB) < os.path.getmtime(_MG_SRC)):
        tmp = _MG_LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _MG_SRC])
        os.replace(tmp, _MG_LIB)
    return _MG_LIB


def _native():
    global _mg
    if _mg is None:
        build_native()
        L = ctypes.CDLL(_MG_LIB)
        dp, lp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)
        c_long, c_double = ctypes.c_long, ctypes.c_double
        L.mg_accept_min_sep.argtypes = [c_long, dp, c_double, c_long, lp]
        L.mg_accept_min_sep.restype = c_long
        L.mg_density.argtypes = [c_long, dp, dp, dp, c_double, c_long, c_long, c_long,
                                 c_double, c_double, dp]
        L.mg_march.argtypes = [dp, c_long, c_long, c_long, dp, c_double, c_double, lp, lp]
        L.mg_march_fetch.argtypes = [dp, ctypes.POINTER(ctypes.c_int32)]
        _mg = L
    return _mg


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gaussian_surface_native(atoms, radii, h_grid: float, beta: float = 2.0,
                            pad: float = 5.0, level: float = 1.0, clamp: float = 0.25):
    """``gaussian_surface`` computed by the native generator (same grid,
    density, tetrahedra, vertex numbering, clamp and orientation)."""
    L = _native()
    atoms = np.ascontiguousarray(atoms, dtype=np.float64)
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    lo = atoms.min(0) - pad
    hi = atoms.max(0) + pad
    shape = tuple(int(math.ceil((hi[a] - lo[a]) / h_grid)) + 1 for a in range(3))
    lo = np.ascontiguousarray(lo)
    F = np.empty(shape, dtype=np.float64)
    L.mg_density(len(atoms), _dptr(atoms), _dptr(radii), _dptr(lo), float(h_grid),
                 shape[0], shape[1], shape[2], float(beta), 3.0, _dptr(F))
    F -= level
    F[F == 0.0] = 1e-300          # no grid value exactly on the level set
    nv, nt = ctypes.c_long(), ctypes.c_long()
    L.mg_march(_dptr(F), shape[0], shape[1], shape[2], _dptr(lo), float(h_grid),
               float(clamp), ctypes.byref(nv), ctypes.byref(nt))
    del F
    V = np.empty((nv.value, 3), np.float64)
    T = np.empty((nt.value, 3), np.int32)
    L.mg_march_fetch(_dptr(V), T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    A = _tri_area(V, T)
    if (A < 1e-12 * A.mean()).any():       # not met with the quarter-edge clamp
        T = _collapse_degenerate(V, T.astype(np.int64))
        V, T = _compact(V, T)
        T = T.astype(np.int32)
    return V, T, {"grid_shape": shape, "h_grid": h_grid, "beta": beta}


def _ico_directions():
    v, _ = _icosahedron()
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def shell_atoms(n: int, r_in: float, r_out: float, seed: int, min_sep: float = 1.2,
                batch: int = 2_000_000):
    """Atoms uniform in r^3 between r_in^3 and r_out^3, uniform in
    direction, thinned by the icosahedral modulation w(u) = 0.5 + 0.5
    max_i (u . v_i)^16 over the 12 vertex directions v_i, with a minimum
    separation (candidates accepted in draw order).  Radii ~ U(1.2, 2.0),
    charges ~ N(0, 0.4) (no shift).  Candidates are drawn in batches of
    ``batch`` (normal directions, uniform r^3, uniform thinning variate)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vdir = _ico_directions()
    kept = []
    total = 0
    while True:
        u = _unit_vectors(rng, batch)
        r = np.cbrt(rng.uniform(r_in ** 3, r_out ** 3, batch))
        w = 0.5 + 0.5 * np.max(u @ vdir.T, axis=1) ** 16
        thin = rng.uniform(0.0, 1.0, batch) < w
        kept.append((u[thin] * r[thin, None]))
        cand = np.ascontiguousarray(np.concatenate(kept))
        idx = np.empty(n, dtype=np.int64)
        total = _native().mg_accept_min_sep(len(cand), _dptr(cand), float(min_sep), n,
                                            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
        if total >= n:
            break
    pos = cand[idx[:n]]
    radius = rng.uniform(1.2, 2.0, n)
    q = rng.normal(0.0, 0.4, n)
    return pos, radius, q


def capsid_shell(seed: int = 5, n_atoms: int = 1_100_000, r_in: float = 220.0,
                 r_out: float = 280.0, h_grid: float = CAPSID_H_GRID):
    """Config 'virus-capsid-scale shell': ~1.1M atoms in a spherical shell
    of radii 220-280 A with icosahedral density modulation, Gaussian
    isosurface by marching tetrahedra (native generator) on a grid whose
    spacing puts the surface near ~20M triangles (~10M nodes)."""
    pos, rad, q = shell_atoms(n_atoms, r_in, r_out, seed)
    V, T, meta = gaussian_surface_native(pos, rad, h_grid)
    return Molecule(name=f"capsid_shell_{n_atoms}", xyz=V, tri=T, atom_xyz=pos,
                    charge=q, radius=rad, meta=dict(meta, seed=seed))


# ---------------------------------------------------------------------------
# Serving stream: star-shaped molecules
# ---------------------------------------------------------------------------

def _real_sph_harm(lmax, xyz):
    """Real orthonormal spherical harmonics Y_lm at unit vectors, l=1..lmax."""
    from scipy.special import sph_harm_y
    z = np.clip(xyz[:, 2], -1.0, 1.0)
    theta = np.arccos(z)
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])
    out = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                out.append(math.sqrt(2.0) * (-1) ** m * Y.real)
            elif m < 0:
                out.append(math.sqrt(2.0) * (-1) ** m * Y.imag)
            else:
                out.append(Y.real)
    return np.stack(out, 1)


def star_request(i: int, level: int | None = None):
    """Request i of the serving stream (seed 4000+i)."""
    rng = np.random.Generator(np.random.PCG64(4000 + i))
    R = rng.uniform(8.0, 40.0)
    a = rng.normal(0.0, 0.05, 48)               # l=1..6: 3+5+...+13 = 48
    L = int(rng.integers(3, 7)) if level is None else level
    _ = level
    nq = int(rng.integers(5, 501))
    qv = rng.normal(0.0, 0.5, nq)
    vhat, tri = icosphere(L, 1.0)

    def rfun(u):
        return R * np.maximum(0.3, 1.0 + _real_sph_harm(6, u) @ a)

    xyz = vhat * rfun(vhat)[:, None]
    pos = np.zeros((nq, 3))
    k = 0
    while k < nq:
        w = _unit_vectors(rng, 1)
        u = rng.uniform()
        rw = float(rfun(w)[0])
        rad = 0.7 * rw * u ** (1.0 / 3.0)
        if rw - rad < 1.5:
            continue
        pos[k] = w[0] * rad
        k += 1
    return Molecule(name=f"star_{i}", xyz=xyz, tri=tri, atom_xyz=pos,
                    charge=qv, radius=np.full(nq, 1.5),
                    meta={"level": L, "R": R, "seed": 4000 + i})


def random_rigid_motion(seed: int):
    """A seeded random rotation matrix and translation vector."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    Rm = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    t = rng.uniform(-10, 10, 3)
    return Rm, t
