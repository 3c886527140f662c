"""FP64 CPU oracle (Python half): loading the C oracle, the node-patch
operator of Section 2 (Eq. 5), restarted GMRES, right-hand side and energy.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

# Coulomb constant e^2 N_A / (4 pi eps0) in kcal A / mol from CODATA 2018
# (e and N_A exact, eps0 = 8.8541878128e-12 F/m, 4184 J per kcal).
_E = 1.602176634e-19
_NA = 6.02214076e23
_EPS0 = 8.8541878128e-12
COULOMB_KCAL = _E * _E * _NA / (4.0 * math.pi * _EPS0) * 1e10 / 4184.0
# Internal potentials follow Eq. (3)'s normalisation (a unit point charge in a
# uniform dielectric eps gives 1/(4 pi eps r)); multiplying by 4 pi C_e turns
# them into kcal/(mol e).
UNIT_SCALE = 4.0 * math.pi * COULOMB_KCAL


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        c_long, c_double = ctypes.c_long, ctypes.c_double
        L.orc_kernels.argtypes = [dp, dp, dp, dp, c_double, dp]
        L.orc_geometry.argtypes = [c_long, dp, c_long, ip, dp, dp, dp, dp, dp]
        L.orc_near_count.argtypes = [c_long, dp, dp, c_double, c_long, lp, lp]
        L.orc_near_fill.argtypes = [c_long, dp, dp, c_double, c_long, lp, lp, lp]
        L.orc_patch_coeffs.argtypes = [c_long, dp, c_long, ip, dp, dp, lp, lp,
                                       c_double, c_double, c_long, lp, lp, dp]
        L.orc_point_coeffs.argtypes = [dp, dp, dp, c_double, c_double, c_long,
                                       lp, lp, dp]
        L.orc_matvec_rows.argtypes = [c_long, dp, dp, dp, c_double, c_double,
                                      c_long, lp, lp, lp, dp, dp, dp]
        L.orc_rhs.argtypes = [c_long, dp, dp, c_long, dp, dp, c_double, dp]
        L.orc_energy_sum.argtypes = [c_long, dp, dp, dp, c_long, dp, dp,
                                     c_double, dp, dp, dp]
        L.orc_energy_sum.restype = c_double
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (for timing it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------------------
# Kernels (Section 2, Eq. 3)
# ---------------------------------------------------------------------------

KERNEL_NAMES = ("G", "u", "dG_dny", "du_dny", "dG_dnx", "du_dnx",
                "d2G", "d2u", "G_minus_u", "d2G_minus_d2u")


def kernels(x, nx, y, ny, kappa):
    """All point kernels for target x (normal nx) and source y (normal ny)."""
    out = np.zeros(10)
    lib().orc_kernels(_d(f64(x)), _d(f64(nx)), _d(f64(y)), _d(f64(ny)),
                      float(kappa), _d(out))
    return dict(zip(KERNEL_NAMES, out))


# ---------------------------------------------------------------------------
# Mesh validation (problem statement: a closed, outward-oriented surface)
# ---------------------------------------------------------------------------

class MeshError(ValueError):
    pass


def validate_mesh(xyz, tri):
    """Reject open/non-manifold meshes, duplicate vertices, degenerate
    triangles and inward orientation."""
    V = f64(xyz)
    T = np.asarray(tri, dtype=np.int64)
    n = V.shape[0]
    if V.ndim != 2 or V.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 3:
        raise MeshError("bad array shapes")
    if n < 4 or len(T) < 4:
        raise MeshError("too few nodes/triangles")
    if not np.isfinite(V).all():
        raise MeshError("non-finite coordinates")
    if T.min() < 0 or T.max() >= n:
        raise MeshError("triangle index out of range")
    if len(np.unique(T)) != n:
        raise MeshError("unused vertex")
    if len(np.unique(V, axis=0)) != n:
        raise MeshError("duplicate vertex")
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    key = e[:, 0] * n + e[:, 1]
    rkey = e[:, 1] * n + e[:, 0]
    u, c = np.unique(key, return_counts=True)
    if (c != 1).any() or not np.isin(rkey, u).all():
        raise MeshError("open or non-manifold surface")
    cr = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    A = 0.5 * np.linalg.norm(cr, axis=1)
    if (A < 1e-12 * A.mean()).any():
        raise MeshError("degenerate triangle")
    vol = np.einsum("ij,ij->i", V[T[:, 0]], np.cross(V[T[:, 1]], V[T[:, 2]])).sum() / 6
    if not vol > 0:
        raise MeshError("surface not oriented outward (non-positive volume)")


# ---------------------------------------------------------------------------
# Geometry (Section 2, Figure 1)
# ---------------------------------------------------------------------------

@dataclass
class Geometry:
    xyz: np.ndarray
    tri: np.ndarray          # int32
    tri_area: np.ndarray
    tri_n: np.ndarray
    area: np.ndarray         # patch areas a_t
    normal: np.ndarray       # node normals n_t
    rho2: np.ndarray         # squared patch radius
    inc_ptr: np.ndarray      # node -> incident triangles (ascending)
    inc_tri: np.ndarray


def geometry(xyz, tri) -> Geometry:
    V = f64(xyz)
    T = np.ascontiguousarray(tri, dtype=np.int32)
    n, m = V.shape[0], T.shape[0]
    ta, tn = np.zeros(m), np.zeros((m, 3))
    na, nn, r2 = np.zeros(n), np.zeros((n, 3)), np.zeros(n)
    lib().orc_geometry(n, _d(V), m, _i(T), _d(ta), _d(tn), _d(na), _d(nn), _d(r2))
    owner = T.reshape(-1).astype(np.int64)
    tri_of = np.repeat(np.arange(m, dtype=np.int64), 3)
    order = np.lexsort((tri_of, owner))
    inc_tri = np.ascontiguousarray(tri_of[order])
    inc_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(owner, minlength=n), out=inc_ptr[1:])
    return Geometry(V, T, ta, tn, na, nn, r2, inc_ptr, inc_tri)


# ---------------------------------------------------------------------------
# Near set and patch integrals (Section 2, Eq. 6)
# ---------------------------------------------------------------------------

def near_set(geo: Geometry, eta: float, rows=None):
    """CSR (ptr, col) of N(p) for the requested rows (all rows by default)."""
    n = geo.xyz.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else i64(rows)
    cnt = np.zeros(len(rows), dtype=np.int64)
    lib().orc_near_count(n, _d(geo.xyz), _d(geo.rho2), float(eta), len(rows),
                         _l(rows), _l(cnt))
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    col = np.zeros(int(ptr[-1]), dtype=np.int64)
    lib().orc_near_fill(n, _d(geo.xyz), _d(geo.rho2), float(eta), len(rows),
                        _l(rows), _l(ptr), _l(col))
    return rows, ptr, col


def patch_coeffs(geo: Geometry, kappa, ebar, p, t):
    """Patch integrals {A,B,C,D}_{pt} of Eq. (6): array [npairs, 4]."""
    p, t = i64(p), i64(t)
    out = np.zeros((len(p), 4))
    lib().orc_patch_coeffs(geo.xyz.shape[0], _d(geo.xyz), geo.tri.shape[0],
                           _i(geo.tri), _d(geo.tri_n), _d(geo.normal),
                           _l(geo.inc_ptr), _l(geo.inc_tri), float(kappa),
                           float(ebar), len(p), _l(p), _l(t), _d(out))
    return out


def point_coeffs(geo: Geometry, kappa, ebar, p, t):
    """Point-rule {A,B,C,D}_{pt} (integrand at node t times a_t)."""
    p, t = i64(p), i64(t)
    out = np.zeros((len(p), 4))
    lib().orc_point_coeffs(_d(geo.xyz), _d(geo.normal), _d(geo.area),
                           float(kappa), float(ebar), len(p), _l(p), _l(t), _d(out))
    return out


# ---------------------------------------------------------------------------
# The operator of Eq. (5)
# ---------------------------------------------------------------------------

@dataclass
class Operator:
    """Direct O(N^2) node-patch operator M of Eq. (5) on the requested rows."""
    geo: Geometry
    eps_p: float
    eps_s: float
    kappa: float
    eta: float
    rows: np.ndarray
    near_ptr: np.ndarray
    near_col: np.ndarray
    near_coef: np.ndarray
    setup_s: float = 0.0
    matvecs: int = 0

    @property
    def n(self):
        return self.geo.xyz.shape[0]

    @property
    def ebar(self):
        return self.eps_s / self.eps_p

    @property
    def alpha(self):
        return 0.5 / self.ebar + 0.5

    def apply_rows(self, x):
        """(yf, yh) at self.rows for x = [f; h]."""
        x = f64(x)
        y = np.zeros(2 * len(self.rows))
        lib().orc_matvec_rows(self.n, _d(self.geo.xyz), _d(self.geo.normal),
                              _d(self.geo.area), float(self.kappa),
                              float(self.ebar), len(self.rows), _l(self.rows),
                              _l(self.near_ptr), _l(self.near_col),
                              _d(self.near_coef), _d(x), _d(y))
        self.matvecs += 1
        return y[0::2].copy(), y[1::2].copy()

    def matvec(self, x):
        assert len(self.rows) == self.n, "operator built on a row subset"
        yf, yh = self.apply_rows(x)
        return np.concatenate([yf, yh])

    def dense(self):
        """Explicit 2N x 2N matrix (small N only), column by column."""
        n2 = 2 * self.n
        M = np.zeros((n2, n2))
        e = np.zeros(n2)
        for j in range(n2):
            e[j] = 1.0
            M[:, j] = self.matvec(e)
            e[j] = 0.0
        return M


def operator(xyz, tri, eps_p, eps_s, kappa, eta=4.0, rows=None,
             validate=True) -> Operator:
    if validate:
        validate_mesh(xyz, tri)
    t0 = time.perf_counter()
    geo = geometry(xyz, tri)
    r, ptr, col = near_set(geo, eta, rows)
    pr = np.repeat(r, np.diff(ptr))
    coef = patch_coeffs(geo, kappa, eps_s / eps_p, pr, col)
    return Operator(geo, float(eps_p), float(eps_s), float(kappa), float(eta),
                    r, ptr, col, np.ascontiguousarray(coef),
                    setup_s=time.perf_counter() - t0)


def rhs(geo: Geometry, atom_xyz, charge, eps_s):
    """Right-hand side of Eq. (5) (second row with dG/dn0, cf. Eq. 3)."""
    n = geo.xyz.shape[0]
    ax, q = f64(atom_xyz), f64(charge)
    b = np.zeros(2 * n)
    lib().orc_rhs(n, _d(geo.xyz), _d(geo.normal), len(q), _d(ax), _d(q),
                  float(eps_s), _d(b))
    return b


def reaction_energy(geo: Geometry, atom_xyz, charge, ebar, f, h):
    """Polar energy (kcal/mol) = 1/2 sum_k q_k phi_reac(r_k) * 4 pi C_e, with
    phi_reac from the interior Green representation (point rule)."""
    ax, q = f64(atom_xyz), f64(charge)
    phi = np.zeros(len(q))
    s = lib().orc_energy_sum(geo.xyz.shape[0], _d(geo.xyz), _d(geo.normal),
                             _d(geo.area), len(q), _d(ax), _d(q), float(ebar),
                             _d(f64(f)), _d(f64(h)), _d(phi))
    return 0.5 * s * UNIT_SCALE, phi


# ---------------------------------------------------------------------------
# Restarted GMRES (textbook restarted GMRES(m) with modified Gram-Schmidt and
# Givens rotations, no preconditioner; stopping rule Eq. 7)
# ---------------------------------------------------------------------------

@dataclass
class GmresInfo:
    iterations: int = 0
    restarts: int = 0
    inner_products: int = 0
    converged: bool = False
    resid_estimate: float = float("nan")
    true_rel_residual: float = float("nan")
    history: list = field(default_factory=list)


def gmres(matvec, b, x0=None, restart=80, max_restarts=5, rel_tol=1e-6,
          abs_tol=0.0):
    b = f64(b)
    nb = float(np.sqrt(b @ b))
    tol = rel_tol * nb + abs_tol
    x = np.zeros_like(b) if x0 is None else f64(x0).copy()
    info = GmresInfo()
    for cycle in range(max_restarts + 1):
        r = b - matvec(x) if (x0 is not None or cycle > 0) else b.copy()
        beta = float(np.sqrt(r @ r))
        info.inner_products += 1
        info.resid_estimate = beta
        if beta <= tol:
            info.converged = True
            break
        if cycle > 0:
            info.restarts += 1
        m = restart
        Vb = np.zeros((m + 1, len(b)))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Vb[0] = r / beta
        k = 0
        done = False
        for j in range(m):
            w = matvec(Vb[j])
            info.iterations += 1
            for i in range(j + 1):
                H[i, j] = w @ Vb[i]
                w = w - H[i, j] * Vb[i]
                info.inner_products += 1
            H[j + 1, j] = float(np.sqrt(w @ w))
            info.inner_products += 1
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            hj1 = H[j + 1, j]
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info.resid_estimate = abs(g[j + 1])
            info.history.append(info.resid_estimate)
            if abs(g[j + 1]) <= tol or hj1 == 0.0:
                done = True
                break
            Vb[j + 1] = w / hj1
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Vb[:k].T @ y
        if done:
            info.converged = True
            break
    rr = b - matvec(x)
    info.true_rel_residual = float(np.sqrt(rr @ rr)) / nb if nb > 0 else 0.0
    return x, info


@dataclass
class Solution:
    f: np.ndarray            # kcal/(mol e)
    h: np.ndarray            # kcal/(mol e A)
    energy: float            # kcal/mol
    info: GmresInfo
    op: Operator
    b: np.ndarray
    x: np.ndarray            # internal units, [f; h]


def solve(mol, eta=4.0, restart=80, max_restarts=5, rel_tol=1e-6, abs_tol=0.0,
          x0=None) -> Solution:
    """Full oracle solve of Eq. (5) for a workloads.Molecule."""
    op = operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa, eta)
    b = rhs(op.geo, mol.atom_xyz, mol.charge, mol.eps_s)
    x, info = gmres(op.matvec, b, x0=x0, restart=restart,
                    max_restarts=max_restarts, rel_tol=rel_tol, abs_tol=abs_tol)
    n = op.n
    E, _ = reaction_energy(op.geo, mol.atom_xyz, mol.charge, op.ebar, x[:n], x[n:])
    return Solution(x[:n] * UNIT_SCALE, x[n:] * UNIT_SCALE, E, info, op, b, x)
