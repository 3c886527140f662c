"""Pins for the oracle's patch integrals {A,B,C,D} of Eq. (6) (Section 2):
  * self patch against a polar-coordinate closed form of the radial integral;
  * neighbour patches against brute-force uniform subdivision (checked for
    convergence) with an independent numpy integrand;
  * the double-layer row sum against the polyhedron's solid angle
    (Van Oosterom-Strackee), with every pair integrated over its patch;
  * sphere row sums of A and B converging to their surface-integral values.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
import workloads as W
from oracle.closed_forms import solid_angle

EBAR = 40.0


def _octahedron():
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    t = []
    for sx in (0, 1):
        for sy in (2, 3):
            for sz in (4, 5):
                f = [sx, sy, sz]
                nrm = np.cross(v[sy] - v[sx], v[sz] - v[sx])
                if nrm @ v[f].mean(0) < 0:
                    f = [sx, sz, sy]
                t.append(f)
    return v, np.array(t, np.int32)


def _patch_pieces(g, t):
    """Flat pieces (P0,P1,P2, facet normal) of node t's patch."""
    out = []
    for k in g.inc_tri[g.inc_ptr[t]:g.inc_ptr[t + 1]]:
        tv = g.tri[k]
        j = int(np.nonzero(tv == t)[0][0])
        pt, pu, pw = g.xyz[tv[j]], g.xyz[tv[(j + 1) % 3]], g.xyz[tv[(j + 2) % 3]]
        c = g.xyz[tv].sum(0) / 3
        out.append((pt, (pt + pu) / 2, c, g.tri_n[k]))
        out.append((pt, c, (pt + pw) / 2, g.tri_n[k]))
    return out


# --- self patch: closed-form radial integrals --------------------------------

def _self_piece(P0, P1, P2, kappa):
    e1 = P1 - P0
    l1 = np.linalg.norm(e1)
    e1 = e1 / l1
    n = np.cross(P1 - P0, P2 - P0)
    n /= np.linalg.norm(n)
    e2 = np.cross(n, e1)
    x2, y2 = (P2 - P0) @ e1, (P2 - P0) @ e2
    th_max = math.atan2(y2, x2)

    def R(th):
        return l1 / (math.cos(th) - math.sin(th) * (x2 - l1) / y2)

    def a_fac(s):
        return -math.expm1(-s) - s * math.exp(-s)

    def A_radial(th):          # int_0^R (1 - e^{-k r})/(4 pi r) r dr
        r = R(th)
        return (r + math.expm1(-kappa * r) / kappa) / (4 * math.pi)

    def D_radial(th):          # int_0^R a(k r)/(4 pi r^3) r dr
        r = R(th)
        return quad(lambda s: a_fac(kappa * s) / s ** 2 if s > 0 else kappa ** 2 / 2,
                    0, r, epsabs=0, epsrel=1e-13, limit=200)[0] / (4 * math.pi)

    A = quad(A_radial, 0, th_max, epsabs=0, epsrel=1e-13, limit=200)[0]
    D = quad(D_radial, 0, th_max, epsabs=0, epsrel=1e-12, limit=200)[0] / EBAR
    return A, D


@pytest.mark.parametrize("kappa", [0.1, 1.3])
def test_self_patch_against_polar_closed_form(kappa):
    mol = W.star_request(3, level=2)
    g = O.geometry(mol.xyz, mol.tri)
    for p in (0, 17, 101):
        ref = np.zeros(2)
        for P0, P1, P2, _ in _patch_pieces(g, p):
            ref += _self_piece(P0, P1, P2, kappa)
        c = O.patch_coeffs(g, kappa, EBAR, [p], [p])[0]
        assert c[0] == pytest.approx(ref[0], rel=1e-11)
        assert c[3] == pytest.approx(ref[1], rel=1e-10)
        assert c[1] == 0.0 and c[2] == 0.0


# --- neighbour patches: brute force ------------------------------------------

def _integrand(x, nx, y, ny, kappa):
    R = x[None, :] - y
    r = np.linalg.norm(R, axis=1)
    s = kappa * r
    e = np.exp(-s)
    Rnx, Rny = R @ nx, (R * ny).sum(-1) if ny.ndim == 2 else R @ ny
    nxny = (ny @ nx) if ny.ndim == 1 else ny @ nx
    fp = 4 * np.pi
    G, u = 1 / (fp * r), e / (fp * r)
    dGy, duy = Rny / (fp * r ** 3), e * (1 + s) * Rny / (fp * r ** 3)
    dGx, dux = -Rnx / (fp * r ** 3), -e * (1 + s) * Rnx / (fp * r ** 3)
    d2 = (nxny * (1 - e * (1 + s)) / r ** 3 - Rnx * Rny * (3 - e * (3 + 3 * s + s * s)) / r ** 5) / fp
    return np.stack([G - u, dGy / EBAR - duy, dGx - dux / EBAR, d2 / EBAR], 1)


def _uniform_rule(P0, P1, P2, level, nq=6):
    """Uniform midpoint subdivision into 4^level pieces, nq x nq collapsed
    Gauss-Legendre (numpy's leggauss) on each piece."""
    tris = [(P0, P1, P2)]
    for _ in range(level):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (bc, ca, ab)]
        tris = nxt
    T = np.array(tris)                                     # [m,3,3]
    z, w = np.polynomial.legendre.leggauss(nq)
    z, w = (z + 1) / 2, w / 2
    U, Vv = np.meshgrid(z, z, indexing="ij")
    WW = np.outer(w, w) * U
    a, b, c = T[:, 0], T[:, 1], T[:, 2]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    pts = (a[:, None, :] + U.reshape(-1)[None, :, None] * (b - a)[:, None, :]
           + (U * Vv).reshape(-1)[None, :, None] * (c - b)[:, None, :])
    wts = 2 * area[:, None] * WW.reshape(-1)[None, :]
    return pts.reshape(-1, 3), wts.reshape(-1)


def _brute(g, p, t, kappa, level):
    acc = np.zeros(4)
    for P0, P1, P2, ny in _patch_pieces(g, t):
        pts, wts = _uniform_rule(P0, P1, P2, level)
        acc += (wts[:, None] * _integrand(g.xyz[p], g.normal[p], pts, ny, kappa)).sum(0)
    return acc


@pytest.mark.parametrize("mesh", ["octahedron", "ico0", "ico1"])
@pytest.mark.parametrize("kappa", [0.1, 1.0])
def test_neighbour_patches_against_brute_force(mesh, kappa):
    if mesh == "octahedron":
        v, t = _octahedron()
    else:
        v, t = W.icosphere(int(mesh[-1]), 1.0)
    g = O.geometry(v, t)
    rng = np.random.default_rng(5)
    rows, ptr, col = O.near_set(g, 4.0)
    pairs = [(p, c) for p in range(len(v)) for c in col[ptr[p]:ptr[p + 1]] if c != p]
    pairs = [pairs[i] for i in rng.choice(len(pairs), size=min(6, len(pairs)), replace=False)]
    P = np.array(pairs)
    got = O.patch_coeffs(g, kappa, EBAR, P[:, 0], P[:, 1])
    for (p, c), gv in zip(pairs, got):
        r5 = _brute(g, p, c, kappa, 5)
        r6 = _brute(g, p, c, kappa, 6)
        scale = np.abs(r6).max()
        assert np.abs(r6 - r5).max() < 1e-12 * scale           # brute force converged
        assert np.abs(gv - r6).max() < 1e-9 * scale, (p, c, gv, r6)


# --- double-layer row sums = solid angle --------------------------------------

@pytest.mark.parametrize("mesh", ["octahedron", "ico1", "star2"])
def test_double_layer_row_sum_is_solid_angle(mesh):
    if mesh == "octahedron":
        v, t = _octahedron()
    elif mesh == "ico1":
        v, t = W.icosphere(1, 1.0)
    else:
        m = W.star_request(4, level=2)
        v, t = m.xyz, m.tri
    g = O.geometry(v, t)
    n = len(v)
    p_idx = [0, n // 2, n - 1]
    for p in p_idx:
        cf = O.patch_coeffs(g, 0.0, EBAR, np.full(n, p), np.arange(n))
        mask = ~(t == p).any(1)
        omega = solid_angle(v[p], v[t[mask, 0]], v[t[mask, 1]], v[t[mask, 2]]).sum()
        expect = (1 / EBAR - 1) * (-omega / (4 * np.pi))
        assert cf[:, 1].sum() == pytest.approx(expect, rel=1e-9)
        assert cf[:, 0].sum() == 0.0 and cf[:, 3].sum() == 0.0   # kappa = 0


# --- sphere row sums -----------------------------------------------------------

def test_sphere_row_sums_converge():
    a, kappa = 2.0, 0.1
    exact_A = a - (1 - math.exp(-2 * kappa * a)) / (2 * kappa)
    exact_B = (1 / EBAR - 1) * (-0.5)
    errA, errB = [], []
    for L in (2, 3, 4):
        v, t = W.icosphere(L, a)
        n = len(v)
        op = O.operator(v, t, 2.0, 2.0 * EBAR, kappa)
        y = op.matvec(np.r_[np.zeros(n), np.ones(n)])
        errA.append(np.abs(-y[:n] - exact_A).max() / exact_A)
        op0 = O.operator(v, t, 2.0, 2.0 * EBAR, 0.0)
        y0 = op0.matvec(np.r_[np.ones(n), np.zeros(n)])
        errB.append(np.abs(y0[:n] - op0.alpha - exact_B).max() / exact_B)
    # single layer: second-order convergence (error / 4 per level); double
    # layer: first order (error / 2 per level), from the point rule on the
    # curved surface's far patches
    assert errA[0] > 3 * errA[1] > 9 * errA[2] and errA[2] < 2e-3
    assert errB[0] > 1.7 * errB[1] > 2.89 * errB[2] and errB[2] < 5e-2
