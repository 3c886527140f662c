"""Pins for the oracle's GMRES, right-hand side and energy (Section 2 Eq. 5,
Section 3.4, Section 5): dense LU, the paper's inner-product counts, the Born
and Kirkwood closed forms, special cases and invariances."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.closed_forms import born_energy, born_surface_values, kirkwood_energy

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _ip_count(k):
    """Inner products of one GMRES cycle of k steps with modified Gram-Schmidt:
    the initial norm, j projections and one norm at step j."""
    return k * (k + 3) // 2 + 1


def test_gmres_matches_dense_lu():
    for mol in (W.born_ion(2), W.star_request(5, level=2)):
        op = O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa)
        b = O.rhs(op.geo, mol.atom_xyz, mol.charge, mol.eps_s)
        M = op.dense()
        x_lu = np.linalg.solve(M, b)
        x, info = O.gmres(op.matvec, b, rel_tol=1e-13, restart=80)
        assert info.converged
        assert np.linalg.norm(x - x_lu) <= 1e-9 * np.linalg.norm(x_lu)
        assert info.inner_products == _ip_count(info.iterations)
        # the small restart also converges and counts per cycle
        x2, info2 = O.gmres(op.matvec, b, rel_tol=1e-12, restart=3, max_restarts=40)
        assert info2.converged and info2.restarts >= 1
        assert np.linalg.norm(x2 - x_lu) <= 1e-9 * np.linalg.norm(x_lu)


def test_inner_product_formula_reproduces_paper_counts():
    restart = GOLD["gmres_counts"]["restart"]
    for run in GOLD["gmres_counts"]["runs"]:
        k, printed = run["iterations"], run["inner_products"]
        total, left = 0, k
        while left > 0:
            c = min(left, restart)
            total += _ip_count(c)
            left -= c
        assert abs(total - printed) <= 3, run


def test_born_constant_reproduces_paper_analytic_sphere():
    s = GOLD["sphere_test"]
    E = born_energy(s["charge"], s["radius"], 2.0, 80.0, 0.0)
    assert E == pytest.approx(s["analytic_kcal_mol"], rel=5e-4)


def test_kirkwood_reduces_to_born_and_classic_series():
    q, a, ep, es = 1.3, 2.5, 2.0, 80.0
    for kappa in (0.0, 0.1, 1.0):
        assert kirkwood_energy([q], [[0, 0, 0]], a, ep, es, kappa) == pytest.approx(
            born_energy(q, a, ep, es, kappa), rel=1e-14)
    # kappa = 0: classic dielectric-sphere reaction field
    pos = np.array([[0.3, -0.2, 0.5], [-0.6, 0.4, 0.1], [0.0, 0.7, -0.9]])
    qs = np.array([1.0, -0.5, 0.8])
    ref = 0.0
    from scipy.special import eval_legendre
    for i in range(3):
        for j in range(3):
            bi, bj = np.linalg.norm(pos[i]), np.linalg.norm(pos[j])
            c = pos[i] @ pos[j] / (bi * bj)
            for n in range(200):
                ref += qs[i] * qs[j] * (bi * bj) ** n / a ** (2 * n + 1) * (n + 1) * (ep - es) / (
                    ep * (n * ep + (n + 1) * es)) * eval_legendre(n, c)
    ref *= 0.5 * O.COULOMB_KCAL
    assert kirkwood_energy(qs, pos, a, ep, es, 0.0) == pytest.approx(ref, rel=1e-12)
    # small kappa approaches the kappa = 0 value
    e1 = kirkwood_energy(qs, pos, a, ep, es, 1e-7)
    assert e1 == pytest.approx(ref, rel=1e-6)


def test_born_ion_energy_and_convergence():
    Eb = born_energy(1.0, 2.0, 2.0, 80.0, 0.1)
    assert Eb == pytest.approx(-40.6432, abs=1e-4)
    fex, hex_ = born_surface_values(1.0, 2.0, 80.0, 0.1)
    eE, ef, eh = [], [], []
    for L in (2, 3, 4):
        sol = O.solve(W.born_ion(L))
        n = len(sol.f)
        assert sol.info.converged and sol.info.true_rel_residual < 1e-6
        eE.append(abs(sol.energy / Eb - 1))
        ef.append(abs(sol.x[:n].mean() / fex - 1))
        eh.append(abs(sol.x[n:].mean() / hex_ - 1))
    assert eE[2] < 0.01 and eE[1] > eE[2]
    assert ef[0] > ef[1] > ef[2]
    assert eh[2] < 0.01


def test_paper_sphere_at_small_mesh():
    s = GOLD["sphere_test"]
    mol = W.born_ion(4, radius=s["radius"], charge=s["charge"], kappa=0.0)
    sol = O.solve(mol)
    assert sol.energy == pytest.approx(s["analytic_kcal_mol"], rel=0.01)


def test_kirkwood_multi_charge_sphere():
    a = 4.0
    pos = np.array([[0.5, 0.8, -0.3], [-1.2, 0.2, 0.9], [0.1, -1.5, -0.6], [1.4, -0.2, 0.7]])
    q = np.array([1.0, -0.7, 0.5, -0.3])
    v, t = W.icosphere(4, a)
    mol = W.Molecule("kirkwood", v, t, pos, q, np.full(4, 1.5), 2.0, 80.0, 0.1)
    sol = O.solve(mol)
    E = kirkwood_energy(q, pos, a, 2.0, 80.0, 0.1)
    assert sol.energy == pytest.approx(E, rel=0.01)


def test_identity_case_is_exact():
    mol = W.star_request(6, level=2)
    op = O.operator(mol.xyz, mol.tri, 3.0, 3.0, 0.0)
    x = np.random.default_rng(1).normal(size=2 * op.n)
    assert (op.matvec(x) == x).all()
    b = O.rhs(op.geo, mol.atom_xyz, mol.charge, 3.0)
    xs, info = O.gmres(op.matvec, b, rel_tol=1e-12)
    assert info.iterations == 1
    assert np.allclose(xs, b, rtol=1e-14, atol=0)


def test_kappa_zero_makes_A_and_D_vanish():
    mol = W.star_request(7, level=2)
    op = O.operator(mol.xyz, mol.tri, 2.0, 80.0, 0.0)
    assert (op.near_coef[:, 0] == 0).all() and (op.near_coef[:, 3] == 0).all()
    n = op.n
    P = np.repeat(np.arange(n), n)
    T = np.tile(np.arange(n), n)
    pc = O.point_coeffs(op.geo, 0.0, 40.0, P[P != T], T[P != T])
    assert (pc[:, 0] == 0).all() and (pc[:, 3] == 0).all()
    # block-triangular: f-row does not see h
    x = np.r_[np.zeros(n), np.random.default_rng(2).normal(size=n)]
    assert (op.matvec(x)[:n] == 0).all()


def _solve_E(mol, **kw):
    return O.solve(mol, rel_tol=1e-12, **kw)


def test_rigid_motion_charge_scaling_and_permutation_invariance():
    mol = W.star_request(8, level=2)
    base = _solve_E(mol)
    Rm, tv = W.random_rigid_motion(3)
    moved = W.Molecule("moved", mol.xyz @ Rm.T + tv, mol.tri, mol.atom_xyz @ Rm.T + tv,
                       mol.charge, mol.radius, mol.eps_p, mol.eps_s, mol.kappa)
    mv = _solve_E(moved)
    assert mv.energy == pytest.approx(base.energy, rel=1e-10)
    assert np.allclose(mv.f, base.f, rtol=1e-9, atol=1e-12 * np.abs(base.f).max())
    scaled = W.Molecule("scaled", mol.xyz, mol.tri, mol.atom_xyz, 3.0 * mol.charge,
                        mol.radius, mol.eps_p, mol.eps_s, mol.kappa)
    assert _solve_E(scaled).energy == pytest.approx(9.0 * base.energy, rel=1e-11)
    perm = np.random.default_rng(4).permutation(mol.n_nodes)
    inv = np.argsort(perm)
    pm = W.Molecule("perm", mol.xyz[perm], inv[mol.tri].astype(np.int32), mol.atom_xyz,
                    mol.charge, mol.radius, mol.eps_p, mol.eps_s, mol.kappa)
    ps = _solve_E(pm)
    assert ps.energy == pytest.approx(base.energy, rel=1e-10)
    assert np.allclose(ps.f, base.f[perm], rtol=1e-9, atol=1e-12 * np.abs(base.f).max())
    # linearity in the charges
    q1 = mol.charge.copy()
    q1[::2] = 0
    m1 = W.Molecule("q1", mol.xyz, mol.tri, mol.atom_xyz, q1, mol.radius,
                    mol.eps_p, mol.eps_s, mol.kappa)
    m2 = W.Molecule("q2", mol.xyz, mol.tri, mol.atom_xyz, mol.charge - q1, mol.radius,
                    mol.eps_p, mol.eps_s, mol.kappa)
    s1, s2 = _solve_E(m1), _solve_E(m2)
    assert np.allclose(s1.f + s2.f, base.f, rtol=1e-9, atol=1e-11 * np.abs(base.f).max())


def test_rhs_against_coulomb_sum():
    mol = W.star_request(9, level=2)
    g = O.geometry(mol.xyz, mol.tri)
    b = O.rhs(g, mol.atom_xyz, mol.charge, mol.eps_s)
    n = len(g.area)
    p = 5
    d = g.xyz[p] - mol.atom_xyz
    r = np.linalg.norm(d, axis=1)
    assert b[p] == pytest.approx((mol.charge / (4 * np.pi * r)).sum() / mol.eps_s, rel=1e-13)
    # dG/dn0 by central differences along the node normal
    hh = 1e-5
    pot = lambda x: (mol.charge / (4 * np.pi * np.linalg.norm(x - mol.atom_xyz, axis=1))).sum()
    fd = (pot(g.xyz[p] + hh * g.normal[p]) - pot(g.xyz[p] - hh * g.normal[p])) / (2 * hh)
    assert b[n + p] == pytest.approx(fd / mol.eps_s, rel=1e-6)
