"""Seeded synthetic inputs: closed, outward-oriented, valid meshes with the
stated sizes; determinism under a fixed seed."""
import numpy as np

import oracle as O
import workloads as W


def test_globular_size_validity_and_determinism():
    m = W.globular()
    assert 40_000 < m.n_nodes < 65_000 and 80_000 < len(m.tri) < 130_000
    O.validate_mesh(m.xyz, m.tri)
    assert abs(m.charge.sum()) < 1e-9 and len(m.charge) == 5000
    assert (np.linalg.norm(m.atom_xyz, axis=1) <= 25.0 + 1e-9).all()
    m2 = W.globular()
    assert (m2.xyz == m.xyz).all() and (m2.tri == m.tri).all()


def test_single_atom_isosurface_is_its_vdw_sphere():
    V, T, _ = W.gaussian_surface(np.zeros((1, 3)), np.array([1.7]), 0.1)
    O.validate_mesh(V, T)
    r = np.linalg.norm(V, axis=1)
    # vertices are clamped a quarter of a tetrahedron edge (<= sqrt(3) h) away
    # from grid points, so they sit within sqrt(3)/4 h of the exact level set
    assert np.abs(r - 1.7).max() < 3 ** 0.5 / 4 * 0.1 + 1e-3


def test_star_requests_valid_and_sized():
    for i in range(6):
        m = W.star_request(i)
        assert m.n_nodes in (642, 2562, 10242, 40962)
        assert 5 <= len(m.charge) <= 500
        O.validate_mesh(m.xyz, m.tri)
        # charges are inside the surface, at least 1.5 A from it along the ray
        assert (np.linalg.norm(m.atom_xyz, axis=1) < np.linalg.norm(m.xyz, axis=1).max()).all()
