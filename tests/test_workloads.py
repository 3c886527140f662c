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


def test_native_surface_generator_equals_python_generator():
    """The native marching tetrahedra (used for the capsid-scale shell) build
    the same mesh as the Python generator: identical triangles and vertex
    numbering, vertices equal up to the last bits of the exponential."""
    for seed, n, rmax, h in ((2, 300, 10.0, 1.0), (3, 2000, 18.0, 1.25), (7, 800, 12.0, 0.7)):
        pos, rad, _ = W.saw_atoms(n, rmax, seed)
        V1, T1, m1 = W.gaussian_surface(pos, rad, h)
        V2, T2, m2 = W.gaussian_surface_native(pos, rad, h)
        assert m1["grid_shape"] == m2["grid_shape"]
        assert np.array_equal(T1, T2)
        assert np.abs(V1 - V2).max() < 1e-12 * np.abs(V1).max()


def test_shell_atoms_recipe():
    """Shell atoms: radii within [r_in, r_out], minimum separation kept,
    denser towards the icosahedral vertex directions, deterministic."""
    pos, rad, q = W.shell_atoms(20_000, 60.0, 80.0, 5, batch=50_000)
    r = np.linalg.norm(pos, axis=1)
    assert r.min() >= 60.0 - 1e-9 and r.max() <= 80.0 + 1e-9
    assert rad.min() >= 1.2 and rad.max() <= 2.0 and len(q) == 20_000
    from scipy.spatial import cKDTree
    d, _ = cKDTree(pos).query(pos, k=2)
    assert d[:, 1].min() >= 1.2
    u = pos / r[:, None]
    near_vertex = np.max(u @ W._ico_directions().T, axis=1) > 0.98
    frac_cap = near_vertex.mean()
    # w = 0.5 + 0.5 c^16 >= 0.5 + 0.5 * 0.98^16 = 0.86 in the caps; the largest
    # cosine to a vertex direction is >= 0.79 everywhere (w >= 0.51), so the
    # caps hold a clearly larger share than their solid angle
    cap_solid = 12 * 2 * np.pi * (1 - 0.98) / (4 * np.pi)
    assert frac_cap > 1.25 * cap_solid
    pos2, _, _ = W.shell_atoms(20_000, 60.0, 80.0, 5, batch=50_000)
    assert np.array_equal(pos, pos2)


def test_capsid_shell_small_replica_is_a_valid_surface():
    """The capsid recipe at a small scale (20,000 atoms in a 60-80 A shell):
    a closed, outward-oriented, valid mesh."""
    pos, rad, q = W.shell_atoms(20_000, 60.0, 80.0, 5, batch=50_000)
    V, T, _ = W.gaussian_surface_native(pos, rad, W.CAPSID_H_GRID)
    O.validate_mesh(V, T)
    assert W.check_closed_manifold(T)
