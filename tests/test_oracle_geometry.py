"""Pins for mesh validation, patch geometry (Section 2, Figure 1) and the near
set."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_euler(L):
    v, t = W.icosphere(L, 1.0)
    assert v.shape[0] == 10 * 4 ** L + 2 and t.shape[0] == 20 * 4 ** L
    edges = {tuple(sorted(e)) for tri in t for e in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0]))}
    assert v.shape[0] - len(edges) + t.shape[0] == 2
    O.validate_mesh(v, t)


def test_patch_areas_tile_the_surface():
    for mol in (W.born_ion(3), W.star_request(1, level=3)):
        g = O.geometry(mol.xyz, mol.tri)
        assert g.area.sum() == pytest.approx(g.tri_area.sum(), rel=1e-13)
        assert np.allclose(np.linalg.norm(g.normal, axis=1), 1.0, atol=1e-14)
        # each patch is one third of each incident triangle
        per = np.zeros(len(g.area))
        np.add.at(per, g.tri.reshape(-1), np.repeat(g.tri_area / 3, 3))
        assert np.allclose(per, g.area, rtol=1e-13)


def test_sphere_normals_are_radial_to_second_order():
    errs = []
    for L in (2, 3, 4):
        v, t = W.icosphere(L, 2.0)
        g = O.geometry(v, t)
        errs.append(np.abs(1 - (g.normal * v / 2.0).sum(1)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-4


def test_facet_normals_point_outward_and_patch_radius():
    v, t = W.icosphere(2, 1.0)
    g = O.geometry(v, t)
    cen = v[t].mean(1)
    assert ((g.tri_n * cen).sum(1) > 0).all()
    # the farthest patch vertex is a centroid or an edge midpoint
    assert (g.rho2 > 0).all()
    edge = np.linalg.norm(v[t[:, 0]] - v[t[:, 1]], axis=1).max()
    assert np.sqrt(g.rho2).max() < edge


def test_mesh_validation_rejects_bad_meshes():
    v, t = W.icosphere(1, 1.0)
    with pytest.raises(O.MeshError):
        O.validate_mesh(v, t[1:])                      # open
    with pytest.raises(O.MeshError):
        O.validate_mesh(v, t[:, [0, 2, 1]])            # inward
    v2 = np.vstack([v, v[:1]])
    t2 = t.copy()
    t2[t2 == 0] = len(v)                               # vertex 0 unused, 42 duplicate
    t2[0] = t[0]
    with pytest.raises(O.MeshError):
        O.validate_mesh(v2, t2)
    vd = v.copy()
    vd[1] = vd[0]
    with pytest.raises(O.MeshError):
        O.validate_mesh(vd, t)                         # duplicate vertex
    with pytest.raises(O.MeshError):
        O.validate_mesh(v[:, :2], t)
    vn = v.copy()
    vn[3, 0] = np.nan
    with pytest.raises(O.MeshError):
        O.validate_mesh(vn, t)


def test_near_set_is_symmetric_contains_self_and_is_about_the_two_ring():
    mol = W.star_request(2, level=3)
    g = O.geometry(mol.xyz, mol.tri)
    rows, ptr, col = O.near_set(g, 4.0)
    n = len(g.area)
    S = np.zeros((n, n), bool)
    S[np.repeat(rows, np.diff(ptr)), col] = True
    assert (S == S.T).all() and S.diagonal().all()
    for i in range(n):
        assert (np.diff(col[ptr[i]:ptr[i + 1]]) > 0).all()
    # brute-force definition
    d2 = ((g.xyz[:, None, :] - g.xyz[None, :, :]) ** 2).sum(-1)
    ref = d2 < 16.0 * np.maximum(g.rho2[:, None], g.rho2[None, :])
    np.fill_diagonal(ref, True)
    assert (ref == S).all()
    assert 10 < S.sum(1).mean() < 40
