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


# ---------------------------------------------------------------------------
# Patch radius rho_t (Figure 1: the patch of node t is bounded by the edge
# midpoints and triangle centroids around t; rho_t is the farthest of them).
# Values worked by hand, on shapes chosen so that a radius taken from the
# midpoints only, from the centroids only, or from the full edges fails.
# ---------------------------------------------------------------------------

def _octahedron():
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    t = []
    for sx in (0, 1):
        for sy in (2, 3):
            for sz in (4, 5):
                f = [sx, sy, sz]
                if np.cross(v[sy] - v[sx], v[sz] - v[sx]) @ v[f].mean(0) < 0:
                    f = [sx, sz, sy]
                t.append(f)
    return v, np.array(t, np.int32)


def _bipyramid():
    """Triangular bipyramid: ring of 3 vertices at radius 1 in z = 0 (angles
    90, 210, 330 degrees), apices at z = +4 and z = -4."""
    ang = np.deg2rad([90.0, 210.0, 330.0])
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], 1)
    v = np.vstack([ring, [[0, 0, 4.0]], [[0, 0, -4.0]]])
    t = []
    for i in range(3):
        j = (i + 1) % 3
        t.append([i, j, 3])            # ring counter-clockwise seen from above
        t.append([j, i, 4])
    return v, np.array(t, np.int32)


def test_patch_radius_octahedron_hand_worked():
    # unit octahedron: edges sqrt(2); midpoint at sqrt(2)/2 (rho^2 = 1/2), the
    # centroid (1/3, 1/3, 1/3) of a face at squared distance 4/9 + 1/9 + 1/9 =
    # 2/3 from (1, 0, 0): the centroids decide, rho^2 = 2/3 at every node
    v, t = _octahedron()
    O.validate_mesh(v, t)
    g = O.geometry(v, t)
    assert np.allclose(g.rho2, 2.0 / 3.0, rtol=1e-15, atol=0)


def test_patch_radius_icosahedron_hand_worked():
    # vertices (0, +-1, +-phi) and cyclic: edge 2; equilateral faces, so the
    # centroid (a / sqrt(3) = 2 / sqrt(3)) is farther than a midpoint (1):
    # rho^2 = 4/3 at every node
    v, t = W.icosphere(0, 1.0)
    v = v * np.sqrt(1.0 + ((1.0 + np.sqrt(5.0)) / 2.0) ** 2)   # back to edge 2
    g = O.geometry(v, t)
    edge = np.linalg.norm(v[t[:, 0]] - v[t[:, 1]], axis=1)
    assert np.allclose(edge, 2.0, rtol=1e-14)
    assert np.allclose(g.rho2, 4.0 / 3.0, rtol=1e-14, atol=0)


def test_patch_radius_irregular_fan_hand_worked():
    # ring node (0, 1, 0): its edge to an apex has length sqrt(17), midpoint
    # at sqrt(17)/2 (rho^2 = 17/4); the centroid of (ring0, ring1, apex) is
    # (-sqrt(3)/6, 1/6, 4/3), squared distance 3/36 + 25/36 + 64/36 = 23/9
    # < 17/4, and the ring edge midpoint lies at sqrt(3)/2: the midpoint to the
    # apex decides.  Apex (0, 0, 4): midpoints at sqrt(17)/2 again, the same
    # centroid at 1/12 + 1/36 + 64/9 = 65/9 > 17/4: the centroid decides.
    v, t = _bipyramid()
    O.validate_mesh(v, t)
    g = O.geometry(v, t)
    assert np.allclose(g.rho2[:3], 17.0 / 4.0, rtol=1e-14, atol=0)
    assert np.allclose(g.rho2[3:], 65.0 / 9.0, rtol=1e-14, atol=0)


def test_near_set_hand_worked_on_the_fan():
    # ring-ring distance sqrt(3) (d^2 = 3), ring-apex sqrt(17) (d^2 = 17),
    # apex-apex 8 (d^2 = 64).  With eta = 1 the rule d^2 < eta^2 max(rho^2):
    # ring-ring 3 < 17/4 near; ring-apex 17 >= 65/9 far; apex-apex far.
    # With eta = 2: ring-apex 17 < 4 * 65/9 near, apex-apex 64 >= 4 * 65/9 far.
    v, t = _bipyramid()
    g = O.geometry(v, t)
    _, ptr, col = O.near_set(g, 1.0)
    rows1 = [list(col[ptr[i]:ptr[i + 1]]) for i in range(5)]
    assert rows1 == [[0, 1, 2], [0, 1, 2], [0, 1, 2], [3], [4]]
    _, ptr, col = O.near_set(g, 2.0)
    rows2 = [list(col[ptr[i]:ptr[i + 1]]) for i in range(5)]
    assert rows2 == [[0, 1, 2, 3, 4]] * 3 + [[0, 1, 2, 3], [0, 1, 2, 4]]
