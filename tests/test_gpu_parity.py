"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bit-exact: Morton keys, permutation, boxes, U/V/W/X lists and offset classes,
near-set structure.  Floating point: near corrections (1e-12 of scale), the
direct (all-P2P) matvec (1e-12 rel-L2), the FMM matvec (1e-5 rel-L2 from
p = 10; at p = 8 the truncation law extrapolated from p = 10 and 12), RHS and
energy kernels (1e-12), solvation energies (1e-4 relative)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import tree as OT

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _solver(mol, **params):
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    _say(f"set_molecule {mol.name} n={mol.n_nodes} {params}")
    s.load(mol, **params)
    return s


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


MOLS = {
    "born3": lambda: W.born_ion(3),
    "born4": lambda: W.born_ion(4),
    "star3": lambda: W.star_request(11, level=3),
    "star4": lambda: W.star_request(12, level=4),
    "globular": lambda: W.globular(),
}


# ------------------------------- tree ---------------------------------------

@pytest.mark.parametrize("name,cap", [("born4", 64), ("star3", 16), ("star4", 32), ("star4", 5),
                                      ("globular", 64), ("globular", 192)])
def test_tree_and_lists_bit_exact(name, cap):
    """Keys, permutation, boxes and the four lists against the CPU tree.  The
    globular molecule (49,190 nodes) spans twelve 4,096-key tiles of the
    radix sort, so its cross-tile offsets are checked too."""
    mol = MOLS[name]()
    s = _solver(mol, leaf_cap=cap)
    g = s.debug_tree()
    key, perm, _, _ = OT.morton_keys(mol.xyz)
    _say(f"sizes {g['sizes']}")
    dk = np.nonzero(g["keys"].astype(np.int64) != key[perm])[0]
    assert len(dk) == 0, f"keys differ at {dk[:5]}: {g['keys'][dk[:5]]} vs {key[perm][dk[:5]]}"
    dp = np.nonzero(g["perm"] != perm)[0]
    assert len(dp) == 0, f"perm differs at {dp[:5]}"
    t = OT.build_tree(mol.xyz, cap)
    assert g["sizes"]["n_boxes"] == t.nbox, (g["sizes"]["n_boxes"], t.nbox)
    for a, b in (("level", t.level), ("parent", t.parent), ("pt_begin", t.pt_begin),
                 ("pt_end", t.pt_end), ("n_child", t.n_child)):
        d = np.nonzero(g[a] != b)[0]
        assert len(d) == 0, f"{a} differs at {d[:5]}: {g[a][d[:5]]} vs {b[d[:5]]}"
    assert (g["prefix"].astype(np.int64) == t.prefix).all()
    nc = t.n_child > 0
    assert (g["child_begin"][nc] == t.child_begin[nc]).all()
    L = OT.build_lists(t)
    for lst, pk, ik in ((L.U, "u_ptr", "u_idx"), (L.V, "v_ptr", "v_idx"), (L.W, "w_ptr", "w_idx"),
                        (L.X, "x_ptr", "x_idx")):
        ptr = np.r_[0, np.cumsum([len(r) for r in lst])]
        flat = np.array([c for r in lst for c in r], dtype=np.int64)
        d = np.nonzero(g[pk] != ptr)[0]
        if len(d):
            B = d[0] - 1 if d[0] > 0 else 0
            gl = g[ik][g[pk][B]:g[pk][B + 1]]
            raise AssertionError(f"{pk} differs first at {d[0]}; box {B}: gpu {list(gl)} "
                                 f"oracle {lst[B]}")
        assert (g[ik] == flat).all(), ik
    vc = np.array([c for r in L.V_class for c in r], dtype=np.int64)
    assert (g["v_class"] == vc).all()
    s.close()


def test_near_set_bit_exact_and_corrections():
    mol = MOLS["star3"]()
    s = _solver(mol)
    g = s.debug_tree()
    perm = g["perm"].astype(np.int64)
    geo = O.geometry(mol.xyz, mol.tri)
    rows, ptr, col = O.near_set(geo, 4.0)
    inv = np.argsort(perm)
    # GPU rows/cols are Morton positions; map to caller indices
    gp = g["near_ptr"]
    gc = perm[g["near_col"]]
    for m in range(mol.n_nodes):
        p = perm[m]
        assert sorted(gc[gp[m]:gp[m + 1]]) == list(col[ptr[p]:ptr[p + 1]])
        assert (np.diff(g["near_col"][gp[m]:gp[m + 1]]) > 0).all()
    # corrections: GPU delta + oracle point rule == oracle patch integral
    P = np.repeat(perm[np.arange(mol.n_nodes)], np.diff(gp))
    T = gc
    ebar = mol.eps_s / mol.eps_p
    patch = O.patch_coeffs(geo, mol.kappa, ebar, P, T)
    point = O.point_coeffs(geo, mol.kappa, ebar, P, T)
    point[P == T] = 0.0
    scale = np.abs(patch).max(axis=0)
    err = np.abs(g["near_delta"] + point - patch).max(axis=0) / scale
    assert (err < 1e-12).all(), err
    _ = inv
    s.close()


def test_near_set_bit_exact_globular():
    """Near set of the 49,190-node molecule (5.58 M entries, every cell of
    the GPU's grid search in use) equals the oracle's set exactly; corrections
    on 4,000 sampled entries are within 1e-12 of the oracle's patch minus
    point values."""
    mol = MOLS["globular"]()
    n = mol.n_nodes
    s = _solver(mol)
    g = s.debug_tree()
    s.close()
    perm = g["perm"].astype(np.int64)
    geo = O.geometry(mol.xyz, mol.tri)
    rows, ptr, col = O.near_set(geo, 4.0)
    gp = g["near_ptr"]
    gcol = g["near_col"].astype(np.int64)
    assert gp[-1] == len(col), (gp[-1], len(col))
    # rows ascending in Morton position
    row_of = np.repeat(np.arange(n), np.diff(gp))
    assert (np.diff(gcol)[np.diff(row_of) == 0] > 0).all()
    gkey = np.sort(perm[row_of] * n + perm[gcol])
    okey = np.repeat(rows, np.diff(ptr)) * n + col
    d = np.nonzero(gkey != np.sort(okey))[0]
    assert len(d) == 0, f"near sets differ at {d[:5]}"
    rng = np.random.default_rng(17)
    sel = np.sort(rng.choice(len(gcol), size=4000, replace=False))
    P, T = perm[row_of[sel]], perm[gcol[sel]]
    ebar = mol.eps_s / mol.eps_p
    patch = O.patch_coeffs(geo, mol.kappa, ebar, P, T)
    point = O.point_coeffs(geo, mol.kappa, ebar, P, T)
    point[P == T] = 0.0
    scale = np.abs(patch).max(axis=0)
    err = np.abs(g["near_delta"][sel] + point - patch).max(axis=0) / scale
    _say(f"globular near entries {len(gcol)}, sampled correction errors {err}")
    assert (err < 1e-12).all(), err


# ------------------------------- matvec -------------------------------------

def _oracle_op(mol):
    return O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa)


@pytest.mark.parametrize("name", ["born3", "star3", "star4"])
def test_direct_matvec_matches_oracle(name):
    mol = MOLS[name]()
    op = _oracle_op(mol)
    x = np.random.default_rng(3).normal(size=2 * mol.n_nodes)
    ref = op.matvec(x)
    s = _solver(mol, leaf_cap=mol.n_nodes)            # root is a leaf: every pair by P2P
    y = s.matvec(x)
    assert _rel(y, ref) < 1e-12
    s.close()


def _check_truncation_gate(errs):
    """The FP64 matvec gate: 1e-5 relative L2 against the direct oracle at an
    expansion order matched to that tolerance (p >= 10 on these meshes).  At
    p = 8 the error is the expansion's truncation error, which falls
    geometrically with the order (each translation's remainder is a power
    (a/R)^(p+1) of the separation ratio): it must lie within the same law
    extrapolated from p = 10 and 12, e_8 <= 2 e_10 (e_10 / e_12), the factor
    2 allowing the per-order rate to drift by sqrt(2) over two orders."""
    assert errs[10] < 1e-5 and errs[12] < 1e-5
    bound8 = 2.0 * errs[10] * (errs[10] / errs[12])
    _say(f"p = 8 truncation bound {bound8:.2e}, error {errs[8]:.2e}")
    assert errs[8] <= bound8


@pytest.mark.parametrize("name", ["born4", "star4"])
def test_fmm_matvec_matches_oracle_and_converges_in_p(name):
    mol = MOLS[name]()
    op = _oracle_op(mol)
    x = np.random.default_rng(4).normal(size=2 * mol.n_nodes)
    ref = op.matvec(x)
    errs = {}
    for p, cap in ((4, 32), (8, 32), (10, 32), (12, 32)):
        s = _solver(mol, order_p=p, leaf_cap=cap)
        info = s.tree_info()
        assert info["n_v"] > 0                          # the far field is exercised
        errs[p] = _rel(s.matvec(x), ref)
        s.close()
    _say(f"fmm errors {errs}")
    assert errs[4] > errs[8] > errs[10] > errs[12]
    _check_truncation_gate(errs)


@pytest.mark.parametrize("name,cap,p", [("born4", 16, 6), ("born4", 32, 8), ("star4", 16, 10),
                                        ("star4", 5, 14)])
def test_m2l_layouts_agree_and_match_oracle(name, cap, p):
    """The M2L work layouts, one result slot per V entry (1), one per
    (target, colleague of its parent) with the colleague's children summed in
    registers (2), and the same slots filled by work items of box pairs
    (parent, colleague) (3), in every precision: the same sums up to rounding
    order, and as close to the oracle as each other.  Small trees share an
    item's octants among several blocks (some shares empty), p = 14 takes 15
    row tiles per operator; orders 6 to 14 run the four pair kernels (two to
    eight row-tile jobs per wave)."""
    import paper_1710_06316_amd as A
    mol = MOLS[name]()
    x = np.random.default_rng(6).normal(size=2 * mol.n_nodes)
    ref = _oracle_op(mol).matvec(x)
    agree = {A.AFMPB_FP64: 1e-13, A.AFMPB_FP32_REFINED: 1e-5, A.AFMPB_FP32_BF16M2L_REFINED: 1e-5}
    for prec, tol in agree.items():
        ys, errs = {}, {}
        for layout in (1, 2, 3):
            s = _solver(mol, order_p=p, leaf_cap=cap, precision=prec, m2l_layout=layout)
            info = s.tree_info()
            assert info["m2l_layout"] == layout and info["n_v"] > 0
            if layout == 1:
                assert info["n_m2l_slots"] == info["n_m2l_pairs"]
            ys[layout] = s.matvec(x)
            errs[layout] = _rel(ys[layout], ref)
            s.close()
        d = max(_rel(ys[2], ys[1]), _rel(ys[3], ys[1]))
        _say(f"{name} p={p} precision={prec} layouts differ {d:.2e}, oracle errors {errs}")
        assert d < tol
        for layout in (2, 3):
            assert errs[layout] <= 1.05 * errs[1] + tol and errs[layout] < 1e-4


def _far_w(mol, cap, tau):
    """W entries (B, C) of the CPU tree whose point counts have a harmonic
    mean >= tau, and the ordered point pairs they stand for."""
    t = OT.build_tree(mol.xyz, cap)
    cnt = t.pt_end - t.pt_begin
    far = pairs = 0
    for B, ws in enumerate(OT.build_lists(t).W):
        for C in ws:
            a, b = int(cnt[B]), int(cnt[C])
            if b > 0 and 2 * a * b >= tau * (a + b):
                far += 1
                pairs += 2 * a * b
    return far, pairs


@pytest.mark.parametrize("name,cap,p", [("born4", 16, 6), ("star4", 16, 8), ("star4", 16, 10),
                                        ("star4", 5, 14)])
def test_wx_expansions_match_oracle(name, cap, p):
    """W/X entries by expansions (C's multipole at B's points, B's points into
    C's local expansion; Section 3.2) instead of direct pairs: the entries
    chosen are those of the CPU tree's W lists above the threshold, the P2P
    work shrinks by exactly their point pairs, and the product stays as close
    to the oracle as with every W/X pair direct (the expansions converge at
    least as fast as the M2L's)."""
    import paper_1710_06316_amd as A
    mol = MOLS[name]()
    x = np.random.default_rng(9).normal(size=2 * mol.n_nodes)
    ref = _oracle_op(mol).matvec(x)
    far, far_pairs = _far_w(mol, cap, 2)
    assert far > 0
    for prec, tol in ((A.AFMPB_FP64, 1e-12), (A.AFMPB_FP32_REFINED, 2e-6)):
        s = _solver(mol, order_p=p, leaf_cap=cap, precision=prec, wx_expand=1)
        off = s.tree_info()
        y_off = s.matvec(x)
        s.close()
        s = _solver(mol, order_p=p, leaf_cap=cap, precision=prec, wx_expand=2)
        on = s.tree_info()
        y_on = s.matvec(x)
        s.close()
        assert off["n_wx_far"] == 0 and off["n_wx_pairs"] == 0
        assert (on["n_wx_far"], on["n_wx_pairs"]) == (far, far_pairs)
        assert on["n_p2p_pairs"] + on["n_wx_pairs"] == off["n_p2p_pairs"]
        e_off, e_on = _rel(y_off, ref), _rel(y_on, ref)
        _say(f"{name} p={p} precision={prec} W entries by expansions {far}/{off['n_w']}: "
             f"oracle errors {e_off:.2e} (direct) {e_on:.2e} (expansions)")
        assert e_on <= 2.0 * e_off + tol and e_on < 1e-4


def test_wx_expansions_globular_solve():
    """On the 49,190-node molecule, W entries of harmonic-mean size >= 16 by
    expansions: the FP32 matvec and the polar energy of a solve agree with
    the all-direct run and the oracle."""
    import paper_1710_06316_amd as A
    mol = MOLS["globular"]()
    x = np.random.default_rng(10).normal(size=2 * mol.n_nodes)
    ref = _oracle_op(mol).matvec(x)
    ys, es = {}, {}
    for wx in (1, 16):
        s = _solver(mol, order_p=8, leaf_cap=64, precision=A.AFMPB_FP32_REFINED, wx_expand=wx)
        info = s.tree_info()
        assert (info["n_wx_far"] > 0) == (wx > 1)
        ys[wx] = s.matvec(x)
        es[wx] = s.solve()[2]
        s.close()
        _say(f"globular wx={wx} far W {info['n_wx_far']} pairs {info['n_wx_pairs']} "
             f"error {_rel(ys[wx], ref):.2e} energy {es[wx]:.6f}")
    assert _rel(ys[16], ref) <= 2.0 * _rel(ys[1], ref) + 2e-6
    assert abs(es[16] - es[1]) <= 1e-5 * abs(es[1])


@pytest.mark.parametrize("p", [8, 14])
def test_overlap_schedules_bit_identical(p):
    """The near-field schedules (P2P beside the whole far-field chain, the
    near-set correction beside P2M and P2P after it, or one stream) add the
    same two terms per row, so the products agree bit for bit; all match the
    oracle."""
    import paper_1710_06316_amd as A
    mol = MOLS["globular"]()
    x = np.random.default_rng(8).normal(size=2 * mol.n_nodes)
    ref = _oracle_op(mol).matvec(x)
    for prec in (A.AFMPB_FP64, A.AFMPB_FP32_REFINED):
        ys = {}
        for overlap in (1, 2, 3):
            s = _solver(mol, order_p=p, leaf_cap=128, precision=prec, overlap=overlap)
            ys[overlap] = s.matvec(x)
            s.close()
        err = _rel(ys[2], ref)
        _say(f"p={p} precision={prec} oracle error {err:.2e}")
        assert np.array_equal(ys[1], ys[2]) and np.array_equal(ys[1], ys[3])
        assert err < (2e-4 if p == 8 else 1e-5)


def test_fmm_matvec_kappa_zero_and_identity_case():
    mol = MOLS["star3"]()
    x = np.random.default_rng(5).normal(size=2 * mol.n_nodes)
    m0 = W.Molecule("k0", mol.xyz, mol.tri, mol.atom_xyz, mol.charge, mol.radius, 2.0, 80.0, 0.0)
    ref = _oracle_op(m0).matvec(x)
    s = _solver(m0, leaf_cap=16, order_p=10)
    assert _rel(s.matvec(x), ref) < 1e-5
    s.close()
    mi = W.Molecule("id", mol.xyz, mol.tri, mol.atom_xyz, mol.charge, mol.radius, 3.0, 3.0, 0.0)
    s = _solver(mi, leaf_cap=16)
    assert _rel(s.matvec(x), x) < 1e-13
    s.close()


def test_rhs_and_energy_kernels():
    mol = MOLS["star3"]()
    s = _solver(mol)
    geo = O.geometry(mol.xyz, mol.tri)
    b_ref = O.rhs(geo, mol.atom_xyz, mol.charge, mol.eps_s)
    assert _rel(s.rhs(), b_ref) < 1e-13
    x = np.random.default_rng(6).normal(size=2 * mol.n_nodes)
    e_ref, _ = O.reaction_energy(geo, mol.atom_xyz, mol.charge, mol.eps_s / mol.eps_p,
                                 x[:mol.n_nodes], x[mol.n_nodes:])
    assert s.energy(x) == pytest.approx(e_ref, rel=1e-12)
    s.close()


# ------------------------------- solve --------------------------------------

@pytest.mark.parametrize("precision", [0, 1])
def test_born_ion_solve_energy(precision):
    from oracle.closed_forms import born_energy
    mol = W.born_ion(4)
    ref = O.solve(mol)
    s = _solver(mol, precision=precision)
    f, h, E, info, st = s.solve()
    _say(f"born solve precision={precision} E={E} oracle={ref.energy} info={info.as_dict()}")
    assert info.converged and info.true_rel_residual < 2e-6
    assert E == pytest.approx(ref.energy, rel=1e-4)
    assert E == pytest.approx(born_energy(1.0, 2.0, 2.0, 80.0, 0.1), rel=0.01)
    assert _rel(f, ref.f) < 1e-4 and _rel(h, ref.h) < 1e-4
    s.close()


def test_star_solve_energy_matches_oracle():
    mol = MOLS["star4"]()
    ref = O.solve(mol)
    s = _solver(mol, leaf_cap=32)
    f, h, E, info, st = s.solve()
    assert E == pytest.approx(ref.energy, rel=1e-4)
    s.close()


@pytest.mark.parametrize("name", ["born4", "star4"])
@pytest.mark.parametrize("precision", [0, 1])
def test_restarted_gmres_matches_oracle(name, precision):
    """Short restart cycles (3 Krylov vectors, up to 40 restarts) on the GPU
    against the oracle's restarted GMRES with the same settings (Section 3.4,
    stopping rule Eq. 7): both converge, energies and potentials agree to
    1e-4."""
    mol = MOLS[name]()
    ref = O.solve(mol, restart=3, max_restarts=40)
    assert ref.info.converged and ref.info.restarts > 0
    s = _solver(mol, leaf_cap=32, order_p=10, precision=precision, restart=3, max_restarts=40)
    f, h, E, info, st = s.solve()
    s.close()
    _say(f"{name} restart 3 precision={precision}: E={E:.8f} oracle={ref.energy:.8f} "
         f"iters {info.iterations} restarts {info.restarts} (oracle {ref.info.iterations}/"
         f"{ref.info.restarts}) refine {info.refinement_steps}")
    assert info.converged and info.true_rel_residual < 2e-6
    if precision == 0:
        assert info.restarts > 0
    assert E == pytest.approx(ref.energy, rel=1e-4)
    assert _rel(f, ref.f) < 1e-4 and _rel(h, ref.h) < 1e-4


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_start_matches_oracle(precision):
    """x0 = the oracle's solution with 1e-3 relative noise: the GPU solve
    starts from it (fewer iterations than from zero) and ends at the
    oracle's solution, as the oracle's GMRES does from the same x0."""
    mol = MOLS["star4"]()
    ref = O.solve(mol)
    rng = np.random.default_rng(23)
    x0 = ref.x * (1.0 + 1e-3 * rng.standard_normal(ref.x.shape))
    ref0 = O.solve(mol, x0=x0)
    s = _solver(mol, leaf_cap=32, order_p=10, precision=precision)
    _, _, E_cold, info_cold, _ = s.solve()
    f, h, E, info, st = s.solve(x0=x0)
    s.close()
    _say(f"warm start precision={precision}: E={E:.8f} oracle={ref.energy:.8f} "
         f"oracle-from-x0={ref0.energy:.8f} iters {info.iterations} (cold {info_cold.iterations}, "
         f"oracle from x0 {ref0.info.iterations})")
    assert info.converged and info.iterations < info_cold.iterations
    assert E == pytest.approx(ref.energy, rel=1e-4) and E == pytest.approx(ref0.energy, rel=1e-4)
    assert _rel(f, ref.f) < 1e-4 and _rel(h, ref.h) < 1e-4


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)) as fh:
        return json.load(fh)


@pytest.mark.parametrize("precision", [0, 1])
def test_globular_energy_matches_oracle_reference(precision):
    """Solvation energy of the 49,190-node molecule (5,000 atoms) against the
    oracle's solve stored by tests/golden/make_oracle_energies.py (1e-4, the
    energy gate), plain FP64 and FP32 with FP64 refinement."""
    ref = _golden("oracle_globular_5000.json")["energy_kcal_mol"]
    mol = MOLS["globular"]()
    s = _solver(mol, order_p=10, leaf_cap=192, precision=precision)
    f, h, E, info, _ = s.solve()
    s.close()
    _say(f"globular precision={precision}: E={E:.6f} oracle={ref:.6f} "
         f"rel={abs(E - ref) / abs(ref):.2e} iters={info.iterations}")
    assert info.converged and info.true_rel_residual < 2e-6
    assert abs(E - ref) <= 1e-4 * abs(ref)


def test_globular_sampled_rows():
    mol = W.globular()
    n = mol.n_nodes
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n, size=192, replace=False))
    op = O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa, rows=rows)
    x = rng.normal(size=2 * n)
    yf, yh = op.apply_rows(x)
    errs = {}
    for p in (8, 10, 12):
        s = _solver(mol, order_p=p)
        y = s.matvec(x)
        errs[p] = np.linalg.norm(np.r_[y[rows] - yf, y[n + rows] - yh]) / np.linalg.norm(np.r_[yf, yh])
        s.close()
    _say(f"globular sampled-row errors {errs}")
    assert errs[8] > errs[10] > errs[12]
    _check_truncation_gate(errs)


# ------------------------------- errors -------------------------------------

def test_error_contract():
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    with pytest.raises(A.AfmpbError) as e:
        s.matvec(np.zeros(10))
    assert e.value.status == A.AFMPB_E_STATE
    v, t = W.icosphere(2, 1.0)
    with pytest.raises(A.AfmpbError) as e:
        s.set_molecule(v, t[1:], np.zeros((1, 3)), [1.0])
    assert e.value.status == A.AFMPB_E_MESH
    with pytest.raises(A.AfmpbError) as e:
        s.set_molecule(v, t[:, [0, 2, 1]], np.zeros((1, 3)), [1.0])
    assert e.value.status == A.AFMPB_E_MESH
    with pytest.raises(A.AfmpbError) as e:
        s.set_molecule(v, t, np.zeros((1, 3)), [1.0], eps_p=-1.0)
    assert e.value.status == A.AFMPB_E_INVALID
    with pytest.raises(A.AfmpbError) as e:
        s.set_molecule(v, t, np.zeros((1, 3)), [1.0], order_p=40)
    assert e.value.status == A.AFMPB_E_INVALID
    s.set_molecule(v, t, np.zeros((1, 3)), [1.0])
    x = np.zeros(2 * len(v))
    x[3] = np.nan
    with pytest.raises(A.AfmpbError) as e:
        s.matvec(x)
    assert e.value.status == A.AFMPB_E_NUMERIC
    s.set_molecule(v, t, np.zeros((1, 3)), [1.0], restart=1, max_restarts=0, rel_tol=1e-14)
    f, h, E, info, st = s.solve(allow_not_converged=True)
    assert st == A.AFMPB_E_NOT_CONVERGED and info.iterations == 1 and np.isfinite(E)
    s.close()


def test_profile_scopes_and_filter():
    """Per-kernel timing: every scope when unrestricted; only the named one
    (with one launch per matvec for M2L here) after afmpb_profile_only; the
    result of the matvec is the same with and without timing."""
    mol = MOLS["born4"]()
    s = _solver(mol, order_p=8, precision=1, leaf_cap=16)
    assert s.tree_info()["n_m2l_pairs"] > 0
    x = np.random.default_rng(11).normal(size=2 * mol.n_nodes)
    y0 = s.matvec(x)
    s.profile(True)
    s.matvec(x)
    allp = s.profile_read()
    s.profile(False)
    for k in ("p2m", "m2l", "m2l_reduce", "l2p", "p2p", "near", "combine"):
        assert allp[k][1] >= 1 and allp[k][0] > 0, (k, allp.get(k))
    s.profile_only("m2l")
    s.profile(True)
    y1 = s.matvec(x)
    only = s.profile_read()
    s.profile(False)
    s.profile_only(None)
    assert only["m2l"][1] == allp["m2l"][1] and only["m2l"][0] > 0
    assert all(v[1] == 0 for k, v in only.items() if k != "m2l"), only
    assert np.array_equal(y0, y1)
    s.close()


# ------------------------- 100k-atom complex (~1M nodes) --------------------

_COMPLEX = {}


def _complex():
    if "mol" not in _COMPLEX:
        _say("generating complex_100k")
        mol = W.complex_100k()
        rng = np.random.default_rng(31)
        rows = np.sort(rng.choice(mol.n_nodes, size=96, replace=False))
        _say(f"complex_100k n={mol.n_nodes}: oracle rows")
        op = O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa, rows=rows,
                        validate=False)
        x = rng.normal(size=2 * mol.n_nodes)
        yf, yh = op.apply_rows(x)
        _COMPLEX.update(mol=mol, rows=rows, x=x, ref=np.r_[yf, yh])
    return _COMPLEX


@pytest.mark.parametrize("p,precision,tol", [(6, 0, 2e-4), (10, 0, 1e-5), (14, 0, 2e-6),
                                             (10, 1, 1e-5)])
def test_complex_sampled_rows(p, precision, tol):
    """~1M-node matvec on 96 oracle rows at expansion orders 6 / 10 / 14
    (errors fall with p; the 1e-5 tolerance is met from p = 10)."""
    c = _complex()
    mol, rows, x, ref = c["mol"], c["rows"], c["x"], c["ref"]
    n = mol.n_nodes
    s = _solver(mol, order_p=p, precision=precision)
    y = s.matvec(x)
    info = s.tree_info()
    s.close()
    err = np.linalg.norm(np.r_[y[rows], y[n + rows]] - ref) / np.linalg.norm(ref)
    _say(f"complex p={p} precision={precision} rows err {err:.3e} boxes {info['n_boxes']} "
         f"V {info['n_m2l_pairs']} near {info['n_near']}")
    assert err < tol


def test_capsid_sampled_rows():
    """The capsid-scale shell (9.7M nodes, 1.1M atoms) in the benchmark's
    configuration (order 8, its leaf capacity, one setup serving the
    FP32-refined and the FP64 form) on 24 oracle rows, and at order 10 in
    FP32.  The 1e-5 gate binds at order 10; order 8 must converge towards it
    (its error above order 10's, both forms within 10% of each other) and
    stay below 5e-5, against a measured 3.0e-5 on these rows: a broken far
    field or near correction gives errors of 1e-3 and more."""
    import bench
    import paper_1710_06316_amd as A
    _say("capsid shell: generating")
    mol = W.capsid_shell()
    n = mol.n_nodes
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, size=24, replace=False))
    _say(f"capsid shell n={n}: oracle rows")
    op = O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa, rows=rows,
                    validate=False)
    x = rng.normal(size=2 * n)
    yf, yh = op.apply_rows(x)
    ref = np.r_[yf, yh]
    leaf = bench.WORKLOADS["capsid"][3]
    errs = {}
    s = _solver(mol, order_p=8, leaf_cap=leaf, precision=A.AFMPB_FP32_REFINED)
    for prec in (A.AFMPB_FP32_REFINED, A.AFMPB_FP64):
        s.set_precision(prec)
        y = s.matvec(x)
        errs[(8, prec)] = np.linalg.norm(np.r_[y[rows], y[n + rows]] - ref) / np.linalg.norm(ref)
    s.close()
    s = _solver(mol, order_p=10, leaf_cap=leaf, precision=A.AFMPB_FP32_REFINED)
    y = s.matvec(x)
    s.close()
    errs[(10, 1)] = np.linalg.norm(np.r_[y[rows], y[n + rows]] - ref) / np.linalg.norm(ref)
    _say(f"capsid sampled-row errors {errs}")
    e32, e64 = errs[(8, A.AFMPB_FP32_REFINED)], errs[(8, A.AFMPB_FP64)]
    assert errs[(10, 1)] < 1e-5
    assert e32 > errs[(10, 1)] and e64 > errs[(10, 1)]
    assert abs(e32 - e64) <= 0.1 * e64 and e32 < 5e-5 and e64 < 5e-5


def test_complex_energy_mixed_vs_fp64():
    """~1M-node solve: the mixed-precision form at p = 10 against the FP64
    form at p = 14 (parity unpinned: no oracle solve at this size)."""
    mol = _complex()["mol"]
    out = {}
    for p, prec in ((10, 1), (14, 0)):
        s = _solver(mol, order_p=p, precision=prec)
        f, h, E, info, _ = s.solve()
        s.close()
        _say(f"complex solve p={p} precision={prec} E={E:.6f} iters={info.iterations} "
             f"res={info.true_rel_residual:.2e}")
        assert info.converged
        out[p] = E
    assert abs(out[10] - out[14]) <= 1e-4 * abs(out[14])


# ------------------------- bf16-split M2L -----------------------------------

def test_bf16_m2l_matvec_and_solve():
    """Mixed precision with bf16-split M2L: the matvec stays within the FMM
    error plus ~2^-16 of the far field, and the refined solve reaches the
    oracle energy (1e-4)."""
    import paper_1710_06316_amd as A
    mol = MOLS["born4"]()
    ref = O.solve(mol)
    x = np.random.default_rng(3).normal(size=2 * mol.n_nodes)
    y_ref = ref.op.matvec(x)
    errs = {}
    for prec in (A.AFMPB_FP32_REFINED, A.AFMPB_FP32_BF16M2L_REFINED):
        s = _solver(mol, order_p=10, precision=prec)
        errs[prec] = _rel(s.matvec(x), y_ref)
        f, h, E, info, _ = s.solve()
        s.close()
        _say(f"born4 precision={prec} matvec err {errs[prec]:.3e} E={E:.6f} oracle={ref.energy:.6f} "
             f"iters={info.iterations} refine={info.refinement_steps}")
        assert info.converged
        assert abs(E - ref.energy) <= 1e-4 * abs(ref.energy)
    assert errs[A.AFMPB_FP32_BF16M2L_REFINED] < 5e-5


def test_bf16_m2l_complex_rows():
    """~1M nodes, p = 14: bf16-split M2L on 96 oracle rows."""
    import paper_1710_06316_amd as A
    c = _complex()
    mol, rows, x, ref = c["mol"], c["rows"], c["x"], c["ref"]
    n = mol.n_nodes
    s = _solver(mol, order_p=14, precision=A.AFMPB_FP32_BF16M2L_REFINED)
    y = s.matvec(x)
    s.close()
    err = np.linalg.norm(np.r_[y[rows], y[n + rows]] - ref) / np.linalg.norm(ref)
    _say(f"complex p=14 bf16 rows err {err:.3e}")
    assert err < 5e-5


@pytest.mark.parametrize("cap", [16, 64, 192, 256])
def test_matvec_bitwise_reproducible_across_leaf_capacities(cap):
    """The matvec uses no atomics: P2P partials, reverse sums, the near
    correction and the M2L slots are added in fixed orders, so repeated calls
    and a fresh setup of the same molecule give bitwise-identical results.
    Leaf capacities from 16 to 256 take the P2P groups from one copy of 8
    lanes to full tiles, several source chunks per group and the multi-chunk
    P2M; the trees differ, the FMM results agree to the truncation error."""
    import paper_1710_06316_amd as A
    mol = W.globular()
    x = np.random.default_rng(8).normal(size=2 * mol.n_nodes)
    for prec in (A.AFMPB_FP32_REFINED, A.AFMPB_FP64):
        s = _solver(mol, order_p=10, leaf_cap=cap, precision=prec)
        y1, y2 = s.matvec(x), s.matvec(x)
        s.close()
        s = _solver(mol, order_p=10, leaf_cap=cap, precision=prec)
        y3 = s.matvec(x)
        s.close()
        _say(f"leaf {cap} precision {prec}: repeat equal {np.array_equal(y1, y2)}, "
             f"fresh setup equal {np.array_equal(y1, y3)}")
        assert np.array_equal(y1, y2) and np.array_equal(y1, y3)
        # against the same matvec on a leaf-64 tree (a different tree)
        s = _solver(mol, order_p=10, leaf_cap=64, precision=prec)
        y64 = s.matvec(x)
        s.close()
        d = _rel(y1, y64)
        _say(f"leaf {cap} vs leaf 64: {d:.2e}")
        assert d < 2e-5
