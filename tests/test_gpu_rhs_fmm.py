"""GPU tests of the fast multipole right-hand side and reaction potential
(one octree over the surface nodes and the atoms; atom charges to node
potentials and normal derivatives for Eq. (5)'s right-hand side, node charges
and dipoles to atom potentials for the energy) against the direct GPU sums
and the FP64 oracle.  Tolerance: 1e-5 relative (the FP64 matvec gate; the pass
runs at expansion order max(p, 14) in FP64, whose worst case, one charge on a
box corner, converges like 0.43^(p+1))."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _solver(mol, **params):
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    _say(f"set_molecule {mol.name} n={mol.n_nodes} atoms={len(mol.charge)} {params}")
    s.load(mol, **params)
    return s


CASES = {
    "born4": lambda: W.born_ion(4),                       # one atom
    "star3": lambda: W.star_request(11, level=3),         # small tree
    "star5": lambda: W.star_request(20, level=5),
    "globular": lambda: W.globular(),                     # 49k nodes, 5,000 atoms
}


@pytest.mark.parametrize("name", list(CASES))
def test_fmm_rhs_and_energy_match_direct_and_oracle(name):
    mol = CASES[name]()
    n = mol.n_nodes
    geo = O.geometry(mol.xyz, mol.tri)
    b_ref = O.rhs(geo, mol.atom_xyz, mol.charge, mol.eps_s)
    # a smooth surface field for the energy: the right-hand side itself
    # (random node values would make the energy a cancelling sum)
    x = b_ref / np.abs(b_ref).max()
    s = _solver(mol, rhs_fmm=1)
    b_dir, e_dir = s.rhs(), s.energy(x)
    assert s.tree_info()["rhs_mode"] == 1
    s.close()
    s = _solver(mol, rhs_fmm=2)
    b_fmm, e_fmm = s.rhs(), s.energy(x)
    t_tree = s.setup_times()["rhs_tree"]
    info = s.tree_info()
    assert info["rhs_mode"] == 2 and info["rhs_boxes"] >= 1
    s.close()
    e_ref, _ = O.reaction_energy(geo, mol.atom_xyz, mol.charge, mol.eps_s / mol.eps_p,
                                 x[:n], x[n:])
    _say(f"{name}: rhs fmm/direct {_rel(b_fmm, b_dir):.2e} fmm/oracle {_rel(b_fmm, b_ref):.2e} "
         f"direct/oracle {_rel(b_dir, b_ref):.2e}; energy fmm {e_fmm!r} direct {e_dir!r} "
         f"oracle {e_ref!r}; tree {t_tree:.1f} ms, {info['rhs_boxes']} boxes")
    assert _rel(b_dir, b_ref) < 1e-13
    assert _rel(b_fmm, b_ref) < 1e-5
    # each half of the right-hand side on its own
    assert _rel(b_fmm[:n], b_ref[:n]) < 1e-5 and _rel(b_fmm[n:], b_ref[n:]) < 1e-5
    assert abs(e_fmm - e_ref) <= 1e-5 * abs(e_ref)
    assert e_dir == pytest.approx(e_ref, rel=1e-12)


def test_fmm_rhs_solve_matches_direct_solve():
    """A full solve with the FMM right-hand side and energy reaches the
    energy of the solve with direct sums (1e-4, the energy gate)."""
    mol = CASES["star5"]()
    out = {}
    for mode in (1, 2):
        s = _solver(mol, rhs_fmm=mode, order_p=10, leaf_cap=64)
        f, h, E, info, _ = s.solve()
        s.close()
        assert info.converged
        out[mode] = (E, f, h)
    _say(f"solve energies direct {out[1][0]!r} fmm {out[2][0]!r}")
    assert abs(out[2][0] - out[1][0]) <= 1e-5 * abs(out[1][0])
    assert _rel(out[2][1], out[1][1]) < 1e-5 and _rel(out[2][2], out[1][2]) < 1e-5


def test_rhs_mode_is_validated():
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    with pytest.raises(A.AfmpbError) as e:
        s.load(W.born_ion(2), rhs_fmm=3)
    assert e.value.status == A.AFMPB_E_INVALID
    s.close()
