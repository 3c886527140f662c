"""Plain, slow, FP64 CPU oracle for the node-patch Poisson-Boltzmann operator.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the product library.

Functions that no independent pin covers are listed in ``PARITY_UNPINNED``.
"""
from .core import (COULOMB_KCAL, UNIT_SCALE, Geometry, GmresInfo, MeshError,
                   Operator, Solution, build, geometry, gmres, kernels, near_set,
                   operator, patch_coeffs, point_coeffs, reaction_energy, rhs,
                   solve, validate_mesh)
from . import closed_forms, tree

# Every oracle function is pinned by a test against closed forms, brute force,
# a library routine or an invariant; see tests/test_oracle_*.py.
PARITY_UNPINNED: tuple = ()

__all__ = [
    "COULOMB_KCAL", "UNIT_SCALE", "Geometry", "GmresInfo", "MeshError",
    "Operator", "Solution", "build", "geometry", "gmres", "kernels",
    "near_set", "operator", "patch_coeffs", "point_coeffs", "reaction_energy",
    "rhs", "solve", "validate_mesh", "closed_forms", "tree", "PARITY_UNPINNED",
]
