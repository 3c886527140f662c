"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only, gcc): every entry point runs on a small molecule without a
sanitizer report, and its results equal those of the library the other tests
use (same source, same contraction-free FP64 arithmetic)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import core as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path):
    exe = str(tmp_path / "orc_sanitized")
    cmd = ["gcc", "-O1", "-g", "-ffp-contract=off", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("gcc without the address/undefined sanitizer runtimes: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_entry_points_clean_under_sanitizers(tmp_path):
    mol = W.star_request(3, level=2)            # 162 nodes, charges inside
    geo = C.geometry(mol.xyz, mol.tri)
    n, m, na = geo.xyz.shape[0], geo.tri.shape[0], len(mol.charge)
    ebar, eta = mol.eps_s / mol.eps_p, 4.0
    x = np.random.default_rng(3).normal(size=2 * n)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.array([n, m, na], dtype=np.int64).tofile(f)
        np.array([mol.kappa, ebar, mol.eps_s, eta], dtype=np.float64).tofile(f)
        geo.xyz.astype(np.float64).tofile(f)
        geo.tri.astype(np.int32).tofile(f)
        geo.inc_ptr.astype(np.int64).tofile(f)
        geo.inc_tri.astype(np.int64).tofile(f)
        np.asarray(mol.atom_xyz, dtype=np.float64).tofile(f)
        np.asarray(mol.charge, dtype=np.float64).tofile(f)
        x.tofile(f)
    out = tmp_path / "out.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([_build(tmp_path), str(inp), str(out)], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR" not in r.stderr, \
        r.stderr[-3000:]

    raw = open(out, "rb").read()
    pos = 0

    def take(count, dtype):
        nonlocal pos
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    ta, tn = take(m, np.float64), take(3 * m, np.float64)
    area, nn, rho2 = take(n, np.float64), take(3 * n, np.float64), take(n, np.float64)
    nnz = int(take(1, np.int64)[0])
    ptr, col = take(n + 1, np.int64), take(nnz, np.int64)
    coef, point = take(4 * nnz, np.float64), take(4 * nnz, np.float64)
    y, b = take(2 * n, np.float64), take(2 * n, np.float64)
    esum, phi = take(1, np.float64)[0], take(na, np.float64)
    assert pos == len(raw)

    # the same quantities from the library the other tests use
    assert np.array_equal(ta, geo.tri_area) and np.array_equal(tn, geo.tri_n.reshape(-1))
    assert np.array_equal(area, geo.area) and np.array_equal(nn, geo.normal.reshape(-1))
    assert np.array_equal(rho2, geo.rho2)
    rows, rptr, rcol = C.near_set(geo, eta)
    assert np.array_equal(ptr, rptr) and np.array_equal(col, rcol)
    pr = np.repeat(rows, np.diff(rptr))
    assert np.allclose(coef, C.patch_coeffs(geo, mol.kappa, ebar, pr, rcol).reshape(-1),
                       rtol=1e-13, atol=0)
    # the point rule is undefined on the diagonal (r = 0), where the stored
    # value is the patch integral alone
    off = np.repeat(pr != rcol, 4)
    assert np.allclose(point[off],
                       C.point_coeffs(geo, mol.kappa, ebar, pr, rcol).reshape(-1)[off],
                       rtol=1e-13, atol=0)
    op = O.operator(mol.xyz, mol.tri, mol.eps_p, mol.eps_s, mol.kappa, eta=eta)
    assert np.allclose(y, np.ravel(np.column_stack(op.apply_rows(x))), rtol=1e-12, atol=0)
    assert np.allclose(b, C.rhs(geo, mol.atom_xyz, mol.charge, mol.eps_s), rtol=1e-13, atol=0)
    e_ref, phi_ref = C.reaction_energy(geo, mol.atom_xyz, mol.charge, ebar, x[:n], x[n:])
    assert np.isclose(0.5 * esum * C.UNIT_SCALE, e_ref, rtol=1e-12, atol=0)
    assert np.allclose(phi, phi_ref, rtol=1e-12, atol=0)
