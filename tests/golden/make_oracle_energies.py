"""Writes oracle reference solves used by the GPU parity tests and the serving
benchmark.  Calls only ``oracle`` (the FP64 CPU oracle) and ``workloads`` (the
seeded input generators); nothing here touches the GPU library.

    python tests/golden/make_oracle_energies.py globular
    python tests/golden/make_oracle_energies.py stars [--count 512] [--max-nodes 10242]

Each reference is the oracle's restarted GMRES solve of Eq. (5) (direct
O(N^2) operator, near set eta = 4) to a relative residual of 1e-8, two orders
below the solver's default 1e-6, so that the GMRES error of the reference is
negligible against the 1e-4 energy tolerance.  Output: JSON next to this file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O          # noqa: E402
import workloads as W       # noqa: E402

REL_TOL = 1e-8


def _solve(mol):
    t0 = time.perf_counter()
    sol = O.solve(mol, rel_tol=REL_TOL, restart=80, max_restarts=5)
    return {
        "name": mol.name,
        "n_nodes": mol.n_nodes,
        "n_atoms": int(len(mol.charge)),
        "energy_kcal_mol": sol.energy,
        "iterations": sol.info.iterations,
        "converged": bool(sol.info.converged),
        "true_rel_residual": sol.info.true_rel_residual,
        "seconds": time.perf_counter() - t0,
    }


def globular(out):
    mol = W.globular()
    rec = _solve(mol)
    rec.update({"workload": "globular_5000 (seed 2, 5,000 atoms, 1.25 A grid)",
                "eps_p": mol.eps_p, "eps_s": mol.eps_s, "kappa": mol.kappa,
                "eta": 4.0, "rel_tol": REL_TOL})
    print(json.dumps(rec), flush=True)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)


def stars(out, count, max_nodes):
    done = {}
    if os.path.exists(out):
        with open(out) as fh:
            done = {r["index"]: r for r in json.load(fh)["requests"]}
    recs = dict(done)
    for i in range(count):
        if i in recs:
            continue
        mol = W.star_request(i)
        if mol.n_nodes > max_nodes:
            continue
        rec = _solve(mol)
        rec["index"] = i
        recs[i] = rec
        print(json.dumps(rec), flush=True)
        with open(out + ".tmp", "w") as fh:
            json.dump({"stream": "star_request(i), i < %d, seed 4000 + i" % count,
                       "max_nodes": max_nodes, "eta": 4.0, "rel_tol": REL_TOL,
                       "requests": [recs[k] for k in sorted(recs)]}, fh, indent=1)
        os.replace(out + ".tmp", out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["globular", "stars"])
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--max-nodes", type=int, default=10242)
    a = ap.parse_args()
    if a.what == "globular":
        globular(os.path.join(HERE, "oracle_globular_5000.json"))
    else:
        stars(os.path.join(HERE, "oracle_star_stream.json"), a.count, a.max_nodes)


if __name__ == "__main__":
    main()
