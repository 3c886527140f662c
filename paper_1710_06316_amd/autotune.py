"""Per-size tuning of the solve server: leaf capacity and expansion order.

For every size bucket of the serving stream (icosphere levels 3-6, i.e. up to
642 / 2,562 / 10,242 / 40,962 nodes) this times a few seeded sample requests
with each candidate (leaf capacity, expansion order) -- setup plus a full
solve through the library, the way the server runs them -- and keeps the
fastest candidate whose polar energies stay within `tol` (relative) of an FP64
order-14 solve of the same requests.  The table is written as JSON next to
this file (`serving_tuning.json`) and read by `load_table()`; the server takes
it through `afmpb_server_set_tuning` (entries ascending in max_nodes).

Run on the GPU:  python -m paper_1710_06316_amd.autotune
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "serving_tuning.json")
LEVEL_NODES = {3: 642, 4: 2562, 5: 10242, 6: 40962}


def _solve(A, mol, **params):
    s = A.Solver(0)
    t0 = time.perf_counter()
    s.load(mol, **params)
    _, _, E, info, _ = s.solve(allow_not_converged=True)
    dt = time.perf_counter() - t0
    s.close()
    return E, dt, bool(info.converged)


def tune(levels=(3, 4, 5, 6), samples=2, leafs=(16, 32, 64, 128, 192, 256), orders=(6, 8, 10),
         precision=1, tol=2e-5, seed0=9000, log=print):
    import paper_1710_06316_amd as A
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as W
    table, detail = [], {}
    for L in levels:
        mols = [W.star_request(seed0 + 10 * L + i, level=L) for i in range(samples)]
        refs = [_solve(A, m, order_p=14, leaf_cap=64, precision=A.AFMPB_FP64)[0] for m in mols]
        for m in mols:                  # warm-up (first-use costs out of the timings)
            _solve(A, m, order_p=orders[0], leaf_cap=leafs[0], precision=precision)
        cand = []
        for leaf in leafs:
            for p in orders:
                ts, errs, ok = [], [], True
                for m, e_ref in zip(mols, refs):
                    E, dt, conv = _solve(A, m, order_p=p, leaf_cap=leaf, precision=precision)
                    ts.append(dt)
                    errs.append(abs(E - e_ref) / abs(e_ref))
                    ok &= conv
                rec = {"leaf_cap": leaf, "order_p": p, "ms": 1e3 * sum(ts) / len(ts),
                       "max_rel_energy_err": max(errs), "converged": ok}
                cand.append(rec)
                log(f"level {L} leaf {leaf:3d} p {p:2d}: {rec['ms']:8.2f} ms, "
                    f"err {rec['max_rel_energy_err']:.2e}")
        good = [c for c in cand if c["converged"] and c["max_rel_energy_err"] <= tol]
        best = min(good or cand, key=lambda c: c["ms"])
        table.append([LEVEL_NODES[L], best["leaf_cap"], best["order_p"]])
        detail[str(L)] = {"chosen": best, "candidates": cand}
    out = {"table": table, "tol": tol, "precision": precision, "samples": samples,
           "detail": detail}
    return out


def save(result, path=TABLE):
    with open(path, "w") as f:
        json.dump(result, f, indent=1)


def load_table(path=TABLE):
    """[(max_nodes, leaf_cap, order_p), ...] or None when no table exists."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return [tuple(x) for x in json.load(f)["table"]]


if __name__ == "__main__":
    res = tune()
    save(res)
    print(json.dumps({"table": res["table"]}), flush=True)
