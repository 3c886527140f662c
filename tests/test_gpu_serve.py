"""GPU tests of the solve server (continuous batching) through the C ABI.

Every served solve runs the same algorithm, kernels and order as afmpb_solve
on its own, so each result must be the same whether the request ran alone,
in a mix with others, or through afmpb_solve directly (compared here to
1e-12 relative; the stated tolerance is 1e-4 on the energy).  Small requests
are also checked against the FP64 CPU oracle (1e-4 relative energy)."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _server(**kw):
    import paper_1710_06316_amd as A
    _say(f"server {kw}")
    return A.Server(**kw)


def _solo(mol, **params):
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    s.load(mol, **params)
    f, h, E, info, _ = s.solve()
    s.close()
    return f, h, E, info


def _mix(levels):
    return [W.star_request(100 + i, level=L) for i, L in enumerate(levels)]


@pytest.mark.parametrize("precision", [0, 1])
def test_server_matches_direct_solve(precision):
    mols = _mix([3, 4, 3])
    srv = _server(max_active=8, precision=precision, order_p=8, leaf_cap=64)
    tickets = [srv.submit(m) for m in mols]
    for m, t in zip(mols, tickets):
        st, res, f, h = srv.poll(t, wait=True)
        assert res.status == 0, res.message
        f0, h0, E0, info0 = _solo(m, precision=precision, order_p=8, leaf_cap=64)
        _say(f"{m.name} n={m.n_nodes} E_server={res.energy:.10f} E_direct={E0:.10f} "
             f"iters {res.info.iterations}/{info0.iterations}")
        assert res.info.iterations == info0.iterations
        assert abs(res.energy - E0) <= 1e-12 * abs(E0)
        assert np.allclose(f, f0, rtol=1e-12, atol=0) and np.allclose(h, h0, rtol=1e-12, atol=0)
    srv.close()


def test_alone_equals_in_mix_and_oracle():
    mols = _mix([3, 5, 4, 3, 6, 4, 3, 5])
    # alone: one request in flight at a time
    srv = _server(max_active=1, order_p=8, leaf_cap=64)
    alone = {}
    for m in mols:
        t = srv.submit(m)
        _, res, f, h = srv.poll(t, wait=True)
        assert res.status == 0, res.message
        alone[m.name] = (res.energy, f, h)
    srv.close()
    # the same requests submitted together, several in flight
    srv = _server(max_active=6, order_p=8, leaf_cap=64)
    t0 = time.perf_counter()
    tickets = [srv.submit(m) for m in mols]
    peak_active = 0
    while srv.stats()["completed"] + srv.stats()["failed"] < len(mols):
        peak_active = max(peak_active, srv.stats()["active"])
        time.sleep(0.002)
    dt = time.perf_counter() - t0
    for m, t in zip(mols, tickets):
        _, res, f, h = srv.poll(t, wait=True)
        assert res.status == 0, res.message
        Ea, fa, ha = alone[m.name]
        assert abs(res.energy - Ea) <= 1e-12 * abs(Ea)
        assert np.array_equal(f, fa) and np.array_equal(h, ha)
    _say(f"mix of {len(mols)} in {dt:.3f} s, peak active {peak_active}, stats {srv.stats()}")
    assert peak_active >= 2
    srv.close()
    # the small ones against the oracle
    for m in mols:
        if m.n_nodes <= 642:
            ref = O.solve(m)
            Ea = alone[m.name][0]
            _say(f"{m.name} oracle {ref.energy:.6f} server {Ea:.6f}")
            assert abs(Ea - ref.energy) <= 1e-4 * abs(ref.energy)


def test_budget_admission_and_errors():
    import paper_1710_06316_amd as A
    mols = _mix([3, 3, 4])
    # a budget below one request: they run one after another, all complete
    srv = _server(hbm_budget_bytes=1, max_active=8, order_p=8)
    tickets = [srv.submit(m) for m in mols]
    seen = 0
    while srv.stats()["completed"] + srv.stats()["failed"] < len(mols):
        seen = max(seen, srv.stats()["active"])
        time.sleep(0.001)
    assert seen <= 1
    for t in tickets:
        _, res, _, _ = srv.poll(t, wait=True)
        assert res.status == 0, res.message
        assert res.device_bytes > 0
    # a bad mesh fails alone, with its own status
    bad = _mix([3])[0]
    tb = A.afmpb_server_submit(srv.srv, bad.xyz, bad.tri[:, [0, 2, 1]], bad.atom_xyz, bad.charge)
    srv.n_of[tb] = bad.n_nodes
    good = srv.submit(_mix([4])[0])
    _, rb, _, _ = srv.poll(tb, wait=True)
    _, rg, _, _ = srv.poll(good, wait=True)
    assert rb.status == A.AFMPB_E_MESH and rg.status == 0
    assert srv.stats()["device_bytes"] == 0
    srv.close()


def test_cancel_queued():
    import paper_1710_06316_amd as A
    mols = _mix([5, 5, 3])
    srv = _server(max_active=1, order_p=8)
    ts = [srv.submit(m) for m in mols]
    srv.cancel(ts[2])
    _, r2, _, _ = srv.poll(ts[2], wait=True)
    assert r2.status == A.AFMPB_E_CANCELLED
    for t in ts[:2]:
        _, r, _, _ = srv.poll(t, wait=True)
        assert r.status == 0, r.message
    srv.close()


def _busy_polling(setup_threads):
    mols = [W.star_request(200 + i, level=3) for i in range(24)]
    srv = _server(max_active=16, setup_threads=setup_threads, order_p=6)
    tickets = [srv.submit(m) for m in mols]
    pending = dict(zip(tickets, mols))
    energies = {}
    t0 = time.perf_counter()
    while pending and time.perf_counter() - t0 < 120:
        for t in list(pending):
            st, res, f, h = srv.poll(t)
            if st == 0:
                assert res.status == 0, res.message
                assert np.all(np.isfinite(f)) and np.all(np.isfinite(h))
                energies[t] = res.energy
                del pending[t]
    assert not pending
    _say(f"{len(mols)} small requests in {time.perf_counter() - t0:.3f} s, stats {srv.stats()}")
    srv.close()
    # each equals the same request served alone
    srv = _server(max_active=1, setup_threads=1, order_p=6)
    for t, m in zip(tickets, mols):
        _, r, _, _ = srv.poll(srv.submit(m), wait=True)
        assert abs(r.energy - energies[t]) <= 1e-12 * abs(r.energy)
    srv.close()


def test_many_small_requests_busy_polling():
    """Many small requests polled without waiting while others finish
    (regression: a finished request must be handed over only after the
    server has stopped writing to it)."""
    _busy_polling(1)


@pytest.mark.skip(reason="parallel setup (setup_threads > 1) is switched off: the serving "
                         "benchmark crashed on the host with 8 setup threads and the cause "
                         "is not found yet")
def test_many_small_requests_parallel_setup():
    _busy_polling(8)


def test_parallel_setup_rejected():
    import paper_1710_06316_amd as A
    with pytest.raises(A.AfmpbError) as e:
        A.Server(setup_threads=2)
    assert e.value.status == A.AFMPB_E_INVALID


def test_tuned_stream_all_finite():
    """The benchmark's request stream (48 star requests, tuned leaf/order per
    size) served twice at saturation: every request converges with a finite
    energy (regression: M2M/L2L operator fragments past the operator's last
    k-step, read from the next matrix or from unwritten levels, turned some
    requests' far field into NaN although their operand rows were zero)."""
    import paper_1710_06316_amd as A
    from paper_1710_06316_amd import autotune
    table = autotune.load_table()
    mols = [W.star_request(i) for i in range(48)]
    for rep in range(2):
        srv = _server(hbm_budget_bytes=64 << 30, max_active=32, tuning=table,
                      precision=A.AFMPB_FP32_REFINED, order_p=0, leaf_cap=0)
        tickets = [srv.submit(m) for m in mols]
        res = [srv.poll(t, wait=True)[1] for t in tickets]
        srv.close()
        bad = [(i, r.status, r.message) for i, r in enumerate(res) if r.status != 0]
        _say(f"tuned stream pass {rep}: failures {bad}")
        assert not bad
        assert all(np.isfinite(r.energy) for r in res)


def test_server_orders_after_caller_stream():
    """A server created with a caller stream: requests submitted after work
    queued on it give the results of direct solves (their work starts after
    the caller's)."""
    import torch
    import paper_1710_06316_amd as A
    torch.cuda.set_device(0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(8):
            a = a @ a.T / 4096.0        # queued work on the caller's stream
    mols = _mix([3, 4])
    srv = _server(max_active=4, order_p=8, leaf_cap=64, stream=st.cuda_stream)
    tickets = [srv.submit(m) for m in mols]
    for m, t in zip(mols, tickets):
        _, res, f, h = srv.poll(t, wait=True)
        assert res.status == 0, res.message
        f0, h0, E0, info0 = _solo(m, order_p=8, leaf_cap=64)
        assert abs(res.energy - E0) <= 1e-12 * abs(E0)
    srv.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", [1, 0])
def test_served_energies_match_oracle_references(precision):
    """Requests of the benchmark's stream (up to 10,242 nodes) served with
    the tuning table's leaf capacity and order: every energy within 1e-4 of
    the oracle's solve of the same request (tests/golden)."""
    import json
    import os
    import paper_1710_06316_amd as A
    from paper_1710_06316_amd import autotune
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_star_stream.json")
    with open(path) as fh:
        golden = {r["index"]: r["energy_kcal_mol"] for r in json.load(fh)["requests"]}
    idx = sorted(golden)[:24]
    assert len(idx) >= 8
    mols = [W.star_request(i) for i in idx]
    srv = _server(hbm_budget_bytes=32 << 30, max_active=16, tuning=autotune.load_table(),
                  precision=precision, order_p=0, leaf_cap=0)
    tickets = [srv.submit(m) for m in mols]
    res = [srv.poll(t, wait=True)[1] for t in tickets]
    srv.close()
    errs = {}
    for i, m, r in zip(idx, mols, res):
        assert r.status == 0, r.message
        errs[i] = abs(r.energy - golden[i]) / abs(golden[i])
    _say(f"served vs oracle (precision {precision}): max {max(errs.values()):.2e} over "
         f"{len(errs)} requests of {sorted(set(m.n_nodes for m in mols))} nodes")
    assert max(errs.values()) <= 1e-4
