"""GPU test of the allocation-free energy entry point through the C ABI.

afmpb_energy_dev_noalloc reads x from device memory in the caller's order and
writes the polar energy to a device scalar, with a fixed static scratch in
place of the per-atom buffers of afmpb_energy.  Two calls in a row on one
device, the second on a smaller input (fewer atoms, fewer nodes, so fewer
partial sums than the first left in the scratch), each against afmpb_energy
and against the FP64 oracle's energy sum (1e-12 relative)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _run(s, mol, seed):
    import torch
    n = mol.n_nodes
    x = np.random.default_rng(seed).normal(size=2 * n)
    e_host = s.energy(x)
    xd = torch.from_numpy(x).to("cuda:0")
    ed = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    s.energy_dev_noalloc(xd.data_ptr(), ed.data_ptr())
    torch.cuda.synchronize()
    e_dev = float(ed.cpu()[0])
    geo = O.geometry(mol.xyz, mol.tri)
    e_ref, _ = O.reaction_energy(geo, mol.atom_xyz, mol.charge, mol.eps_s / mol.eps_p,
                                 x[:n], x[n:])
    _say(f"{mol.name} n={n} atoms={len(mol.charge)} noalloc={e_dev!r} "
         f"energy={e_host!r} oracle={e_ref!r}")
    assert e_dev == pytest.approx(e_host, rel=1e-12)
    assert e_dev == pytest.approx(e_ref, rel=1e-12)


def test_energy_noalloc_matches_energy_twice_shrinking():
    import torch
    import paper_1710_06316_amd as A
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    big = W.globular()                         # 5,000 atoms: 20 partial sums
    small = W.star_request(12, level=3)        # fewer atoms, one or two partials
    assert len(small.charge) < len(big.charge) and small.n_nodes < big.n_nodes
    s = A.Solver(0, stream)
    _say(f"load {big.name}")
    s.load(big)
    _run(s, big, 1)
    _say(f"load {small.name}")
    s.load(small)
    _run(s, small, 2)
    s.close()


def test_energy_noalloc_errors():
    import torch
    import paper_1710_06316_amd as A
    s = A.Solver(0)
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(A.AfmpbError) as e:
        s.energy_dev_noalloc(out.data_ptr(), out.data_ptr())
    assert e.value.status == A.AFMPB_E_STATE
    mol = W.born_ion(2)
    s.load(mol)
    with pytest.raises(A.AfmpbError) as e:
        s.energy_dev_noalloc(0, out.data_ptr())
    assert e.value.status == A.AFMPB_E_INVALID
    s.close()
