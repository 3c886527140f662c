"""GPU tests of the device memory supplier of afmpb_create (C ABI): with
PyTorch's caching allocator bound, every device buffer of the context comes
through the callback, results are bitwise those of a context that allocates
for itself, and everything is returned on destroy."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_every_device_buffer_comes_from_the_allocator():
    import torch
    import paper_1710_06316_amd as A
    torch.cuda.set_device(0)
    mol = W.globular()
    params = dict(order_p=10, leaf_cap=192, precision=A.AFMPB_FP32_REFINED, rhs_fmm=2)
    x = np.random.default_rng(5).normal(size=2 * mol.n_nodes)
    # reference: the library's own allocations (also loads every code object)
    s = A.Solver(0)
    s.load(mol, **params)
    y_ref = s.matvec(x)
    E_ref = s.solve()[2]
    s.close()
    # one more context on the allocator first: the runtime's private memory
    # for register spills is set aside per hardware queue the first time a
    # spilling kernel runs there (not a buffer of any context), and each
    # context's streams may land on queues not used before (at most four
    # per process here)
    warm = A.TorchAllocator(0)
    s = A.Solver(0, allocator=warm)
    s.load(mol, **params)
    s.matvec(x)
    s.solve()
    s.close()
    assert warm.live_bytes == 0
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    res0 = torch.cuda.memory_reserved()
    al = A.TorchAllocator(0)
    s = A.Solver(0, allocator=al)
    s.load(mol, **params)
    y = s.matvec(x)
    E = s.solve()[2]
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    res1 = torch.cuda.memory_reserved()
    used, pooled = free0 - free1, res1 - res0
    _say(f"callback buffers {len(al.live)} ({al.live_bytes / 2**20:.1f} MiB live, "
         f"{al.calls} calls); device memory taken {used / 2**20:.1f} MiB, "
         f"PyTorch pool grew {pooled / 2**20:.1f} MiB")
    assert al.calls > 50 and al.live_bytes > (100 << 20)
    assert torch.cuda.memory_allocated() >= al.live_bytes
    # what the process took beyond PyTorch's pool is runtime state only
    assert used - pooled < (64 << 20)
    assert np.array_equal(y, y_ref) and E == E_ref
    s.close()
    assert al.live_bytes == 0 and not al.live


def test_allocator_failure_is_reported():
    """An allocator that refuses: set_molecule fails with AFMPB_E_OOM and the
    context stays usable."""
    import paper_1710_06316_amd as A

    class Refusing(A.TorchAllocator):
        def _do_alloc(self, nbytes, stream, user):
            self.calls += 1
            return None

    al = Refusing(0)
    s = A.Solver(0, allocator=al)
    with pytest.raises(A.AfmpbError) as e:
        s.load(W.born_ion(2))
    assert e.value.status == A.AFMPB_E_OOM and al.calls >= 1
    s.close()
