"""Device memory from the caller: the library's buffers taken from PyTorch's caching allocator
(tc_set_allocator) and sized from a caller's budget (tc_set_memory_budget), through the C ABI.

The allocator changes where the memory comes from, never the results: outputs equal those of a context
on hipMalloc bit for bit.  A budget changes the batching (and whether the resident pair store is kept),
so outputs agree to rounding."""
import numpy as np
import pytest

import tcinputs as T

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")


def _say(msg):
    print(msg, flush=True)


def _case():
    return T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.8, 0.5])


def test_torch_allocator_owns_the_library_memory():
    import torch

    w = _case()
    _say("[gpu] library device memory from torch's caching allocator")
    ref = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    hc_ref = ref.apply()
    E_ref = ref.energy()[0]
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, torch_alloc=True)
    loaded = torch.cuda.memory_allocated()
    hc = op.apply()
    E = op.energy()[0]
    held = torch.cuda.memory_allocated()
    _say(f"    torch.cuda.memory_allocated: {base} before, {loaded} after load, {held} after the application")
    assert loaded > base                 # coefficients and plane-wave data
    assert held > loaded + (1 << 20)     # fields, tables and pair buffers
    for a, b in zip(hc, hc_ref):
        np.testing.assert_array_equal(a, b)
    assert E == E_ref
    op.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


@pytest.mark.parametrize("budget_mib", [1, 8, 64])
def test_memory_budget_sizes_store_and_batches(budget_mib):
    """1 MiB: one target per batch, no store; 8 MiB: a few targets per batch; 64 MiB: the store and
    large batches.  The operator and energy agree with the default sizing."""
    import torch

    w = _case()
    _say(f"[gpu] memory budget {budget_mib} MiB (torch allocator)")
    ref = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    hc_ref = ref.apply()
    E_ref = ref.energy()[0]
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, torch_alloc=True, mem_budget=budget_mib << 20)
    hc = op.apply()
    E = op.energy()[0]
    held = torch.cuda.memory_allocated() - base
    op.close()
    scale = max(np.abs(x).max() for x in hc_ref)
    err = max(np.abs(a - b).max() for a, b in zip(hc, hc_ref)) / scale
    _say(f"    held {held / 2**20:.1f} MiB; max rel difference {err:.2e}")
    assert err < 1e-12
    assert abs(E - E_ref) < 1e-12 * abs(E_ref)


def test_allocator_argument_errors():
    _say("[gpu] tc_set_allocator with one function")
    op = tc.TCOperator(0)
    with pytest.raises(tc.TCError, match="status -1"):
        op._check(op._L.tc_set_allocator(op._h, tc.ALLOC_FN(lambda n, u: None), tc.FREE_FN(), None),
                  "tc_set_allocator")
    op.close()
