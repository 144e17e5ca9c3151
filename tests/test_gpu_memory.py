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


def relerr(a, b):
    scale = max(np.abs(x).max() for x in b)
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / scale


def _store_budget(w, q1, elem_bytes, bitc=False):
    """Caller budget of a batch of 8 targets of pair buffers plus q1 full partner columns of 5 fields (one
    spin channel): the triangular store of TC mode fits q1 columns in it and not q1 + 1 (P > q1 (q1 + 1) / 2)."""
    P, NR = w.nk * w.nband, int(np.prod(w.grid))
    per_target = P * ((8 if bitc else 5) + 4) * NR * elem_bytes
    return per_target * min(8, P) + q1 * 5 * P * NR * elem_bytes


@pytest.mark.parametrize("prec,elem", [("fp64", 16), ("fp32", 8)])
def test_partial_pair_store_equals_no_store(prec, elem):
    """A caller budget between an eighth and all of the store: the triangular store keeps the first Q1 = 3
    partner columns (the pairs (t, q) of q <= t, q < 3; the others of min(t, q) < 3 read reflected and
    conjugated); the occupied pass reads them for its rows below Q1 and forms its own pairs for the others,
    and pass A forms the pairs of targets and partners at or above Q1.  Same operator, energy and orbital
    energies as without the store (to rounding), and as the oracle; the occupied pass's own pair densities
    run for some rows only."""
    from oracle.fftroute import ALL_TERMS, MULT, Problem

    w = T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.8])
    P = w.nk * w.nband
    pr = Problem(w)
    ref = [c.numpy() for c in pr.to_coeff(sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL_TERMS))]
    p = tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32
    tol = 1e-10 if prec == "fp64" else 2e-6
    res = {}
    # batches of 2 targets: without the store the occupied pass forms pairs for rows 0-1, 2-3, 4-5, 6-7; with
    # 3 stored columns it reads rows 0-1 and 2 and forms pairs for 3-4, 5-6 and 7
    for name, kw in (("none", dict(pair_store=False)), ("partial", dict(mem_budget=_store_budget(w, 3, elem))),
                     ("full", dict())):
        kw["batch"] = 2
        _say(f"[gpu] partial pair store {prec}: {name}")
        op = tc.from_workload(w, precision=p, **kw)
        op.set_profiling(True)
        op.kernel_stats(reset=True)
        out = op.apply()
        st = op.kernel_stats()
        res[name] = (out, op.energy()[0], op.orbital_energies(), st["k_pair_xy<R,N,true>"]["launches"])
        op.close()
    occ = {k: v[3] for k, v in res.items()}
    _say(f"    occupied-pass pair launches: {occ}")
    assert occ == {"none": 4, "partial": 3, "full": 0}
    for name in ("partial", "full"):
        assert relerr(res[name][0], res["none"][0]) < (1e-12 if prec == "fp64" else 1e-6), name
        assert abs(res[name][1] - res["none"][1]) < (1e-12 if prec == "fp64" else 1e-7) * abs(res["none"][1])
    assert relerr(res["partial"][0], ref) < tol


def _refusing_op(w, cap, refused, budget=0, batch=0, pair_store=True):
    """An FP64 operator of w whose device memory comes from PyTorch's caching allocator through callbacks
    that refuse (return NULL for) every request above cap bytes, recording the refused sizes."""
    import torch

    op = tc.TCOperator(0)
    stream = op.stream()

    def _alloc(nbytes, user):
        if nbytes > cap:
            refused.append(int(nbytes))
            return None
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)

    def _free(ptr, nbytes, user):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (tc.ALLOC_FN(_alloc), tc.FREE_FN(_free))
    op._check(op._L.tc_set_allocator(op._h, cbs[0], cbs[1], None), "tc_set_allocator")
    op._refusing_cbs = cbs
    if budget:
        op.set_memory_budget(budget)
    if batch:
        op.set_batch(batch)
    if not pair_store:
        op.set_pair_store(False)
    op.set_cell(w.lattice)
    op.set_kmesh(*w.kmesh)
    op.set_grid(*w.grid)
    for ik, m in enumerate(w.miller):
        op.set_basis(ik, m)
    op.set_jastrow(w.A, w.C)
    op.set_options(tc.TC_PREC_FP64, w.alpha, True, tc.TERM_ALL)
    for ik in range(w.nk):
        op.load_orbitals(ik, w.right[ik], w.occ[ik])
    return op


def test_store_takes_fewer_columns_when_an_allocation_fails():
    """An allocator that refuses every request above 8 MiB: the whole triangular store (78 pairs, 10.8 MB in
    FP64) is refused, and the store settles on the most partner columns that it grants (6 of 12: 57 pairs,
    7.9 MB); the next application asks for no refused size again.  The operator equals the one without the
    store."""
    w = _case()
    P = w.nk * w.nband
    _say("[gpu] pair store under an allocator that refuses requests above 8 MiB")
    ref = tc.from_workload(w, precision=tc.TC_PREC_FP64, pair_store=False, batch=4)
    ref.set_profiling(True)
    ref.kernel_stats(reset=True)
    hc_ref = ref.apply()
    own_ref = ref.kernel_stats()["k_pair_xy<R,N,true>"]["launches"]
    ref.close()
    cap, refused = 8 << 20, []
    op = _refusing_op(w, cap, refused, budget=64 << 20, batch=4)
    op.set_profiling(True)
    outs = []
    for _ in range(2):
        op.kernel_stats(reset=True)
        outs.append((op.apply(), op.kernel_stats()["k_pair_xy<R,N,true>"]["launches"], len(refused)))
    op.close()
    pair = 5 * int(np.prod(w.grid)) * 16
    _say(f"    refused {[r // pair for r in refused]} pairs; own occupied-pass pair launches "
         f"{[o[1] for o in outs]} (without the store {own_ref})")
    assert refused and all(r > cap for r in refused) and P * (P + 1) // 2 * pair in refused
    assert outs[1][2] == outs[0][2]                         # no refused size asked for again
    assert own_ref == 3 and outs[0][1] == outs[1][1] == 2   # rows 6-9 and 10-11 form their own pairs
    for hc, _, _ in outs:
        assert relerr(hc, hc_ref) < 1e-12


def test_batch_shrinks_when_its_buffers_are_refused():
    """Without a budget the 12 targets of the case make one batch (bufA 16 MB, bufB 20 MB in FP64); under
    an allocator that refuses requests above 12 MB the batch halves to 6 targets, and the operator equals
    the unrestricted one."""
    w = _case()
    _say("[gpu] batch buffers under an allocator that refuses requests above 12 MB")
    ref = tc.from_workload(w, precision=tc.TC_PREC_FP64, pair_store=False)
    hc_ref = ref.apply()
    E_ref = ref.energy()[0]
    ref.close()
    refused = []
    op = _refusing_op(w, 12 << 20, refused, pair_store=False)
    hc = op.apply()
    E = op.energy()[0]
    op.close()
    _say(f"    refused {refused} bytes")
    assert refused
    assert relerr(hc, hc_ref) < 1e-12
    assert abs(E - E_ref) < 1e-12 * abs(E_ref)
