"""tc_apply_all_dev_noalloc: the application with every device buffer carved from the library's fixed
scratch, through the C ABI.  Its output and energy must equal those of tc_apply_all_dev on the same
context (FP64 1e-10, FP32 2e-6 relative; the batching may differ), on two calls in a row where the
second has a smaller input (the scratch keeps the first call's contents)."""
import numpy as np
import pytest

import tcinputs as T

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")


def _say(msg):
    print(msg, flush=True)


def _pair_of_runs(w, prec):
    import torch

    op = tc.from_workload(w, precision=prec)
    shape = (w.nk, w.right[0].shape[0], op.npw_max)
    ref = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    got = torch.full(shape, float("nan"), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    op.apply_dev(ref.data_ptr())
    op.sync()
    E_ref = op.energy()[0]
    op.apply_dev_noalloc(got.data_ptr())
    E = op.energy()[0]
    op.apply_dev(ref.data_ptr())   # the ordinary path still works after it
    op.sync()
    E_ref2 = op.energy()[0]
    op.close()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy(), E_ref, E, E_ref2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_noalloc_equals_apply_all_dev_twice_second_smaller(prec, tol):
    P = tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32
    cases = [T.tiny_fcc(kmesh=(2, 2, 2), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.9, 0.4]),
             T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])]
    for w in cases:
        _say(f"[gpu] no-allocation application {w.name} {prec} vs tc_apply_all_dev")
        ref, got, E_ref, E, E_ref2 = _pair_of_runs(w, P)
        assert np.isfinite(got).all()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        _say(f"    max rel difference {err:.2e}; energies {E!r} vs {E_ref!r}")
        assert err < tol
        assert abs(E - E_ref) < tol * abs(E_ref)
        assert E_ref2 == E_ref


def test_noalloc_errors():
    import torch

    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0)
    _say("[gpu] no-allocation application: unprepared context, NULL output, scratch too small")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    out = torch.zeros((w.nk, 2, op.npw_max), dtype=torch.complex128, device="cuda")
    with pytest.raises(tc.TCError, match="status -2"):
        op.apply_dev_noalloc(out.data_ptr())
    op.apply_dev(out.data_ptr())
    with pytest.raises(tc.TCError, match="status -1"):
        op._check(op._L.tc_apply_all_dev_noalloc(op._h, None), "tc_apply_all_dev_noalloc")
    op.close()
    big = T.workload("fcc_si_k444_g24")
    op = tc.from_workload(big, precision=tc.TC_PREC_FP64)
    out = torch.zeros((big.nk, big.nband, op.npw_max), dtype=torch.complex128, device="cuda")
    op.apply_dev(out.data_ptr())
    with pytest.raises(tc.TCError, match="status -7"):
        op.apply_dev_noalloc(out.data_ptr())
    op.apply_dev(out.data_ptr())   # still usable
    op.close()
