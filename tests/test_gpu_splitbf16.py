"""Split-BF16 precision mode: z-direction DFTs on the matrix cores (hi + lo BF16, three products,
FP32 accumulation), everything else as in the FP32 mode.

Error model: each operand is carried to about 16 significant bits (BF16 hi + lo) and the dropped
lo*lo product is ~2^-16 of the result, so one DFT stage is accurate to a few 1e-6 relative; an
output element passes through a few such stages plus the FP32 work (measured: 1e-6 to 5e-6 of the
largest element, energies within 1e-7).  Stated per-result bounds (relative to the largest
element): 2e-5 for operator elements, 1e-6 for the energy.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem
from oracle.heg import heg_energy, heg_terms

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")

ELEM_TOL = 2e-5
ENERGY_TOL = 1e-6


def _say(msg):
    print(msg, flush=True)


def _rel(a, b):
    scale = max(np.abs(x).max() for x in b)
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / scale


@pytest.mark.parametrize("grid,kmesh,nb", [(8, (2, 1, 1), 2), (16, (1, 2, 1), 2), (48, (2, 1, 1), 2)])
def test_small_cases_vs_oracle(grid, kmesh, nb):
    w = T.tiny_fcc(kmesh=kmesh, grid=grid, ecut=2.0 if grid == 8 else 3.0, nb=nb, a=6.0 if grid == 8 else 7.0,
                   occ=[1.0, 0.7][:nb])
    pr = Problem(w)
    ref = [c.numpy() for c in pr.to_coeff(sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL_TERMS))]
    E = float(pr.energy())
    op = tc.from_workload(w, precision=tc.TC_PREC_FP32_SPLITBF16)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    err, eerr = _rel(hc, ref), abs(Eg - E) / abs(E)
    _say(f"[gpu] split-bf16 {grid}^3 {kmesh}: element error {err:.3e}, energy error {eerr:.3e}")
    assert err < ELEM_TOL
    assert eerr < ENERGY_TOL


def test_electron_gas_54_vs_closed_forms():
    w = T.workload("heg54_twist2_g32")
    eps, p, f = heg_terms(w)
    lam = sum(MULT.get(t, 1) * e for t, e in eps.items())
    op = tc.from_workload(w, precision=tc.TC_PREC_FP32_SPLITBF16)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    nb = w.right[0].shape[0]
    exp = [lam[ik * nb:(ik + 1) * nb, None] * w.right[ik] for ik in range(w.nk)]
    err = _rel(hc, exp)
    Eh, _ = heg_energy(w)
    _say(f"[gpu] split-bf16 heg54 32^3: element error {err:.3e}, energy error {abs(Eg - Eh) / abs(Eh):.3e}")
    assert err < ELEM_TOL
    assert abs(Eg - Eh) < ENERGY_TOL * abs(Eh)


def test_bench_workload_vs_fp64():
    w = T.workload("fcc_si_k444_g24")
    out = {}
    for name, prec in (("fp64", tc.TC_PREC_FP64), ("split", tc.TC_PREC_FP32_SPLITBF16)):
        op = tc.from_workload(w, precision=prec)
        out[name] = (op.apply(), op.energy()[0])
        op.close()
    err = _rel(out["split"][0], out["fp64"][0])
    eerr = abs(out["split"][1] - out["fp64"][1]) / abs(out["fp64"][1])
    _say(f"[gpu] split-bf16 fcc_si_k444_g24: element error {err:.3e}, energy error {eerr:.3e}")
    assert err < ELEM_TOL
    assert eerr < ENERGY_TOL


def test_supercell_48_vs_fp32_repeatable():
    """48^3 (six 16-row tiles per DFT): every element finite, close to FP32, identical on a second run."""
    w = T.workload("fcc_si_x2_k222_g48")
    out = {}
    for name, prec in (("fp32", tc.TC_PREC_FP32), ("split", tc.TC_PREC_FP32_SPLITBF16), ("split2", tc.TC_PREC_FP32_SPLITBF16)):
        op = tc.from_workload(w, precision=prec)
        out[name] = (op.apply(), op.energy()[0])
        op.close()
    assert all(np.isfinite(x).all() for x in out["split"][0])
    err = _rel(out["split"][0], out["fp32"][0])
    _say(f"[gpu] split-bf16 supercell 48^3: element difference to FP32 {err:.3e}")
    assert err < ELEM_TOL
    assert all(np.array_equal(a, b) for a, b in zip(out["split"][0], out["split2"][0]))
    assert abs(out["split"][1] - out["fp32"][1]) < ENERGY_TOL * abs(out["fp32"][1])


def test_grid_not_divisible_by_8_is_rejected():
    w = T.tiny_fcc(kmesh=(2, 2, 2), grid=12, ecut=2.0, nb=2, a=6.0)
    op = tc.from_workload(w, precision=tc.TC_PREC_FP32_SPLITBF16)
    with pytest.raises(tc.TCError, match="status -5"):
        op.apply()
    op.close()
