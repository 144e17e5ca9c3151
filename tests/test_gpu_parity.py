"""Parity of the HIP path with the FP64 oracle, element by element, through the C ABI (one case on a
shifted Monkhorst-Pack mesh); the cusp-tied Jastrow entry point against explicit C."""
import numpy as np
import pytest

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem
from oracle.heg import heg_energy

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")

FP64_TOL = 1e-10      # relative, FP64 GPU vs FP64 oracle
FP32_TOL = 2e-6       # relative per result (max norm), FP32 GPU vs FP64 oracle


def _say(msg):
    print(msg, flush=True)


def oracle(w, terms=ALL_TERMS, div=True):
    pr = Problem(w, div_correction=div)
    per = {t: [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))] for t in terms}
    tot = [sum(per[t][k] for t in terms) for k in range(w.nk)]
    return per, tot, float(pr.energy(terms=terms))


def oracle_energies(w):
    """Energy with each term alone (kinetic included) and the orbital energies <chi|T + h|phi>."""
    pr = Problem(w)
    g = {t: pr.term(t, 0) for t in ALL_TERMS}
    kin = pr.kinetic().numpy()
    f = pr.orb[0]["f"].numpy()
    T = 2 * np.sum(f * kin).real / pr.nk
    E1 = {}
    for t in ALL_TERMS:
        fac = 0.5 if t.startswith("2") else MULT.get(t, 1) / 3.0
        E1[t] = T + 2 * fac * float(np.sum(f * pr.braket(0, g[t]).numpy()).real) / pr.nk
    eps = kin + pr.braket(0, sum(MULT.get(t, 1) * g[t] for t in ALL_TERMS)).numpy()
    return E1, eps


def relerr(a, b):
    scale = max(np.abs(x).max() for x in b)
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / scale


CASES = {
    "fcc_k211_g8_partial": lambda: T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]),
    "fcc_k222_g12_empty_band": lambda: T.tiny_fcc(kmesh=(2, 2, 2), grid=12, ecut=2.0, nb=3, a=6.0,
                                                   occ=[1.0, 0.9, 0.0]),
    "fcc_k121_g16_nb1": lambda: T.tiny_fcc(kmesh=(1, 2, 1), grid=16, ecut=3.0, nb=1, a=7.0),
    # Monkhorst-Pack shifted mesh: k = (i + s) / n
    "fcc_k221_g12_shifted": lambda: T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.8],
                                               kshift=(0.5, 0.25, 0.0)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    w = CASES[request.param]()
    return request.param, w, oracle(w)


def test_every_term_fp64(case):
    name, w, (per, tot, E) = case
    for t in ALL_TERMS:
        _say(f"[gpu] {name} fp64 term {t}")
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=tc.TERM_BITS[t] | tc.TERM_BITS["corr"])
        hc = op.apply()
        op.close()
        scale = max(max(np.abs(x).max() for x in tot), 1e-300)
        err = max(np.abs(h - r).max() for h, r in zip(hc, per[t])) / scale
        assert err < FP64_TOL, (t, err)


@pytest.mark.parametrize("batch,store", [(0, True), (1, True), (3, True), (0, False), (3, False)])
def test_total_and_energy_fp64_with_batching(case, batch, store):
    name, w, (per, tot, E) = case
    _say(f"[gpu] {name} fp64 all terms batch={batch} pair_store={store}")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, batch=batch, pair_store=store)
    hc = op.apply()
    Eg, parts = op.energy()
    op.close()
    assert relerr(hc, tot) < FP64_TOL
    assert abs(Eg - E) < FP64_TOL * abs(E)


def test_total_and_energy_fp32(case):
    name, w, (per, tot, E) = case
    _say(f"[gpu] {name} fp32 all terms")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP32, batch=2)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    assert relerr(hc, tot) < FP32_TOL
    assert abs(Eg - E) < 1e-6 * abs(E)


def test_electron_gas_closed_form_fp64():
    w = T.workload("heg14_g16")
    _say("[gpu] heg14 gamma 16^3 fp64 vs closed forms")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    Eg, parts = op.energy()
    op.close()
    Eh, _ = heg_energy(w)
    assert abs(Eg - Eh) < 1e-10 * abs(Eh)


def test_hartree_fock_limit_fp64():
    w = T.workload("heg14_g16").replace(A=(0.0, 0.0))
    _say("[gpu] heg14 A=0 (Hartree-Fock) fp64")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    Eg, parts = op.energy()
    op.close()
    # exchange = total - kinetic; closed form with the GB correction
    assert parts["two_body"] == pytest.approx(-1.8003924344714473, rel=1e-10)
    assert parts["three_body"] == pytest.approx(0.0, abs=1e-14)


def test_no_correction_option_fp64():
    w = CASES["fcc_k211_g8_partial"]()
    _, tot, E = oracle(w, div=False)
    _say("[gpu] fcc_k211 fp64 without divergence corrections")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, div_correction=False)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    assert relerr(hc, tot) < FP64_TOL
    assert abs(Eg - E) < FP64_TOL * abs(E)


def test_error_paths():
    _say("[gpu] error paths")
    op = tc.TCOperator(0)
    with pytest.raises(tc.TCError, match="status -5"):
        op.set_grid(20, 20, 20)
    with pytest.raises(tc.TCError, match="status -2"):
        op.apply()
    op.set_cell(T.fcc_lattice(6.0))
    op.set_kmesh(1, 1, 1)
    op.set_grid(8, 8, 8)
    with pytest.raises(tc.TCError, match="status -3"):
        op.set_basis(0, np.array([[4, 0, 0]]))
    with pytest.raises(tc.TCError, match="status -1"):
        op.set_jastrow([1.0, 1.0], [0.0, 1.0])
    op.close()


def test_energy_of_every_single_term_fp64(case):
    """Every term alone (with its correction), including 2bh2 and 2bx2 without their partners."""
    name, w, _ = case
    E1, _ = oracle_energies(w)
    for t in ALL_TERMS:
        _say(f"[gpu] {name} fp64 energy of term {t} alone")
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=tc.TERM_BITS[t] | tc.TERM_BITS["corr"])
        Eg, _ = op.energy()
        op.close()
        assert abs(Eg - E1[t]) < FP64_TOL * abs(E1[t]), (t, Eg, E1[t])


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_orbital_energies(case, prec, tol):
    name, w, _ = case
    _, eps = oracle_energies(w)
    _say(f"[gpu] {name} {prec} orbital energies")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    got = op.orbital_energies().reshape(-1)
    g2 = op.orbital_energies().reshape(-1)
    op.close()
    err = np.abs(got - eps).max() / np.abs(eps).max()
    _say(f"    max |eps - eps_oracle| / max |eps| = {err:.3e}")
    assert err < tol
    np.testing.assert_array_equal(got, g2)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_shared_last_z_stage_equals_separate_stages(case, prec, tol):
    """3b6 selected with pass-B terms runs one shared z stage and one partner sum; selected apart, each
    keeps its own.  The operator is linear in the selected terms, so the two must agree."""
    name, w, _ = case
    _say(f"[gpu] {name} {prec} shared 3b6 / pass-B z stage vs separate")
    P = tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32
    b3b6 = tc.TERM_BITS["3b6"]
    bB = tc.TERM_BITS["2bx2"] | tc.TERM_BITS["3b3"] | tc.TERM_BITS["3b4"] | tc.TERM_BITS["3b5"]
    out = {}
    for key, mask in (("both", b3b6 | bB), ("3b6", b3b6), ("B", bB)):
        op = tc.from_workload(w, precision=P, terms=mask, div_correction=False)
        out[key] = op.apply()
        op.close()
    sep = [a + b for a, b in zip(out["3b6"], out["B"])]
    assert relerr(out["both"], sep) < tol


def test_pair_store_switch_on_a_live_context(case):
    """The resident store can be switched off (released at once) and on again between applications."""
    name, w, (per, tot, E) = case
    _say(f"[gpu] {name} fp64 pair store on -> off -> on")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    runs = [op.apply()]
    op.set_pair_store(False)
    runs.append(op.apply())
    op.set_pair_store(True)
    runs.append(op.apply())
    op.close()
    for hc in runs:
        assert relerr(hc, tot) < FP64_TOL
    assert relerr(runs[1], runs[0]) < 1e-13 and relerr(runs[2], runs[0]) < 1e-15


@pytest.mark.parametrize("reading", ["printed", "limit"])
def test_reading_of_the_mesh_corrections_fp64(case, reading):
    """Both readings of the mesh corrections (TC_DIV_PRINTED: one u~_short(0)/N_k in the G = G' = 0 corrections
    of 3a2 and 3b6, no 2bx1 correction; TC_DIV_LIMIT: two, and the 2bx1 remainder), term by term and in
    total, against the oracle under the same reading."""
    name, w, _ = case
    pr = Problem(w, reading=reading)
    for t in ("2bx1", "3a2", "3b6", "2ax"):
        _say(f"[gpu] {name} fp64 reading={reading} term {t}")
        ref = [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))]
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=tc.TERM_BITS[t] | tc.TERM_BITS["corr"],
                              reading=reading)
        hc = op.apply()
        op.close()
        assert relerr(hc, ref) < FP64_TOL, (t, relerr(hc, ref))
    _say(f"[gpu] {name} fp64 reading={reading} all terms + energy")
    tot = [c.numpy() for c in pr.to_coeff(sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL_TERMS))]
    E = float(pr.energy())
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, reading=reading)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    assert relerr(hc, tot) < FP64_TOL
    assert abs(Eg - E) < FP64_TOL * abs(E)


def test_readings_differ_and_bad_code_is_rejected():
    w = CASES["fcc_k211_g8_partial"]()
    _say("[gpu] fcc_k211 fp64 printed vs limit energies; invalid div_correction code")
    es = []
    for reading in ("printed", "limit"):
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, reading=reading)
        es.append(op.energy()[0])
        op.close()
    assert abs(es[0] - es[1]) > 1e-6 * abs(es[0])
    op = tc.TCOperator(0)
    with pytest.raises(tc.TCError, match="status -1"):
        op._check(op._L.tc_set_options(op._h, 0, 1.0, 3, tc.TERM_ALL), "tc_set_options")
    op.close()


def test_cusp_tied_jastrow_equals_explicit_c():
    """tc_set_jastrow_cusp(A) gives the operator of tc_set_jastrow(A, C) with C from Eq. cusp."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    A = (0.7, 0.45)
    C = (np.sqrt(2 * A[0]), np.sqrt(A[1]))
    _say("[gpu] cusp-tied Jastrow vs explicit C")
    out = []
    for tied in (False, True):
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, A=A, C=C)
        if tied:
            op.set_jastrow_cusp(A)
        out.append((op.apply(), op.energy()[0]))
        op.close()
    assert out[1][1] == out[0][1]
    for a, b in zip(out[1][0], out[0][0]):
        np.testing.assert_array_equal(a, b)
    op = tc.TCOperator()
    with pytest.raises(tc.TCError, match="status"):
        op.set_jastrow_cusp((0.0, 1.0))
    op.close()
