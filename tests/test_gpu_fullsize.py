"""Parity at full workload sizes, in the launch configuration the benchmark times.

The oracle cannot evaluate every output at these sizes in seconds, so each test
checks what it can compute independently:
  * the 54-electron gas on a 2x2x2 twist mesh (216 orbitals, 32^3 grid): every
    term and every output element against the plane-wave closed forms;
  * the fcc bench workload (256 orbitals, 24^3 grid) and its 2x2x2 supercell
    (48^3 grid): sampled target orbitals against the FP64 oracle restricted to
    those targets, for every term whose oracle cost does not grow with the
    number of orbital pairs (all but 3a2, 3a4, 3b2, 3b5);
  * the terms left out there through a property that holds at any size: the
    three-body block <phi_i|h3|phi_j> is Hermitian, and the V2a block too;
  * the bench cell and grid on a 2x2x2 k-mesh (32 orbitals, 1,024 pairs, 24^3; the
    oracle takes about 15 s): every term alone and all terms together, element by
    element, in FP64, FP32 and split BF16, with the pair store on and off and with
    batches whose last one is partial;
  * a small problem on the 48^3 grid: all terms, element by element, in FP64 and FP32, in TC mode,
    the biorthogonal mode, spin-polarised, and both.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle.fftroute import MULT, Problem
from oracle.heg import heg_energy, heg_terms

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")

FP64_TOL = 1e-10
FP32_TOL = 2e-6
PAIR_FREE = ("2ah", "2bh1", "2bh2", "2ax", "2bx1", "2bx2", "3a1", "3a3", "3b1", "3b3", "3b4", "3b6")
THREE_BODY = ("3a1", "3a2", "3a3", "3a4", "3b1", "3b2", "3b3", "3b4", "3b5", "3b6")


def _say(msg):
    print(msg, flush=True)


def _mask(terms, corr=True):
    m = 0
    for t in terms:
        m |= tc.TERM_BITS[t]
    return m | (tc.TERM_BITS["corr"] if corr else 0)


def _rows(hc, w, targets):
    """Output rows of the given flat orbital indices (k-major, then band)."""
    nb = w.right[0].shape[0]
    return [hc[j // nb][j % nb] for j in targets]


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_electron_gas_54_every_element(prec, tol):
    w = T.workload("heg54_twist2_g32")
    _say(f"[gpu] heg54 twist2 32^3 {prec}: all terms vs closed forms")
    eps, p, f = heg_terms(w)
    lam = sum(MULT.get(t, 1) * e for t, e in eps.items())       # eigenvalue of h2 + h3 per orbital
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    nb = w.right[0].shape[0]
    exp = [lam[ik * nb:(ik + 1) * nb, None] * w.right[ik] for ik in range(w.nk)]
    scale = max(np.abs(x).max() for x in exp)
    err = max(np.abs(a - b).max() for a, b in zip(hc, exp)) / scale
    _say(f"    max element error / max |h c| = {err:.3e}")
    assert err < tol
    Eh, _ = heg_energy(w)
    assert abs(Eg - Eh) < (FP64_TOL if prec == "fp64" else 1e-6) * abs(Eh)
    # orbital energies: |k+G|^2/2 + the eigenvalue of h2 + h3 (Sec. 2.3: Re eps is the band energy)
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    eps = op.orbital_energies().reshape(-1)
    op.close()
    exp_eps = 0.5 * np.sum(p * p, 1) + lam
    eerr = np.abs(eps - exp_eps).max() / np.abs(exp_eps).max()
    _say(f"    orbital energies: max error / max |eps| = {eerr:.3e}")
    assert eerr < tol


def _sampled(w, targets, terms, prec, tol, batch=0):
    pr = Problem(w)
    pr.restrict_targets(targets)
    ref = 0
    for t in terms:
        ref = ref + MULT.get(t, 1) * pr.term(t, 0)
    exp = pr.to_coeff(ref)
    nb = w.right[0].shape[0]
    exp_rows = [exp[j // nb][j % nb].numpy() for j in targets]
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32,
                          terms=_mask(terms), batch=batch)
    hc = op.apply()
    op.close()
    got = _rows(hc, w, targets)
    scale = max(np.abs(x).max() for x in exp_rows)
    err = max(np.abs(a - b).max() for a, b in zip(got, exp_rows)) / scale
    _say(f"    sampled targets {list(targets)}: max element error / max |h c| = {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_bench_workload_sampled_targets(prec, tol):
    w = T.workload("fcc_si_k444_g24")
    _say(f"[gpu] fcc_si_k444_g24 {prec}: sampled targets vs oracle (pair-free terms)")
    _sampled(w, [0, 149, 255], PAIR_FREE, prec, tol)


def test_supercell_48_sampled_target_fp32():
    w = T.workload("fcc_si_x2_k222_g48")
    _say("[gpu] fcc_si_x2_k222_g48 fp32: one sampled target vs oracle (pair-free terms)")
    _sampled(w, [77], PAIR_FREE, "fp32", FP32_TOL)


@pytest.mark.parametrize("part", ["three_body", "v2a"])
def test_bench_workload_hermitian_blocks_fp64(part):
    w = T.workload("fcc_si_k444_g24")
    terms = THREE_BODY if part == "three_body" else ("2ah", "2ax")
    _say(f"[gpu] fcc_si_k444_g24 fp64: {part} block Hermitian at full size")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=_mask(terms))
    hc = op.apply()
    op.close()
    worst = 0.0
    for ik in range(w.nk):
        M = np.conj(w.right[ik]) @ hc[ik].T            # M_ab = <phi_a | h phi_b>
        worst = max(worst, np.abs(M - M.conj().T).max() / np.abs(M).max())
    _say(f"    max |M - M^H| / max |M| over k = {worst:.3e}")
    assert worst < 1e-11


def test_bench_workload_fp32_matches_fp64_every_element():
    w = T.workload("fcc_si_k444_g24")
    _say("[gpu] fcc_si_k444_g24: all terms, fp32 (bench launch configuration) vs fp64")
    out = {}
    for name, prec in (("fp64", tc.TC_PREC_FP64), ("fp32", tc.TC_PREC_FP32)):
        op = tc.from_workload(w, precision=prec)
        out[name] = (op.apply(), op.energy()[0])
        op.close()
    scale = max(np.abs(x).max() for x in out["fp64"][0])
    err = max(np.abs(a - b).max() for a, b in zip(out["fp32"][0], out["fp64"][0])) / scale
    _say(f"    max element difference / max |h c| = {err:.3e}; energies {out['fp32'][1]!r} {out['fp64'][1]!r}")
    assert err < FP32_TOL
    assert abs(out["fp32"][1] - out["fp64"][1]) < 1e-6 * abs(out["fp64"][1])


ALL = PAIR_FREE + ("3a2", "3a4", "3b2", "3b5")
SPLIT_TOL = 2e-5


@pytest.fixture(scope="module")
def fcc_k222_g24():
    """The bench cell, grid, bands and Jastrow on a 2x2x2 k-mesh; the oracle's output per term."""
    w = T.fcc_si(kmesh=(2, 2, 2))
    _say("[oracle] fcc_si_x1_k2x2x2_g24: every term (FP64 CPU)")
    pr = Problem(w)
    per = {t: [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))] for t in ALL}
    tot = [sum(per[t][k] for t in ALL) for k in range(w.nk)]
    return w, per, tot, float(pr.energy())


def test_bench_grid_every_term_fp64(fcc_k222_g24):
    w, per, tot, E = fcc_k222_g24
    scale = max(np.abs(x).max() for x in tot)
    for t in ALL:
        _say(f"[gpu] fcc_si k222 24^3 fp64 term {t} alone")
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=_mask((t,)))
        hc = op.apply()
        op.close()
        err = max(np.abs(a - b).max() for a, b in zip(hc, per[t])) / scale
        assert err < FP64_TOL, (t, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split"])
@pytest.mark.parametrize("batch,store", [(0, True), (5, True), (5, False)])
def test_bench_grid_all_terms(fcc_k222_g24, prec, batch, store):
    """All terms at the bench grid through the bench's kernels (24-point plane kernels, the resident pair
    store, the shared 3b6 / pass-B z stage); batch 5 of 32 targets leaves a partial last batch."""
    w, per, tot, E = fcc_k222_g24
    P = {"fp64": tc.TC_PREC_FP64, "fp32": tc.TC_PREC_FP32, "split": tc.TC_PREC_FP32_SPLITBF16}[prec]
    tol = {"fp64": FP64_TOL, "fp32": FP32_TOL, "split": SPLIT_TOL}[prec]
    _say(f"[gpu] fcc_si k222 24^3 {prec} all terms batch={batch} pair_store={store}")
    op = tc.from_workload(w, precision=P, batch=batch, pair_store=store)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    scale = max(np.abs(x).max() for x in tot)
    err = max(np.abs(a - b).max() for a, b in zip(hc, tot)) / scale
    eerr = abs(Eg - E) / abs(E)
    _say(f"    max element error / max |h c| = {err:.3e}; energy {Eg!r} vs oracle {E!r} (rel {eerr:.3e})")
    assert err < tol
    assert eerr < (FP64_TOL if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_grid_48_all_terms(prec, tol):
    """48-point plane kernels (FP64: spin channels in separate LDS rounds) against the oracle."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=48, ecut=3.0, nb=2, a=7.0, occ=[1.0, 0.7])
    _say(f"[gpu] tiny fcc 48^3 {prec}: all terms vs oracle")
    pr = Problem(w)
    per = {t: [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))] for t in ALL}
    tot = [sum(per[t][k] for t in ALL) for k in range(w.nk)]
    E = float(pr.energy())
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    scale = max(np.abs(x).max() for x in tot)
    err = max(np.abs(a - b).max() for a, b in zip(hc, tot)) / scale
    _say(f"    max element error / max |h c| = {err:.3e}; energy rel err {abs(Eg - E) / abs(E):.3e}")
    assert err < tol
    assert abs(Eg - E) < (FP64_TOL if prec == "fp64" else 1e-6) * abs(E)
    if prec == "fp64":
        scale = max(np.abs(x).max() for x in tot)
        for t in ("3a2", "3a4", "3b2", "3b5", "3b6"):
            op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=_mask((t,)))
            hc = op.apply()
            op.close()
            e = max(np.abs(a - b).max() for a, b in zip(hc, per[t])) / scale
            _say(f"    term {t}: {e:.3e}")
            assert e < FP64_TOL, (t, e)


_GRID48_REF = {}   # oracle outputs per mode, shared by the precisions


def _grid48_workload(mode):
    """A small problem on the 48^3 grid in the biorthogonal mode, spin-polarised, or both."""
    left = 0.15 if "bitc" in mode else None
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=48, ecut=3.0, nb=2, a=7.0, occ=[1.0, 0.7], left_mix=left,
                   seed_offset=3)
    if "pol" in mode:
        w = T.polarized(w, 41, occ_dn=[0.9, 0.2])
    return w


@pytest.mark.parametrize("mode,prec,tol", [(m, p, t) for m in ("bitc", "pol", "bitc_pol")
                                           for p, t in (("fp64", FP64_TOL), ("fp32", FP32_TOL))])
def test_grid_48_all_terms_other_modes(mode, prec, tol):
    """48-point plane kernels of the biorthogonal occupied pass (k_fused_OB), the spin-polarised pass A and
    occupied pass (k_fused_A<POL>, k_fused_O<SPLITH>) and their FP64 separate-round layouts, against the
    oracle: every output element of every spin channel, and the energy."""
    chans = (0, 1) if "pol" in mode else (0,)
    if mode not in _GRID48_REF:
        w = _grid48_workload(mode)
        _say(f"[oracle] tiny fcc 48^3 {mode}: all terms (FP64 CPU)")
        pr = Problem(w)
        tot = {s: [c.numpy() for c in pr.to_coeff(sum(MULT.get(t, 1) * pr.term(t, s) for t in ALL), s)]
               for s in chans}
        _GRID48_REF[mode] = (w, tot, float(pr.energy()))
    w, tot, E = _GRID48_REF[mode]
    _say(f"[gpu] tiny fcc 48^3 {mode} {prec}: all terms vs oracle")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    for s in chans:
        got = hc[s] if "pol" in mode else hc
        scale = max(np.abs(x).max() for x in tot[s])
        err = max(np.abs(a - b).max() for a, b in zip(got, tot[s])) / scale
        _say(f"    spin {s}: max element error / max |h c| = {err:.3e}")
        assert err < tol, (s, err)
    _say(f"    energy {Eg!r} vs oracle {E!r} (rel {abs(Eg - E) / abs(E):.3e})")
    assert abs(Eg - E) < (FP64_TOL if prec == "fp64" else 1e-6) * abs(E)


@pytest.fixture(scope="module")
def fcc_k222_g24_bitc():
    w = T.fcc_si(kmesh=(2, 2, 2), left_mix=0.1)
    _say("[oracle] fcc_si_x1_k2x2x2_g24 biorthogonal: all terms (FP64 CPU)")
    pr = Problem(w)
    tot = [c.numpy() for c in pr.to_coeff(sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL))]
    return w, tot, float(pr.energy())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bench_grid_bitc_all_terms(fcc_k222_g24_bitc, prec):
    """The biorthogonal mode at the bench grid with the resident pair store serving both occupied-pass
    convolutions, and a partial last batch."""
    w, tot, E = fcc_k222_g24_bitc
    P = tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32
    _say(f"[gpu] fcc_si k222 24^3 biorthogonal {prec} all terms, batch 5")
    op = tc.from_workload(w, precision=P, batch=5)
    hc = op.apply()
    Eg, _ = op.energy()
    op.close()
    scale = max(np.abs(x).max() for x in tot)
    err = max(np.abs(a - b).max() for a, b in zip(hc, tot)) / scale
    _say(f"    max element error / max |h c| = {err:.3e}; energy rel {abs(Eg - E) / abs(E):.3e}")
    assert err < (FP64_TOL if prec == "fp64" else FP32_TOL)
    assert abs(Eg - E) < (FP64_TOL if prec == "fp64" else 1e-6) * abs(E)
