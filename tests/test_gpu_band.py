"""Band (zero-weight) k-points off the SCF mesh through the C ABI (tc_apply_band).

Against the FP64 oracle, whose band orbitals are targets of every term and partners of none: every term
and the total on random off-mesh k-points (FP64), the total and the orbital energies in FP32, without and
with the band forms of the divergence corrections.
Independent of the oracle: a band k-point placed on a mesh k-point with that k-point's orbitals gives the
mesh result, also when shifted by a reciprocal lattice vector with its plane waves shifted back.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")

FP64_TOL = 1e-10
FP32_TOL = 2e-6


def _say(msg):
    print(msg, flush=True)


def relerr(a, b):
    scale = max(np.abs(x).max() for x in b)
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / scale


def _band_kinetic(w):
    B = T.reciprocal(w.lattice)
    out = []
    for kf, m, c in zip(w.band_k, w.band_miller, w.band_right):
        kg = (np.asarray(kf)[None, :] + np.asarray(m)) @ B
        out.append(np.sum(np.abs(c) ** 2 * 0.5 * np.sum(kg * kg, 1)[None, :], 1))
    return np.stack(out)


CASES = {
    "fcc_k211_g8_band3": lambda: T.with_band(
        T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]),
        [[0.13, 0.27, 0.41], [0.5, 0.25, 0.0], [-0.2, 0.6, 0.35]], seed=5, ecut=2.0, occ=[1.0, 0.5]),
    "fcc_k221_g12_band2": lambda: T.with_band(
        T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.8, 0.0], seed_offset=5),
        [[0.31, -0.12, 0.07], [0.75, 0.5, 0.25]], seed=6, ecut=2.0, nb=2),
}


@pytest.fixture(scope="module", params=[(c, d) for c in CASES for d in (False, True)],
                ids=[f"{c}-{'corr' if d else 'nocorr'}" for c in CASES for d in (False, True)])
def case(request):
    name, div = request.param
    w = CASES[name]()
    pr = Problem(w, div_correction=div)
    nk = w.nk
    per = {t: [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))][nk:] for t in ALL_TERMS}
    tot = [sum(per[t][b] for t in ALL_TERMS) for b in range(len(w.band_k))]
    g = sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL_TERMS)
    eps = pr.braket(0, g).numpy()[pr.Pm:].reshape(len(w.band_k), -1) + _band_kinetic(w)
    return f"{name}-{'corr' if div else 'nocorr'}", div, w, per, tot, eps


def test_every_term_fp64(case):
    name, div, w, per, tot, eps = case
    scale = max(np.abs(x).max() for x in tot)
    for t in ALL_TERMS:
        _say(f"[gpu] band {name} fp64 term {t}")
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=tc.TERM_BITS[t] | tc.TERM_BITS["corr"],
                              div_correction=div)
        got, _ = op.apply_band()
        op.close()
        err = max(np.abs(g - r).max() for g, r in zip(got, per[t])) / scale
        assert err < FP64_TOL, (t, err)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_total_and_orbital_energies(case, prec, tol):
    name, div, w, per, tot, eps = case
    _say(f"[gpu] band {name} {prec} total")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32, div_correction=div)
    got, eg = op.apply_band()
    op.close()
    err = relerr(got, tot)
    erre = np.abs(eg - eps).max() / np.abs(eps).max()
    _say(f"    max |H c - oracle| / max = {err:.3e}, orbital energies {erre:.3e}")
    assert err < tol
    assert erre < tol


def test_band_point_on_the_mesh_and_shifted():
    w0 = T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.8, 0.0], seed_offset=5)
    k = 3
    w = T.with_band(w0, [w0.kfrac[k], w0.kfrac[k] + np.array([1.0, 0.0, -1.0])], source=[k, k],
                    shift=[[0, 0, 0], [1, 0, -1]])
    _say("[gpu] band: points on the mesh")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64, div_correction=False)
    mesh = op.apply()
    em = op.orbital_energies()
    got, eg = op.apply_band()
    op.close()
    for b in range(2):
        assert np.abs(got[b] - mesh[k]).max() < 1e-12 * np.abs(mesh[k]).max()
        assert np.abs(eg[b] - em[k]).max() < 1e-12 * np.abs(em[k]).max()


def test_band_rejections():
    w = CASES["fcc_k211_g8_band3"]()
    _say("[gpu] band: rejections")
    # with corrections, a band k-point on the mesh (modulo G) is the mesh k-point
    w0 = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    wm = T.with_band(w0, [w0.kfrac[1] + np.array([0.0, 1.0, 0.0])], source=[1], shift=[[0, 1, 0]])
    op = tc.from_workload(wm, precision=tc.TC_PREC_FP64, div_correction=True)
    with pytest.raises(tc.TCError, match="on the mesh"):
        op.apply_band()
    op.close()
    op = tc.from_workload(w.replace(band_k=None), precision=tc.TC_PREC_FP64, div_correction=False)
    with pytest.raises(tc.TCError, match="no band"):
        op._check(op._L.tc_apply_band(op._h, None, None), "tc_apply_band")
    op.close()
