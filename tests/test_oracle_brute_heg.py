"""The FFT-route oracle against the literal permutation integrals (brute force) and the plane-wave closed forms."""
import numpy as np
import pytest

import tcinputs as T
from oracle.brute import Brute
from oracle.fftroute import Problem, TERMS3
from oracle.heg import heg_energy, heg_terms

# 3c_k equals 3b_{k'} after x2 <-> x3, q1 <-> q2 (Sec. 2.6.4)
C_TO_B = {"1": "1", "2": "2", "3": "6", "4": "5", "5": "4", "6": "3"}


def _cases():
    yield T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    yield T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.15,
                     seed_offset=7)


@pytest.mark.parametrize("w", list(_cases()), ids=["tc", "bitc"])
def test_fftroute_equals_literal_permutation_integrals(w):
    pr = Problem(w, div_correction=False)
    br = Brute(w, coeff=[c.numpy() for c in pr.cr], left=None if pr.cl is None else [c.numpy() for c in pr.cl])
    for j in range(pr.P):
        b2 = br.two_body(j)
        for t, ref in b2.items():
            g = pr.term(t, 0)[j].numpy().reshape(-1)
            assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-300, t
    for j in (0, pr.P - 1):
        b3 = br.three_body(j)
        for t in TERMS3:
            g = pr.term(t, 0)[j].numpy().reshape(-1)
            lit = [t] if t[1] == "b" else [t]
            if t == "3a3":
                lit = ["3a3", "3a6"]
            if t == "3a4":
                lit = ["3a4", "3a5"]
            if t[1] == "b":
                lit = [t, "3c" + C_TO_B[t[2]]]
            for name in lit:
                ref = b3[name]
                assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(np.abs(ref)), (t, name)


@pytest.mark.parametrize("reading", ["printed", "limit"])
def test_electron_gas_gamma_every_term_closed_form(reading):
    w = T.workload("heg14_g16")
    E, parts = Problem(w, reading=reading).energy(per_term=True)
    Eh, ph = heg_energy(w, reading=reading)
    for k, v in ph.items():
        assert float(parts[k]) == pytest.approx(v, abs=1e-12 * max(1.0, abs(Eh))), k
    assert float(E) == pytest.approx(Eh, rel=1e-12)


@pytest.mark.parametrize("reading", ["printed", "limit"])
def test_electron_gas_twists_operator_is_diagonal_and_matches(reading):
    # 2x2x2 twists, the 3 lowest |k+G|^2 plane waves per twist, partially filled
    w = T.heg_twist(rs=2.0, nelec=10, tw=2, grid=12, ecut=3.0, nocc=3)
    w = w.replace(occ=[np.array([1.0, 0.8, 0.5]) for _ in w.occ])
    pr = Problem(w, reading=reading)
    eps, p, f = heg_terms(w, reading=reading)
    for t in eps:
        g = pr.term(t, 0)
        for j in range(pr.P):
            phi = pr.orb[0]["phi"][j]
            ref = eps[t][j] * phi
            err = float(np.max(np.abs((g[j] - ref).numpy())))
            assert err <= 1e-11 * max(1.0, float(np.max(np.abs(ref.numpy())))), (t, j)
