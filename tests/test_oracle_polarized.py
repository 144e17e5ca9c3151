"""Spin-polarised input in the oracle: each spin channel with its own orbitals and fillings.

Pins: the FFT-route oracle O1 equals the literal permutation integrals O2 for targets of both spins
(every two-body term; the three-body terms on one target per spin); identical channels reproduce
the unpolarised results; exchanging the channels exchanges the outputs and keeps the energy.
"""
import numpy as np
import pytest
import torch

import tcinputs as T
from oracle.brute import Brute
from oracle.fftroute import ALL_TERMS, MULT, Problem, TERMS3

C_TO_B = {"1": "1", "2": "2", "3": "6", "4": "5", "5": "4", "6": "3"}


def _pol_cases():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    yield T.polarized(w, 31, occ_dn=[0.9, 0.2])
    wb = T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.15, seed_offset=7)
    yield T.polarized(wb, 32, occ_dn=[1.0, 0.0])


@pytest.mark.parametrize("w", list(_pol_cases()), ids=["tc", "bitc"])
def test_polarized_fftroute_equals_literal_integrals(w):
    pr = Problem(w, div_correction=False)
    up, dn = pr.spin_sets
    wb = w.replace(right_dn=[c.numpy() for c in dn[0]],
                   left_dn=None if dn[1] is None else [c.numpy() for c in dn[1]])
    br = Brute(wb, coeff=[c.numpy() for c in up[0]], left=None if up[1] is None else [c.numpy() for c in up[1]])
    P = pr.P
    for s in (0, 1):
        for j in range(P):
            b2 = br.two_body(j + s * P)
            for t, ref in b2.items():
                g = pr.term(t, s)[j].numpy().reshape(-1)
                assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-300, (s, j, t)
        b3 = br.three_body(s * P)
        for t in TERMS3:
            g = pr.term(t, s)[0].numpy().reshape(-1)
            lit = [t]
            if t == "3a3":
                lit = ["3a3", "3a6"]
            if t == "3a4":
                lit = ["3a4", "3a5"]
            if t[1] == "b":
                lit = [t, "3c" + C_TO_B[t[2]]]
            for name in lit:
                ref = b3[name]
                assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(np.abs(ref)), (s, t, name)


def _outputs(w):
    pr = Problem(w)
    return {s: {t: pr.term(t, s) for t in ALL_TERMS} for s in (0, 1)}, float(pr.energy())


def test_identical_channels_reproduce_unpolarized():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    wp = w.replace(right_dn=list(w.right), occ_dn=list(w.occ))
    o0, E0 = _outputs(w)
    o1, E1 = _outputs(wp)
    assert E1 == pytest.approx(E0, rel=1e-14)
    for s in (0, 1):
        for t in ALL_TERMS:
            torch.testing.assert_close(o1[s][t], o0[0][t], rtol=1e-13, atol=1e-15)


def test_exchanging_channels_exchanges_outputs():
    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]), 9,
                    occ_dn=[0.8, 0.1])
    ws = w.replace(right=w.right_dn, right_dn=w.right, occ=w.occ_dn, occ_dn=w.occ)
    o, E = _outputs(w)
    os_, Es = _outputs(ws)
    assert Es == pytest.approx(E, rel=1e-13)
    for t in ALL_TERMS:
        for s in (0, 1):
            torch.testing.assert_close(os_[1 - s][t], o[s][t], rtol=1e-12, atol=1e-14)
