"""Shifted Monkhorst-Pack k-meshes in the oracle (k = (i + s) / n, Sec. "Functionalities" of the TC++
description: meshes with or without a shift).

Pins: the FFT-route oracle equals the literal permutation integrals O2 for every term on a shifted mesh
(TC and BITC); on the electron gas with a shifted twist grid every term is the plane-wave closed form
(O3); the Gygi-Baldereschi constant depends on mesh differences only, so the shift leaves it unchanged.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle.brute import Brute
from oracle.fftroute import Problem, TERMS3
from oracle.heg import heg_energy, heg_terms

C_TO_B = {"1": "1", "2": "2", "3": "6", "4": "5", "5": "4", "6": "3"}
SHIFT = (0.5, 0.5, 0.5)


def _cases():
    yield T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7], kshift=SHIFT)
    yield T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.15,
                     seed_offset=7, kshift=(0.5, 0.0, 0.25))


@pytest.mark.parametrize("w", list(_cases()), ids=["tc", "bitc"])
def test_shifted_mesh_fftroute_equals_literal_integrals(w):
    pr = Problem(w, div_correction=False)
    assert np.allclose(pr.kfrac[0], np.asarray(w.kshift) / np.asarray(w.kmesh))
    br = Brute(w, coeff=[c.numpy() for c in pr.cr], left=None if pr.cl is None else [c.numpy() for c in pr.cl])
    for j in range(pr.P):
        for t, ref in br.two_body(j).items():
            g = pr.term(t, 0)[j].numpy().reshape(-1)
            assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-300, t
    b3 = br.three_body(0)
    for t in TERMS3:
        g = pr.term(t, 0)[0].numpy().reshape(-1)
        lit = {"3a3": ["3a3", "3a6"], "3a4": ["3a4", "3a5"]}.get(t, [t] if t[1] == "a" else [t, "3c" + C_TO_B[t[2]]])
        for name in lit:
            ref = b3[name]
            assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(np.abs(ref)), (t, name)


@pytest.mark.parametrize("reading", ["printed", "limit"])
def test_electron_gas_on_a_shifted_twist_grid_matches_the_closed_forms(reading):
    w = T.heg_twist(rs=2.0, nelec=10, tw=2, grid=12, ecut=3.0, nocc=3, kshift=SHIFT)
    w = w.replace(occ=[np.array([1.0, 0.8, 0.5]) for _ in w.occ])
    pr = Problem(w, reading=reading)
    eps, p, f = heg_terms(w, reading=reading)
    for t in eps:
        g = pr.term(t, 0)
        for j in range(pr.P):
            ref = eps[t][j] * pr.orb[0]["phi"][j]
            err = float(np.max(np.abs((g[j] - ref).numpy())))
            assert err <= 1e-11 * max(1.0, float(np.max(np.abs(ref.numpy())))), (t, j)
    E, _ = heg_energy(w, reading=reading)
    assert float(pr.energy()) == pytest.approx(E, rel=1e-12)
    # the shift matters: the twist grid's plane-wave momenta are not those of the unshifted grid
    w0 = T.heg_twist(rs=2.0, nelec=10, tw=2, grid=12, ecut=3.0, nocc=3)
    w0 = w0.replace(occ=[np.array([1.0, 0.8, 0.5]) for _ in w0.occ])
    assert abs(heg_energy(w0, reading=reading)[0] - E) > 1e-4 * abs(E)


def test_gb_constant_is_shift_independent():
    w0 = T.tiny_fcc(kmesh=(2, 2, 1), grid=8, ecut=1.5, nb=1, a=6.0)
    w1 = T.tiny_fcc(kmesh=(2, 2, 1), grid=8, ecut=1.5, nb=1, a=6.0, kshift=SHIFT)
    p0, p1 = Problem(w0), Problem(w1)
    assert p1.delta_gb == pytest.approx(p0.delta_gb, rel=1e-14)
    assert p1.sigma_aux == pytest.approx(p0.sigma_aux, rel=1e-14)
