"""Pins of the SCF oracle (O5, exact diagonalisation per iteration) on the electron gas.

Plane waves solve the SCF equation of the electron gas, so from a perturbed start the loop must
return to the occupied plane waves and the energy of the closed forms (O3), in the TC mode and in the
biorthogonal mode (which coincides with TC for the electron gas, Sec. 4.2).
"""
import numpy as np
import pytest

import tcinputs as T
from oracle import scf as S
from oracle.heg import heg_energy


@pytest.fixture(scope="module")
def heg2():
    # 2 electrons (one doubly occupied plane wave, m = 0) in the basis |m|^2 <= 1, 8^3 grid
    return T.heg_gamma(rs=4.0, nelec=2, grid=8, mmax2=1, occ_m2=0)


@pytest.mark.parametrize("left_amp", [None, 0.3])
def test_heg2_returns_to_the_plane_wave(heg2, left_amp):
    E0, _ = heg_energy(heg2)
    start = T.perturbed_start(heg2, 0.4, 3, left_amp=left_amp)
    hist, right, left, evals, Ef = S.scf(start, max_iter=60, etol=1e-14)
    assert abs(Ef - E0) < 1e-12 * abs(E0) + 1e-14
    c = right[0][0]
    assert abs(abs(c[0]) - 1.0) < 1e-6 and np.abs(c[1:]).max() < 1e-6
    assert abs(hist[0] - E0) > 1e-4                                   # the start was away from it


def test_operator_matrix_of_plane_waves_is_diagonal(heg2):
    H = S.operator_matrices(heg2, heg2.right)[0]
    off = H - np.diag(np.diag(H))
    assert np.abs(off).max() < 1e-12 * np.abs(H).max()


@pytest.mark.parametrize("reading", ["printed", "limit"])
def test_operator_matrix_diagonal_is_the_closed_form(heg2, reading):
    """Pins the coefficient-space output of the FFT-route oracle (to_coeff: sqrt(Omega), 1/N_r and the
    plane-wave gather): every diagonal element of [T + h] on the plane-wave set equals |p|^2/2 plus the
    closed-form eigenvalue of that plane wave as a zero-filling target (O3, no grid and no FFT)."""
    from oracle.fftroute import MULT
    from oracle.heg import heg_terms

    H = S.operator_matrices(heg2, heg2.right, reading=reading)[0]
    npw = heg2.miller[0].shape[0]
    E = np.eye(npw, dtype=np.complex128)
    wx = heg2.replace(right=[np.concatenate([heg2.right[0], E])],
                      occ=[np.concatenate([np.asarray(heg2.occ[0], float), np.zeros(npw)])])
    eps, p, f = heg_terms(wx, reading=reading)
    nb = heg2.right[0].shape[0]
    lam = sum(MULT.get(t, 1) * e for t, e in eps.items())[nb:]
    ref = 0.5 * np.sum(p[nb:] ** 2, 1) + lam
    assert np.abs(np.diag(H) - ref).max() < 1e-12 * np.abs(ref).max()
    # the closed forms differ between the plane waves, so a wrong scale of any entry shows
    assert np.ptp(ref.real) > 1e-2 * np.abs(ref).max()


def test_polarized_operator_matrices_with_equal_channels():
    """The per-channel plane-wave matrices of a polarised workload with two identical channels are the
    unpolarised matrix, for both channels."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=6, ecut=1.5, nb=1, a=6.0)
    wp = w.replace(right_dn=[c.copy() for c in w.right], occ_dn=[o.copy() for o in w.occ])
    H0 = S.operator_matrices(w, w.right)
    for s in (0, 1):
        Hs = S.operator_matrices(wp, wp.right, spin=s)
        for a, b in zip(Hs, H0):
            assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
