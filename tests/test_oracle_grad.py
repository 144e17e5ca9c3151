"""The oracle gradient (autograd of the discrete energy) against central finite differences, h = 1e-5."""
import numpy as np
import pytest
import torch

import tcinputs as T
from oracle import grad as OG


@pytest.fixture(scope="module")
def case():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6])
    return w, OG.energy_and_grad(w)


def test_orbital_gradient_matches_central_differences(case):
    w, (E, gc, gA, gC) = case
    rng = np.random.default_rng(1)
    h = 1e-5
    for trial in range(3):
        d = [rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape) for c in w.right]
        ep = OG.energy(w, coeff=[c + h * x for c, x in zip(w.right, d)])
        em = OG.energy(w, coeff=[c - h * x for c, x in zip(w.right, d)])
        fd = (ep - em) / (2 * h)
        an = sum(np.sum((np.conj(g) * x).real) for g, x in zip(gc, d))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("which", ["A0", "A1", "C0", "C1"])
def test_jastrow_parameter_gradient(case, which):
    w, (E, gc, gA, gC) = case
    h = 1e-5
    A = np.array(w.A, dtype=float)
    C = np.array(w.C, dtype=float)
    i = int(which[1])
    if which[0] == "A":
        Ap, Am = A.copy(), A.copy()
        Ap[i] += h
        Am[i] -= h
        fd = (OG.energy(w, A=Ap, C=C) - OG.energy(w, A=Am, C=C)) / (2 * h)
        assert gA[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    else:
        Cp, Cm = C.copy(), C.copy()
        Cp[i] += h
        Cm[i] -= h
        fd = (OG.energy(w, A=A, C=Cp) - OG.energy(w, A=A, C=Cm)) / (2 * h)
        assert gC[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------- biorthogonal mode
@pytest.fixture(scope="module")
def bitc_case():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.2)
    r, l = OG.bitc_pair(w)
    return w, r, l, OG.energy_and_grad_bitc(w, r, l)


@pytest.mark.parametrize("side", ["right", "left"])
def test_bitc_gradients_match_central_differences(bitc_case, side):
    w, r, l, (E, gr, gl, dA, dC) = bitc_case
    rng = np.random.default_rng(5 if side == "right" else 6)
    g = gr if side == "right" else gl
    d = [0.3 * (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)) for c in r]
    h = 1e-5
    e = []
    for sgn in (1, -1):
        rr = [a + sgn * h * b for a, b in zip(r, d)] if side == "right" else r
        ll = [a + sgn * h * b for a, b in zip(l, d)] if side == "left" else l
        e.append(OG.energy_bitc(w, rr, ll))
    fd = (e[0] - e[1]) / (2 * h)
    an = sum(np.sum((np.conj(gk) * dk).real) for gk, dk in zip(g, d))
    assert an == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_bitc_gradient_reduces_to_tc_when_left_equals_right():
    """E_TC(c) = E_BITC(c, c): the two partial gradients add up to the TC gradient."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6])
    E0, g0, _, _ = OG.energy_and_grad(w)
    E, gr, gl, _, _ = OG.energy_and_grad_bitc(w, w.right, w.right)
    assert E == pytest.approx(E0, rel=1e-13)
    for a, b, c in zip(gr, gl, g0):
        np.testing.assert_allclose(a + b, c, atol=1e-12 * np.abs(c).max())


# ---------------------------------------------------------------- spin-polarised channels
@pytest.fixture(scope="module")
def pol_case():
    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6]), 41,
                    occ_dn=[0.9, 0.3])
    return w, OG.energy_and_grad_polarized(w)


@pytest.mark.parametrize("side", ["up", "dn"])
def test_polarized_gradient_matches_central_differences(pol_case, side):
    w, (E, gu, gd, gA, gC) = pol_case
    rng = np.random.default_rng(11 if side == "up" else 12)
    h = 1e-5
    base = w.right if side == "up" else w.right_dn
    g = gu if side == "up" else gd
    for trial in range(2):
        d = [rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape) for c in base]
        plus = [c + h * x for c, x in zip(base, d)]
        minus = [c - h * x for c, x in zip(base, d)]
        if side == "up":
            fd = (OG.energy_polarized(w, up=plus) - OG.energy_polarized(w, up=minus)) / (2 * h)
        else:
            fd = (OG.energy_polarized(w, dn=plus) - OG.energy_polarized(w, dn=minus)) / (2 * h)
        an = sum(np.sum((np.conj(a) * x).real) for a, x in zip(g, d))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9)
    Ap = np.array(w.A, dtype=float)
    Am = Ap.copy()
    Ap[0] += h
    Am[0] -= h
    fdA = (OG.energy_polarized(w, A=Ap, C=np.array(w.C)) - OG.energy_polarized(w, A=Am, C=np.array(w.C))) / (2 * h)
    assert gA[0] == pytest.approx(fdA, rel=1e-6, abs=1e-9)


def test_equal_channels_share_the_unpolarized_gradient():
    """Two identical channels: each channel's gradient is half of the unpolarised one (which differentiates
    the coefficients that both spins share), and dA, dC are the same."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6])
    E0, g0, gA0, gC0 = OG.energy_and_grad(w)
    wp = w.replace(right_dn=[c.copy() for c in w.right], occ_dn=[o.copy() for o in w.occ])
    E, gu, gd, gA, gC = OG.energy_and_grad_polarized(wp)
    assert E == pytest.approx(E0, rel=1e-13)
    for a, b, c in zip(gu, gd, g0):
        np.testing.assert_allclose(a + b, c, rtol=0, atol=1e-12 * np.abs(c).max())
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(c).max())
    np.testing.assert_allclose(gA, gA0, rtol=1e-12)
    np.testing.assert_allclose(gC, gC0, rtol=1e-12)


@pytest.fixture(scope="module")
def bitc_pol_case():
    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.15,
                               seed_offset=7), 43, occ_dn=[0.9, 0.3])
    pairs = OG.bitc_pair_polarized(w)
    return w, pairs, OG.energy_and_grad_bitc_polarized(w, *pairs)


def _energy_bitc_pol(w, ru, lu, rd, ld):
    from oracle.fftroute import CD, Problem

    with torch.no_grad():
        t = lambda x: [torch.as_tensor(c, dtype=CD) for c in x]
        return float(Problem(w, coeff=t(ru), left=t(lu), coeff_dn=t(rd), left_dn=t(ld),
                             biorthogonalize=False).energy())


@pytest.mark.parametrize("which", [0, 1, 2, 3], ids=["right_up", "left_up", "right_dn", "left_dn"])
def test_bitc_polarized_gradients_match_central_differences(bitc_pol_case, which):
    """Each of the four partial gradients of the spin-polarised biorthogonal energy (pairs held fixed)
    against central differences along random directions."""
    w, pairs, res = bitc_pol_case
    g = res[1 + which]
    rng = np.random.default_rng(50 + which)
    h = 1e-5
    d = [rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape) for c in pairs[which]]
    e = []
    for sgn in (1, -1):
        p = [list(x) for x in pairs]
        p[which] = [c + sgn * h * x for c, x in zip(pairs[which], d)]
        e.append(_energy_bitc_pol(w, *p))
    fd = (e[0] - e[1]) / (2 * h)
    an = sum(np.sum((np.conj(a) * x).real) for a, x in zip(g, d))
    assert an == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_bitc_polarized_equal_channels_share_the_unpolarized_gradients():
    """Two identical biorthogonal channels: each channel's right and left gradients are half of the
    unpolarised ones (whose pair both spins share); E, dA and dC are the same."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6], left_mix=0.15, seed_offset=7)
    r, l = OG.bitc_pair(w)
    E0, gr0, gl0, gA0, gC0 = OG.energy_and_grad_bitc(w, r, l)
    wp = w.replace(right_dn=[c.copy() for c in w.right], left_dn=[c.copy() for c in w.left],
                   occ_dn=[o.copy() for o in w.occ])
    E, gru, glu, grd, gld, gA, gC = OG.energy_and_grad_bitc_polarized(wp, r, l, r, l)
    assert E == pytest.approx(E0, rel=1e-13)
    for up, dn, ref in ((gru, grd, gr0), (glu, gld, gl0)):
        for a, b, c in zip(up, dn, ref):
            np.testing.assert_allclose(a + b, c, rtol=0, atol=1e-12 * np.abs(c).max())
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(c).max())
    np.testing.assert_allclose(gA, gA0, rtol=1e-12)
    np.testing.assert_allclose(gC, gC0, rtol=1e-12)
