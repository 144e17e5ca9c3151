"""Band (zero-weight) k-points in the FP64 oracle, and the band forms of the divergence corrections.

Pins (no GPU), with band orbitals carried over from a mesh k-point k0 to k = k0 + delta d:
  * on the mesh (delta = 0, corrections off) and shifted by a reciprocal lattice vector, every term of a
    band orbital equals the mesh one (the shift is never reduced modulo G);
  * every singular exchange sum is regularised: without corrections the band operator diverges as
    delta -> 0 (1/delta^2 or 1/delta), with them it has a finite limit (its sign and size are what
    cancel the divergence, readings R13, R14);
  * where the partner factor at the singular point does not depend on the partner's momentum (2ax,
    2bx2, 3a3, 3b3, 3b4) the limit is the mesh operator itself, linearly in delta;
  * 2bx1: the limit is the mesh operator plus the isotropic remainder -(4 pi A / N_k) sum_mu f
    rho~_{mu j}(0) phi_mu of (nabla + ik) acting on the partner's Bloch phase; the printed mesh form has no
    on-mesh correction, the "limit" reading (R4) adds exactly this remainder;
  * electron gas (uniform density, plane waves): 3b6 tends to the mesh operator of the "limit" reading
    (two u~_short(0)/N_k in its G = G' = 0 correction), and the printed mesh operator (one) misses it by
    the u~_short term (reading R4).
"""
import math

import numpy as np
import pytest
import torch

import tcinputs as T
from oracle.fftroute import ALL_TERMS, FOURPI, MULT, Problem

D = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
SINGULAR = ("2ax", "2bx1", "2bx2", "3a3", "3a4", "3b3", "3b4", "3b5", "3b6")
MOMENTUM_FREE = ("2ax", "2bx2", "3a3", "3b3", "3b4")


def _fcc():
    return T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])


def _band_out(w0, k0, delta, terms, div=True, reading="printed"):
    w = T.with_band(w0, [w0.kfrac[k0] + delta * D], source=[k0])
    pr = Problem(w, div_correction=div, reading=reading)
    return {t: pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))[w0.nk].numpy() for t in terms}


def _mesh_out(w0, k0, terms, div=True, reading="printed"):
    pr = Problem(w0, div_correction=div, reading=reading)
    return {t: pr.to_coeff(MULT.get(t, 1) * pr.term(t, 0))[k0].numpy() for t in terms}


def test_band_point_on_the_mesh_and_shifted():
    w0 = _fcc()
    k0 = 1
    w = T.with_band(w0, [w0.kfrac[k0], w0.kfrac[k0] + np.array([1.0, -1.0, 0.0])], source=[k0, k0],
                    shift=[[0, 0, 0], [1, -1, 0]])
    pr = Problem(w, div_correction=False)
    for t in ALL_TERMS:
        g = pr.to_coeff(pr.term(t, 0))
        ref = g[k0].numpy()
        sc = max(np.abs(ref).max(), 1e-300)
        for b in (0, 1):
            assert np.abs(g[w0.nk + b].numpy() - ref).max() <= 1e-13 * sc + 1e-300, (t, b)


@pytest.fixture(scope="module")
def fcc_limits():
    w0 = _fcc()
    k0 = 1
    return w0, k0, _mesh_out(w0, k0, ALL_TERMS), {d: _band_out(w0, k0, d, ALL_TERMS) for d in (1e-3, 1e-4, 1e-5)}


def test_corrections_remove_the_divergences(fcc_limits):
    w0, k0, mesh, band = fcc_limits
    raw = {d: _band_out(w0, k0, d, SINGULAR, div=False) for d in (1e-3, 1e-4)}
    for t in SINGULAR:
        sc = np.abs(mesh[t]).max()
        # without corrections: at least a 1/delta growth
        grow = np.abs(raw[1e-4][t] - mesh[t]).max() / np.abs(raw[1e-3][t] - mesh[t]).max()
        assert grow > 8.0, (t, grow)
        # with them: a finite limit (Cauchy in delta)
        step = np.abs(band[1e-4][t] - band[1e-5][t]).max()
        assert step < 1e-3 * max(sc, np.abs(band[1e-5][t]).max()), (t, step)


def test_momentum_free_terms_tend_to_the_mesh_operator(fcc_limits):
    w0, k0, mesh, band = fcc_limits
    for t in MOMENTUM_FREE:
        sc = np.abs(mesh[t]).max()
        e3 = np.abs(band[1e-3][t] - mesh[t]).max() / sc
        e4 = np.abs(band[1e-4][t] - mesh[t]).max() / sc
        assert e4 < 0.15 * e3 and e4 < 1e-3, (t, e3, e4)


def test_2bx1_limit_is_the_mesh_operator_plus_the_isotropic_remainder(fcc_limits):
    w0, k0, mesh, band = fcc_limits
    ref = Problem(w0)
    o = ref.orb[0]
    Q = ref.sel(0, k0)
    rem = []
    for j in Q:
        r0 = ref.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])
        rem.append(-FOURPI * ref.A[0] / ref.nk * torch.sum((o["f"][Q] * r0)[:, None, None, None] * o["phi"][Q], 0))
    full = torch.zeros_like(o["phi"])
    full[torch.as_tensor(Q)] = torch.stack(rem)
    P = ref.to_coeff(full)[k0].numpy()
    err = np.abs(band[1e-5]["2bx1"] - mesh["2bx1"] - P).max() / np.abs(P).max()
    assert err < 1e-3, err
    # the "limit" reading's mesh operator is that limit (its remainder is the one derived above)
    lim = _mesh_out(w0, k0, ("2bx1",), reading="limit")["2bx1"]
    assert np.abs(lim - mesh["2bx1"] - P).max() <= 1e-12 * np.abs(P).max()
    err = np.abs(band[1e-5]["2bx1"] - lim).max() / np.abs(lim).max()
    assert err < 1e-3, err


def test_heg_3b6_band_limit_fixes_the_readings():
    """Plane waves: the 3b6 sum is isotropic at its singular point, so the band operator of
    Eq. 3b6_div_band1 tends to the mesh operator exactly when the mesh correction holds the full finite
    remainder 2 (4 pi A) u~_short(0) of Q^2 u~(Q)^2 (the "limit" reading).  The printed coefficient (one
    u~_short(0)/N_k) leaves a finite gap."""
    w0 = T.heg_gamma(rs=2.0, nelec=14, grid=16, mmax2=9, occ_m2=1)
    mesh = _mesh_out(w0, 0, ("3b6", "2ax"), reading="limit")
    printed = _mesh_out(w0, 0, ("3b6", "2ax"), reading="printed")
    e = {}
    for d in (1e-3, 1e-4):
        b = _band_out(w0, 0, d, ("3b6", "2ax"))   # band forms: the same in both readings
        e[d] = {t: np.abs(b[t] - mesh[t]).max() / np.abs(mesh[t]).max() for t in b}
    for t in ("3b6", "2ax"):
        assert e[1e-4][t] < 0.15 * e[1e-3][t] and e[1e-4][t] < 1e-3, (t, e)
    assert np.abs(printed["2ax"] - mesh["2ax"]).max() == 0.0
    gap = np.abs(printed["3b6"] - mesh["3b6"]).max() / np.abs(mesh["3b6"]).max()
    assert gap > 1e-2, gap
