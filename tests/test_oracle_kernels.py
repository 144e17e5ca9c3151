"""Pins of the oracle's kernels and Gygi-Baldereschi constant against quadrature and textbook values."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy import integrate

import tcinputs as T
from oracle.fftroute import jastrow_kernels, Problem
from oracle.heg import gb_delta

A, C = 1.6389, 1.8104


def radial_ft(f, G):
    """(4 pi / G) int_0^inf r sin(G r) f(r) dr by oscillatory quadrature (QUADPACK QAWF)."""
    val, _ = integrate.quad(lambda r: r * f(r), 0.0, np.inf, weight="sin", wvar=G, limlst=200)
    return 4.0 * math.pi / G * val


def u(r):
    return A / r * (1.0 - math.exp(-r / C))


def du(r):  # d u / d r
    return A * (math.exp(-r / C) / (C * r) - (1.0 - math.exp(-r / C)) / r ** 2)


@pytest.mark.parametrize("G", [0.3, 0.7, 1.5, 3.0])
def test_kernels_match_radial_quadrature(G):
    ut, lap, W = [float(x) for x in jastrow_kernels(torch.tensor([G * G], dtype=torch.float64),
                                                     torch.tensor(A, dtype=torch.float64),
                                                     torch.tensor(C, dtype=torch.float64))]
    # u = A/r - A e^{-r/C}/r: Coulomb part analytic 4 pi A / G^2, Yukawa part by quadrature
    yuk = radial_ft(lambda r: A * math.exp(-r / C) / r if r > 0 else A / C, G)
    assert ut == pytest.approx(4 * math.pi * A / G ** 2 - yuk, rel=1e-8)
    # lap u = (1/r) d^2(r u)/dr^2 = -A e^{-r/C} / (C^2 r)
    q_lap = radial_ft(lambda r: -A * math.exp(-r / C) / (C * C * r) if r > 0 else -A / C ** 3, G)
    assert lap == pytest.approx(q_lap, rel=1e-8)
    # (grad u)^2 = (du/dr)^2, absolutely convergent
    q_w = radial_ft(lambda r: du(r) ** 2 if r > 1e-12 else A * A / (4 * C ** 4), G)
    assert W == pytest.approx(q_w, rel=1e-6)


def test_w_small_g_branch_and_limits():
    Q2 = torch.tensor([1e-14, 1e-10, (0.9e-3 / C) ** 2, (1.1e-3 / C) ** 2, 1e-4], dtype=torch.float64)
    ut, lap, W = jastrow_kernels(Q2, torch.tensor(A, dtype=torch.float64), torch.tensor(C, dtype=torch.float64))
    # W(0) = 2 pi A^2 / C, lap(0) = -4 pi A; linear cusp W ~ 2 pi A^2/C - pi^2 A^2 Q
    assert float(W[0]) == pytest.approx(2 * math.pi * A * A / C - math.pi ** 2 * A * A * 1e-7, rel=1e-12)
    assert float(lap[0]) == pytest.approx(-4 * math.pi * A, rel=1e-12)
    Q = math.sqrt(1e-10)
    assert float(W[1]) == pytest.approx(2 * math.pi * A * A / C - math.pi ** 2 * A * A * Q, rel=1e-9)
    # continuity across the series / closed-form switch
    assert abs(float(W[2]) - float(W[3])) < 1e-3 * float(W[2])


def test_gb_madelung_limit_and_hf_closed_form():
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "heg_hf_exchange.json")))
    w = T.workload("heg14_g16")
    L = w.lattice[0, 0]
    # alpha -> 0: 4 pi Delta_GB / Omega is the simple-cubic Madelung constant / L
    for a in (0.5, 1.0):
        assert 4 * math.pi * gb_delta(w.lattice, w.kmesh, a) / w.omega == pytest.approx(2.837297 / L, rel=3e-7)
    assert 4 * math.pi * gb_delta(w.lattice, w.kmesh, w.alpha) / w.omega == pytest.approx(
        ref["four_pi_dgb_over_omega"], rel=1e-12)
    # Hartree-Fock limit (u = 0) of the FFT-route oracle on the 14-electron gas
    pr = Problem(w.replace(A=(0.0, 0.0)), div_correction=False)
    _, parts = pr.energy(per_term=True, terms=("2ax",))
    assert float(parts["2ax"]) == pytest.approx(ref["exchange_uncorrected_Ha"], rel=1e-12)
    pr = Problem(w.replace(A=(0.0, 0.0)))
    _, parts = pr.energy(per_term=True, terms=("2ax",))
    assert float(parts["2ax"]) == pytest.approx(ref["exchange_corrected_Ha"], rel=1e-12)
    assert float(parts["2ax"]) == pytest.approx(-1.800392, abs=1e-6)


@pytest.mark.parametrize("mesh", [(2, 2, 2), (4, 4, 4), (3, 1, 2)])
def test_gb_vector_correction_vanishes_on_uniform_mesh(mesh):
    w = T.fcc_si(kmesh=(1, 1, 1), grid=8, ecut=1.0, nb=1).replace(kmesh=mesh)
    w = w.replace(miller=w.miller * int(np.prod(mesh)), right=w.right * int(np.prod(mesh)),
                  occ=w.occ * int(np.prod(mesh)))
    pr = Problem(w)
    assert np.max(np.abs(pr.gb_vector)) < 1e-12 * max(1.0, pr.sigma_aux)
