"""Crystal symmetry: the transformation laws used by the symmetry-reduced path, pinned on the FP64 oracle.

The synthetic orbitals are invariant under the 48 operations of the diamond structure on the fcc lattice
(x -> R (x + tau), half of them with tau = R^-1 (1/4, 1/4, 1/4)).  The oracle computes everything for
every k-point without symmetry; its results must obey the relations of Sec. 2.6.1 (orbitals) and
Sec. 2.6.4 (the h5 field of Alg. 3a2 and the vector field h3 of Alg. 3a4, with the operation applied to
the vector), which the library uses to compute only the representatives:
  h5_k(n)  = h5_k0((R n + R N tau) mod N),
  h3_k(n)  = exp(2 pi i b.n / N) S^T h3_k0((R n + R N tau) mod N),   S = L^T R L^-T,
  (H c)_k  = the image of (H c)_k0, as the orbitals.
"""
import math

import numpy as np
import pytest
import torch

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem


@pytest.fixture(scope="module")
def sym_case():
    base = T.tiny_fcc(kmesh=(2, 2, 2), grid=12, ecut=2.0, nb=4, a=6.0)
    ops = T.diamond_ops(base.lattice)
    w = T.symmetric_orbitals(base, ops, 4242)
    rep, opi, bb = T.k_orbits(ops, w.kmesh)
    pr = Problem(w, div_correction=False)
    return w, ops, rep, opi, bb, pr


def _perm(R, tau, N):
    """Flat source index of (R n + R N tau) mod N for every grid point n (C order [n1][n2][n3])."""
    n = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 3)
    v = np.rint(R @ (np.asarray(tau) * N)).astype(int)
    m = np.mod(n @ R.T + v[None, :], N)
    return (m[:, 0] * N + m[:, 1]) * N + m[:, 2], n


def test_ops_form_a_group_and_reduce_the_mesh(sym_case):
    w, ops, rep, opi, bb, pr = sym_case
    assert len(ops) == 48
    for R, tau in ops:
        S = w.lattice.T @ R @ np.linalg.inv(w.lattice.T)
        np.testing.assert_allclose(S @ S.T, np.eye(3), atol=1e-12)
    assert sorted(set(rep)) == [0, 1, 3]          # Gamma, L and X orbits of the 2x2x2 mesh


def test_density_is_invariant(sym_case):
    w, ops, rep, opi, bb, pr = sym_case
    N = w.grid[0]
    n = pr.n[0].numpy().reshape(-1)
    for R, tau in ops:
        src, _ = _perm(R, tau, N)
        np.testing.assert_allclose(n[src], n, rtol=0, atol=1e-13 * np.abs(n).max())


def test_h5_and_h3_transformation_laws(sym_case):
    w, ops, rep, opi, bb, pr = sym_case
    N = w.grid[0]
    nb = w.nband
    for k in range(w.nk):
        if rep[k] == k:
            continue
        R, tau = ops[opi[k]]
        src, n = _perm(R, tau, N)
        St = np.linalg.inv(w.lattice) @ R.T @ w.lattice          # S^T
        phase = np.exp(2j * math.pi * (n @ bb[k]) / N)
        for mu in range(nb):
            q, q0 = k * nb + mu, rep[k] * nb + mu
            h5 = pr.h5_3a2(0, q, 0).numpy().reshape(-1)
            h50 = pr.h5_3a2(0, q0, 0).numpy().reshape(-1)
            np.testing.assert_allclose(h50[src], h5, rtol=0, atol=1e-12 * np.abs(h5).max())
            h3 = pr.h3_3a4(0, q).numpy().reshape(3, -1)
            h30 = pr.h3_3a4(0, q0).numpy().reshape(3, -1)
            img = phase[None, :] * (St @ h30[:, src])
            np.testing.assert_allclose(img, h3, rtol=0, atol=1e-12 * np.abs(h3).max())


def test_operator_output_follows_the_orbitals(sym_case):
    w, ops, rep, opi, bb, pr = sym_case
    prd = Problem(w)   # with the divergence corrections
    out = prd.to_coeff(sum(MULT.get(t, 1) * prd.term(t, 0) for t in ALL_TERMS))
    for k in range(w.nk):
        if rep[k] == k:
            continue
        R, tau = ops[opi[k]]
        g0, ph = T.image_map(R, tau, bb[k], w.miller[rep[k]], w.miller[k])
        ref = out[k].numpy()
        img = out[rep[k]].numpy()[:, g0] * ph[None, :]
        np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_generated_orbitals_are_the_images(sym_case):
    w, ops, rep, opi, bb, pr = sym_case
    for k in range(w.nk):
        R, tau = ops[max(opi[k], 0)] if opi[k] >= 0 else (np.eye(3, dtype=int), np.zeros(3))
        g0, ph = T.image_map(R, tau, bb[k], w.miller[rep[k]], w.miller[k])
        np.testing.assert_array_equal(w.right[k], w.right[rep[k]][:, g0] * ph[None, :])
